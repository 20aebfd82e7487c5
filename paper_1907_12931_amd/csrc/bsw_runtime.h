// bsw_runtime.h -- host-side internals shared by the runtime (bsw_host.cpp)
// and the serving loop (bsw_server.cpp).  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/bsw.h"
#include "bsw_internal.h"

namespace bsw {

// Device pointers of one call.
struct Args {
  int64_t n;
  const uint8_t* q;
  const uint64_t* q_off;
  const uint8_t* t;
  const uint64_t* t_off;
  const int32_t* h0;
  const uint8_t* pid;
  int32_t n_params;
  bsw_result* out;
  bsw_diag* diag;
  // end offsets (pair k ends at q_end[k]); null = q_off + 1
  const uint64_t* q_end;
  const uint64_t* t_end;
  bool codes_checked;  // the sequence bytes were validated beforehand
};

// Set the calling thread's error text; returns code.
int set_error(int code, const char* fmt, ...);

// Load a context's scoring table (validated).
int ctx_set_params(bsw_ctx* c, const bsw_params* params, int32_t n_params);
// Allocate a context's device buffers for calls of up to n pairs with its
// current scoring table, so that such calls allocate nothing.
int ctx_reserve(bsw_ctx* c, int64_t n, int32_t n_params);
// Enqueue one call on stream s (the context's path), ending with the copy
// of its status to the host.
int ctx_enqueue(bsw_ctx* c, const Args& a, hipStream_t s);
// After the stream has passed the call: its status, then its timing.
int ctx_finish(bsw_ctx* c);
// Band cells settled by the last finished call.
unsigned long long ctx_last_cells(const bsw_ctx* c);
hipStream_t ctx_stream(const bsw_ctx* c);

void launch_fill(uint32_t* p, int64_t nwords, hipStream_t s);
void launch_codes(const uint8_t* seq, const uint64_t* off, int64_t n, Status* st,
                  uint64_t bytes, hipStream_t s);
void launch_assemble(const ReqSlice* tab, int m, int64_t n, uint64_t* qb, uint64_t* qe,
                     uint64_t* tb, uint64_t* te, int32_t* h0, uint8_t* pid, hipStream_t s);

}  // namespace bsw
