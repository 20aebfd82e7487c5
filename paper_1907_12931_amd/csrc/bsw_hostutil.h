// bsw_hostutil.h -- host-only parts of the runtime: the serving arena's
// allocator, validation of the host-memory inputs, the launch shapes the
// tuner picks and the tune cache's file format.  Nothing here touches a
// device or includes HIP, so the same code is also built on its own with
// the host compiler's address and undefined-behaviour sanitizers.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/bsw.h"

namespace bsw {

// First-fit allocator over a byte range [0, size), with coalescing of free
// neighbours.  Offsets only: the caller owns the memory behind them.
class Arena {
 public:
  void reset(size_t bytes) {
    free_.clear();
    if (bytes) free_[0] = bytes;
    size_ = bytes;
  }
  bool alloc(size_t bytes, size_t* at) {
    if (bytes == 0) return false;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *at = it->first;
      const size_t rest = it->second - bytes;
      const size_t next = it->first + bytes;
      free_.erase(it);
      if (rest) free_[next] = rest;
      return true;
    }
    return false;
  }
  void release(size_t at, size_t bytes) {
    if (bytes == 0) return;
    auto it = free_.emplace(at, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }
  size_t free_bytes() const {
    size_t s = 0;
    for (auto& kv : free_) s += kv.second;
    return s;
  }
  size_t free_blocks() const { return free_.size(); }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0;
};

// Launch shapes of the batched path that the tuner chooses.
struct Tune {
  int nside = 2;    // side streams the classes are spread over (1..4); two
                    // keep the caller's stream, the runtime's default
                    // stream and the side streams within the four
                    // hardware queues a process gets by default
  int occ8 = 100;   // percent of the resident groups per CU for 8-bit classes
  int spec16 = 1;   // try pairs whose bound needs 16 bits at 8 bits first
  int wave32 = 64;  // 32-bit classes with a query cap >= this run one pair
                    // per wave (wave mode); the others one pair per lane
                    // (512: every 32-bit class in lane mode)
  bool operator==(const Tune& o) const {
    return nside == o.nside && occ8 == o.occ8 && spec16 == o.spec16 && wave32 == o.wave32;
  }
};

// ---------------------------------------------------------------------------
// Input validation.  Each returns the index of the first bad element, or -1.

// Why a scoring set is rejected, or nullptr when it is fine.
inline const char* params_problem(const bsw_params& p) {
  if (p.o_del < 0 || p.o_ins < 0 || p.o_del > BSW_MAX_GAP || p.o_ins > BSW_MAX_GAP)
    return "gap open out of range";
  if (p.e_del < 1 || p.e_ins < 1 || p.e_del > BSW_MAX_GAP || p.e_ins > BSW_MAX_GAP)
    return "gap extend out of range";
  if (p.w < 0) return "w < 0";
  if (p.end_bonus < 0 || p.end_bonus > BSW_MAX_BONUS) return "end_bonus out of range";
  return nullptr;
}

enum PairFault { PF_NONE = 0, PF_OFFSETS, PF_H0, PF_PID, PF_QCODE, PF_TCODE };

// A host-memory pair batch (the bsw_extend_batch arguments); *why receives
// the PairFault.  q and t may be null only when no pair has bytes there.
inline int64_t first_bad_pair(int64_t n, const uint8_t* q, const uint64_t* q_off,
                              const uint8_t* t, const uint64_t* t_off, const int32_t* h0,
                              const uint8_t* pid, int32_t n_params, int* why) {
  *why = PF_NONE;
  for (int64_t k = 0; k < n; ++k) {
    if (q_off[k + 1] < q_off[k] || t_off[k + 1] < t_off[k] ||
        q_off[k + 1] - q_off[k] > BSW_MAX_LEN || t_off[k + 1] - t_off[k] > BSW_MAX_LEN ||
        (!q && q_off[k + 1] > q_off[k]) || (!t && t_off[k + 1] > t_off[k])) {
      *why = PF_OFFSETS;
      return k;
    }
    if (h0[k] < 1 || h0[k] > BSW_MAX_H0) {
      *why = PF_H0;
      return k;
    }
    if (pid && pid[k] >= n_params) {
      *why = PF_PID;
      return k;
    }
    for (uint64_t x = q_off[k]; x < q_off[k + 1]; ++x)
      if (q[x] > 4) {
        *why = PF_QCODE;
        return k;
      }
    for (uint64_t x = t_off[k]; x < t_off[k + 1]; ++x)
      if (t[x] > 4) {
        *why = PF_TCODE;
        return k;
      }
  }
  return -1;
}

// Read offsets of the seed driver: non-decreasing, lengths <= BSW_MAX_LEN.
inline int64_t first_bad_read(const uint64_t* read_off, int64_t n_reads) {
  for (int64_t i = 0; i < n_reads; ++i)
    if (read_off[i + 1] < read_off[i] || read_off[i + 1] - read_off[i] > BSW_MAX_LEN) return i;
  return -1;
}

// Seeds of the seed driver against valid read offsets: read index, read
// interval, h0, reference range, and reference windows of both sides no
// longer than BSW_MAX_LEN (w = the scoring's band limit).
inline int64_t first_bad_seed(const bsw_seed* seeds, int64_t n, const uint64_t* read_off,
                              int64_t n_reads, uint64_t ref_len, int64_t w) {
  for (int64_t k = 0; k < n; ++k) {
    const bsw_seed& sd = seeds[k];
    bool ok = sd.read >= 0 && sd.read < n_reads;
    const int64_t len = ok ? (int64_t)(read_off[sd.read + 1] - read_off[sd.read]) : 0;
    ok = ok && sd.qb >= 0 && sd.qb <= sd.qe && sd.qe <= len && sd.h0 >= 1 &&
         sd.h0 <= BSW_MAX_H0 && sd.rb >= 0 && (uint64_t)sd.rb <= ref_len &&
         (uint64_t)(sd.qe - sd.qb) <= ref_len - (uint64_t)sd.rb;
    if (ok) {
      const int64_t lt = std::min<int64_t>(sd.rb, (int64_t)sd.qb + w);
      const uint64_t re = (uint64_t)sd.rb + (uint64_t)(sd.qe - sd.qb);
      const uint64_t rt = std::min<uint64_t>(ref_len - re, (uint64_t)(len - sd.qe) + w);
      ok = lt <= BSW_MAX_LEN && rt <= (uint64_t)BSW_MAX_LEN;
    }
    if (!ok) return k;
  }
  return -1;
}

// ---------------------------------------------------------------------------
// Tune cache: a small JSON object, one entry per line,
//   "gfx950:cu256:w100:sym1:mb0": {"nside": 4, "occ8": 100, "spec16": 1, "wave32": 64, "ms": 57.1},
// Lines that do not have that form are ignored.

using CacheEntries = std::vector<std::pair<std::string, std::string>>;

inline CacheEntries cache_read(const char* path) {
  CacheEntries e;
  FILE* f = std::fopen(path, "r");
  if (!f) return e;
  std::string line;
  char buf[256];
  bool more = true;
  while (more) {
    line.clear();
    // whole lines, however long
    for (;;) {
      if (!std::fgets(buf, sizeof buf, f)) {
        more = false;
        break;
      }
      line += buf;
      if (!line.empty() && line.back() == '\n') break;
    }
    const size_t a = line.find('"');
    const size_t b = a == std::string::npos ? a : line.find('"', a + 1);
    const size_t v = b == std::string::npos ? b : line.find('{', b);
    const size_t z = v == std::string::npos ? v : line.find('}', v);
    if (z != std::string::npos)
      e.emplace_back(line.substr(a + 1, b - a - 1), line.substr(v, z - v + 1));
  }
  std::fclose(f);
  return e;
}

// A cache value: true when it has every field and each is in range.
inline bool parse_tune(const std::string& v, int nside_max, Tune* t) {
  Tune x;
  double ms = 0;
  if (std::sscanf(v.c_str(),
                  "{\"nside\": %d, \"occ8\": %d, \"spec16\": %d, \"wave32\": %d, \"ms\": %lf}",
                  &x.nside, &x.occ8, &x.spec16, &x.wave32, &ms) != 5)
    return false;
  if (x.nside < 1 || x.nside > nside_max || x.occ8 < 1 || x.occ8 > 100 ||
      (x.spec16 != 0 && x.spec16 != 1) || x.wave32 < 32 || x.wave32 > 512)
    return false;
  *t = x;
  return true;
}

inline std::string format_tune(const Tune& t, double ms) {
  char v[160];
  std::snprintf(v, sizeof v,
                "{\"nside\": %d, \"occ8\": %d, \"spec16\": %d, \"wave32\": %d, \"ms\": %.3f}",
                t.nside, t.occ8, t.spec16, t.wave32, ms);
  return v;
}

// Replace or add key's entry and rewrite the file (through a temporary and
// a rename, so a reader never sees half a file).  False on an I/O error.
inline bool cache_put(const char* path, const std::string& key, const std::string& value) {
  CacheEntries e = cache_read(path);
  bool found = false;
  for (auto& kv : e)
    if (kv.first == key) {
      kv.second = value;
      found = true;
    }
  if (!found) e.emplace_back(key, value);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "{\n");
  for (size_t i = 0; i < e.size(); ++i)
    std::fprintf(f, " \"%s\": %s%s\n", e[i].first.c_str(), e[i].second.c_str(),
                 i + 1 < e.size() ? "," : "");
  std::fprintf(f, "}\n");
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

}  // namespace bsw
