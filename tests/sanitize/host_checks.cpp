// host_checks.cpp -- exercises the host-only parts of the runtime
// (paper_1907_12931_amd/csrc/bsw_hostutil.h: the serving arena, input
// validation, the tune cache format) in a build with the address and
// undefined-behaviour sanitizers.  Every input array sits in a heap block of
// exactly its size, so a read one past an end is caught.  Prints OK and
// exits 0 when every check holds.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <string>
#include <vector>

#include "../../paper_1907_12931_amd/csrc/bsw_hostutil.h"

using namespace bsw;

static int failures = 0;
#define CHECK(x)                                                        \
  do {                                                                  \
    if (!(x)) {                                                         \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #x); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

template <class T>
static T* exact(const std::vector<T>& v) {
  T* p = static_cast<T*>(std::malloc(v.size() * sizeof(T) + (v.empty() ? 1 : 0)));
  for (size_t i = 0; i < v.size(); ++i) p[i] = v[i];
  return p;
}

static void arena_checks() {
  std::mt19937_64 rng(7);
  for (int round = 0; round < 4; ++round) {
    const size_t size = (size_t)1 << (16 + round * 2);
    Arena a;
    a.reset(size);
    std::map<size_t, size_t> live;
    for (int op = 0; op < 50000; ++op) {
      if (live.empty() || rng() % 3 != 0) {
        const size_t bytes = 256 * (1 + rng() % (size / 256 / 16));
        size_t at = 0;
        if (!a.alloc(bytes, &at)) continue;
        CHECK(at + bytes <= size);
        auto nx = live.lower_bound(at);
        if (nx != live.end()) CHECK(at + bytes <= nx->first);
        if (nx != live.begin()) {
          auto pv = std::prev(nx);
          CHECK(pv->first + pv->second <= at);
        }
        live[at] = bytes;
      } else {
        auto it = live.begin();
        std::advance(it, rng() % live.size());
        a.release(it->first, it->second);
        live.erase(it);
      }
      size_t used = 0;
      for (auto& kv : live) used += kv.second;
      if (op % 997 == 0) CHECK(a.free_bytes() + used == size);
    }
    for (auto& kv : live) a.release(kv.first, kv.second);
    CHECK(a.free_bytes() == size);
    CHECK(a.free_blocks() == 1);
    size_t at = 0;
    CHECK(a.alloc(size, &at) && at == 0);
    CHECK(!a.alloc(1, &at));
    CHECK(!a.alloc(0, &at));
  }
  Arena z;
  z.reset(0);
  size_t at = 0;
  CHECK(!z.alloc(256, &at));
}

static void pair_checks() {
  // pairs: (3, 2), (0, 0), (4, 1); codes at the very ends of q and t
  const std::vector<uint8_t> qv = {0, 1, 2, 3, 4, 0, 1}, tv = {4, 3, 2};
  const std::vector<uint64_t> qo = {0, 3, 3, 7}, to = {0, 2, 2, 3};
  const std::vector<int32_t> h0v = {5, 1, BSW_MAX_H0};
  const std::vector<uint8_t> pidv = {0, 1, 1};
  uint8_t* q = exact(qv);
  uint8_t* t = exact(tv);
  uint64_t* q_off = exact(qo);
  uint64_t* t_off = exact(to);
  int32_t* h0 = exact(h0v);
  uint8_t* pid = exact(pidv);
  int why = -1;
  CHECK(first_bad_pair(3, q, q_off, t, t_off, h0, pid, 2, &why) == -1 && why == PF_NONE);
  CHECK(first_bad_pair(3, q, q_off, t, t_off, h0, nullptr, 1, &why) == -1);
  CHECK(first_bad_pair(3, q, q_off, t, t_off, h0, pid, 1, &why) == 1 && why == PF_PID);
  q[6] = 5;
  CHECK(first_bad_pair(3, q, q_off, t, t_off, h0, pid, 2, &why) == 2 && why == PF_QCODE);
  q[6] = 1;
  t[2] = 9;
  CHECK(first_bad_pair(3, q, q_off, t, t_off, h0, pid, 2, &why) == 2 && why == PF_TCODE);
  t[2] = 2;
  h0[2] = BSW_MAX_H0 + 1;
  CHECK(first_bad_pair(3, q, q_off, t, t_off, h0, pid, 2, &why) == 2 && why == PF_H0);
  h0[2] = 0;
  CHECK(first_bad_pair(3, q, q_off, t, t_off, h0, pid, 2, &why) == 2 && why == PF_H0);
  h0[2] = 1;
  q_off[2] = 2;  // decreasing
  CHECK(first_bad_pair(3, q, q_off, t, t_off, h0, pid, 2, &why) == 1 && why == PF_OFFSETS);
  q_off[2] = 3;
  // no sequence bytes where a pair has some
  CHECK(first_bad_pair(3, nullptr, q_off, t, t_off, h0, pid, 2, &why) == 0 &&
        why == PF_OFFSETS);
  CHECK(first_bad_pair(3, q, q_off, nullptr, t_off, h0, pid, 2, &why) == 0);
  // empty pairs need no sequence pointer
  const std::vector<uint64_t> zo = {0, 0, 0};
  uint64_t* z_off = exact(zo);
  CHECK(first_bad_pair(2, nullptr, z_off, nullptr, z_off, h0, nullptr, 1, &why) == -1);
  // a length past the limit
  const std::vector<uint64_t> lo = {0, (uint64_t)BSW_MAX_LEN + 1};
  uint64_t* l_off = exact(lo);
  CHECK(first_bad_pair(1, q, l_off, t, z_off, h0, nullptr, 1, &why) == 0 && why == PF_OFFSETS);
  for (void* p : {(void*)q, (void*)t, (void*)q_off, (void*)t_off, (void*)h0, (void*)pid,
                  (void*)z_off, (void*)l_off})
    std::free(p);
}

static void seed_checks() {
  const std::vector<uint64_t> ro = {0, 151, 151, 302};
  uint64_t* read_off = exact(ro);
  CHECK(first_bad_read(read_off, 3) == -1);
  read_off[2] = 100;
  CHECK(first_bad_read(read_off, 3) == 1);
  read_off[2] = 151;
  const uint64_t ref_len = 1000;
  const std::vector<bsw_seed> sv = {
      {0, 10, 40, 30, 100},   // fine
      {1, 0, 0, 1, 0},        // empty read, empty seed at the reference start
      {2, 151, 151, 1, 1000}, // empty seed at both ends
      {2, 0, 151, 151, 849},  // whole read at the reference end
  };
  bsw_seed* seeds = exact(sv);
  CHECK(first_bad_seed(seeds, 4, read_off, 3, ref_len, 100) == -1);
  seeds[3].rb = 850;  // one past the reference end
  CHECK(first_bad_seed(seeds, 4, read_off, 3, ref_len, 100) == 3);
  seeds[3].rb = 849;
  seeds[0].read = 3;  // no such read
  CHECK(first_bad_seed(seeds, 4, read_off, 3, ref_len, 100) == 0);
  seeds[0].read = -1;
  CHECK(first_bad_seed(seeds, 4, read_off, 3, ref_len, 100) == 0);
  seeds[0].read = 0;
  seeds[0].qe = 152;
  CHECK(first_bad_seed(seeds, 4, read_off, 3, ref_len, 100) == 0);
  seeds[0].qe = 40;
  seeds[0].h0 = 0;
  CHECK(first_bad_seed(seeds, 4, read_off, 3, ref_len, 100) == 0);
  seeds[0].h0 = 30;
  // a left window past BSW_MAX_LEN: long reference, huge band
  CHECK(first_bad_seed(seeds, 1, read_off, 3, (uint64_t)1 << 40, 100) == -1);
  seeds[0].rb = (int64_t)1 << 20;
  CHECK(first_bad_seed(seeds, 1, read_off, 3, (uint64_t)1 << 40, 1 << 20) == 0);
  std::free(read_off);
  std::free(seeds);
}

static void params_checks() {
  bsw_params p{};
  for (int i = 0; i < 25; ++i) p.mat[i] = (i % 6 == 0) ? 1 : -4;
  p.o_del = p.o_ins = 6;
  p.e_del = p.e_ins = 1;
  p.w = 100;
  p.zdrop = 100;
  p.end_bonus = 5;
  CHECK(params_problem(p) == nullptr);
  bsw_params b = p;
  b.e_ins = 0;
  CHECK(params_problem(b) != nullptr);
  b = p;
  b.o_del = BSW_MAX_GAP + 1;
  CHECK(params_problem(b) != nullptr);
  b = p;
  b.w = -1;
  CHECK(params_problem(b) != nullptr);
  b = p;
  b.end_bonus = -1;
  CHECK(params_problem(b) != nullptr);
}

static void cache_checks(const std::string& dir) {
  const std::string path = dir + "/tune.json";
  std::remove(path.c_str());
  CHECK(cache_read(path.c_str()).empty());
  Tune t;
  t.nside = 2;
  t.occ8 = 75;
  t.spec16 = 0;
  t.wave32 = 128;
  CHECK(cache_put(path.c_str(), "k1", format_tune(t, 12.5)));
  Tune u;
  CHECK(cache_put(path.c_str(), "k2", format_tune(u, 3.0)));
  auto e = cache_read(path.c_str());
  CHECK(e.size() == 2 && e[0].first == "k1" && e[1].first == "k2");
  Tune r;
  CHECK(parse_tune(e[0].second, 4, &r) && r == t);
  CHECK(parse_tune(e[1].second, 4, &r) && r == u);
  CHECK(!parse_tune(e[0].second, 1, &r));  // nside above the limit
  t.occ8 = 50;
  CHECK(cache_put(path.c_str(), "k1", format_tune(t, 9.0)));
  e = cache_read(path.c_str());
  CHECK(e.size() == 2 && parse_tune(e[0].second, 4, &r) && r.occ8 == 50);
  // damaged and overlong lines are skipped, whole lines are still read
  FILE* f = std::fopen(path.c_str(), "w");
  CHECK(f != nullptr);
  if (f) {
    std::fprintf(f, "{\n \"only a key\n \"k\": no value\n \"k\": {unclosed\n");
    std::fprintf(f, " \"%s\": {\"nside\": 1}\n", std::string(3000, 'x').c_str());
    std::fprintf(f, " \"k3\": {\"nside\": 3, \"occ8\": 100, \"spec16\": 1, \"wave32\": 600,"
                    " \"ms\": 1.0},\n \"k4\": {\"nside\": 1, \"occ8\": 100, \"spec16\": 1, "
                    "\"wave32\": 32, \"ms\": 1.0}\n}");  // no final newline
    std::fclose(f);
  }
  e = cache_read(path.c_str());
  CHECK(e.size() == 3);
  CHECK(e.size() == 3 && e[0].first.size() == 3000 && !parse_tune(e[0].second, 4, &r));
  CHECK(e.size() == 3 && e[1].first == "k3" && !parse_tune(e[1].second, 4, &r));
  CHECK(e.size() == 3 && e[2].first == "k4" && parse_tune(e[2].second, 4, &r) &&
        r.wave32 == 32);
  CHECK(!parse_tune("", 4, &r));
  CHECK(!parse_tune("{\"nside\": 2, \"occ8\": 0, \"spec16\": 1, \"wave32\": 64, \"ms\": 1}",
                    4, &r));
  CHECK(!cache_put((dir + "/no/such/dir/tune.json").c_str(), "k", format_tune(u, 1.0)));
  std::remove(path.c_str());
}

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: host_checks SCRATCH_DIR\n");
    return 2;
  }
  arena_checks();
  pair_checks();
  seed_checks();
  params_checks();
  cache_checks(argv[1]);
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("OK\n");
  return 0;
}
