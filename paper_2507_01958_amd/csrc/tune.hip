// Autotuner of the launch shapes (struct Tune) of the preconditioner passes
// and the A kernel.
//
// The choices change how work is split among blocks (rows per block of the
// row transforms, column pairs per block of the column solves, column blocks
// per wave and the persistent form of the time GEMM) and which FFT form runs
// (register-resident or LDS-staged), never what is computed beyond rounding. They are measured with HIP events on the plan's stream:
// each candidate times a few applications of the preconditioner to a fixed
// vector, the best (minimum over trials) is kept, one parameter at a time.
// Results are cached per (d, grid, N_t, boundary, precision, l, GPU
// architecture) for the process, applied to every later plan of that key,
// and, when MFG_TUNE_CACHE names a file, read from and appended to it.
#include <cstdio>
#include <cstdlib>
#include <initializer_list>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "plan.h"

namespace mfg {

int fail(int code, const std::string& msg);

namespace {

using Key = std::tuple<int, int, int, int, int, int, int, std::string>;

std::mutex g_mu;
std::map<Key, Tune> g_cache;
bool g_file_loaded = false;

std::string arch_of(int device) {
  static std::map<int, std::string> names;
  auto it = names.find(device);
  if (it != names.end()) return it->second;
  hipDeviceProp_t prop;
  std::string name = "unknown";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    name = prop.gcnArchName;
    const size_t colon = name.find(':');
    if (colon != std::string::npos) name = name.substr(0, colon);
  }
  names[device] = name;
  return name;
}

Key key_of(const Plan& P) {
  return Key{P.pb.d, P.g.n0, P.g.n1, P.g.nt, P.pb.bc, P.precision, P.l, arch_of(P.device)};
}

// One cache line: "d n0 n1 nt bc precision l arch f64_cb lp_cb rows_elems cols_lines pers
// fft_reg aat_tc lp_waves lp_cb_i lp_waves_i aat_big".
void load_file_locked() {
  if (g_file_loaded) return;
  g_file_loaded = true;
  const char* path = std::getenv("MFG_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char arch[64];
  int d, n0, n1, nt, bc, prec, l;
  Tune t;
  while (std::fscanf(f, "%d %d %d %d %d %d %d %63s %d %d %d %d %d %d %d %d %d %d %d", &d, &n0,
                     &n1, &nt, &bc, &prec, &l, arch, &t.f64_cb, &t.lp_cb, &t.rows_elems,
                     &t.cols_lines, &t.tgemm_pers, &t.fft_reg, &t.aat_tc, &t.lp_waves,
                     &t.lp_cb_i, &t.lp_waves_i, &t.aat_big) == 19)
    g_cache[Key{d, n0, n1, nt, bc, prec, l, arch}] = t;
  std::fclose(f);
}

void store(const Plan& P, const Tune& t) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_file_locked();
  const Key k = key_of(P);
  g_cache[k] = t;
  const char* path = std::getenv("MFG_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%d %d %d %d %d %d %d %s %d %d %d %d %d %d %d %d %d %d %d\n",
               std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
               std::get<5>(k), std::get<6>(k), std::get<7>(k).c_str(), t.f64_cb, t.lp_cb,
               t.rows_elems, t.cols_lines, t.tgemm_pers, t.fft_reg, t.aat_tc, t.lp_waves,
               t.lp_cb_i, t.lp_waves_i, t.aat_big);
  std::fclose(f);
}

// Timed units: the preconditioner as PCG applies it (with its fused dot
// products), and the fused A apply (PCG direction update
// p = z + beta p_old with q = A p), each tuned on its own launch shapes.
enum Unit { U_PRECOND = 0, U_AAT = 1 };

void tune_unit(Plan& P, int unit, hipStream_t s) {
  if (unit == U_PRECOND) launch_precond(P, P.r, P.z, true, P.q, s);
  else launch_pdir_AAt(P, P.z, P.r, P.p, P.q, false, s);
}

// Mean time (ms) of `reps` units, best of `trials`.
int time_unit(Plan& P, int unit, hipEvent_t a, hipEvent_t b, int reps, int trials,
              float* best) {
  hipStream_t s = P.stream;
  tune_unit(P, unit, s);  // warm caches and code
  *best = 1e30f;
  for (int t = 0; t < trials; ++t) {
    if (hipEventRecord(a, s) != hipSuccess) return fail(MFG_ERR_HIP, "event record failed");
    for (int i = 0; i < reps; ++i) tune_unit(P, unit, s);
    if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess)
      return fail(MFG_ERR_HIP, "event record failed");
    if (hipGetLastError() != hipSuccess) return fail(MFG_ERR_HIP, "launch failed while tuning");
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return fail(MFG_ERR_HIP, "event timing failed");
    if (ms / reps < *best) *best = ms / reps;
  }
  return MFG_OK;
}

}  // namespace

// Launch shapes the batched kernels support: the blocked time GEMM with one
// shape (column blocks per wave, waves per block) for both directions, the
// default A-kernel tile.
void batch_shape(Tune& t) {
  t.tgemm_pers = 0;
  t.aat_big = Tune{}.aat_big;
  t.lp_waves_i = t.lp_waves;
  t.lp_cb_i = t.lp_cb;
}

bool tune_lookup(const Plan& P, Tune* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_file_locked();
  auto it = g_cache.find(key_of(P));
  if (it == g_cache.end()) return false;
  *out = it->second;
  return true;
}

// The fields that are choices of method or fixed by the plan's settings, not
// tuned launch shapes: a cached entry never replaces them.
void keep_untuned(const Tune& from, Tune& to) {
  to.flex = from.flex;
  to.lp_stream = from.lp_stream;
  to.rhs_tc = from.rhs_tc;
  to.fuse_fwd = from.fuse_fwd;
  to.fuse_upd = from.fuse_upd;
  to.fuse_inv = from.fuse_inv;
  to.batch_queue = from.batch_queue;
}

// allow_pers = false keeps the time GEMM in the form the batched launches use.
int autotune(Plan& P, int effort, bool allow_pers) {
  if (effort < 2) {
    Tune t;
    if (tune_lookup(P, &t)) {
      if (!allow_pers) batch_shape(t);
      keep_untuned(P.tune, t);
      P.tune = t;
      return MFG_OK;
    }
  }
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return fail(MFG_ERR_HIP, "event creation failed");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(MFG_ERR_HIP, "event creation failed");
  }
  // inputs: constant vectors (the passes take the same time for any values)
  launch_fill(P.r, P.g.n, 1.0, P.stream);
  launch_fill(P.q, P.g.n, 1.0, P.stream);
  const long long work = P.g.n;
  const int reps = work >= (1LL << 22) ? 5 : (work >= (1LL << 18) ? 10 : 40);
  const int trials = 3;
  // A parameter is a list of candidate settings, each setting one or more
  // fields (joint choices where fields interact, e.g. column blocks x waves).
  using Setting = std::vector<std::pair<int Tune::*, int>>;
  struct Param {
    int unit;
    std::vector<Setting> values;
  };
  auto single = [](int Tune::*f, std::initializer_list<int> vs) {
    std::vector<Setting> out;
    for (int v : vs) out.push_back(Setting{{f, v}});
    return out;
  };
  auto joint = [](int Tune::*fa, int Tune::*fb, std::initializer_list<std::pair<int, int>> vs) {
    std::vector<Setting> out;
    for (auto v : vs) out.push_back(Setting{{fa, v.first}, {fb, v.second}});
    return out;
  };
  std::vector<Param> params;
  if (P.precision == MFG_FP64) {
    params.push_back({U_PRECOND, single(&Tune::f64_cb, {1, 2})});
  } else if (allow_pers) {
    params.push_back({U_PRECOND, joint(&Tune::lp_cb, &Tune::lp_waves,
                                       {{2, 4}, {1, 4}, {2, 8}, {1, 8}})});
    params.push_back({U_PRECOND, joint(&Tune::lp_cb_i, &Tune::lp_waves_i,
                                       {{2, 4}, {1, 4}, {2, 8}, {1, 8}})});
  } else {  // batched GEMMs: one shape for both directions
    std::vector<Setting> both;
    for (auto cw : {std::make_pair(2, 4), std::make_pair(1, 4), std::make_pair(2, 8),
                    std::make_pair(1, 8)})
      both.push_back(Setting{{&Tune::lp_cb, cw.first}, {&Tune::lp_waves, cw.second},
                             {&Tune::lp_cb_i, cw.first}, {&Tune::lp_waves_i, cw.second}});
    params.push_back({U_PRECOND, both});
  }
  if (P.ntp > 0 && allow_pers) params.push_back({U_PRECOND, single(&Tune::tgemm_pers, {0, 1})});
  params.push_back({U_PRECOND, single(&Tune::fft_reg, {1, 0})});
  params.push_back({U_PRECOND, single(&Tune::rows_elems, {256, 512, 1024, 2048, 4096})});
  if (P.g.has0) params.push_back({U_PRECOND, single(&Tune::cols_lines, {1, 2, 4, 8, 16})});
  if (P.g.has0 && allow_pers) {
    params.push_back({U_AAT, joint(&Tune::aat_big, &Tune::aat_tc,
                                   {{0, 0}, {0, 8}, {0, 16}, {0, 32}, {1, 0}, {1, 8}, {1, 16},
                                    {1, 32}, {2, 0}, {2, 4}, {2, 8}, {2, 16}})});
  } else {
    params.push_back({U_AAT, single(&Tune::aat_tc, {0, 4, 8, 16, 32})});
  }
  if (!allow_pers) batch_shape(P.tune);
  int rc = MFG_OK;
  float cur[2] = {0.0f, 0.0f};
  launch_precond(P, P.r, P.z, false, nullptr, P.stream);  // a z for the A unit
  for (int u = 0; u < 2 && !rc; ++u) rc = time_unit(P, u, a, b, reps, trials, &cur[u]);
  const int passes = effort >= 2 ? 2 : 1;
  for (int pass = 0; pass < passes && !rc; ++pass) {
    for (const Param& prm : params) {
      const Tune keep = P.tune;
      Tune best = keep;
      for (const Setting& st : prm.values) {
        Tune t = keep;
        for (const auto& fv : st) t.*(fv.first) = fv.second;
        bool same = true;
        for (const auto& fv : st) same = same && (keep.*(fv.first) == fv.second);
        if (same) continue;
        P.tune = t;
        float ms;
        if ((rc = time_unit(P, prm.unit, a, b, reps, trials, &ms))) break;
        if (ms < 0.985f * cur[prm.unit]) {  // switch only on a clear gain
          cur[prm.unit] = ms;
          best = t;
        }
      }
      P.tune = best;
      if (rc) break;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc) return rc;
  if (!allow_pers) batch_shape(P.tune);  // both GEMM directions share the tuned shape
  store(P, P.tune);
  return MFG_OK;
}

}  // namespace mfg
