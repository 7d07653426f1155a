// Batched Chambolle-Pock solves: many independent plans advanced together.
//
// Every phase of a CP step (right-hand side, PCG initialisation, each PCG
// iteration's reduced-matrix product, update, preconditioner passes and
// reductions, back-projection + prox) runs as ONE launch over all instances:
// the launch takes a device array of per-instance arguments and block offsets
// and each block runs the single-plan body for its instance (batch_args.h).
// Instances keep their own launch shapes, so a batched solve performs exactly
// the arithmetic of solving each plan alone.
//
// The step sizes of the Section 5 schedule do not depend on the data: they are
// computed on the host for every instance and iteration and copied to the
// device, where a small kernel loads those of the current iteration into each
// instance's scalar block. With that, a CP step up to a fixed number of PCG
// iterations contains no host decision and is captured once into a hipGraph
// and replayed; instances that have converged skip their work through their
// done flags, and any instance that needs more iterations continues with
// eager batched launches before the back-projection.
#include <algorithm>
#include <cmath>
#include <string>
#include <tuple>
#include <vector>

#include "batch_args.h"
#include "plan.h"
#include "tgemm.h"

namespace mfg {

int fail(int code, const std::string& msg);

namespace {

template <typename A>
struct Phase {
  A* args = nullptr;
  int* off = nullptr;
  int ninst = 0;
  int total = 0;
  size_t shm = 0;
};

// Spatial launches of one FFT size class (0: LDS path, else the axis length);
// T is the preconditioner's intermediate (float in the mixed modes, double in
// FP64).
template <typename T>
struct SpatialGroup {
  int cls = 0, threads = 256;
  Phase<RowsArgs<T>> rows_fwd, rows_inv;
};
template <typename T>
struct ColsGroup {
  int cls = 0, threads = 256;
  Phase<ColsArgs<T>> cols;
};

// One time-GEMM launch class: low precision (N_t padding class, column blocks
// per wave, waves per block) or float64 (k rows per block kb, column blocks cb).
struct GemmGroup {
  int ntp = 0, cb = 2, waves = 4, kb = 8;
  Phase<GemmArgs<double, float>> fwd_init, fwd;  // fwd: with the r.r stopping test
  Phase<GemmArgs<float, double>> inv_init, inv_iter;
  Phase<GemmArgs<double, double>> fwd64_init, fwd64, inv64_init, inv64_iter;
};

}  // namespace

struct Batch {
  std::vector<mfg_plan_t> plans;
  int count = 0;
  int mode = GM_F32;  // GM_F64: the float64 preconditioner
  hipStream_t user = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  double* scal_all = nullptr;  // count x S_COUNT scalar blocks (the plans' own)
  double* host_scal = nullptr;
  double* tol2 = nullptr;
  double* sched = nullptr;
  int sched_cap = 0;
  std::vector<GemmGroup> groups;
  Phase<UpdArgs> upd_first, upd_odd, upd_even;
  Phase<AatArgs> aat_first, aat_odd, aat_even;
  std::vector<SpatialGroup<float>> rows;
  std::vector<ColsGroup<float>> cols;
  std::vector<SpatialGroup<double>> rows64;
  std::vector<ColsGroup<double>> cols64;
  Phase<RhsArgs> rhs;
  // back-projection of the last step of a call (writes xi', ybar') and of the
  // other steps (hands z = xi' + sigma' ybar' to the next right-hand side)
  Phase<BackprojArgs> bp, bp_mid;
  FinishArgs *f_bb = nullptr, *f_dm = nullptr;
  std::vector<const double*> bound;  // state vectors the rhs/bp phases were built for
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_k = 0;
  std::vector<void*> dev;
  // persistent A phase over a tile queue (Tune::batch_queue): the counter and
  // the resident grid
  int* queue = nullptr;
  int qgrid = 0;
};

}  // namespace mfg

struct mfg_batch_s {
  mfg::Batch B;
};

namespace mfg {

namespace {

int dmalloc(Batch& B, void** p, size_t bytes) {
  if (hipMalloc(p, bytes ? bytes : 16) != hipSuccess) {
    (void)hipGetLastError();
    return fail(MFG_ERR_OOM, "batch allocation failed");
  }
  B.dev.push_back(*p);
  return MFG_OK;
}

template <typename A>
int upload_phase(Batch& B, const std::vector<A>& args, const std::vector<int>& blocks,
                 Phase<A>& ph, size_t shm = 0) {
  std::vector<int> off(args.size() + 1, 0);
  for (size_t i = 0; i < args.size(); ++i) off[i + 1] = off[i] + blocks[i];
  int rc;
  if (!ph.args) {
    void *pa, *po;
    if ((rc = dmalloc(B, &pa, args.size() * sizeof(A))) ||
        (rc = dmalloc(B, &po, off.size() * sizeof(int))))
      return rc;
    ph.args = static_cast<A*>(pa);
    ph.off = static_cast<int*>(po);
  }
  if (hipMemcpy(ph.args, args.data(), args.size() * sizeof(A), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(ph.off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return fail(MFG_ERR_HIP, "batch argument upload failed");
  ph.ninst = (int)args.size();
  ph.total = off.back();
  ph.shm = shm;
  return MFG_OK;
}

int upload_finish(Batch& B, const std::vector<FinishArgs>& f, FinishArgs** out) {
  int rc;
  if (!*out) {
    void* p;
    if ((rc = dmalloc(B, &p, f.size() * sizeof(FinishArgs)))) return rc;
    *out = static_cast<FinishArgs*>(p);
  }
  if (hipMemcpy(*out, f.data(), f.size() * sizeof(FinishArgs), hipMemcpyHostToDevice) !=
      hipSuccess)
    return fail(MFG_ERR_HIP, "batch argument upload failed");
  return MFG_OK;
}

Plan& plan_of(Batch& B, int i) { return B.plans[i]->P; }
const double* done_of(Batch& B, int i) { return B.scal_all + (size_t)i * S_COUNT + S_DONE; }

// Spatial-solve launches of every instance, grouped by size class.
template <typename T>
int build_spatial(Batch& B, std::vector<SpatialGroup<T>>& rows_out,
                  std::vector<ColsGroup<T>>& cols_out) {
  const int n = B.count;
  std::vector<int> rcls(n), ccls(n), rthr(n), cthr(n);
  std::vector<RowsArgs<T>> rf(n), ri(n);
  std::vector<ColsArgs<T>> cl(n);
  std::vector<int> b_rows(n), b_cols(n);
  std::vector<size_t> rshm(n), cshm(n);
  for (int i = 0; i < n; ++i) {
    Plan& P = plan_of(B, i);
    const double* done = done_of(B, i);
    T* tmp = reinterpret_cast<T*>(P.tmp);
    rcls[i] = batch_rows_args<T>(P, tmp, 0, done, &rf[i], &b_rows[i], &rshm[i], &rthr[i]);
    batch_rows_args<T>(P, tmp, 1, done, &ri[i], &b_rows[i], &rshm[i], &rthr[i]);
    ccls[i] = batch_cols_args<T>(P, tmp, done, &cl[i], &b_cols[i], &cshm[i], &cthr[i]);
  }
  int rc;
  std::vector<int> classes(rcls);
  std::sort(classes.begin(), classes.end());
  classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
  rows_out.assign(classes.size(), SpatialGroup<T>{});
  for (size_t c = 0; c < classes.size(); ++c) {
    std::vector<RowsArgs<T>> f, v;
    std::vector<int> blocks;
    size_t shm = 0;
    for (int i = 0; i < n; ++i)
      if (rcls[i] == classes[c]) {
        f.push_back(rf[i]);
        v.push_back(ri[i]);
        blocks.push_back(b_rows[i]);
        shm = std::max(shm, rshm[i]);
        rows_out[c].threads = rthr[i];
      }
    rows_out[c].cls = classes[c];
    if ((rc = upload_phase(B, f, blocks, rows_out[c].rows_fwd, shm)) ||
        (rc = upload_phase(B, v, blocks, rows_out[c].rows_inv, shm)))
      return rc;
  }
  classes = ccls;
  std::sort(classes.begin(), classes.end());
  classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
  cols_out.assign(classes.size(), ColsGroup<T>{});
  for (size_t c = 0; c < classes.size(); ++c) {
    std::vector<ColsArgs<T>> f;
    std::vector<int> blocks;
    size_t shm = 0;
    for (int i = 0; i < n; ++i)
      if (ccls[i] == classes[c]) {
        f.push_back(cl[i]);
        blocks.push_back(b_cols[i]);
        shm = std::max(shm, cshm[i]);
        cols_out[c].threads = cthr[i];
      }
    cols_out[c].cls = classes[c];
    if ((rc = upload_phase(B, f, blocks, cols_out[c].cols, shm))) return rc;
  }
  return MFG_OK;
}

// Build the argument arrays of the PCG phases (state independent).
int build_pcg_phases(Batch& B) {
  const int n = B.count;
  const bool f64 = B.mode == GM_F64;
  std::vector<UpdArgs> u0, uo, ue;
  std::vector<AatArgs> af, ao, ae;
  std::vector<int> b_upd, b_aat;
  std::vector<FinishArgs> fbb;
  for (int i = 0; i < n; ++i) {
    Plan& P = plan_of(B, i);
    const double* done = done_of(B, i);
    UpdArgs u1 = update_args(P, P.u, P.r, P.p, P.q, false);   // odd k: p_new = p
    UpdArgs u2 = update_args(P, P.u, P.r, P.p2, P.q, false);  // even k: p_new = p2
    u1.done = u2.done = done;
    uo.push_back(u1);
    ue.push_back(u2);
    u1.first = 1;  // k = 1: x = alpha p
    u0.push_back(u1);
    b_upd.push_back(update_grid(P));
    int g;
    af.push_back(aat_args(P, P.z, P.p2, P.p, P.q, true, done, &g));
    ao.push_back(aat_args(P, P.z, P.p2, P.p, P.q, false, done, &g));
    ae.push_back(aat_args(P, P.z, P.p, P.p2, P.q, false, done, &g));
    b_aat.push_back(g);
    u0.back().npq = uo.back().npq = ue.back().npq = g;
    // b.b partials come from the right-hand side kernel, which starts the solve
    fbb.push_back(finish_args(P, T_BB, rhs_grid(P), OP_BB));
  }
  int rc;
  if ((rc = upload_finish(B, fbb, &B.f_bb))) return rc;
  if ((rc = f64 ? build_spatial<double>(B, B.rows64, B.cols64)
                : build_spatial<float>(B, B.rows, B.cols)))
    return rc;
  // time GEMMs: one launch per class: low precision (N_t padding class,
  // column blocks per wave, waves), float64 (k rows per block, column blocks)
  auto shape_of = [&](int i) {
    const Plan& P = plan_of(B, i);
    if (f64) {
      int blk, kb, cb;
      (void)batch_gemm64_args(P, nullptr, nullptr, DOT_NONE, nullptr, nullptr, nullptr, &blk, &kb,
                              &cb);
      return std::make_tuple(kb, cb, 0);
    }
    if (P.ntp == 0) return std::make_tuple(-1, 0, 0);  // N_t > 128: streaming V
    const Tune& t = P.tune;
    return std::make_tuple(P.ntp, t.lp_cb == 1 ? 1 : 2, t.lp_waves == 8 ? 8 : 4);
  };
  std::vector<std::tuple<int, int, int>> classes;
  for (int i = 0; i < n; ++i) classes.push_back(shape_of(i));
  std::sort(classes.begin(), classes.end());
  classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
  B.groups.assign(classes.size(), GemmGroup{});
  std::vector<int> gemm_grid(n, 0);
  for (size_t gi = 0; gi < classes.size(); ++gi) {
    GemmGroup& G = B.groups[gi];
    if (f64) std::tie(G.kb, G.cb, G.waves) = classes[gi];
    else std::tie(G.ntp, G.cb, G.waves) = classes[gi];
    std::vector<GemmArgs<double, float>> fw0, fw;
    std::vector<GemmArgs<float, double>> i0, i1;
    std::vector<GemmArgs<double, double>> d0, d1, e0, e1;
    std::vector<int> blocks, blocks_fwd;
    for (int i = 0; i < n; ++i) {
      Plan& P = plan_of(B, i);
      if (shape_of(i) != classes[gi]) continue;
      int blk;
      if (!f64 && G.ntp < 0) {
        // streaming V: the forward and inverse launches split differently
        float* tmp = reinterpret_cast<float*>(P.tmp);
        int bf;
        fw0.push_back(batch_gemm_lps_args<double, float>(P, B.mode, P.r, tmp, DOT_NONE, nullptr,
                                                         nullptr, done_of(B, i), &bf));
        fw.push_back(fw0.back());
        fw.back().nrr = update_grid(P);
        i0.push_back(batch_gemm_lps_args<float, double>(P, B.mode, tmp, P.z, DOT_INIT, P.r,
                                                        nullptr, done_of(B, i), &blk));
        i1.push_back(batch_gemm_lps_args<float, double>(P, B.mode, tmp, P.z,
                                                        pcg_flexible(P) ? DOT_FLEX : DOT_STD,
                                                        P.r, P.q, done_of(B, i), &blk));
        blocks_fwd.push_back(bf);
        blocks.push_back(blk);
        gemm_grid[i] = blk;
        continue;
      }
      if (f64) {
        int kb, cb;
        d0.push_back(batch_gemm64_args(P, P.r, P.tmp, DOT_NONE, nullptr, nullptr, done_of(B, i),
                                       &blk, &kb, &cb));
        d1.push_back(d0.back());
        d1.back().nrr = update_grid(P);
        e0.push_back(batch_gemm64_args(P, P.tmp, P.z, DOT_INIT, P.r, nullptr, done_of(B, i), &blk,
                                       &kb, &cb));
        e1.push_back(batch_gemm64_args(P, P.tmp, P.z, DOT_STD, P.r, P.q, done_of(B, i), &blk, &kb,
                                       &cb));
      } else {
        float* tmp = reinterpret_cast<float*>(P.tmp);
        fw0.push_back(batch_gemm_args<double, float>(P, B.mode, P.r, tmp, DOT_NONE, nullptr,
                                                     nullptr, done_of(B, i), &blk));
        fw.push_back(fw0.back());
        fw.back().nrr = update_grid(P);
        i0.push_back(batch_gemm_args<float, double>(P, B.mode, tmp, P.z, DOT_INIT, P.r, nullptr,
                                                    done_of(B, i), &blk));
        i1.push_back(batch_gemm_args<float, double>(P, B.mode, tmp, P.z,
                                                    pcg_flexible(P) ? DOT_FLEX : DOT_STD, P.r,
                                                    P.q, done_of(B, i), &blk));
      }
      blocks.push_back(blk);
      blocks_fwd.push_back(blk);
      gemm_grid[i] = blk;
    }
    if (f64) {
      if ((rc = upload_phase(B, d0, blocks, G.fwd64_init)) ||
          (rc = upload_phase(B, d1, blocks, G.fwd64)) ||
          (rc = upload_phase(B, e0, blocks, G.inv64_init)) ||
          (rc = upload_phase(B, e1, blocks, G.inv64_iter)))
        return rc;
    } else if ((rc = upload_phase(B, fw0, blocks_fwd, G.fwd_init)) ||
               (rc = upload_phase(B, fw, blocks_fwd, G.fwd)) ||
               (rc = upload_phase(B, i0, blocks, G.inv_init)) ||
               (rc = upload_phase(B, i1, blocks, G.inv_iter))) {
      return rc;
    }
  }
  // the update and the A kernel sum the inverse GEMM's r.z partials themselves
  for (int i = 0; i < n; ++i) {
    u0[i].nrz = uo[i].nrz = ue[i].nrz = gemm_grid[i];
    af[i].nrz = ao[i].nrz = ae[i].nrz = gemm_grid[i];
  }
  if ((rc = upload_phase(B, u0, b_upd, B.upd_first)) ||
      (rc = upload_phase(B, uo, b_upd, B.upd_odd)) || (rc = upload_phase(B, ue, b_upd, B.upd_even)) ||
      (rc = upload_phase(B, af, b_aat, B.aat_first)) ||
      (rc = upload_phase(B, ao, b_aat, B.aat_odd)) || (rc = upload_phase(B, ae, b_aat, B.aat_even)))
    return rc;
  return MFG_OK;
}

// Right-hand side and back-projection phases bound to the states' vectors.
int build_state_phases(Batch& B, mfg_state_t* st) {
  std::vector<RhsArgs> rh;
  std::vector<BackprojArgs> bp, bpm;
  std::vector<int> b_rhs, b_bp;
  std::vector<FinishArgs> fdm;
  for (int i = 0; i < B.count; ++i) {
    Plan& P = plan_of(B, i);
    const double* S = B.scal_all + (size_t)i * S_COUNT;
    double* Sw = B.scal_all + (size_t)i * S_COUNT;
    // the right-hand side goes straight into the PCG residual and starts the solve
    RhsArgs ra = rhs_args(P, st[i].xi, st[i].ybar, 0.0, S + S_SIGMA, P.r, P.zn, S + S_ZMODE);
    ra.init = 1;
    ra.tol2_dev = B.tol2 + i;
    rh.push_back(ra);
    b_rhs.push_back(rhs_grid(P));
    BackprojArgs a = backproj_args(P, P.u, st[i].xi, st[i].y, st[i].ybar, 0.0, 0.0, S + S_TAU,
                                   S + S_THETA, nullptr);
    a.zflag = Sw + S_ZMODE;
    bp.push_back(a);
    a.zout = P.zn;
    a.sigma_dev = S + S_SIGMA;
    bpm.push_back(a);
    b_bp.push_back(backproj_grid(P));
    fdm.push_back(finish_args(P, T_DM, backproj_grid(P), OP_DM));
  }
  int rc;
  if ((rc = upload_phase(B, rh, b_rhs, B.rhs)) || (rc = upload_phase(B, bp, b_bp, B.bp)) ||
      (rc = upload_phase(B, bpm, b_bp, B.bp_mid)) ||
      (rc = upload_finish(B, fdm, &B.f_dm)))
    return rc;
  return MFG_OK;
}

template <typename T>
void spatial_phase(const std::vector<SpatialGroup<T>>& rows, const std::vector<ColsGroup<T>>& cols,
                   hipStream_t s) {
  for (const auto& G : rows)
    launch_rows_batch<T>(G.cls, G.rows_fwd.args, G.rows_fwd.off, G.rows_fwd.ninst,
                         G.rows_fwd.total, G.rows_fwd.shm, G.threads, s);
  for (const auto& G : cols)
    launch_cols_batch<T>(G.cls, G.cols.args, G.cols.off, G.cols.ninst, G.cols.total, G.cols.shm,
                         G.threads, s);
  for (const auto& G : rows)
    launch_rows_batch<T>(G.cls, G.rows_inv.args, G.rows_inv.off, G.rows_inv.ninst,
                         G.rows_inv.total, G.rows_inv.shm, G.threads, s);
}

void precond_phase(Batch& B, bool init, hipStream_t s) {
  if (B.mode == GM_F64) {
    for (auto& G : B.groups) {
      const auto& ph = init ? G.fwd64_init : G.fwd64;
      launch_gemm64_batch(G.kb, G.cb, ph.args, ph.off, ph.ninst, ph.total, s);
    }
    spatial_phase<double>(B.rows64, B.cols64, s);
    for (auto& G : B.groups) {
      const auto& ph = init ? G.inv64_init : G.inv64_iter;
      launch_gemm64_batch(G.kb, G.cb, ph.args, ph.off, ph.ninst, ph.total, s);
    }
    return;
  }
  for (auto& G : B.groups) {
    const auto& ph = init ? G.fwd_init : G.fwd;
    if (G.ntp < 0) launch_gemm_lps_batch<double, float>(B.mode, ph.args, ph.off, ph.ninst,
                                                        ph.total, s);
    else launch_gemm_batch<double, float>(B.mode, G.ntp, G.cb, G.waves, ph.args, ph.off,
                                          ph.ninst, ph.total, s);
  }
  spatial_phase<float>(B.rows, B.cols, s);
  for (auto& G : B.groups) {
    const auto& ph = init ? G.inv_init : G.inv_iter;
    if (G.ntp < 0) launch_gemm_lps_batch<float, double>(B.mode, ph.args, ph.off, ph.ninst,
                                                        ph.total, s);
    else launch_gemm_batch<float, double>(B.mode, G.ntp, G.cb, G.waves, ph.args, ph.off,
                                          ph.ninst, ph.total, s);
  }
}

// PCG iteration k >= 1 for every instance not yet converged.
void pcg_iteration(Batch& B, int k, hipStream_t s) {
  const auto& aat = (k == 1) ? B.aat_first : ((k & 1) ? B.aat_odd : B.aat_even);
  launch_aat_batch(true, aat.args, aat.off, B.count, aat.total, s, B.queue, B.qgrid);
  const auto& upd = (k == 1) ? B.upd_first : ((k & 1) ? B.upd_odd : B.upd_even);
  launch_update_batch(upd.args, upd.off, B.count, upd.total, s);
  precond_phase(B, false, s);
}

// Everything of one CP step before the host looks at convergence: step sizes,
// right-hand side, PCG initialisation and K iterations.
void step_head(Batch& B, int K, int maxit_sched, hipStream_t s) {
  launch_cp_advance_batch(B.scal_all, S_COUNT, B.count, B.sched, maxit_sched, s);
  launch_rhs_batch(B.rhs.args, B.rhs.off, B.count, B.rhs.total, s);  // also starts the PCG
  launch_finish_batch(B.f_bb, B.count, s);
  precond_phase(B, true, s);
  for (int k = 1; k <= K; ++k) pcg_iteration(B, k, s);
}

int read_all(Batch& B) {
  if (hipMemcpyAsync(B.host_scal, B.scal_all, (size_t)B.count * S_COUNT * sizeof(double),
                     hipMemcpyDeviceToHost, B.stream) != hipSuccess ||
      hipStreamSynchronize(B.stream) != hipSuccess)
    return fail(MFG_ERR_HIP, "batch scalar readback failed");
  return MFG_OK;
}

__global__ void k_batch_set(double* scal, int stride, int ninst, int slot, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst) scal[(size_t)i * stride + slot] = v;
}

void release_graph(Batch& B) {
  if (B.exec) (void)hipGraphExecDestroy(B.exec);
  if (B.graph) (void)hipGraphDestroy(B.graph);
  B.exec = nullptr;
  B.graph = nullptr;
  B.graph_k = 0;
}

}  // namespace

int batch_create(Batch& B, const mfg_problem_t* pbs, const double* const* V,
                 const double* const* m0, int count, hipStream_t stream) {
  B.count = count;
  B.user = stream;
  const int prec = pbs[0].precision;
  B.mode = prec == MFG_FP64 ? GM_F64
           : (prec == MFG_MIXED_FP32 ? GM_F32 : (prec == MFG_MIXED_FP16 ? GM_F16 : GM_BF16));
  for (int i = 0; i < count; ++i) {
    if (pbs[i].precision != prec) return fail(MFG_ERR_INVALID_ARG, "mixed precisions in a batch");
    if (pbs[i].d != 2) return fail(MFG_ERR_UNSUPPORTED, "batched solves need d = 2");

    if (pbs[i].qprime != 2.0) return fail(MFG_ERR_UNSUPPORTED, "batched solves need q' = 2");
  }
  if (hipStreamCreateWithFlags(&B.stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&B.ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&B.ev_out, hipEventDisableTiming) != hipSuccess)
    return fail(MFG_ERR_HIP, "stream creation failed");
  for (int i = 0; i < count; ++i) {
    mfg_plan_t h = nullptr;
    int rc = mfg_plan(&pbs[i], V[i], m0[i], stream, &h);
    if (rc) return rc;
    B.plans.push_back(h);
    batch_shape(h->P.tune);  // launch shapes the batched kernels support
    // above N_t = 128 the batched low-precision time GEMM is the streaming one
    if (prec != MFG_FP64 && h->P.ntp == 0 && !h->P.tune.lp_stream)
      return fail(MFG_ERR_UNSUPPORTED,
                  "batched mixed-precision solves above N_t = 128 need the streaming time GEMM");
  }
  int rc;
  void* p;
  if ((rc = dmalloc(B, &p, (size_t)count * S_COUNT * sizeof(double)))) return rc;
  B.scal_all = static_cast<double*>(p);
  if (hipMemset(B.scal_all, 0, (size_t)count * S_COUNT * sizeof(double)) != hipSuccess)
    return fail(MFG_ERR_HIP, "memset failed");
  for (int i = 0; i < count; ++i) plan_of(B, i).red.scal = B.scal_all + (size_t)i * S_COUNT;
  if ((rc = dmalloc(B, &p, (size_t)count * sizeof(double)))) return rc;
  B.tol2 = static_cast<double*>(p);
  if (hipHostMalloc(&p, (size_t)count * S_COUNT * sizeof(double), hipHostMallocDefault) !=
      hipSuccess)
    return fail(MFG_ERR_OOM, "pinned allocation failed");
  B.host_scal = static_cast<double*>(p);
  if (plan_of(B, 0).tune.batch_queue) {
    if ((rc = dmalloc(B, &p, sizeof(int)))) return rc;
    B.queue = static_cast<int*>(p);
    B.qgrid = aat_queue_grid(true);
    if (B.qgrid <= 0) B.queue = nullptr;  // occupancy unknown: one block per tile
  }
  return build_pcg_phases(B);
}

void batch_release(Batch& B) {
  if (B.stream) (void)hipStreamSynchronize(B.stream);
  release_graph(B);
  for (mfg_plan_t h : B.plans) mfg_destroy(h);
  B.plans.clear();
  for (void* p : B.dev) (void)hipFree(p);
  B.dev.clear();
  if (B.host_scal) (void)hipHostFree(B.host_scal);
  B.host_scal = nullptr;
  if (B.ev_in) (void)hipEventDestroy(B.ev_in);
  if (B.ev_out) (void)hipEventDestroy(B.ev_out);
  if (B.stream) (void)hipStreamDestroy(B.stream);
  B.stream = nullptr;
}

int batch_autotune(Batch& B, int effort) {
  if (hipStreamSynchronize(B.stream) != hipSuccess) return fail(MFG_ERR_HIP, "stream sync failed");
  for (int i = 0; i < B.count; ++i) {
    int rc = autotune(plan_of(B, i), effort, false);
    if (rc) return rc;
  }
  // launch shapes changed: rebuild the argument arrays, drop the graph
  release_graph(B);
  return build_pcg_phases(B);
}

int batch_cp_solve(Batch& B, mfg_state_t* st, int n_iter, double rtol, int maxit, int use_graph,
                   int* pcg_iters) {
  hipStream_t s = B.stream;
  const int n = B.count;
  if (n_iter <= 0) return MFG_OK;
  // the previous call's last launches may still read the argument arrays
  if (hipStreamSynchronize(s) != hipSuccess) return fail(MFG_ERR_HIP, "stream sync failed");
  // host schedule (same arithmetic as the single-plan driver)
  std::vector<double> sched((size_t)n * n_iter * 3);
  for (int i = 0; i < n; ++i) {
    double sigma = st[i].sigma, tau = st[i].tau;
    const double gamma = plan_of(B, i).gamma;
    for (int j = 0; j < n_iter; ++j) {
      const double theta = 1.0 / std::sqrt(1.0 + 2.0 * gamma * tau);
      double* e = &sched[((size_t)i * n_iter + j) * 3];
      e[0] = sigma;
      e[1] = tau;
      e[2] = theta;
      tau *= theta;
      sigma /= theta;
    }
  }
  if (n_iter > B.sched_cap) {
    void* p;
    int rc = dmalloc(B, &p, sched.size() * sizeof(double));
    if (rc) return rc;
    B.sched = static_cast<double*>(p);
    B.sched_cap = n_iter;
    release_graph(B);  // the graph holds the old schedule pointer
  }
  std::vector<double> t2(n, rtol * rtol);
  if (hipMemcpy(B.tol2, t2.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return fail(MFG_ERR_HIP, "upload failed");
  // the schedule table is laid out for B.sched_cap iterations per instance
  std::vector<double> padded((size_t)n * B.sched_cap * 3, 0.0);
  for (int i = 0; i < n; ++i)
    std::copy(sched.begin() + (size_t)i * n_iter * 3, sched.begin() + (size_t)(i + 1) * n_iter * 3,
              padded.begin() + (size_t)i * B.sched_cap * 3);
  if (hipMemcpy(B.sched, padded.data(), padded.size() * sizeof(double), hipMemcpyHostToDevice) !=
      hipSuccess)
    return fail(MFG_ERR_HIP, "upload failed");
  std::vector<const double*> want;
  for (int i = 0; i < n; ++i) {
    want.push_back(st[i].xi);
    want.push_back(st[i].y);
    want.push_back(st[i].ybar);
  }
  if (want != B.bound) {
    int rc = build_state_phases(B, st);
    if (rc) return rc;
    B.bound = want;
    release_graph(B);
  }
  if (B.graph_k > maxit) release_graph(B);
  // order after the caller's stream
  (void)hipEventRecord(B.ev_in, B.user);
  (void)hipStreamWaitEvent(s, B.ev_in, 0);
  hipLaunchKernelGGL(k_batch_set, dim3((n + 63) / 64), dim3(64), 0, s, B.scal_all, S_COUNT, n,
                     (int)S_CPIT, 0.0);
  // the first step of the call reads the states' xi and ybar
  hipLaunchKernelGGL(k_batch_set, dim3((n + 63) / 64), dim3(64), 0, s, B.scal_all, S_COUNT, n,
                     (int)S_ZMODE, 0.0);
  int final_rc = MFG_OK;
  // an error inside the loop leaves the states part-way through a step (the
  // device vectors moved, the scalars not): they are marked unusable
  auto abandon = [&](int code, const std::string& msg) {
    for (int i = 0; i < n; ++i) st[i].iter = -1;
    return fail(code, msg);
  };
  for (int it = 0; it < n_iter; ++it) {
    int K = std::min(B.graph_k > 0 ? B.graph_k : 8, maxit);
    if (use_graph && !B.exec && it > 0) {
      // capture with the iteration count the first steps needed
      if (hipStreamBeginCapture(s, hipStreamCaptureModeGlobal) != hipSuccess)
        return abandon(MFG_ERR_HIP, "graph capture failed to start");
      step_head(B, K, B.sched_cap, s);
      if (hipStreamEndCapture(s, &B.graph) != hipSuccess ||
          hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0) != hipSuccess) {
        release_graph(B);
        return abandon(MFG_ERR_HIP, "graph instantiation failed");
      }
      B.graph_k = K;
    }
    if (use_graph && B.exec) {
      if (hipGraphLaunch(B.exec, s) != hipSuccess) return abandon(MFG_ERR_HIP, "graph launch failed");
    } else {
      step_head(B, K, B.sched_cap, s);
    }
    int rc = read_all(B);
    if (rc) return abandon(rc, mfg_last_error());
    int k = K;
    int maxits = 0;
    while (true) {
      bool all = true;
      for (int i = 0; i < n; ++i) {
        const double* S = B.host_scal + (size_t)i * S_COUNT;
        if (S[S_BAD] == 2.0) return abandon(MFG_ERR_NONFINITE, "non-finite value in a batched PCG");
        if (S[S_BAD] == 1.0) return abandon(MFG_ERR_BREAKDOWN, "breakdown in a batched PCG");
        if (S[S_DONE] == 0.0) all = false;
      }
      if (all || k >= maxit) break;
      ++k;
      pcg_iteration(B, k, s);
      if ((rc = read_all(B))) return abandon(rc, mfg_last_error());
    }
    for (int i = 0; i < n; ++i) {
      const double* S = B.host_scal + (size_t)i * S_COUNT;
      const int its = (int)S[S_ITS];
      maxits = std::max(maxits, its);
      if (S[S_DONE] == 0.0) final_rc = MFG_ERR_NOT_CONVERGED;
      if (pcg_iters) pcg_iters[(size_t)it * n + i] = its;
      // b = 0: done before the first update, which would have written u
      if (S[S_DONE] != 0.0 && its == 0) launch_fill(plan_of(B, i).u, plan_of(B, i).g.n, 0.0, s);
    }
    if (!B.exec && B.graph_k == 0) B.graph_k = std::min(std::max(maxits + 1, 2), maxit);
    const auto& bp = (it + 1 < n_iter) ? B.bp_mid : B.bp;
    launch_backproj_batch(bp.args, bp.off, n, bp.total, s);
    launch_finish_batch(B.f_dm, n, s);
  }
  (void)hipEventRecord(B.ev_out, s);
  (void)hipStreamWaitEvent(B.user, B.ev_out, 0);
  if (hipGetLastError() != hipSuccess) return fail(MFG_ERR_HIP, "batched launch failed");
  for (int i = 0; i < n; ++i) {
    const double* e = &sched[((size_t)i * n_iter + (n_iter - 1)) * 3];
    st[i].theta = e[2];
    st[i].tau = e[1] * e[2];
    st[i].sigma = e[0] / e[2];
    st[i].iter += n_iter;
  }
  if (final_rc) return fail(final_rc, "some batched PCG solve reached maxit");
  return MFG_OK;
}

}  // namespace mfg

using mfg::fail;

extern "C" {

int mfg_plan_batch(const mfg_problem_t* pbs, const double* const* V, const double* const* m0,
                   int count, hipStream_t stream, mfg_batch_t* out) {
  if (!pbs || !V || !m0 || !out || count < 1) return fail(MFG_ERR_INVALID_ARG, "bad arguments");
  *out = nullptr;
  mfg_batch_s* h = new (std::nothrow) mfg_batch_s();
  if (!h) return fail(MFG_ERR_OOM, "host allocation failed");
  int rc = mfg::batch_create(h->B, pbs, V, m0, count, stream);
  if (rc) {
    std::string msg = mfg_last_error();
    mfg::batch_release(h->B);
    delete h;
    fail(rc, msg);
    return rc;
  }
  *out = h;
  return MFG_OK;
}

int mfg_batch_destroy(mfg_batch_t b) {
  if (!b) return MFG_OK;
  mfg::batch_release(b->B);
  delete b;
  return MFG_OK;
}

int mfg_batch_plan(mfg_batch_t b, int i, mfg_plan_t* out) {
  if (!b || !out || i < 0 || i >= b->B.count) return fail(MFG_ERR_INVALID_ARG, "bad arguments");
  *out = b->B.plans[i];
  return MFG_OK;
}

int mfg_batch_autotune(mfg_batch_t b, int effort) {
  if (!b || (effort != 1 && effort != 2)) return fail(MFG_ERR_INVALID_ARG, "bad arguments");
  return mfg::batch_autotune(b->B, effort);
}

int mfg_batch_cp_solve(mfg_batch_t b, mfg_state_t* states, int n_iter, double pcg_rtol,
                       int pcg_maxit, int use_graph, int* pcg_iters) {
  if (!b || !states || n_iter < 0 || pcg_maxit < 1 || !(pcg_rtol >= 0.0))
    return fail(MFG_ERR_INVALID_ARG, "bad arguments");
  for (int i = 0; i < b->B.count; ++i)
    if (!states[i].xi || !states[i].y || !states[i].ybar || !(states[i].tau > 0.0) ||
        !(states[i].sigma > 0.0))
      return fail(MFG_ERR_INVALID_ARG, "bad state");
  return mfg::batch_cp_solve(b->B, states, n_iter, pcg_rtol, pcg_maxit, use_graph, pcg_iters);
}

}  // extern "C"
