// Orchestration of the randomized SVD (Sec. 4; Halko et al. 2011, Example
// 1.6 with subspace iteration), the zip-up row absorption, controlled bond
// expansion on explicit matrices and the overlap of two environments.
#include "driver.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <future>
#include <map>

namespace fp {

// ---------------------------------------------------------------------------
// dense (data-independent) plans of one rSVD
// ---------------------------------------------------------------------------
namespace {

struct Layout {
  std::vector<int64_t> rows;
  std::vector<int32_t> k;
  std::vector<int64_t> off;
  int64_t total = 0;
  static int64_t total_of(const std::vector<int64_t>& r, const std::vector<int32_t>& kk) {
    int64_t t = 0;
    for (size_t J = 0; J < r.size(); ++J) t += r[J] * (int64_t)kk[J];
    return t;
  }
  void build(const std::vector<int64_t>& r, const std::vector<int32_t>& kk) {
    rows = r;
    k = kk;
    off.assign(r.size(), 0);
    total = 0;
    for (size_t J = 0; J < r.size(); ++J) {
      off[J] = total;
      total += r[J] * (int64_t)kk[J];
    }
  }
};

int ksplit_for(int64_t K, int k) {
  // enough K chunks that the Gram of a tall block fills the machine
  const int64_t tiles = ((k + 63) / 64) * (int64_t)((k + 63) / 64);
  int64_t want = std::max<int64_t>(1, 512 / std::max<int64_t>(tiles, 1));
  want = std::min<int64_t>(want, std::max<int64_t>(1, K / 256));
  return (int)std::min<int64_t>(want, 256);
}

struct DensePlans {
  PlanSet ps;
  int gram[2] = {-1, -1};   // 0: row layout, 1: column layout
  int qmul[2] = {-1, -1};
  int mm = -1;              // per sector: (k x k at v0) times (k x k at S), into [0, S)
  int vtv = -1;             // per sector: V^T V of the k x k V at S, into [0, S)
  int vx = -1;              // per sector: V (at S) times X (at v0), into [0, S)
  std::vector<ReduceDesc> red[2];
  int64_t part_total[2] = {0, 0};
  std::vector<int64_t> small_off, lam_off;
  int64_t S = 0, lam_total = 0;
  int max_k = 0;
  int max_red_mn = 0;
};

Status build_dense(fpeps_ctx_s* ctx, const Layout& L0, const Layout& L1, DensePlans& dp,
                   const std::string& tag) {
  const int ns = (int)L0.k.size();
  dp.small_off.assign(ns, 0);
  dp.lam_off.assign(ns, 0);
  dp.S = 0;
  dp.lam_total = 0;
  for (int J = 0; J < ns; ++J) {
    dp.small_off[J] = dp.S;
    dp.lam_off[J] = dp.lam_total;
    dp.S += (int64_t)L0.k[J] * L0.k[J];
    dp.lam_total += L0.k[J];
    dp.max_k = std::max(dp.max_k, (int)L0.k[J]);
  }
  const Layout* Ls[2] = {&L0, &L1};
  std::string err;
  for (int side = 0; side < 2; ++side) {
    const Layout& L = *Ls[side];
    std::vector<DenseOp> gops, qops;
    dp.red[side].clear();
    int64_t poff = 0;
    for (int J = 0; J < ns; ++J) {
      const int k = L.k[J];
      if (k <= 0 || L.rows[J] <= 0) continue;
      const int ks = ksplit_for(L.rows[J], k);
      DenseOp g{};
      g.a_off = L.off[J];
      g.b_off = L.off[J];
      g.c_off = poff;
      g.M = k;
      g.N = k;
      g.K = (int32_t)L.rows[J];
      g.a_rs = 1;
      g.a_cs = k;
      g.b_rs = k;
      g.b_cs = 1;
      g.c_rs = k;
      g.c_cs = 1;
      g.alpha = 1.0;
      g.ksplit = std::max(ks, 2);
      gops.push_back(g);
      ReduceDesc r{};
      r.c_off = dp.small_off[J];
      r.c_rs = k;
      r.c_cs = 1;
      r.p_off = poff;
      r.M = k;
      r.N = k;
      r.nsplit = g.ksplit;
      dp.red[side].push_back(r);
      dp.max_red_mn = std::max(dp.max_red_mn, k * k);
      poff += (int64_t)g.ksplit * k * k;
      DenseOp q{};
      q.a_off = L.off[J];
      q.b_off = dp.S + dp.small_off[J];
      q.c_off = L.off[J];
      q.M = (int32_t)L.rows[J];
      q.N = k;
      q.K = k;
      q.a_rs = k;
      q.a_cs = 1;
      q.b_rs = k;
      q.b_cs = 1;
      q.c_rs = k;
      q.c_cs = 1;
      q.alpha = 1.0;
      qops.push_back(q);
    }
    dp.part_total[side] = poff;
    GemmPlan gp, qp;
    if (!plan_dense(gops, dp.ps.pool, 64, 64, 1, gp, err)) return fail(FPEPS_ERR_SHAPE, err);
    if (!plan_dense(qops, dp.ps.pool, 64, 64, 1, qp, err)) return fail(FPEPS_ERR_SHAPE, err);
    dp.gram[side] = dp.ps.add(std::move(gp));
    dp.qmul[side] = dp.ps.add(std::move(qp));
  }
  // U~ = V0 V1 of the core factorisation: V0 kept after the S + lam part
  std::vector<DenseOp> mops;
  const int64_t v0_base = 2 * dp.S + dp.lam_total;
  for (int J = 0; J < ns; ++J) {
    const int k = L0.k[J];
    if (k <= 0) continue;
    DenseOp o{};
    o.a_off = v0_base + dp.small_off[J];
    o.b_off = dp.S + dp.small_off[J];
    o.c_off = dp.small_off[J];
    o.M = o.N = o.K = k;
    o.a_rs = k;
    o.a_cs = 1;
    o.b_rs = k;
    o.b_cs = 1;
    o.c_rs = k;
    o.c_cs = 1;
    o.alpha = 1.0;
    mops.push_back(o);
  }
  GemmPlan mp;
  if (!plan_dense(mops, dp.ps.pool, 64, 64, 1, mp, err)) return fail(FPEPS_ERR_SHAPE, err);
  dp.mm = dp.ps.add(std::move(mp));
  // re-orthonormalisation of V (one CholeskyQR pass): V^T V and V X
  std::vector<DenseOp> tops = mops, xops = mops;
  for (size_t i = 0; i < mops.size(); ++i) {
    tops[i].a_off = mops[i].b_off;   // V^T: V read by columns
    tops[i].a_rs = 1;
    tops[i].a_cs = mops[i].M;
    xops[i].a_off = mops[i].b_off;   // V times X (X at the V0 place)
    xops[i].b_off = mops[i].a_off;
  }
  GemmPlan tp, xp;
  if (!plan_dense(tops, dp.ps.pool, 64, 64, 1, tp, err)) return fail(FPEPS_ERR_SHAPE, err);
  if (!plan_dense(xops, dp.ps.pool, 64, 64, 1, xp, err)) return fail(FPEPS_ERR_SHAPE, err);
  dp.vtv = dp.ps.add(std::move(tp));
  dp.vx = dp.ps.add(std::move(xp));
  return dp.ps.upload(ctx, tag);
}

// Widths up to these run on one workgroup per matrix (the matrix in LDS for
// the eigensolver); wider ones on the multi-workgroup blocked kernels. The
// relative-rule eigensolver always runs on one workgroup (plane rotations
// one at a time keep every eigenvalue's relative accuracy).
constexpr int CHOL_ONE_WG_MAX_K = 64;
constexpr int EIG_ONE_WG_MAX_K = 80;

// Shifted Cholesky and inverse of a batch (contract of launch_chol_inv).
Status chol_inv(fpeps_ctx_s* ctx, const SmallDesc* dd, int nd, int max_k, double* small,
                int* status) {
  if (max_k <= CHOL_ONE_WG_MAX_K) {
    FP_HIP(launch_chol_inv(dd, nd, small, status, ctx->stream));
    return Status::ok();
  }
  int* zf = nullptr;
  FP_TRY(ctx->bufT("ch_zf", (size_t)std::max(nd, 1), &zf));
  FP_HIP(launch_chol_inv_blocked(dd, nd, max_k, small, zf, status, ctx->stream));
  return Status::ok();
}

// Symmetric eigen-decomposition of a batch (contract of launch_jacobi_eig).
// The blocked solver (absolute rule, wide matrices; *blocked set) syncs once
// per sweep to test convergence.
Status eig_sym(fpeps_ctx_s* ctx, const SmallDesc* dd, int nd, int max_k, double* small,
               int* status, bool rel, bool* blocked = nullptr) {
  if (blocked) *blocked = false;
  if (rel || max_k <= EIG_ONE_WG_MAX_K) {
    if (max_k > JACOBI_MAX_K)
      return fail(FPEPS_ERR_UNSUPPORTED, "sketch width above " + std::to_string(JACOBI_MAX_K));
    FP_HIP(launch_jacobi_eig(dd, nd, max_k, small, status, ctx->stream, rel));
    return Status::ok();
  }
  if (blocked) *blocked = true;
  int* flags = nullptr;
  double* work = nullptr;
  FP_TRY(ctx->bufT("bj_flags", (size_t)2 * nd + 1, &flags));
  FP_TRY(ctx->bufT("bj_work", bj_work_doubles(nd, max_k), &work));
  FP_HIP(launch_fill_int(flags, 2 * (int64_t)nd + 1, 0, ctx->stream));
  FP_HIP(launch_bj_init(dd, nd, max_k, small, flags, work, ctx->stream));
  bool converged = false;
  for (int sweep = 0; sweep < 30 && !converged; ++sweep) {
    FP_HIP(launch_bj_sweep(dd, nd, max_k, small, flags, work, ctx->stream));
    int left = 0;
    FP_HIP(hipMemcpyAsync(&left, flags + 2 * nd, sizeof(int), hipMemcpyDeviceToHost,
                          ctx->stream));
    FP_TRY(ctx->sync());
    converged = left == 0;
  }
  FP_HIP(launch_bj_finish(dd, nd, max_k, small, work, ctx->stream));
  if (!converged) {
    // the Jacobi limit bit, as the one-workgroup solver reports it
    int hs = 0;
    FP_HIP(hipMemcpyAsync(&hs, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    FP_TRY(ctx->sync());
    hs |= 4;
    FP_HIP(hipMemcpyAsync(status, &hs, sizeof(int), hipMemcpyHostToDevice, ctx->stream));
    FP_TRY(ctx->sync());
  }
  return Status::ok();
}

// Shifted CholeskyQR3 of the per-sector blocks in ``Y`` (layout ``side``),
// ping-ponging with ``Wb``. Returns the buffer that holds Q.
Status orth(fpeps_ctx_s* ctx, DensePlans& dp, int side, const Layout& L, double* Y, double* Wb,
            double** Qout, uint32_t* fallbacks) {
  double *part = nullptr, *small = nullptr;
  int* status = nullptr;
  FP_TRY(ctx->bufT("rs_part", (size_t)std::max<int64_t>(dp.part_total[side], 1), &part));
  FP_TRY(ctx->bufT("rs_small", (size_t)(3 * dp.S + dp.lam_total + 1), &small));
  FP_TRY(ctx->bufT("rs_status", L.k.size() + 2, &status));
  ReduceDesc* dred = nullptr;
  FP_TRY(ctx->upload("rs_red" + std::to_string(side), dp.red[side].data(),
                     dp.red[side].size() * sizeof(ReduceDesc), (void**)&dred));
  std::vector<SmallDesc> ch;
  for (size_t J = 0; J < L.k.size(); ++J) {
    if (L.k[J] <= 0 || L.rows[J] <= 0) continue;
    SmallDesc d{};
    d.a_off = dp.small_off[J];
    d.b_off = dp.S + dp.small_off[J];
    d.c_off = 2 * dp.S + dp.lam_off[J];
    d.k = L.k[J];
    d.rows = (int32_t)std::min<int64_t>(L.rows[J], INT32_MAX);
    d.shift = 0.0;
    ch.push_back(d);
  }
  SmallDesc* dch = nullptr;
  std::vector<SmallDesc> ch_shift = ch;
  for (auto& d : ch_shift) d.shift = 11.0;
  FP_TRY(ctx->upload("rs_chol0", ch_shift.data(), ch_shift.size() * sizeof(SmallDesc), (void**)&dch));
  SmallDesc* dch1 = nullptr;
  FP_TRY(ctx->upload("rs_chol1", ch.data(), ch.size() * sizeof(SmallDesc), (void**)&dch1));
  const int64_t small_n = 3 * dp.S + dp.lam_total + 1;
  // Shifted CholeskyQR3 (Fukaya et al.): one shifted pass, then two plain
  // passes. A plain pass whose Cholesky breaks down (a rank-deficient
  // sketch: its null directions are still at rounding level after the
  // shifted pass) is replaced by one more shifted pass, which lifts the
  // smallest directions by a factor of about 1/sqrt(shift) each time; null
  // directions at rounding level become an arbitrary orthonormal completion
  // (as with Householder QR) and small but genuine directions keep their
  // share of the range. A sketch that is rank-deficient exactly (an operator
  // block with fewer nonzero rows than sketch columns: no shift can lift
  // what is structurally zero) still breaks down after three shifted
  // passes; by then every genuine direction is of order one, and two SVQB
  // passes (Stathopoulos & Wu) finish it, turning the exact null directions
  // (Gram eigenvalues below 1e-8 of the largest) into zero columns.
  auto pass = [&](bool shifted) -> Status {
    FP_TRY(run_gemm(ctx, dp.ps, dp.gram[side], Y, L.total, Y, L.total, part,
                    std::max<int64_t>(dp.part_total[side], 1)));
    FP_HIP(launch_reduce_partials(dred, (int)dp.red[side].size(), dp.max_red_mn, small, part,
                                  ctx->stream));
    FP_TRY(chol_inv(ctx, shifted ? dch : dch1, (int)ch.size(), dp.max_k, small, status));
    return Status::ok();
  };
  auto apply_r = [&]() -> Status {
    FP_TRY(run_gemm(ctx, dp.ps, dp.qmul[side], Y, L.total, small, small_n, Wb, L.total));
    std::swap(Y, Wb);
    return Status::ok();
  };
  int nshift = 1;
  bool svqb = false;
  FP_TRY(pass(true));
  FP_TRY(apply_r());
  for (;;) {
    FP_HIP(launch_fill_int(status, (int64_t)L.k.size() + 2, 0, ctx->stream));
    FP_TRY(pass(false));
    int hs = 0;
    FP_HIP(hipMemcpyAsync(&hs, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
    FP_TRY(ctx->sync());
    if (!(hs & 1)) break;
    *fallbacks |= 1u;
    if (nshift >= 3) {
      svqb = true;
      break;
    }
    FP_TRY(pass(true));   // the failed factorisation overwrote the Gram matrix
    FP_TRY(apply_r());
    ++nshift;
  }
  if (svqb) {
    *fallbacks |= 4u;
    for (int sp = 0; sp < 2; ++sp) {
      FP_TRY(run_gemm(ctx, dp.ps, dp.gram[side], Y, L.total, Y, L.total, part,
                      std::max<int64_t>(dp.part_total[side], 1)));
      FP_HIP(launch_reduce_partials(dred, (int)dp.red[side].size(), dp.max_red_mn, small, part,
                                    ctx->stream));
      FP_TRY(eig_sym(ctx, dch1, (int)ch.size(), dp.max_k, small, status, false));
      FP_HIP(launch_svqb_scale(dch1, (int)ch.size(), small, 1e-8, ctx->stream));
      FP_TRY(apply_r());
    }
    FP_TRY(ctx->sync());
    *Qout = Y;
    return Status::ok();
  }
  FP_TRY(apply_r());
  FP_HIP(launch_fill_int(status, (int64_t)L.k.size() + 2, 0, ctx->stream));
  FP_TRY(pass(false));
  FP_TRY(apply_r());
  int hs = 0;
  FP_HIP(hipMemcpyAsync(&hs, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  FP_TRY(ctx->sync());
  if (hs & 1) return fail(FPEPS_ERR_NUMERIC, "Cholesky breakdown in the orthonormalisation");
  *Qout = Y;
  return Status::ok();
}

}  // namespace

// ---------------------------------------------------------------------------
// generic randomized SVD over sectors
// ---------------------------------------------------------------------------
namespace {

// Global cut of every group (sectors listed group by group) over the
// eigenvalues in ``out.small``: kept counts, cut statistics and the host
// copy of the eigenvalues.
Status cut_run(fpeps_ctx_s* ctx, const RsvdIO& io, int chi, const std::vector<double>& gfloor,
               RsvdOut& out) {
  const int ns = (int)io.m.size();
  const int ngrp = (int)gfloor.size();
  auto grp_of = [&](int J) { return io.grp.empty() ? 0 : io.grp[J]; };
  double* small = out.small;
  int64_t lam_total = 0;
  for (int J = 0; J < ns; ++J) lam_total += std::max(out.k[J], 0);
  std::vector<int64_t> loff;
  std::vector<int32_t> kk;
  std::vector<int> sidx;
  std::vector<CutGroup> cg(ngrp, CutGroup{0, 0, 0, 0, 0.0});
  int max_ns = 0, max_total = 0;
  for (int g = 0; g < ngrp; ++g) {
    cg[g].s0 = (int32_t)kk.size();
    cg[g].floor = gfloor[g];
    for (int J = 0; J < ns; ++J) {
      if (out.k[J] <= 0 || grp_of(J) != g) continue;
      loff.push_back(2 * out.S + out.lam_off[J]);
      kk.push_back(out.k[J]);
      sidx.push_back(J);
      cg[g].total += out.k[J];
    }
    cg[g].ns = (int32_t)kk.size() - cg[g].s0;
    max_ns = std::max(max_ns, (int)cg[g].ns);
    max_total = std::max(max_total, (int)cg[g].total);
  }
  int64_t* dloff = nullptr;
  int32_t* dkk = nullptr;
  int32_t* dkept = nullptr;
  CutOut* dcut = nullptr;
  CutGroup* dcg = nullptr;
  FP_TRY(ctx->upload("rs_loff", loff.data(), loff.size() * sizeof(int64_t), (void**)&dloff));
  FP_TRY(ctx->upload("rs_kk", kk.data(), kk.size() * sizeof(int32_t), (void**)&dkk));
  FP_TRY(ctx->upload("rs_cg", cg.data(), cg.size() * sizeof(CutGroup), (void**)&dcg));
  FP_TRY(ctx->bufT("rs_kept", kk.size() + 1, &dkept));
  FP_TRY(ctx->bufT("rs_cut", (size_t)ngrp, &dcut));
  if (max_total > 6144 || max_ns > 1024)
    return fail(FPEPS_ERR_UNSUPPORTED, "too many singular values for the on-chip cut");
  FP_HIP(launch_cut(dcg, ngrp, max_ns, max_total, dloff, dkk, chi, small, dkept, dcut,
                    ctx->stream));
  std::vector<int32_t> kept_c(kk.size());
  out.cuts.assign(ngrp, CutOut{});
  FP_HIP(hipMemcpyAsync(kept_c.data(), dkept, kk.size() * sizeof(int32_t),
                        hipMemcpyDeviceToHost, ctx->stream));
  FP_HIP(hipMemcpyAsync(out.cuts.data(), dcut, ngrp * sizeof(CutOut), hipMemcpyDeviceToHost,
                        ctx->stream));
  out.lam.assign(lam_total, 0.0);
  if (lam_total)
    FP_HIP(hipMemcpyAsync(out.lam.data(), small + 2 * out.S, lam_total * sizeof(double),
                          hipMemcpyDeviceToHost, ctx->stream));
  FP_TRY(ctx->sync());
  out.cut = out.cuts[0];
  out.kept.assign(ns, 0);
  for (size_t i = 0; i < sidx.size(); ++i) out.kept[sidx[i]] = kept_c[i];
  for (double v : out.lam)
    if (!std::isfinite(v)) return fail(FPEPS_ERR_NUMERIC, "non-finite singular value");
  return Status::ok();
}

// One factorisation with fixed sketch widths k (Halko et al. Ex. 1.6): range
// finder with q power iterations, B^T = M^T Q, core factorisation of B and
// (do_cut) the global cut of every group. Sectors of width 0 are skipped.
Status rsvd_pass(fpeps_ctx_s* ctx, RsvdIO& io, const std::vector<int32_t>& k, int chi, int q,
                 uint64_t seed, const std::vector<double>& gfloor, RsvdOut& out,
                 bool do_cut = true) {
  const int ns = (int)io.m.size();
  out.k = k;
  FP_TRY(io.prepare(out.k));
  Layout RL, CL;
  RL.build(io.m, out.k);
  CL.build(io.n, out.k);
  DensePlans dp;
  FP_TRY(build_dense(ctx, RL, CL, dp, "rsd"));
  out.small_off = dp.small_off;
  out.lam_off = dp.lam_off;
  out.S = dp.S;
  out.row_off = RL.off;
  out.col_off = CL.off;
  double *c0, *c1, *r0, *r1;
  FP_TRY(ctx->bufT("rs_c0", (size_t)std::max<int64_t>(CL.total, 1), &c0));
  FP_TRY(ctx->bufT("rs_c1", (size_t)std::max<int64_t>(CL.total, 1), &c1));
  FP_TRY(ctx->bufT("rs_r0", (size_t)std::max<int64_t>(RL.total, 1), &r0));
  FP_TRY(ctx->bufT("rs_r1", (size_t)std::max<int64_t>(RL.total, 1), &r1));
  // Gaussian sketch per sector
  std::vector<GaussDesc> gd;
  int64_t maxe = 0;
  for (int J = 0; J < ns; ++J) {
    if (out.k[J] <= 0) continue;
    GaussDesc g{};
    g.off = CL.off[J];
    g.nelem = io.n[J] * (int64_t)out.k[J];
    g.c1 = io.c1[J];
    g.c2 = io.c2v.empty() ? io.c2 : io.c2v[J];
    g.c3 = io.c3;
    gd.push_back(g);
    maxe = std::max(maxe, g.nelem);
  }
  GaussDesc* dgd = nullptr;
  FP_TRY(ctx->upload("rs_gauss", gd.data(), gd.size() * sizeof(GaussDesc), (void**)&dgd));
  FP_HIP(launch_gaussian(dgd, (int)gd.size(), maxe, c0, seed, ctx->stream));
  // stage A
  // the last product of the range finder (it fixes Q) and the projection
  // are "final": FP64 intermediates in mixed precision
  FP_TRY(io.apply(false, q == 0, c0, r0));
  double* Q = nullptr;
  FP_TRY(orth(ctx, dp, 0, RL, r0, r1, &Q, &out.fallbacks));
  for (int it = 0; it < q; ++it) {
    FP_TRY(io.apply(true, false, Q, c0));
    double* Qz = nullptr;
    FP_TRY(orth(ctx, dp, 1, CL, c0, c1, &Qz, &out.fallbacks));
    double* Yb = (Q == r0) ? r1 : r0;
    FP_TRY(io.apply(false, it == q - 1, Qz, Yb));
    double* other = (Yb == r0) ? r1 : r0;
    FP_TRY(orth(ctx, dp, 0, RL, Yb, other, &Q, &out.fallbacks));
  }
  // stage B: B^T = M^T Q
  double* Bt = c0;
  FP_TRY(io.apply(true, true, Q, Bt));
  out.Q = Q;
  out.Bt = Bt;
  // Core factorisation of B without squaring its condition number in the
  // result: (1) V0 = eigenvectors of B B^T (Gram of the columns of B^T,
  // Jacobi); (2) C = B^T V0 has nearly orthogonal columns whose norms are
  // the singular values, so the Jacobi eigen-decomposition of C^T C with
  // the relative stopping rule resolves every value to its own size
  // (Demmel & Veselic 1992); (3) U~ = V0 V1. The values then carry an
  // absolute error of a few eps times the largest, like a backward-stable
  // SVD of B.
  double *part = nullptr, *small = nullptr;
  int* status = nullptr;
  FP_TRY(ctx->bufT("rs_part", (size_t)std::max<int64_t>(dp.part_total[1], 1), &part));
  FP_TRY(ctx->bufT("rs_small", (size_t)(3 * dp.S + dp.lam_total + 1), &small));
  FP_TRY(ctx->bufT("rs_status", 4, &status));
  ReduceDesc* dred = nullptr;
  FP_TRY(ctx->upload("rs_red1", dp.red[1].data(), dp.red[1].size() * sizeof(ReduceDesc),
                     (void**)&dred));
  std::vector<SmallDesc> jd;
  const int64_t v0_base = 2 * dp.S + dp.lam_total;
  for (int J = 0; J < ns; ++J) {
    if (out.k[J] <= 0) continue;
    SmallDesc d{};
    d.a_off = dp.small_off[J];
    d.b_off = dp.S + dp.small_off[J];
    d.c_off = 2 * dp.S + dp.lam_off[J];
    d.k = out.k[J];
    jd.push_back(d);
  }
  SmallDesc* djd = nullptr;
  FP_TRY(ctx->upload("rs_jac", jd.data(), jd.size() * sizeof(SmallDesc), (void**)&djd));
  FP_HIP(launch_fill_int(status, 4, 0, ctx->stream));
  FP_TRY(run_gemm(ctx, dp.ps, dp.gram[1], Bt, CL.total, Bt, CL.total, part,
                  std::max<int64_t>(dp.part_total[1], 1)));
  FP_HIP(launch_reduce_partials(dred, (int)dp.red[1].size(), dp.max_red_mn, small, part,
                                ctx->stream));
  bool blocked = false;
  FP_TRY(eig_sym(ctx, djd, (int)jd.size(), dp.max_k, small, status, false, &blocked));
  const int64_t small_n = 3 * dp.S + dp.lam_total + 1;
  if (blocked && dp.S > 0) {
    // the block solver's V0 is orthogonal to about 1e-13 only; one
    // CholeskyQR pass (V0 <- V0 R^{-1}, R^T R = V0^T V0) brings it to
    // rounding level, so that C below keeps the singular values of B
    std::vector<SmallDesc> od = jd;
    for (size_t i = 0; i < od.size(); ++i) {
      od[i].b_off = v0_base + jd[i].a_off;
      od[i].rows = jd[i].k;
      od[i].shift = 0.0;
    }
    SmallDesc* dod = nullptr;
    int* ostat = nullptr;
    FP_TRY(ctx->upload("rs_reorth", od.data(), od.size() * sizeof(SmallDesc), (void**)&dod));
    FP_TRY(ctx->bufT("rs_ostat", od.size() + 2, &ostat));
    FP_HIP(launch_fill_int(ostat, (int64_t)od.size() + 2, 0, ctx->stream));
    FP_TRY(run_gemm(ctx, dp.ps, dp.vtv, small, small_n, small, small_n, small, small_n));
    FP_TRY(chol_inv(ctx, dod, (int)od.size(), dp.max_k, small, ostat));
    FP_TRY(run_gemm(ctx, dp.ps, dp.vx, small, small_n, small, small_n, small, small_n));
    FP_HIP(hipMemcpyAsync(small + dp.S, small, dp.S * sizeof(double), hipMemcpyDeviceToDevice,
                          ctx->stream));
  }
  if (dp.S > 0)
    FP_HIP(hipMemcpyAsync(small + v0_base, small + dp.S, dp.S * sizeof(double),
                          hipMemcpyDeviceToDevice, ctx->stream));
  FP_TRY(run_gemm(ctx, dp.ps, dp.qmul[1], Bt, CL.total, small, small_n, c1, CL.total));
  FP_TRY(run_gemm(ctx, dp.ps, dp.gram[1], c1, CL.total, c1, CL.total, part,
                  std::max<int64_t>(dp.part_total[1], 1)));
  FP_HIP(launch_reduce_partials(dred, (int)dp.red[1].size(), dp.max_red_mn, small, part,
                                ctx->stream));
  FP_TRY(eig_sym(ctx, djd, (int)jd.size(), dp.max_k, small, status, true));
  // U~ = V0 V1 (into the free [0, S) part, then back to V's place)
  FP_TRY(run_gemm(ctx, dp.ps, dp.mm, small, small_n, small, small_n, small, small_n));
  if (dp.S > 0)
    FP_HIP(hipMemcpyAsync(small + dp.S, small, dp.S * sizeof(double), hipMemcpyDeviceToDevice,
                          ctx->stream));
  int hs = 0;
  FP_HIP(hipMemcpyAsync(&hs, status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  FP_TRY(ctx->sync());
  if (hs & 4) out.fallbacks |= 2u;
  out.small = small;
  if (do_cut) FP_TRY(cut_run(ctx, io, chi, gfloor, out));
  return Status::ok();
}

}  // namespace

Status rsvd_run(fpeps_ctx_s* ctx, RsvdIO& io, int chi, int p, int q, uint64_t seed,
                RsvdOut& out, double sv_cut) {
  const int ns = (int)io.m.size();
  // Sketch widths (Halko et al. Sec. 4.2: the target rank plus p columns):
  // k_J = min(m_J, n_J, h_J + p) with h_J the caller's guess of the kept
  // count (hint) or the share ceil(chi m_J / sum m) of chi in the sector's
  // group. A sector is saturated when its sketch does not cover it and the
  // cut kept more than k_J - p/2 of its values; saturated sectors are
  // widened to min(m_J, n_J, 2 k_J + p) and the factorisation is repeated.
  const std::vector<int64_t>& wm = io.width_m.empty() ? io.m : io.width_m;
  const std::vector<int64_t>& wn = io.width_n.empty() ? io.n : io.width_n;
  if (!io.grp.empty() && (int)io.grp.size() != ns) return fail(FPEPS_ERR_ARG, "group list size");
  if (!io.c2v.empty() && (int)io.c2v.size() != ns) return fail(FPEPS_ERR_ARG, "tag list size");
  if (!io.hint.empty() && (int)io.hint.size() != ns) return fail(FPEPS_ERR_ARG, "hint list size");
  int ngrp = 1;
  for (int g : io.grp) {
    if (g < 0) return fail(FPEPS_ERR_ARG, "negative group");
    ngrp = std::max(ngrp, g + 1);
  }
  auto grp_of = [&](int J) { return io.grp.empty() ? 0 : io.grp[J]; };
  std::vector<int64_t> msum(ngrp, 0), maxdim(ngrp, 0);
  for (int J = 0; J < ns; ++J) {
    msum[grp_of(J)] += std::max<int64_t>(wm[J], 0);
    maxdim[grp_of(J)] = std::max({maxdim[grp_of(J)], wm[J], wn[J]});
  }
  // truncation floor per group: eps * max(m_J, n_J) relative to the largest
  // value (the rank tolerance of Numerical Recipes Sec. 2.6), or sv_cut
  std::vector<double> gfloor(ngrp);
  for (int g = 0; g < ngrp; ++g)
    gfloor[g] = sv_cut > 0.0 ? sv_cut : 2.220446049250313e-16 * (double)maxdim[g];
  std::vector<int32_t> k(ns, 0);
  for (int J = 0; J < ns; ++J) {
    const int64_t ms = msum[grp_of(J)];
    if (wm[J] <= 0 || wn[J] <= 0 || ms <= 0) continue;
    const int64_t h = (!io.hint.empty() && io.hint[J] >= 0) ? io.hint[J]
                                                             : ((int64_t)chi * wm[J] + ms - 1) / ms;
    k[J] = (int32_t)std::min({wm[J], wn[J], h + p});
  }
  out.pass_k.clear();
  out.pass_kept.clear();
  auto log_pass = [&](const std::vector<int32_t>& kp) {
    if (!ctx->verbose) return;
    std::fprintf(stderr, "[fpeps] rsvd pass %zu: widths", out.pass_k.size());
    for (int v : kp) std::fprintf(stderr, " %d", v);
    std::fprintf(stderr, " | kept");
    for (int v : out.kept) std::fprintf(stderr, " %d", v);
    std::fprintf(stderr, "\n");
  };
  out.fallbacks = 0;
  FP_TRY(rsvd_pass(ctx, io, k, chi, q, seed, gfloor, out));
  uint32_t fb = out.fallbacks;
  out.pass_k.push_back(out.k);
  out.pass_kept.push_back(out.kept);
  log_pass(out.k);
  for (;;) {
    std::vector<int32_t> grow(ns, 0);
    bool any = false;
    for (int J = 0; J < ns; ++J) {
      const int64_t cover = std::min(wm[J], wn[J]);
      if (k[J] > 0 && k[J] < cover && 2 * (int64_t)out.kept[J] + p > 2 * (int64_t)k[J]) {
        grow[J] = (int32_t)std::min<int64_t>(cover, 2 * (int64_t)k[J] + p);
        any = true;
      }
    }
    if (!any) break;
    // A sector keeps its sketch (the same Gaussian columns for the same
    // width), so a repeated factorisation of an unwidened sector would give
    // its previous result again: only the widened sectors are factorised,
    // the others keep theirs, and the cut runs over all of them.
    // The current results move aside first (the pass reuses the buffers).
    const int64_t q_n = std::max<int64_t>(Layout::total_of(io.m, k), 1);
    const int64_t b_n = std::max<int64_t>(Layout::total_of(io.n, k), 1);
    const int64_t s_n = 3 * out.S + (int64_t)std::accumulate(k.begin(), k.end(), (int64_t)0) + 1;
    double *kq = nullptr, *kb = nullptr, *ks = nullptr;
    FP_TRY(ctx->bufT("rs_keep_q", (size_t)q_n, &kq));
    FP_TRY(ctx->bufT("rs_keep_b", (size_t)b_n, &kb));
    FP_TRY(ctx->bufT("rs_keep_s", (size_t)s_n, &ks));
    FP_HIP(hipMemcpyAsync(kq, out.Q, q_n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    FP_HIP(hipMemcpyAsync(kb, out.Bt, b_n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    FP_HIP(hipMemcpyAsync(ks, out.small, s_n * sizeof(double), hipMemcpyDeviceToDevice,
                          ctx->stream));
    const RsvdOut prev = out;
    RsvdOut part;
    part.fallbacks = 0;
    FP_TRY(rsvd_pass(ctx, io, grow, chi, q, seed, gfloor, part, false));
    fb |= part.fallbacks;
    // merged layout: widened sectors from this pass, the others from before
    std::vector<int32_t> kf(ns);
    for (int J = 0; J < ns; ++J) kf[J] = grow[J] > 0 ? grow[J] : k[J];
    Layout RL, CL;
    RL.build(io.m, kf);
    CL.build(io.n, kf);
    RsvdOut mg;
    mg.k = kf;
    mg.row_off = RL.off;
    mg.col_off = CL.off;
    mg.small_off.assign(ns, 0);
    mg.lam_off.assign(ns, 0);
    int64_t S = 0, lt = 0;
    for (int J = 0; J < ns; ++J) {
      mg.small_off[J] = S;
      mg.lam_off[J] = lt;
      S += (int64_t)kf[J] * kf[J];
      lt += kf[J];
    }
    mg.S = S;
    FP_TRY(ctx->bufT("rs_merge_q", (size_t)std::max<int64_t>(RL.total, 1), &mg.Q));
    FP_TRY(ctx->bufT("rs_merge_b", (size_t)std::max<int64_t>(CL.total, 1), &mg.Bt));
    FP_TRY(ctx->bufT("rs_merge_s", (size_t)(3 * S + lt + 1), &mg.small));
    auto copy = [&](double* dst, const double* src, int64_t n) -> Status {
      if (n > 0)
        FP_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice,
                              ctx->stream));
      return Status::ok();
    };
    for (int J = 0; J < ns; ++J) {
      const int kj = kf[J];
      if (kj <= 0) continue;
      const bool g = grow[J] > 0;
      const RsvdOut& src = g ? part : prev;
      const double* sq = g ? part.Q : kq;
      const double* sb = g ? part.Bt : kb;
      const double* ss = g ? part.small : ks;
      FP_TRY(copy(mg.Q + mg.row_off[J], sq + src.row_off[J], io.m[J] * (int64_t)kj));
      FP_TRY(copy(mg.Bt + mg.col_off[J], sb + src.col_off[J], io.n[J] * (int64_t)kj));
      FP_TRY(copy(mg.small + S + mg.small_off[J], ss + src.S + src.small_off[J],
                  (int64_t)kj * kj));
      FP_TRY(copy(mg.small + 2 * S + mg.lam_off[J], ss + 2 * src.S + src.lam_off[J], kj));
    }
    FP_TRY(cut_run(ctx, io, chi, gfloor, mg));
    mg.pass_k = std::move(out.pass_k);
    mg.pass_kept = std::move(out.pass_kept);
    out = std::move(mg);
    k = kf;
    out.pass_k.push_back(grow);
    out.pass_kept.push_back(out.kept);
    log_pass(grow);
  }
  out.fallbacks = fb;
  return Status::ok();
}

// U_J = Q_J U~_J[:, :kept_J] into ``Uout`` (offsets uoff, row stride kept_J)
// and R_J = U~_J[:, :kept_J]^T B_J into ``Rout`` (offsets roff, kept_J x n_J).
Status rsvd_factors(fpeps_ctx_s* ctx, const RsvdIO& io, const RsvdOut& r,
                    const std::vector<int64_t>& uoff, double* Uout, int64_t u_size,
                    const std::vector<int64_t>& roff, double* Rout, int64_t r_size) {
  const int ns = (int)io.m.size();
  std::vector<DenseOp> uops, rops;
  for (int J = 0; J < ns; ++J) {
    const int k = r.k[J], c = r.kept[J];
    if (k <= 0 || c <= 0) continue;
    if (Uout) {
      DenseOp u{};
      u.a_off = r.row_off[J];
      u.b_off = r.S + r.small_off[J];
      u.c_off = uoff[J];
      u.M = (int32_t)io.m[J];
      u.N = c;
      u.K = k;
      u.a_rs = k;
      u.a_cs = 1;
      u.b_rs = k;
      u.b_cs = 1;
      u.c_rs = c;
      u.c_cs = 1;
      u.alpha = 1.0;
      uops.push_back(u);
    }
    if (Rout) {
      DenseOp v{};
      v.a_off = r.S + r.small_off[J];
      v.b_off = r.col_off[J];
      v.c_off = roff[J];
      v.M = c;
      v.N = (int32_t)io.n[J];
      v.K = k;
      v.a_rs = 1;
      v.a_cs = k;
      v.b_rs = 1;
      v.b_cs = k;
      v.c_rs = io.n[J];
      v.c_cs = 1;
      v.alpha = 1.0;
      rops.push_back(v);
    }
  }
  PlanSet ps;
  std::string err;
  GemmPlan up, rp;
  if (!plan_dense(uops, ps.pool, 64, 64, 1, up, err)) return fail(FPEPS_ERR_SHAPE, err);
  if (!plan_dense(rops, ps.pool, 64, 64, 1, rp, err)) return fail(FPEPS_ERR_SHAPE, err);
  int iu = ps.add(std::move(up)), ir = ps.add(std::move(rp));
  FP_TRY(ps.upload(ctx, "fac"));
  int64_t rowt = 0, colt = 0;
  for (int J = 0; J < ns; ++J) {
    rowt += io.m[J] * (int64_t)r.k[J];
    colt += io.n[J] * (int64_t)r.k[J];
  }
  const int64_t small_n = 2 * r.S + (int64_t)r.lam.size() + 1;
  if (Uout) FP_TRY(run_gemm(ctx, ps, iu, r.Q, rowt, r.small, small_n, Uout, u_size));
  if (Rout) FP_TRY(run_gemm(ctx, ps, ir, r.small, small_n, r.Bt, colt, Rout, r_size));
  if (Uout) {
    // canonical gauge: largest-magnitude entry of every U column positive
    std::vector<SignDesc> sd;
    std::vector<int32_t> cd;
    int ncols = 0;
    for (int J = 0; J < ns; ++J) {
      const int c = r.kept[J];
      if (r.k[J] <= 0 || c <= 0) continue;
      SignDesc g{};
      g.u_off = uoff[J];
      g.r_off = Rout ? roff[J] : 0;
      g.m = (int32_t)io.m[J];
      g.ncol = c;
      g.n = (int32_t)io.n[J];
      g.col0 = ncols;
      for (int i = 0; i < c; ++i) cd.push_back((int32_t)sd.size());
      sd.push_back(g);
      ncols += c;
    }
    SignDesc* dsd = nullptr;
    int32_t* dcd = nullptr;
    FP_TRY(ctx->upload("sign_d", sd.data(), sd.size() * sizeof(SignDesc), (void**)&dsd));
    FP_TRY(ctx->upload("sign_c", cd.data(), cd.size() * sizeof(int32_t), (void**)&dcd));
    FP_HIP(launch_sign_fix(dsd, (int)sd.size(), ncols, dcd, Uout, Rout, ctx->stream));
  }
  return ctx->sync();
}

// ---------------------------------------------------------------------------
// zip-up absorption of one row
// ---------------------------------------------------------------------------
namespace {

// Writes the structure of one output site; *fits = false (and the required
// sizes in the report) when a capacity is too small.
Status write_structure(const std::vector<LegP>& legs, const std::vector<int>& dirs,
                       const std::vector<std::array<uint16_t, 5>>& blocks,
                       const std::vector<int64_t>& offs, int64_t nelem, fpeps_tensor* t,
                       fpeps_report* rep, bool* fits) {
  int need_sect = 0;
  for (auto& l : legs) need_sect = std::max(need_sect, l->nsect());
  const int nlab = legs[0]->nlab;
  if (rep) {
    rep->required_sect = std::max(rep->required_sect, need_sect);
    rep->required_blocks = std::max(rep->required_blocks, (int32_t)blocks.size());
    rep->required_elem = std::max(rep->required_elem, nelem);
  }
  *fits = !(need_sect > t->max_sect || (int64_t)blocks.size() > t->max_blocks ||
            nelem > t->max_elem);
  if (!*fits) return Status::ok();
  if (!t->nsect || !t->dirs || !t->labels || !t->dims || !t->block_sect || !t->block_off)
    return fail(FPEPS_ERR_ARG, "output tensor has null structure arrays");
  t->nlegs = (int32_t)legs.size();
  t->nlab = nlab;
  for (size_t l = 0; l < legs.size(); ++l) {
    t->nsect[l] = legs[l]->nsect();
    t->dirs[l] = dirs[l];
    for (int s = 0; s < legs[l]->nsect(); ++s) {
      for (int i = 0; i < nlab; ++i)
        t->labels[((int64_t)l * t->max_sect + s) * nlab + i] = legs[l]->label(s)[i];
      t->dims[(int64_t)l * t->max_sect + s] = legs[l]->dim[s];
    }
  }
  t->nblocks = (int32_t)blocks.size();
  for (size_t b = 0; b < blocks.size(); ++b) {
    for (int l = 0; l < 5; ++l) t->block_sect[b * 5 + l] = blocks[b][l];
    t->block_off[b] = offs[b];
  }
  t->nelem = nelem;
  return Status::ok();
}

}  // namespace

namespace {

// Bond expansion of one truncated site (Sec. 4, Figs. 3-5). With the kept
// left space U (m_J x c_J per sector, row stride c_J) and R = U^T M
// (c_J x n_J), the kept right space is V = diag(1/sigma) R. The randomized
// SVD of the discarded part (1 - U U^T) M (1 - V^T V) runs through the
// site's own chain, the projectors split as in Fig. 5 and applied around
// each application (the sketch is folded first: M (Om - V^T (V Om)), then
// Y - U (U^T Y)); one application (q = 0), widths from the residual's
// dimensions (m_J - c_J, n_J - c_J), sketch stream 1, one cut of
// ``cbe_extra`` directions over the sectors. Returns Q (m_J x e_J, row
// stride e_J, canonical signs) and Z = M^T Q (n_J x e_J), whose transpose
// are the expansion's remainder rows.
struct CbeResult {
  std::vector<int32_t> e;
  double* Q = nullptr;
  double* Z = nullptr;
  std::vector<int64_t> qoff, zoff;
  std::vector<std::vector<int32_t>> pass_k;     // widths factorised in each pass
  std::vector<int32_t> k;                       // final widths
  std::vector<std::array<double, 2>> pass_fl;   // chain flops of each pass's plans
  double rem_flops = 0;                         // M^T Q
  uint32_t fallbacks = 0;
};

Status cbe_site(fpeps_ctx_s* ctx, SiteOp& op, const RsvdOut& rs, const double* U,
                const std::vector<int64_t>& uoff, int64_t u_total, const double* R,
                const std::vector<int64_t>& roff, int64_t r_total, const fpeps_opts* o, int x,
                int64_t budget, CbeResult& out) {
  const int ns = (int)op.sect.size();
  const std::vector<int32_t>& c = rs.kept;
  // V = diag(1/sigma) R
  std::vector<double> sc;
  std::vector<SectDesc> vd;
  std::vector<int64_t> voff(ns, 0);
  int64_t vt = 0, maxe = 0;
  for (int J = 0; J < ns; ++J) {
    voff[J] = vt;
    if (c[J] <= 0) continue;
    SectDesc g{};
    g.off_a = roff[J];
    g.off_out = vt;
    g.rows = c[J];
    g.cols = (int32_t)op.sect[J].n;
    g.s0 = (int32_t)sc.size();
    for (int i = 0; i < c[J]; ++i) {
      const double l = rs.lam[rs.lam_off[J] + i];
      sc.push_back(l > 0 ? 1.0 / std::sqrt(l) : 0.0);
    }
    vd.push_back(g);
    vt += (int64_t)c[J] * op.sect[J].n;
    maxe = std::max<int64_t>(maxe, (int64_t)c[J] * op.sect[J].n);
  }
  double* V = nullptr;
  FP_TRY(ctx->bufT("cbe_V", (size_t)std::max<int64_t>(vt, 1), &V));
  if (!vd.empty()) {
    SectDesc* dvd = nullptr;
    double* dsc = nullptr;
    FP_TRY(ctx->upload("cbe_vd", vd.data(), vd.size() * sizeof(SectDesc), (void**)&dvd));
    FP_TRY(ctx->upload("cbe_sc", sc.data(), sc.size() * sizeof(double), (void**)&dsc));
    FP_HIP(launch_row_scale(dvd, (int)vd.size(), maxe, R, V, dsc, ctx->stream));
  }
  RsvdIO io;
  for (int J = 0; J < ns; ++J) {
    io.m.push_back(op.sect[J].m);
    io.n.push_back(op.sect[J].n);
    io.width_m.push_back(op.sect[J].m - c[J]);
    io.width_n.push_back(op.sect[J].n - c[J]);
    io.c1.push_back((uint32_t)J);
  }
  io.c2 = (uint32_t)x;
  io.c3 = (uint32_t)(o->row & 0xFFFF) | (1u << 16);
  std::shared_ptr<SiteOp::Plans> plp;
  PlanSet pj;
  int pv1 = -1, pv2 = -1, pu1 = -1, pu2 = -1;
  int64_t s_total = 0;
  io.prepare = [&](const std::vector<int32_t>& k) -> Status {
    if (plp) out.pass_fl.push_back({plp->flops_fwd, plp->flops_bwd});
    plp = std::make_shared<SiteOp::Plans>();
    FP_TRY(op.plan_host(k, budget, *plp, true, false));
    FP_TRY(op.upload(ctx, *plp));
    std::vector<DenseOp> v1, v2, u1, u2;
    s_total = 0;
    for (int J = 0; J < ns; ++J) {
      const int64_t soff = s_total;
      if (k[J] <= 0 || c[J] <= 0) continue;
      s_total += (int64_t)c[J] * k[J];
      const int32_t m = (int32_t)op.sect[J].m, n = (int32_t)op.sect[J].n;
      DenseOp d{};
      d.alpha = 1.0;
      // s = V x  (c x k), x: n x k in the column layout
      d.a_off = voff[J]; d.a_rs = n; d.a_cs = 1;
      d.b_off = plp->col_off[J]; d.b_rs = k[J]; d.b_cs = 1;
      d.c_off = soff; d.c_rs = k[J]; d.c_cs = 1;
      d.M = c[J]; d.N = k[J]; d.K = n;
      v1.push_back(d);
      // tmp = -V^T s  (n x k)
      DenseOp e{};
      e.alpha = -1.0;
      e.a_off = voff[J]; e.a_rs = 1; e.a_cs = n;
      e.b_off = soff; e.b_rs = k[J]; e.b_cs = 1;
      e.c_off = plp->col_off[J]; e.c_rs = k[J]; e.c_cs = 1;
      e.M = n; e.N = k[J]; e.K = c[J];
      v2.push_back(e);
      // s = U^T y  (c x k), y: m x k in the row layout
      DenseOp f{};
      f.alpha = 1.0;
      f.a_off = uoff[J]; f.a_rs = 1; f.a_cs = c[J];
      f.b_off = plp->row_off[J]; f.b_rs = k[J]; f.b_cs = 1;
      f.c_off = soff; f.c_rs = k[J]; f.c_cs = 1;
      f.M = c[J]; f.N = k[J]; f.K = m;
      u1.push_back(f);
      // tmp = -U s  (m x k)
      DenseOp g{};
      g.alpha = -1.0;
      g.a_off = uoff[J]; g.a_rs = c[J]; g.a_cs = 1;
      g.b_off = soff; g.b_rs = k[J]; g.b_cs = 1;
      g.c_off = plp->row_off[J]; g.c_rs = k[J]; g.c_cs = 1;
      g.M = m; g.N = k[J]; g.K = c[J];
      u2.push_back(g);
    }
    pj = PlanSet();
    std::string err;
    GemmPlan a, b, cc, dd;
    if (!plan_dense(v1, pj.pool, 64, 64, 1, a, err)) return fail(FPEPS_ERR_SHAPE, err);
    if (!plan_dense(v2, pj.pool, 64, 64, 1, b, err)) return fail(FPEPS_ERR_SHAPE, err);
    if (!plan_dense(u1, pj.pool, 64, 64, 1, cc, err)) return fail(FPEPS_ERR_SHAPE, err);
    if (!plan_dense(u2, pj.pool, 64, 64, 1, dd, err)) return fail(FPEPS_ERR_SHAPE, err);
    pv1 = pj.add(std::move(a));
    pv2 = pj.add(std::move(b));
    pu1 = pj.add(std::move(cc));
    pu2 = pj.add(std::move(dd));
    return pj.upload(ctx, "cbe_proj");
  };
  // x <- x - V^T (V x) (column side) or x - U (U^T x) (row side), in place
  auto project = [&](bool row_side, double* xv, int64_t xtotal) -> Status {
    double *sb = nullptr, *tmp = nullptr;
    FP_TRY(ctx->bufT("cbe_s", (size_t)std::max<int64_t>(s_total, 1), &sb));
    FP_TRY(ctx->bufT("cbe_tmp", (size_t)std::max<int64_t>(xtotal, 1), &tmp));
    // sectors without kept directions have no projection product: their
    // part of tmp must add zero
    FP_HIP(launch_fill(tmp, xtotal, 0.0, ctx->stream));
    const int64_t st = std::max<int64_t>(s_total, 1);
    if (!row_side) {
      FP_TRY(run_gemm(ctx, pj, pv1, V, std::max<int64_t>(vt, 1), xv, xtotal, sb, st));
      FP_TRY(run_gemm(ctx, pj, pv2, V, std::max<int64_t>(vt, 1), sb, st, tmp, xtotal));
    } else {
      FP_TRY(run_gemm(ctx, pj, pu1, U, u_total, xv, xtotal, sb, st));
      FP_TRY(run_gemm(ctx, pj, pu2, U, u_total, sb, st, tmp, xtotal));
    }
    return axpy_inplace(ctx, xv, tmp, xtotal);
  };
  io.apply = [&](bool t, bool, const double* xi, double* yo) -> Status {
    double* xc = const_cast<double*>(xi);
    if (!t) {
      FP_TRY(project(false, xc, plp->col_total));
      FP_TRY(op.apply(ctx, *plp, false, xc, yo, false));
      FP_TRY(project(true, yo, plp->row_total));
    } else {
      FP_TRY(project(true, xc, plp->row_total));
      FP_TRY(op.apply(ctx, *plp, true, xc, yo, false));
      FP_TRY(project(false, yo, plp->col_total));
    }
    return Status::ok();
  };
  RsvdOut rc;
  FP_TRY(rsvd_run(ctx, io, o->cbe_extra, o->oversample, 0, o->seed, rc, o->sv_cut));
  out.pass_fl.push_back({plp->flops_fwd, plp->flops_bwd});
  out.pass_k = rc.pass_k;
  out.k = rc.k;
  out.e = rc.kept;
  out.fallbacks = rc.fallbacks;
  // Q = Q_sketch U~[:, :e] (canonical signs), then Z = M^T Q
  out.qoff.assign(ns, 0);
  int64_t qt = 0;
  for (int J = 0; J < ns; ++J) {
    out.qoff[J] = qt;
    qt += op.sect[J].m * (int64_t)out.e[J];
  }
  FP_TRY(ctx->bufT("cbe_Q", (size_t)std::max<int64_t>(qt, 1), &out.Q));
  FP_TRY(rsvd_factors(ctx, io, rc, out.qoff, out.Q, std::max<int64_t>(qt, 1), {}, nullptr, 0));
  SiteOp::Plans pe;
  FP_TRY(op.plan_host(out.e, budget, pe, true, false));
  FP_TRY(op.upload(ctx, pe));
  for (int J = 0; J < ns; ++J)
    if (pe.row_off[J] != out.qoff[J]) return fail(FPEPS_ERR_SHAPE, "expansion layout mismatch");
  out.zoff = pe.col_off;
  out.rem_flops = pe.flops_bwd;
  FP_TRY(ctx->bufT("cbe_Z", (size_t)std::max<int64_t>(pe.col_total, 1), &out.Z));
  FP_TRY(op.apply(ctx, pe, true, out.Q, out.Z, false));
  return Status::ok();
}

}  // namespace

Status absorb_row(fpeps_ctx_s* ctx, int L, const fpeps_tensor* env_in, const fpeps_tensor* ket,
                  const fpeps_tensor* pepo, const fpeps_opts* o, fpeps_tensor* env_out,
                  double* log_norm, fpeps_report* rep) {
  if (L < 1 || !env_in || !ket || !pepo || !o || !env_out || !log_norm)
    return fail(FPEPS_ERR_ARG, "null argument or L < 1");
  if (o->precision != FPEPS_FP64 && o->precision != FPEPS_FP32)
    return fail(FPEPS_ERR_UNSUPPORTED, "precision: FPEPS_FP64 or FPEPS_FP32");
  const bool f32 = o->precision == FPEPS_FP32;
  if (o->cbe_extra < 0) return fail(FPEPS_ERR_ARG, "cbe_extra >= 0 required");
  if (o->chi < 1 || o->oversample < 0 || o->power_iters < 0)
    return fail(FPEPS_ERR_ARG, "chi >= 1, oversample >= 0, power_iters >= 0 required");
  SymInfo sym;
  sym.kind = o->symmetry;
  sym.fermionic = o->fermionic != 0;
  sym.coef_seed = o->coef_seed;
  ctx->tune_into(sym);
  if (sym.kind < 0 || sym.kind > 2) return fail(FPEPS_ERR_ARG, "bad symmetry");
  const int nlab = sym.kind == SYM_U1U1 ? 2 : 1;
  // one budget for the chain intermediates of all streams: up to
  // max_streams slices are live at once, each within its share
  const int64_t budget =
      std::max<int64_t>(1, ctx->total_budget(o) / std::max(1, ctx->max_streams));
  ctx->diag.assign(L, SiteDiag());
  ctx->peak_ws = 0;
  ctx->nslices = 0;
  ctx->time_kernels = (o->flags & FPEPS_FLAG_TIME_KERNELS) != 0;
  ctx->multi_stream = (o->flags & FPEPS_FLAG_ONE_STREAM) == 0;
  ctx->kt_seconds = ctx->kt_flops = 0;
  ctx->kt_launches = 0;
  ctx->evused = 0;
  ctx->evflops.clear();
  ctx->evlabel.clear();
  ctx->evbytes.clear();
  ctx->evshape.clear();
  ctx->kt_by_label.clear();
  {
    const char* v = std::getenv("FPEPS_VERBOSE");
    ctx->verbose = v ? std::max(1, std::atoi(v)) : 0;
  }
  auto wall = [] { return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count(); };
  EventPair evp;
  FP_HIP(evp.create());
  hipEvent_t ev0 = evp.a, ev1 = evp.b;
  FP_HIP(hipEventRecord(ev0, ctx->stream));
  double lg = 0.0, flops = 0.0, alg_bytes = 0.0, disc = 0.0, gap = INFINITY;
  int kept_total = 0;
  uint32_t fallbacks = 0;
  bool cap_fail = false;

  // remainder of the left edge: one element equal to 1
  double* Rbuf[2] = {nullptr, nullptr};
  FP_TRY(ctx->bufT("R_edge", 1, &Rbuf[0]));
  FP_HIP(launch_fill(Rbuf[0], 1, 1.0, ctx->stream));
  BT R;
  int64_t R_size = 1;
  const double* Rdev = Rbuf[0];
  {
    BT T0, K0, W0;
    FP_TRY(tensor_to_bt(&env_in[0], {N_a, N_tk, N_tw, N_tb, N_b}, nlab, T0));
    FP_TRY(tensor_to_bt(&ket[0], {N_p, N_lk, N_rk, N_tk, N_dk}, nlab, K0));
    FP_TRY(tensor_to_bt(&pepo[0], {N_q, N_p, N_lw, N_rw, N_tw, N_dw}, nlab, W0));
    auto zero = std::make_shared<Leg>();
    zero->nlab = nlab;
    zero->dir = 1;
    zero->lab.assign(nlab, 0);
    zero->dim = {1};
    auto fl = [](const LegP& l) {
      auto m = std::make_shared<Leg>(*l);
      m->dir = -m->dir;
      return LegP(m);
    };
    R.names = {N_c, N_a, N_lk, N_lw, N_lb};
    R.cat = {zero, T0.cat[0], K0.cat[1], W0.cat[2], fl(K0.cat[1])};
    for (int i = 1; i < 5; ++i)
      if (R.cat[i]->total() != 1) return fail(FPEPS_ERR_SHAPE, "left boundary legs must have dim 1");
    Block b;
    b.base = 0;
    set_rowmajor(R, b);
    R.blocks.push_back(b);
    R.size = 1;
  }
  int rcur = 0;
  // the remainder's squared norm, summed on the device and not yet divided out
  const double* r_nrm = nullptr;
  int64_t r_len = 0;
  // The previous site's analysis and plans: a site whose structure key,
  // widths, budget and precision are equal reuses them (interior sites of a
  // row often share their block structure) and only uploads them again.
  struct PlanCache {
    std::string key;
    std::vector<Sector> sect;
    std::vector<std::vector<int64_t>> unit_size;
    std::shared_ptr<SiteOp::Plans> pl;
    std::vector<int32_t> k;
  } cache;
  int cache_hits = 0;
  // the remainder-independent part of the last analysis (interior sites of
  // a row share their T, ket and PEPO structure)
  FwdAnalysis fwd_an;
  // kept count per sector label of the previous truncated site: the first
  // guess of this site's sketch widths
  std::map<std::vector<int32_t>, int32_t> prev_kept;
  bool have_prev = false;
  int total_passes = 0;
  for (int x = 0; x < L; ++x) {
    BT T, K, W;
    FP_TRY(tensor_to_bt(&env_in[x], {N_a, N_tk, N_tw, N_tb, N_b}, nlab, T));
    FP_TRY(tensor_to_bt(&ket[x], {N_p, N_lk, N_rk, N_tk, N_dk}, nlab, K));
    FP_TRY(tensor_to_bt(&pepo[x], {N_q, N_p, N_lw, N_rw, N_tw, N_dw}, nlab, W));
    SiteData d;
    d.T = env_in[x].data;
    d.T_size = env_in[x].nelem;
    d.A = ket[x].data;
    d.A_size = ket[x].nelem;
    d.W = pepo[x].data;
    d.W_size = pepo[x].nelem;
    d.R = Rdev;
    d.R_size = R_size;
    if (o->flags & FPEPS_FLAG_CHECK_FINITE) {
      int* flag = nullptr;
      FP_TRY(ctx->bufT("finite_flag", 1, &flag));
      FP_HIP(launch_fill_int(flag, 1, 0, ctx->stream));
      FP_HIP(launch_check_finite(d.T, d.T_size, flag, ctx->stream));
      FP_HIP(launch_check_finite(d.A, d.A_size, flag, ctx->stream));
      FP_HIP(launch_check_finite(d.W, d.W_size, flag, ctx->stream));
      int h = 0;
      FP_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
      FP_TRY(ctx->sync());
      if (h) return fail(FPEPS_ERR_NUMERIC, "non-finite input at site " + std::to_string(x));
    }
    const double tw0 = wall();
    SiteOp op;
    FP_TRY(op.init(sym, nlab, std::move(T), std::move(K), std::move(W), std::move(R), d));
    std::string key = op.structure_key();
    const bool same = !cache.key.empty() && key == cache.key;
    if (same) {
      op.sect = cache.sect;
      op.unit_size = cache.unit_size;
    } else {
      FP_TRY(op.analyse(&fwd_an));
    }
    if (r_nrm) {
      double h = 0;
      FP_HIP(hipMemcpyAsync(&h, r_nrm, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      FP_TRY(ctx->sync());
      if (!(h > 0.0) || !std::isfinite(h))
        return fail(FPEPS_ERR_NUMERIC, "remainder has zero or non-finite norm");
      const double nu = std::sqrt(h);
      FP_HIP(launch_scale(Rbuf[rcur], r_len, 1.0 / nu, ctx->stream));
      lg += std::log(nu);
      r_nrm = nullptr;
    }
    const int ns = (int)op.sect.size();
    SiteDiag& dg = ctx->diag[x];
    for (auto& s : op.sect) {
      dg.m.push_back(s.m);
      dg.n.push_back(s.n);
    }
    std::vector<LegP> olegs = {op.R.cat[0], op.ket.cat[op.ket.pos(N_dk)], op.W.cat[op.W.pos(N_dw)],
                               op.bra.cat[op.bra.pos(N_db)], nullptr};
    if (x == L - 1) {
      int64_t ntot = 0;
      int J1 = -1;
      for (int J = 0; J < ns; ++J) {
        ntot += op.sect[J].n;
        if (op.sect[J].n == 1) J1 = J;
      }
      if (ntot != 1 || J1 < 0) return fail(FPEPS_ERR_SHAPE, "right boundary legs must have dim 1");
      std::vector<int32_t> k(ns, 0);
      k[J1] = 1;
      SiteOp::Plans pl;
      FP_TRY(op.plan(ctx, k, budget, pl, false, f32));
      double *xin = nullptr, *y = nullptr, *part = nullptr, *nrm = nullptr;
      FP_TRY(ctx->bufT("last_x", 1, &xin));
      FP_TRY(ctx->bufT("last_y", (size_t)std::max<int64_t>(pl.row_total, 1), &y));
      FP_TRY(ctx->bufT("nrm_part", 512, &part));
      FP_TRY(ctx->bufT("nrm_out", 1, &nrm));
      FP_HIP(launch_fill(xin, 1, 1.0, ctx->stream));
      FP_TRY(op.apply(ctx, pl, false, xin, y, false));
      FP_HIP(launch_sumsq(y, pl.row_total, part, nrm, ctx->stream));
      double h = 0;
      FP_HIP(hipMemcpyAsync(&h, nrm, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      FP_TRY(ctx->sync());
      if (!(h > 0.0) || !std::isfinite(h)) return fail(FPEPS_ERR_NUMERIC, "last site has zero or non-finite norm");
      const double nu = std::sqrt(h);
      lg += std::log(nu);
      auto jl = std::make_shared<Leg>();
      jl->nlab = nlab;
      jl->lab = op.sect[J1].label;
      jl->dim = {1};
      olegs[4] = jl;
      std::vector<std::array<uint16_t, 5>> blocks;
      std::vector<int64_t> offs;
      for (size_t t = 0; t < op.sect[J1].rows.size(); ++t) {
        auto& r = op.sect[J1].rows[t];
        blocks.push_back({r[0], r[1], r[2], r[3], 0});
        offs.push_back(op.sect[J1].rrow[t]);
      }
      std::vector<int> dirs = {1, op.ket.cat[op.ket.pos(N_dk)]->dir, op.W.cat[op.W.pos(N_dw)]->dir,
                               op.bra.cat[op.bra.pos(N_db)]->dir, -1};
      bool fits = false;
      FP_TRY(write_structure(olegs, dirs, blocks, offs, pl.row_total, &env_out[x], rep, &fits));
      if (fits) {
        FP_HIP(hipMemcpyAsync(env_out[x].data, y, pl.row_total * sizeof(double),
                              hipMemcpyDeviceToDevice, ctx->stream));
        FP_HIP(launch_scale(env_out[x].data, pl.row_total, 1.0 / nu, ctx->stream));
      } else {
        cap_fail = true;
      }
      dg.k = k;
      dg.kept = k;
      break;
    }
    // randomized SVD of M_x
    RsvdIO io;
    std::shared_ptr<SiteOp::Plans> plp;
    for (int J = 0; J < ns; ++J) {
      io.m.push_back(op.sect[J].m);
      io.n.push_back(op.sect[J].n);
      io.c1.push_back((uint32_t)J);
    }
    io.c2 = (uint32_t)x;
    io.c3 = (uint32_t)(o->row & 0xFFFF);
    if (have_prev) {
      io.hint.assign(ns, -1);
      for (int J = 0; J < ns; ++J) {
        auto it = prev_kept.find(op.sect[J].label);
        if (it != prev_kept.end()) io.hint[J] = it->second;
      }
    }
    // chain flops (forward, transposed) of the plans of every factorisation pass
    std::vector<std::array<double, 2>> pass_fl;
    double t_plan = 0;
    // The transposed-chain plans are first used after the sketch product
    // M Omega: they are planned on a host thread while the device runs it,
    // and uploaded before the first transposed application.
    std::future<Status> bwd_job;
    bool bwd_wait = false;
    io.prepare = [&](const std::vector<int32_t>& k) {
      const double t0 = wall();
      Status st = Status::ok();
      if (plp) pass_fl.push_back({plp->flops_fwd, plp->flops_bwd});
      if (same && cache.pl && cache.k == k && cache.pl->f32 == f32) {
        plp = cache.pl;
        st = op.upload(ctx, *plp);
        ++cache_hits;
      } else {
        plp = std::make_shared<SiteOp::Plans>();
        st = op.plan_host(k, budget, *plp, false, f32);
        if (st.good()) st = op.upload(ctx, *plp, 1);
        if (st.good()) {
          const SiteOp* opc = &op;
          std::shared_ptr<SiteOp::Plans> pl = plp;
          bwd_job = std::async(std::launch::async, [opc, k, pl]() { return opc->plan_bwd(k, *pl); });
          bwd_wait = true;
        }
      }
      t_plan += wall() - t0;
      return st;
    };
    auto join_bwd = [&](bool up) -> Status {
      if (!bwd_wait) return Status::ok();
      bwd_wait = false;
      const double t0 = wall();
      FP_TRY(bwd_job.get());
      op.sum_plans(*plp);
      if (up) FP_TRY(op.upload(ctx, *plp, 2));
      t_plan += wall() - t0;
      return Status::ok();
    };
    io.apply = [&](bool t, bool fin, const double* xi, double* yo) {
      if (t) FP_TRY(join_bwd(true));
      return op.apply(ctx, *plp, t, xi, yo, f32 && !fin);
    };
    RsvdOut rs;
    const double tw1 = wall();
    if (f32) FP_TRY(op.make_f32_operands(ctx));
    {
      Status st = rsvd_run(ctx, io, o->chi, o->oversample, o->power_iters, o->seed, rs, o->sv_cut);
      if (st.good()) st = join_bwd(false);
      if (!st.good()) return fail(st.code, "site " + std::to_string(x) + ": " + st.msg);
    }
    fallbacks |= rs.fallbacks;
    pass_fl.push_back({plp->flops_fwd, plp->flops_bwd});
    total_passes += (int)rs.pass_k.size();
    if (ctx->verbose) {
      int64_t mt = 0, nt = 0;
      for (int J = 0; J < ns; ++J) {
        mt += op.sect[J].m;
        nt += op.sect[J].n;
      }
      double xl = 0, pk = 0;
      size_t tabs = 0;
      for (const auto& sl : plp->slices) {
        for (const RtPlan& r : sl.ps->rts) {
          xl += r.x_loads;
          pk += (double)r.pack_size;
        }
        tabs += sl.ps->pool.data.size();
      }
      std::fprintf(stderr,
                   "[fpeps] site %d%s: sectors %d m %lld n %lld analyse %.3fs rsvd %.3fs (plan %.3fs) "
                   "chain flops/app %.3e slices %zu ws %.2f GB table entries %zu layer loads "
                   "%.3e pack %.3e upload %.1f MB %.3fs\n",
                   x, same ? " (plans reused)" : "", ns, (long long)mt, (long long)nt, tw1 - tw0, wall() - tw1, t_plan, plp->flops_fwd,
                   plp->slices.size(), (plp->ws1 + plp->ws2) * 8e-9, tabs, xl, pk,
                   ctx->plan_up_bytes * 1e-6, ctx->plan_up_seconds);
    }
    if (ctx->verbose >= 2) {
      std::fprintf(stderr, "[fpeps] site %d kept", x);
      for (int v : rs.kept) std::fprintf(stderr, " %d", v);
      std::fprintf(stderr, "\n");
      // layer steps: tiles by (rows per tile, staged columns, chunks) over all
      // slices
      for (int st = 1; st <= 3; ++st)
        for (int bwd = 0; bwd < 2; ++bwd) {
          std::map<std::array<int, 3>, double> hist;
          double all = 0;
          for (const auto& sl : plp->slices) {
            const PlanSet* ps = bwd ? sl.psb.get() : sl.ps.get();
            const int idx = bwd ? sl.bwd[st] : sl.fwd[st];
            const bool rt = bwd ? sl.bwd_rt[st] : sl.fwd_rt[st];
            if (!ps || idx < 0 || !rt) continue;
            for (const RtGroup& g : ps->rts[idx].groups) {
              const double nt = (double)((g.M + g.rows - 1) / g.rows);
              const int kb = g.ktot <= 8 ? 8 : g.ktot <= 16 ? 16 : g.ktot <= 32 ? 32 : g.ktot <= 64 ? 64 : 999;
              hist[{g.rows, kb, std::min(g.o1 - g.o0, 9)}] += nt;
              all += nt;
            }
          }
          std::fprintf(stderr, "[fpeps] site %d layer step %s%d tiles:", x, bwd ? "T" : "",
                       bwd ? 5 - st : st + 1);
          for (auto& kv : hist)
            if (kv.second >= 0.02 * all)
              std::fprintf(stderr, " rows%d/k<=%d/nch%d:%.0f%%", kv.first[0], kv.first[1],
                           kv.first[2], 100.0 * kv.second / all);
          std::fprintf(stderr, "\n");
        }
      // GEMM steps: jobs, 16-deep K tiles per job, tile shapes
      const int steps[4] = {1, 5, 11, 15};
      for (int st : steps) {
        double jobs = 0, tiles = 0, small = 0, mts = 0, nts = 0, nplan = 0;
        for (const auto& sl : plp->slices) {
          const bool bwd = st > 10;
          const int idx = bwd ? sl.bwd[st == 15 ? 0 : 4] : sl.fwd[st == 1 ? 0 : 4];
          const PlanSet* ps = bwd ? sl.psb.get() : sl.ps.get();
          if (!ps || idx < 0) continue;
          const GemmPlan& g = ps->plans[idx];
          for (const GemmJob& j : g.jobs) {
            int64_t t = 0;
            for (int q = j.p0; q < j.p1; ++q) {
              const int64_t k0 = std::max(j.k0, 0), k1 = std::min<int64_t>(j.k1, g.pairs[q].K);
              if (k1 > k0) t += (k1 - k0 + 15) / 16;
            }
            jobs += 1;
            tiles += (double)t;
            if (t <= 4) small += 1;
          }
          if (!g.jobs.empty()) {
            mts += g.mt;
            nts += g.nt;
            nplan += 1;
          }
        }
        std::fprintf(stderr,
                     "[fpeps] site %d gemm step %s%d: %.0f jobs, %.1f K tiles per job, %.0f%% of "
                     "jobs with <= 4 tiles, mean tile %.0fx%.0f\n",
                     x, st > 10 ? "T" : "", st > 10 ? st - 10 : st, jobs,
                     jobs > 0 ? tiles / jobs : 0.0, jobs > 0 ? 100.0 * small / jobs : 0.0,
                     mts / std::max(nplan, 1.0), nts / std::max(nplan, 1.0));
      }
    }
    // outputs: environment site (U) and the next remainder (R); with bond
    // expansion [U | Q] and [R ; Q^T M]
    std::vector<int32_t> kept = rs.kept;
    std::vector<int64_t> uoff(ns, 0), roff(ns, 0);
    int64_t ut = 0, rt = 0;
    auto offsets = [&](const std::vector<int32_t>& kk, std::vector<int64_t>& uo,
                       std::vector<int64_t>& ro, int64_t& u_t, int64_t& r_t) {
      u_t = r_t = 0;
      for (int J = 0; J < ns; ++J) {
        uo[J] = u_t;
        ro[J] = r_t;
        u_t += op.sect[J].m * (int64_t)kk[J];
        r_t += op.sect[J].n * (int64_t)kk[J];
      }
    };
    const int rn = 1 - rcur;
    double* ubuf = nullptr;
    CbeResult cb;
    if (o->cbe_extra > 0) {
      std::vector<int64_t> uo0(ns), ro0(ns);
      int64_t ut0 = 0, rt0 = 0;
      offsets(rs.kept, uo0, ro0, ut0, rt0);
      double *u0 = nullptr, *r0 = nullptr;
      FP_TRY(ctx->bufT("U_trunc", (size_t)std::max<int64_t>(ut0, 1), &u0));
      FP_TRY(ctx->bufT("R_trunc", (size_t)std::max<int64_t>(rt0, 1), &r0));
      FP_TRY(rsvd_factors(ctx, io, rs, uo0, u0, std::max<int64_t>(ut0, 1), ro0, r0,
                          std::max<int64_t>(rt0, 1)));
      FP_TRY(cbe_site(ctx, op, rs, u0, uo0, std::max<int64_t>(ut0, 1), r0, ro0,
                      std::max<int64_t>(rt0, 1), o, x, budget, cb));
      fallbacks |= cb.fallbacks;
      for (int J = 0; J < ns; ++J) kept[J] += cb.e[J];
      offsets(kept, uoff, roff, ut, rt);
      FP_TRY(ctx->bufT(rn == 0 ? "R_a" : "R_b", (size_t)std::max<int64_t>(rt, 1), &Rbuf[rn]));
      FP_TRY(ctx->bufT("U_site", (size_t)std::max<int64_t>(ut, 1), &ubuf));
      std::vector<SectDesc> mu, mr;
      int64_t mue = 0, mre = 0;
      for (int J = 0; J < ns; ++J) {
        if (kept[J] <= 0) continue;
        SectDesc a{};
        a.off_a = uo0[J];
        a.off_b = cb.qoff[J];
        a.off_out = uoff[J];
        a.rows = (int32_t)op.sect[J].m;
        a.cols = rs.kept[J];
        a.cols_b = cb.e[J];
        mu.push_back(a);
        mue = std::max<int64_t>(mue, op.sect[J].m * (int64_t)kept[J]);
        SectDesc b{};
        b.off_a = ro0[J];
        b.off_b = cb.zoff[J];
        b.off_out = roff[J];
        b.rows = rs.kept[J];
        b.cols = (int32_t)op.sect[J].n;
        b.cols_b = cb.e[J];
        mr.push_back(b);
        mre = std::max<int64_t>(mre, op.sect[J].n * (int64_t)kept[J]);
      }
      SectDesc *dmu = nullptr, *dmr = nullptr;
      FP_TRY(ctx->upload("cbe_mu", mu.data(), mu.size() * sizeof(SectDesc), (void**)&dmu));
      FP_TRY(ctx->upload("cbe_mr", mr.data(), mr.size() * sizeof(SectDesc), (void**)&dmr));
      FP_HIP(launch_merge_cols(dmu, (int)mu.size(), mue, u0, cb.Q, ubuf, ctx->stream));
      FP_HIP(launch_stack_rows_t(dmr, (int)mr.size(), mre, r0, cb.Z, Rbuf[rn], ctx->stream));
    } else {
      offsets(kept, uoff, roff, ut, rt);
      FP_TRY(ctx->bufT(rn == 0 ? "R_a" : "R_b", (size_t)std::max<int64_t>(rt, 1), &Rbuf[rn]));
      FP_TRY(ctx->bufT("U_site", (size_t)std::max<int64_t>(ut, 1), &ubuf));
      FP_TRY(rsvd_factors(ctx, io, rs, uoff, ubuf, std::max<int64_t>(ut, 1), roff, Rbuf[rn],
                          std::max<int64_t>(rt, 1)));
    }
    std::vector<int> sel;
    for (int J = 0; J < ns; ++J)
      if (kept[J] > 0) sel.push_back(J);
    auto jl = std::make_shared<Leg>();
    jl->nlab = nlab;
    for (int J : sel) {
      for (int32_t v : op.sect[J].label) jl->lab.push_back(v);
      jl->dim.push_back(kept[J]);
    }
    olegs[4] = jl;
    std::vector<std::array<uint16_t, 5>> blocks;
    std::vector<int64_t> offs;
    for (size_t si = 0; si < sel.size(); ++si) {
      const int J = sel[si];
      for (size_t t = 0; t < op.sect[J].rows.size(); ++t) {
        auto& r = op.sect[J].rows[t];
        blocks.push_back({r[0], r[1], r[2], r[3], (uint16_t)si});
        offs.push_back(uoff[J] + op.sect[J].rrow[t] * kept[J]);
      }
    }
    std::vector<int> dirs = {1, op.ket.cat[op.ket.pos(N_dk)]->dir, op.W.cat[op.W.pos(N_dw)]->dir,
                             op.bra.cat[op.bra.pos(N_db)]->dir, -1};
    bool fits = false;
    FP_TRY(write_structure(olegs, dirs, blocks, offs, ut, &env_out[x], rep, &fits));
    if (fits) {
      if (ut > 0)
        FP_HIP(hipMemcpyAsync(env_out[x].data, ubuf, ut * sizeof(double), hipMemcpyDeviceToDevice,
                              ctx->stream));
    } else {
      cap_fail = true;
    }
    // normalise the remainder: its norm is summed here and read after the
    // next site's structure analysis, so that host work overlaps the factor
    // products still running on the device
    {
      double *part = nullptr, *nrm = nullptr;
      FP_TRY(ctx->bufT("nrm_part", 512, &part));
      FP_TRY(ctx->bufT("nrm_out", 1, &nrm));
      FP_HIP(launch_sumsq(Rbuf[rn], rt, part, nrm, ctx->stream));
      r_nrm = nrm;
      r_len = rt;
    }
    // R for the next site: per-sector matrices (kept_J x n_J), blocks by column tuple
    BT Rn;
    Rn.names = {N_c, N_a, N_lk, N_lw, N_lb};
    auto cl = std::make_shared<Leg>(*jl);
    cl->dir = 1;
    Rn.cat = {cl, op.T.cat[op.T.pos(N_b)], op.ket.cat[op.ket.pos(N_rk)], op.W.cat[op.W.pos(N_rw)],
              op.bra.cat[op.bra.pos(N_rb)]};
    for (size_t si = 0; si < sel.size(); ++si) {
      const int J = sel[si];
      const Sector& s = op.sect[J];
      for (size_t t = 0; t < s.cols.size(); ++t) {
        Block b;
        b.sect[0] = (uint16_t)si;
        for (int i = 0; i < 4; ++i) b.sect[i + 1] = s.cols[t][i];
        b.base = roff[J] + s.crow[t];
        int64_t st = 1;
        for (int i = 4; i >= 1; --i) {
          b.stride[i] = st;
          st *= Rn.cat[i]->dim[b.sect[i]];
        }
        b.stride[0] = s.n;
        Rn.blocks.push_back(b);
      }
    }
    Rn.size = std::max<int64_t>(rt, 1);
    R = std::move(Rn);
    Rdev = Rbuf[rn];
    R_size = std::max<int64_t>(rt, 1);
    rcur = rn;
    cache.key = std::move(key);
    cache.sect = op.sect;
    cache.unit_size = op.unit_size;
    ctx->release_later(std::move(cache.pl));
    cache.pl = plp;
    cache.k = rs.pass_k.back();   // the widths plp was planned for
    // diagnostics and report
    dg.k = rs.k;
    dg.kept = rs.kept;
    for (int J = 0; J < ns; ++J)
      for (int i = 0; i < rs.k[J]; ++i) {
        const double l = rs.lam[rs.lam_off[J] + i];
        dg.sigma.push_back(l > 0 ? std::sqrt(l) : 0.0);
        dg.sector.push_back(J);
      }
    // algorithmic flops: every pass applies M and M^T 1 + q times each and
    // factorises; the output factors once
    double site_flops = 0;
    {
      const int q = o->power_iters;
      for (size_t ps = 0; ps < rs.pass_k.size(); ++ps) {
        site_flops += (1 + q) * (pass_fl[ps][0] + pass_fl[ps][1]);
        for (int J = 0; J < ns; ++J) {
          const double m = (double)op.sect[J].m, n = (double)op.sect[J].n,
                       k = rs.pass_k[ps][J];
          if (k <= 0) continue;
          site_flops += (q + 1) * (2 * m * k * k - 2 * k * k * k / 3.0) +
                        q * (2 * n * k * k - 2 * k * k * k / 3.0);
          site_flops += 2 * n * k * k + 11 * k * k * k;
        }
      }
      for (int J = 0; J < ns; ++J) {
        const double m = (double)op.sect[J].m, n = (double)op.sect[J].n, k = rs.k[J],
                     c = rs.kept[J];
        if (k > 0) site_flops += 2 * m * k * c + 2 * k * c * n;
      }
      // bond expansion: per pass one application of M and of M^T with the
      // projector splits (4 c k (m + n) each), one orthonormalisation and
      // the core factorisation; then Q = Q_sketch U~ and M^T Q
      for (size_t ps = 0; ps < cb.pass_k.size(); ++ps) {
        site_flops += cb.pass_fl[ps][0] + cb.pass_fl[ps][1];
        for (int J = 0; J < ns; ++J) {
          const double m = (double)op.sect[J].m, n = (double)op.sect[J].n,
                       k = cb.pass_k[ps][J], c = rs.kept[J];
          if (k <= 0) continue;
          site_flops += 8 * c * k * (m + n);
          site_flops += 2 * m * k * k - 2 * k * k * k / 3.0;
          site_flops += 2 * n * k * k + 11 * k * k * k;
        }
      }
      if (!cb.pass_k.empty()) {
        site_flops += cb.rem_flops;
        for (int J = 0; J < ns; ++J) {
          const double m = (double)op.sect[J].m, k = cb.k[J], e = cb.e[J];
          if (k > 0) site_flops += 2 * m * k * e;
        }
      }
    }
    flops += site_flops;
    // algorithmic bytes: every application reads T, R, the ket and the PEPO
    // once and writes its output (m x k rows or n x k columns) once
    {
      const int q = o->power_iters;
      const double in_b = 8.0 * (double)(d.T_size + d.R_size + d.A_size + d.W_size);
      for (size_t ps = 0; ps < rs.pass_k.size(); ++ps) {
        double rows = 0, cols = 0;
        for (int J = 0; J < ns; ++J) {
          rows += (double)op.sect[J].m * rs.pass_k[ps][J];
          cols += (double)op.sect[J].n * rs.pass_k[ps][J];
        }
        alg_bytes += (1 + q) * (2 * in_b + 8.0 * rows + 8.0 * cols);
      }
    }
    prev_kept.clear();
    for (int J = 0; J < ns; ++J) prev_kept[op.sect[J].label] = kept[J];
    have_prev = true;
    for (int v : kept) kept_total += v;
    dg.cbe = cb.e;
    if (rs.cut.total2 > 0) disc = std::max(disc, 1.0 - rs.cut.kept2 / rs.cut.total2);
    if (rs.cut.s_next >= 0 && rs.cut.s_last > 0)
      gap = std::min(gap, (rs.cut.s_last - rs.cut.s_next) / rs.cut.s_last);
  }
  ctx->release_later(std::move(cache.pl));
  FP_HIP(hipEventRecord(ev1, ctx->stream));
  FP_HIP(hipEventSynchronize(ev1));
  float ms = 0;
  FP_HIP(hipEventElapsedTime(&ms, ev0, ev1));
  FP_TRY(ctx->sync());
  if (cap_fail) return fail(FPEPS_ERR_CAPACITY, "output tensor capacity too small (see report)");
  *log_norm += lg;
  if (rep) {
    rep->alg_flops = flops;
    rep->seconds = ms * 1e-3;
    rep->discarded_weight = disc;
    rep->min_rel_gap = std::isfinite(gap) ? gap : -1.0;
    rep->log_norm = lg;
    rep->peak_workspace = ctx->peak_ws;
    rep->workspace_bytes = (double)ctx->ws_bytes;
    rep->kept_total = kept_total;
    rep->nslices = ctx->nslices;
    rep->fallbacks = fallbacks;
    rep->plan_reuses = cache_hits;
    rep->rsvd_passes = total_passes;
    rep->alg_bytes = alg_bytes;
    rep->kernel_launches = (int32_t)ctx->kt_launches;
    rep->kernel_seconds = ctx->kt_seconds;
    rep->kernel_flops = ctx->kt_flops;
    for (auto& kv : ctx->kt_by_label) {
      const int st = kv.first % 10;
      const bool layer = st >= 2 && st <= 4;
      (layer ? rep->layer_launches : rep->gemm_launches) += (int32_t)kv.second[2];
      (layer ? rep->layer_seconds : rep->gemm_seconds) += kv.second[0];
      (layer ? rep->layer_flops : rep->gemm_flops) += kv.second[1];
      (layer ? rep->layer_bytes : rep->gemm_bytes) += kv.second[3];
    }
  }
  if (ctx->verbose && ctx->time_kernels) {
    for (auto& kv : ctx->kt_by_label) {
      const int base = kv.first % 100, cls = kv.first / 100 - 1;
      const auto& v = kv.second;
      std::fprintf(stderr,
                   "[fpeps] chain step %s%d: %6.0f launches %9.3f s %10.3e flops %7.2f TFLOP/s "
                   "%9.1f GB %7.2f TB/s",
                   base >= 10 ? "T" : "", base >= 10 ? base - 10 : base, v[2], v[0], v[1],
                   v[1] / v[0] * 1e-12, v[3] * 1e-9, v[3] / v[0] * 1e-12);
      if (cls >= 0)
        std::fprintf(stderr, "  class %d: %.0f tiles/launch, %.1f KiB LDS", cls, v[4] / v[2],
                     v[5] / v[2] / 1024.0);
      std::fprintf(stderr, "\n");
    }
  }
  ctx->time_kernels = false;
  return Status::ok();
}

// ---------------------------------------------------------------------------
// site operator shape / application (chain on its own)
// ---------------------------------------------------------------------------
Status make_site(fpeps_ctx_s* ctx, const fpeps_tensor* R, const fpeps_tensor* T,
                 const fpeps_tensor* A, const fpeps_tensor* W, const fpeps_opts* o, SiteOp& op) {
  if (!R || !T || !A || !W || !o) return fail(FPEPS_ERR_ARG, "null argument");
  SymInfo sym;
  sym.kind = o->symmetry;
  sym.fermionic = o->fermionic != 0;
  sym.coef_seed = o->coef_seed;
  ctx->tune_into(sym);
  if (sym.kind < 0 || sym.kind > 2) return fail(FPEPS_ERR_ARG, "bad symmetry");
  const int nlab = sym.kind == SYM_U1U1 ? 2 : 1;
  BT bT, bK, bW, bR;
  FP_TRY(tensor_to_bt(T, {N_a, N_tk, N_tw, N_tb, N_b}, nlab, bT));
  FP_TRY(tensor_to_bt(A, {N_p, N_lk, N_rk, N_tk, N_dk}, nlab, bK));
  FP_TRY(tensor_to_bt(W, {N_q, N_p, N_lw, N_rw, N_tw, N_dw}, nlab, bW));
  FP_TRY(tensor_to_bt(R, {N_c, N_a, N_lk, N_lw, N_lb}, nlab, bR));
  SiteData d;
  d.T = T->data;
  d.T_size = T->nelem;
  d.A = A->data;
  d.A_size = A->nelem;
  d.W = W->data;
  d.W_size = W->nelem;
  d.R = R->data;
  d.R_size = R->nelem;
  FP_TRY(op.init(sym, nlab, std::move(bT), std::move(bK), std::move(bW), std::move(bR), d));
  return op.analyse();
}

// ---------------------------------------------------------------------------
// explicit matrices: rSVD and CBE
// ---------------------------------------------------------------------------
namespace {

struct ExplicitOp {
  std::vector<int64_t> m, n, aoff;
  int64_t atotal = 0;
  double* A = nullptr;          // all matrices, row-major, concatenated
  // optional projectors (CBE): U_i (m x r), V_i (r x n)
  std::vector<int32_t> r;
  std::vector<int64_t> uoff, voff;
  double* U = nullptr;
  double* V = nullptr;
  int64_t utotal = 0, vtotal = 0;
  PlanSet ps;
  int pm = -1, pt = -1;
  // projection plans
  int p_v1 = -1, p_v2 = -1, p_u1 = -1, p_u2 = -1;
  int pt_u1 = -1, pt_u2 = -1, pt_v1 = -1, pt_v2 = -1;
  std::vector<int64_t> col_off, row_off, s_off;
  int64_t col_total = 0, row_total = 0, s_total = 0;
};

Status explicit_prepare(fpeps_ctx_s* ctx, ExplicitOp& e, const std::vector<int32_t>& k) {
  const int nm = (int)e.m.size();
  e.col_off.assign(nm, 0);
  e.row_off.assign(nm, 0);
  e.s_off.assign(nm, 0);
  e.col_total = e.row_total = e.s_total = 0;
  for (int i = 0; i < nm; ++i) {
    e.col_off[i] = e.col_total;
    e.row_off[i] = e.row_total;
    e.s_off[i] = e.s_total;
    e.col_total += e.n[i] * (int64_t)k[i];
    e.row_total += e.m[i] * (int64_t)k[i];
    e.s_total += (e.r.empty() ? 0 : (int64_t)e.r[i]) * k[i];
  }
  std::vector<DenseOp> fm, ft, v1, v2, u1, u2, tu1, tu2, tv1, tv2;
  for (int i = 0; i < nm; ++i) {
    if (k[i] <= 0) continue;
    DenseOp d{};
    d.alpha = 1.0;
    // y = A x
    d.a_off = e.aoff[i]; d.a_rs = e.n[i]; d.a_cs = 1;
    d.b_off = e.col_off[i]; d.b_rs = k[i]; d.b_cs = 1;
    d.c_off = e.row_off[i]; d.c_rs = k[i]; d.c_cs = 1;
    d.M = (int32_t)e.m[i]; d.N = k[i]; d.K = (int32_t)e.n[i];
    fm.push_back(d);
    // y = A^T x
    DenseOp t{};
    t.alpha = 1.0;
    t.a_off = e.aoff[i]; t.a_rs = 1; t.a_cs = e.n[i];
    t.b_off = e.row_off[i]; t.b_rs = k[i]; t.b_cs = 1;
    t.c_off = e.col_off[i]; t.c_rs = k[i]; t.c_cs = 1;
    t.M = (int32_t)e.n[i]; t.N = k[i]; t.K = (int32_t)e.m[i];
    ft.push_back(t);
    if (!e.r.empty() && e.r[i] > 0) {
      const int ri = e.r[i];
      // s = V x (r x k) ; x -= V^T s   (on the column side)
      DenseOp a{};
      a.alpha = 1.0;
      a.a_off = e.voff[i]; a.a_rs = e.n[i]; a.a_cs = 1;
      a.b_off = e.col_off[i]; a.b_rs = k[i]; a.b_cs = 1;
      a.c_off = e.s_off[i]; a.c_rs = k[i]; a.c_cs = 1;
      a.M = ri; a.N = k[i]; a.K = (int32_t)e.n[i];
      v1.push_back(a);
      DenseOp b{};
      b.alpha = -1.0;
      b.a_off = e.voff[i]; b.a_rs = 1; b.a_cs = e.n[i];
      b.b_off = e.s_off[i]; b.b_rs = k[i]; b.b_cs = 1;
      b.c_off = e.col_off[i]; b.c_rs = k[i]; b.c_cs = 1;
      b.M = (int32_t)e.n[i]; b.N = k[i]; b.K = ri;
      v2.push_back(b);
      // s = U^T y ; y -= U s  (on the row side)
      DenseOp c{};
      c.alpha = 1.0;
      c.a_off = e.uoff[i]; c.a_rs = 1; c.a_cs = ri;
      c.b_off = e.row_off[i]; c.b_rs = k[i]; c.b_cs = 1;
      c.c_off = e.s_off[i]; c.c_rs = k[i]; c.c_cs = 1;
      c.M = ri; c.N = k[i]; c.K = (int32_t)e.m[i];
      u1.push_back(c);
      DenseOp dd{};
      dd.alpha = -1.0;
      dd.a_off = e.uoff[i]; dd.a_rs = ri; dd.a_cs = 1;
      dd.b_off = e.s_off[i]; dd.b_rs = k[i]; dd.b_cs = 1;
      dd.c_off = e.row_off[i]; dd.c_rs = k[i]; dd.c_cs = 1;
      dd.M = (int32_t)e.m[i]; dd.N = k[i]; dd.K = ri;
      u2.push_back(dd);
    }
  }
  std::string err;
  e.ps = PlanSet();
  GemmPlan a, b, c1, c2, c3, c4;
  if (!plan_dense(fm, e.ps.pool, 64, 64, 1, a, err)) return fail(FPEPS_ERR_SHAPE, err);
  if (!plan_dense(ft, e.ps.pool, 64, 64, 1, b, err)) return fail(FPEPS_ERR_SHAPE, err);
  if (!plan_dense(v1, e.ps.pool, 64, 64, 1, c1, err)) return fail(FPEPS_ERR_SHAPE, err);
  if (!plan_dense(v2, e.ps.pool, 64, 64, 1, c2, err)) return fail(FPEPS_ERR_SHAPE, err);
  if (!plan_dense(u1, e.ps.pool, 64, 64, 1, c3, err)) return fail(FPEPS_ERR_SHAPE, err);
  if (!plan_dense(u2, e.ps.pool, 64, 64, 1, c4, err)) return fail(FPEPS_ERR_SHAPE, err);
  e.pm = e.ps.add(std::move(a));
  e.pt = e.ps.add(std::move(b));
  e.p_v1 = e.ps.add(std::move(c1));
  e.p_v2 = e.ps.add(std::move(c2));
  e.p_u1 = e.ps.add(std::move(c3));
  e.p_u2 = e.ps.add(std::move(c4));
  return e.ps.upload(ctx, "expl");
}

// The subtractions x - V^T (V x) and y - U (U^T y) accumulate into the
// operand in place: the GEMM writes C = alpha * A B, so they are done as
// separate products into scratch followed by an in-place axpy-free form:
// here the projected vector is formed as x' = x + (-V^T) s by a GEMM whose
// output is a scratch copy, then copied back.
Status project(fpeps_ctx_s* ctx, ExplicitOp& e, bool row_side, double* x, int64_t xtotal) {
  double *s = nullptr, *tmp = nullptr;
  FP_TRY(ctx->bufT("expl_s", (size_t)std::max<int64_t>(e.s_total, 1), &s));
  FP_TRY(ctx->bufT("expl_tmp", (size_t)std::max<int64_t>(xtotal, 1), &tmp));
  // matrices without kept directions have no projection product: their part
  // of tmp must add zero
  FP_HIP(launch_fill(tmp, xtotal, 0.0, ctx->stream));
  if (!row_side) {
    FP_TRY(run_gemm(ctx, e.ps, e.p_v1, e.V, e.vtotal, x, xtotal, s, std::max<int64_t>(e.s_total, 1)));
    FP_TRY(run_gemm(ctx, e.ps, e.p_v2, e.V, e.vtotal, s, std::max<int64_t>(e.s_total, 1), tmp, xtotal));
  } else {
    FP_TRY(run_gemm(ctx, e.ps, e.p_u1, e.U, e.utotal, x, xtotal, s, std::max<int64_t>(e.s_total, 1)));
    FP_TRY(run_gemm(ctx, e.ps, e.p_u2, e.U, e.utotal, s, std::max<int64_t>(e.s_total, 1), tmp, xtotal));
  }
  return axpy_inplace(ctx, x, tmp, xtotal);
}

}  // namespace

Status axpy_inplace(fpeps_ctx_s* ctx, double* x, const double* y, int64_t n) {
  FP_HIP(launch_add(x, y, n, ctx->stream));
  return Status::ok();
}

Status explicit_rsvd(fpeps_ctx_s* ctx, int nmat, const int64_t* m, const int64_t* n,
                     const double* const* A, const fpeps_opts* o, double* const* U_out,
                     double* const* R_out, int32_t* kept, double* sigma, fpeps_report* rep,
                     const int32_t* rr, const double* const* Uin, const double* const* Vin,
                     bool cbe, const int32_t* group) {
  if (nmat < 1 || !m || !n || !A || !o || !kept) return fail(FPEPS_ERR_ARG, "null argument");
  if (group)
    for (int i = 0; i < nmat; ++i)
      if (group[i] < 0 || group[i] >= nmat) return fail(FPEPS_ERR_ARG, "group ids must be 0 .. nmat-1");
  if (o->precision != FPEPS_FP64)
    return fail(FPEPS_ERR_UNSUPPORTED, "explicit matrices: only FPEPS_FP64 is available");
  EventPair evp;
  FP_HIP(evp.create());
  hipEvent_t ev0 = evp.a, ev1 = evp.b;
  FP_HIP(hipEventRecord(ev0, ctx->stream));
  ExplicitOp e;
  for (int i = 0; i < nmat; ++i) {
    if (m[i] < 0 || n[i] < 0 || m[i] > INT32_MAX || n[i] > INT32_MAX)
      return fail(FPEPS_ERR_ARG, "bad matrix size");
    if (m[i] * n[i] > 0 && !A[i]) return fail(FPEPS_ERR_ARG, "null matrix");
    e.m.push_back(m[i]);
    e.n.push_back(n[i]);
    e.aoff.push_back(e.atotal);
    e.atotal += m[i] * n[i];
  }
  FP_TRY(ctx->bufT("expl_A", (size_t)std::max<int64_t>(e.atotal, 1), &e.A));
  for (int i = 0; i < nmat; ++i)
    if (m[i] * n[i] > 0)
      FP_HIP(hipMemcpyAsync(e.A + e.aoff[i], A[i], m[i] * n[i] * sizeof(double),
                            hipMemcpyDeviceToDevice, ctx->stream));
  std::vector<int64_t> mm = e.m, nn = e.n;
  if (cbe) {
    if (!rr || !Uin || !Vin) return fail(FPEPS_ERR_ARG, "null projector argument");
    for (int i = 0; i < nmat; ++i) {
      if (rr[i] < 0 || rr[i] > m[i] || rr[i] > n[i]) return fail(FPEPS_ERR_ARG, "bad kept rank");
      e.r.push_back(rr[i]);
      e.uoff.push_back(e.utotal);
      e.voff.push_back(e.vtotal);
      e.utotal += m[i] * rr[i];
      e.vtotal += rr[i] * n[i];
      mm[i] = m[i] - rr[i];
      nn[i] = n[i] - rr[i];
    }
    FP_TRY(ctx->bufT("expl_U", (size_t)std::max<int64_t>(e.utotal, 1), &e.U));
    FP_TRY(ctx->bufT("expl_V", (size_t)std::max<int64_t>(e.vtotal, 1), &e.V));
    for (int i = 0; i < nmat; ++i) {
      if (rr[i] == 0) continue;
      FP_HIP(hipMemcpyAsync(e.U + e.uoff[i], Uin[i], m[i] * rr[i] * sizeof(double),
                            hipMemcpyDeviceToDevice, ctx->stream));
      FP_HIP(hipMemcpyAsync(e.V + e.voff[i], Vin[i], rr[i] * n[i] * sizeof(double),
                            hipMemcpyDeviceToDevice, ctx->stream));
    }
  }
  RsvdIO io;
  io.m = e.m;
  io.n = e.n;
  if (!group) {
    for (int i = 0; i < nmat; ++i) io.c1.push_back((uint32_t)i);
    io.c2 = (uint32_t)o->tag;
  } else {
    // every group is the problem of its own call: sketch counters (ordinal
    // inside the group, tag + group), widths and cut per group
    std::vector<uint32_t> ord(nmat, 0);
    for (int i = 0; i < nmat; ++i) {
      io.c1.push_back(ord[group[i]]++);
      io.c2v.push_back((uint32_t)(o->tag + group[i]));
      io.grp.push_back(group[i]);
    }
  }
  io.c3 = cbe ? (1u << 16) : 0u;
  // widths follow the (residual) sizes: k_i = min(m_i', n_i', ceil(chi m_i'/sum m') + p)
  const int chi = cbe ? o->cbe_extra : o->chi;
  io.width_m = mm;
  io.width_n = nn;
  io.prepare = [&](const std::vector<int32_t>& k) { return explicit_prepare(ctx, e, k); };
  io.apply = [&](bool t, bool, const double* x, double* y) -> Status {
    if (!t) {
      double* xc = const_cast<double*>(x);
      if (cbe) FP_TRY(project(ctx, e, false, xc, e.col_total));
      FP_TRY(run_gemm(ctx, e.ps, e.pm, e.A, e.atotal, xc, e.col_total, y, e.row_total));
      if (cbe) FP_TRY(project(ctx, e, true, y, e.row_total));
    } else {
      double* xc = const_cast<double*>(x);
      if (cbe) FP_TRY(project(ctx, e, true, xc, e.row_total));
      FP_TRY(run_gemm(ctx, e.ps, e.pt, e.A, e.atotal, xc, e.row_total, y, e.col_total));
      if (cbe) FP_TRY(project(ctx, e, false, y, e.col_total));
    }
    return Status::ok();
  };
  RsvdOut rs;
  FP_TRY(rsvd_run(ctx, io, chi, o->oversample, cbe ? 0 : o->power_iters, o->seed, rs, o->sv_cut));
  // outputs
  std::vector<int64_t> uoff(nmat), roff(nmat);
  int64_t ut = 0, rt = 0;
  for (int i = 0; i < nmat; ++i) {
    uoff[i] = ut;
    roff[i] = rt;
    ut += e.m[i] * (int64_t)rs.kept[i];
    rt += e.n[i] * (int64_t)rs.kept[i];
  }
  double *ub = nullptr, *rb = nullptr;
  FP_TRY(ctx->bufT("expl_Uo", (size_t)std::max<int64_t>(ut, 1), &ub));
  if (!cbe) FP_TRY(ctx->bufT("expl_Ro", (size_t)std::max<int64_t>(rt, 1), &rb));
  FP_TRY(rsvd_factors(ctx, io, rs, uoff, ub, std::max<int64_t>(ut, 1), roff, cbe ? nullptr : rb,
                      std::max<int64_t>(rt, 1)));
  int64_t sp = 0;
  for (int i = 0; i < nmat; ++i) {
    kept[i] = rs.kept[i];
    const int64_t c = rs.kept[i];
    if (c > 0 && U_out && U_out[i])
      FP_HIP(hipMemcpyAsync(U_out[i], ub + uoff[i], e.m[i] * c * sizeof(double),
                            hipMemcpyDeviceToDevice, ctx->stream));
    if (!cbe && c > 0 && R_out && R_out[i])
      FP_HIP(hipMemcpyAsync(R_out[i], rb + roff[i], e.n[i] * c * sizeof(double),
                            hipMemcpyDeviceToDevice, ctx->stream));
    if (sigma)
      for (int j = 0; j < c; ++j) {
        const double l = rs.lam[rs.lam_off[i] + j];
        sigma[sp++] = l > 0 ? std::sqrt(l) : 0.0;
      }
  }
  FP_HIP(hipEventRecord(ev1, ctx->stream));
  FP_HIP(hipEventSynchronize(ev1));
  float ms = 0;
  FP_HIP(hipEventElapsedTime(&ms, ev0, ev1));
  if (rep) {
    // algorithmic flops, counted as for a site of the absorption: (2 + 2q)
    // dense products (plus the projector splits of the expansion),
    // orthonormalisation, core factorisation and the output factors
    const int qq = cbe ? 0 : o->power_iters;
    double fl = 0;
    for (const auto& pk : rs.pass_k)
      for (int i = 0; i < nmat; ++i) {
        const double mi = (double)e.m[i], ni = (double)e.n[i], k = pk[i];
        if (k <= 0) continue;
        fl += (2 + 2 * qq) * 2.0 * mi * ni * k;
        if (cbe) fl += (2 + 2 * qq) * 4.0 * (rr ? rr[i] : 0) * k * (mi + ni);
        fl += (qq + 1) * (2 * mi * k * k - 2 * k * k * k / 3.0) +
              qq * (2 * ni * k * k - 2 * k * k * k / 3.0);
        fl += 2 * ni * k * k + 11 * k * k * k;
      }
    for (int i = 0; i < nmat; ++i) {
      const double mi = (double)e.m[i], ni = (double)e.n[i], k = rs.k[i], c = rs.kept[i];
      if (k > 0) fl += 2 * mi * k * c + (cbe ? 0.0 : 2 * k * c * ni);
    }
    rep->alg_flops = fl;
    rep->rsvd_passes = (int32_t)rs.pass_k.size();
    rep->workspace_bytes = (double)ctx->ws_bytes;
    rep->seconds = ms * 1e-3;
    rep->fallbacks = rs.fallbacks;
    int tot = 0;
    for (int v : rs.kept) tot += v;
    rep->kept_total = tot;
    // over the groups: the smallest relative gap and the largest discarded weight
    double gap = INFINITY, disc = 0.0;
    for (const CutOut& c : rs.cuts) {
      if (c.s_next >= 0 && c.s_last > 0) gap = std::min(gap, (c.s_last - c.s_next) / c.s_last);
      if (c.total2 > 0) disc = std::max(disc, 1.0 - c.kept2 / c.total2);
    }
    rep->min_rel_gap = std::isfinite(gap) ? gap : -1.0;
    rep->discarded_weight = disc;
  }
  return Status::ok();
}

// ---------------------------------------------------------------------------
// overlap of two environments
// ---------------------------------------------------------------------------
Status overlap(fpeps_ctx_s* ctx, int L, const fpeps_tensor* top, const fpeps_tensor* bot,
               double log_norm, int32_t* sign, double* log_abs) {
  if (L < 1 || !top || !bot || !sign || !log_abs) return fail(FPEPS_ERR_ARG, "null argument");
  if (!std::isfinite(log_norm)) return fail(FPEPS_ERR_ARG, "non-finite log-norm");
  // E is divided by its Frobenius norm after every site; the logarithms are
  // accumulated, so the value is returned as (sign, log |value|) whatever
  // its magnitude
  double lg = log_norm;
  double *npart = nullptr, *nout = nullptr;
  FP_TRY(ctx->bufT("ov_npart", 512, &npart));
  FP_TRY(ctx->bufT("ov_nout", 1, &nout));
  const int nlab = top[0].nlab;
  SymInfo none;
  // E[at, ab]
  BT E;
  double* Ebuf[2] = {nullptr, nullptr};
  FP_TRY(ctx->bufT("ov_E0", 1, &Ebuf[0]));
  FP_HIP(launch_fill(Ebuf[0], 1, 1.0, ctx->stream));
  int cur = 0;
  int64_t Esize = 1;
  for (int x = 0; x < L; ++x) {
    BT T, B;
    FP_TRY(tensor_to_bt(&top[x], {N_a, N_tk, N_tw, N_tb, N_b}, nlab, T));
    FP_TRY(tensor_to_bt(&bot[x], {N_c, N_tk, N_tw, N_tb, N_j}, nlab, B));
    if (x == 0) {
      if (T.cat[0]->total() != 1 || B.cat[0]->total() != 1)
        return fail(FPEPS_ERR_SHAPE, "left bonds of the environments must have dim 1");
      E.names = {N_a, N_c};
      E.cat = {T.cat[0], B.cat[0]};
      Block b;
      b.base = 0;
      set_rowmajor(E, b);
      E.blocks.push_back(b);
      E.size = 1;
    }
    PlanSet ps;
    std::string err;
    StepSpec s1;
    s1.step = 1;
    s1.m_is_x = false;
    s1.out_names = {N_c, N_tk, N_tw, N_tb, N_b};
    s1.key_order = {N_a, N_c};
    StepResult r1;
    if (!plan_step(E, T, s1, none, ps.pool, nullptr, r1, err)) return fail(FPEPS_ERR_SHAPE, err);
    StepSpec s2;
    s2.step = 2;
    s2.m_is_x = true;
    s2.out_names = {N_b, N_j};
    s2.key_order = {N_c, N_tk, N_tw, N_tb, N_b};
    StepResult r2;
    if (!plan_step(r1.out, B, s2, none, ps.pool, nullptr, r2, err))
      return fail(FPEPS_ERR_SHAPE, err);
    const int64_t xs = std::max<int64_t>(r1.out.size, 1), es = std::max<int64_t>(r2.out.size, 1);
    int i1 = ps.add(std::move(r1.plan)), i2 = ps.add(std::move(r2.plan));
    FP_TRY(ps.upload(ctx, "ov"));
    double* X = nullptr;
    FP_TRY(ctx->bufT("ov_X", (size_t)xs, &X));
    const int nx = 1 - cur;
    FP_TRY(ctx->bufT(nx ? "ov_E1" : "ov_E0b", (size_t)es, &Ebuf[nx]));
    FP_TRY(run_gemm(ctx, ps, i1, top[x].data, top[x].nelem, Ebuf[cur], Esize, X, xs));
    FP_TRY(run_gemm(ctx, ps, i2, X, xs, bot[x].data, bot[x].nelem, Ebuf[nx], es));
    if (x + 1 < L) {
      FP_HIP(launch_sumsq(Ebuf[nx], es, npart, nout, ctx->stream));
      double h = 0;
      FP_HIP(hipMemcpyAsync(&h, nout, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      FP_TRY(ctx->sync());
      if (!std::isfinite(h)) return fail(FPEPS_ERR_NUMERIC, "non-finite environment overlap");
      if (h > 0.0) {
        const double nu = std::sqrt(h);
        FP_HIP(launch_scale(Ebuf[nx], es, 1.0 / nu, ctx->stream));
        lg += std::log(nu);
      }
    }
    FP_TRY(ctx->sync());
    E = BT();
    E.names = {N_a, N_c};
    E.cat = r2.out.cat;
    E.blocks = r2.out.blocks;
    E.size = es;
    Esize = es;
    cur = nx;
  }
  // sum of all entries of the final (1 x 1 per block) E
  std::vector<double> h(Esize);
  FP_HIP(hipMemcpyAsync(h.data(), Ebuf[cur], Esize * sizeof(double), hipMemcpyDeviceToHost,
                        ctx->stream));
  FP_TRY(ctx->sync());
  double v = 0;
  for (const Block& b : E.blocks) v += h[b.base];
  if (!std::isfinite(v)) return fail(FPEPS_ERR_NUMERIC, "non-finite environment overlap");
  *sign = v > 0.0 ? 1 : (v < 0.0 ? -1 : 0);
  *log_abs = v != 0.0 ? lg + std::log(std::fabs(v)) : -INFINITY;
  return Status::ok();
}

}  // namespace fp
