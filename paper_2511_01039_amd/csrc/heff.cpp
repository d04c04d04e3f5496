// The effective single-site operator of the Davidson step applied to a PEPS
// tensor: contraction pattern 2(b) of Sec. 3, ((T L) C) (B R) with the
// PEPS-PEPO sandwich C applied layer by layer, every step a grouped
// block-pair GEMM on the device.
#include "driver.hpp"

#include <algorithm>

namespace fp {

namespace {
// leg orders of the intermediates (the keys of the per-pair scalars)
const std::vector<int> H_T = {N_a, N_tk, N_tw, N_tb, N_b};
const std::vector<int> H_L = {N_a, N_lk, N_lw, N_lb, N_c};
const std::vector<int> H_B = {N_c, N_dk, N_dw, N_db, N_d};
const std::vector<int> H_R = {N_b, N_rk, N_rw, N_rb, N_d};
const std::vector<int> H_KET = {N_p, N_lk, N_rk, N_tk, N_dk};
const std::vector<int> H_PEPO = {N_q, N_p, N_lw, N_rw, N_tw, N_dw};
const std::vector<int> H_X1 = {N_tk, N_tw, N_tb, N_b, N_lk, N_lw, N_lb, N_c};
const std::vector<int> H_X2 = {N_tw, N_tb, N_b, N_lw, N_lb, N_c, N_p, N_rk, N_dk};
const std::vector<int> H_X3 = {N_tb, N_b, N_lb, N_c, N_rk, N_dk, N_q, N_rw, N_dw};
const std::vector<int> H_X4 = {N_c, N_dk, N_dw, N_db, N_b, N_rk, N_rw, N_rb};
const std::vector<int> H_Y = {N_q, N_lb, N_rb, N_tb, N_db};
}  // namespace

Status heff_apply(fpeps_ctx_s* ctx, const fpeps_tensor* T, const fpeps_tensor* L,
                  const fpeps_tensor* B, const fpeps_tensor* R, const fpeps_tensor* W,
                  const fpeps_tensor* A, const fpeps_opts* o, fpeps_tensor* y,
                  fpeps_report* rep) {
  if (!T || !L || !B || !R || !W || !A || !o || !y) return fail(FPEPS_ERR_ARG, "null argument");
  if (o->precision != FPEPS_FP64) return fail(FPEPS_ERR_UNSUPPORTED, "precision: FPEPS_FP64");
  SymInfo sym;
  sym.kind = o->symmetry;
  sym.fermionic = o->fermionic != 0;
  sym.coef_seed = o->coef_seed;
  if (sym.kind < 0 || sym.kind > 2) return fail(FPEPS_ERR_ARG, "bad symmetry");
  const int nlab = sym.kind == SYM_U1U1 ? 2 : 1;
  BT bT, bL, bB, bR, bW, bA;
  FP_TRY(tensor_to_bt(T, H_T, nlab, bT));
  FP_TRY(tensor_to_bt(L, H_L, nlab, bL));
  FP_TRY(tensor_to_bt(B, H_B, nlab, bB));
  FP_TRY(tensor_to_bt(R, H_R, nlab, bR));
  FP_TRY(tensor_to_bt(W, H_PEPO, nlab, bW));
  FP_TRY(tensor_to_bt(A, H_KET, nlab, bA));
  struct Step {
    const BT* X;
    const BT* S;
    const std::vector<int>* out;
    const std::vector<int>* key;
    int step;
  };
  // X1 = T L, X2 = X1 A, X3 = X2 W, X4 = B R, y = X3 X4; the M index of each
  // product comes from X (its free legs lead in the output order)
  PlanSet ps;
  std::string err;
  BT X1, X2, X3, X4, Y;
  BT* outs[5] = {&X1, &X2, &X3, &X4, &Y};
  const Step steps[5] = {{&bT, &bL, &H_X1, &H_T, 11},
                         {&X1, &bA, &H_X2, &H_X1, 12},
                         {&X2, &bW, &H_X3, &H_X2, 13},
                         {&bB, &bR, &H_X4, &H_B, 14},
                         {&X3, &X4, &H_Y, &H_X3, 15}};
  int idx[5];
  double flops = 0;
  for (int s = 0; s < 5; ++s) {
    StepSpec sp;
    sp.step = steps[s].step;
    sp.m_is_x = true;
    sp.key_side = 0;
    sp.out_names = *steps[s].out;
    sp.key_order = *steps[s].key;
    StepResult r;
    if (!plan_step(*steps[s].X, *steps[s].S, sp, sym, ps.pool, nullptr, r, err))
      return fail(FPEPS_ERR_SHAPE, "effective-operator step " + std::to_string(s + 1) + ": " + err);
    flops += r.plan.flops;
    idx[s] = ps.add(std::move(r.plan));
    *outs[s] = std::move(r.out);
  }
  // output structure: the bra-side legs, blocks as the last step made them
  {
    int need_sect = 0;
    for (auto& l : Y.cat) need_sect = std::max(need_sect, l->nsect());
    if (rep) {
      rep->required_sect = need_sect;
      rep->required_blocks = (int32_t)Y.blocks.size();
      rep->required_elem = Y.size;
    }
    if (need_sect > y->max_sect || (int64_t)Y.blocks.size() > y->max_blocks || Y.size > y->max_elem)
      return fail(FPEPS_ERR_CAPACITY, "output tensor capacity too small (see report)");
    if (!y->nsect || !y->dirs || !y->labels || !y->dims || !y->block_sect || !y->block_off ||
        (Y.size > 0 && !y->data))
      return fail(FPEPS_ERR_ARG, "output tensor has null arrays");
    y->nlegs = 5;
    y->nlab = nlab;
    for (int l = 0; l < 5; ++l) {
      const Leg& g = *Y.cat[l];
      y->nsect[l] = g.nsect();
      y->dirs[l] = g.dir;
      for (int s = 0; s < g.nsect(); ++s) {
        for (int i = 0; i < nlab; ++i) y->labels[((int64_t)l * y->max_sect + s) * nlab + i] = g.label(s)[i];
        y->dims[(int64_t)l * y->max_sect + s] = g.dim[s];
      }
    }
    y->nblocks = (int32_t)Y.blocks.size();
    for (size_t b = 0; b < Y.blocks.size(); ++b) {
      for (int l = 0; l < 5; ++l) y->block_sect[b * 5 + l] = Y.blocks[b].sect[l];
      y->block_off[b] = Y.blocks[b].base;
    }
    y->nelem = Y.size;
  }
  FP_TRY(ps.upload(ctx, "heff"));
  EventPair evp;
  FP_HIP(evp.create());
  FP_HIP(hipEventRecord(evp.a, ctx->stream));
  double *x1 = nullptr, *x2 = nullptr, *x3 = nullptr, *x4 = nullptr;
  const int64_t s1 = std::max<int64_t>(X1.size, 1), s2 = std::max<int64_t>(X2.size, 1),
                s3 = std::max<int64_t>(X3.size, 1), s4 = std::max<int64_t>(X4.size, 1);
  FP_TRY(ctx->bufT("heff_x1", (size_t)s1, &x1));
  FP_TRY(ctx->bufT("heff_x2", (size_t)s2, &x2));
  FP_TRY(ctx->bufT("heff_x3", (size_t)s3, &x3));
  FP_TRY(ctx->bufT("heff_x4", (size_t)s4, &x4));
  FP_TRY(run_gemm(ctx, ps, idx[0], T->data, T->nelem, L->data, L->nelem, x1, s1));
  FP_TRY(run_gemm(ctx, ps, idx[1], x1, s1, A->data, A->nelem, x2, s2));
  FP_TRY(run_gemm(ctx, ps, idx[2], x2, s2, W->data, W->nelem, x3, s3));
  FP_TRY(run_gemm(ctx, ps, idx[3], B->data, B->nelem, R->data, R->nelem, x4, s4));
  if (Y.size > 0) FP_TRY(run_gemm(ctx, ps, idx[4], x3, s3, x4, s4, y->data, Y.size));
  FP_HIP(hipEventRecord(evp.b, ctx->stream));
  FP_HIP(hipEventSynchronize(evp.b));
  float ms = 0;
  FP_HIP(hipEventElapsedTime(&ms, evp.a, evp.b));
  if (rep) {
    rep->alg_flops = flops;
    rep->seconds = ms * 1e-3;
    rep->workspace_bytes = (double)ctx->ws_bytes;
  }
  return Status::ok();
}

}  // namespace fp
