// The effective single-site operator of the Davidson step applied to a PEPS
// tensor: contraction pattern 2(b) of Sec. 3, ((T L) C) (B R) with the
// PEPS-PEPO sandwich C applied layer by layer, every step a grouped
// block-pair GEMM on the device.
#include "driver.hpp"

#include <algorithm>
#include <atomic>
#include <memory>

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

// The five steps planned: X1 = T L, X2 = X1 A, X3 = X2 W, X4 = B R,
// y = X3 X4; the M index of each product comes from X (its free legs lead
// in the output order).
struct HeffPlan {
  PlanSet ps;
  BT X1, X2, X3, X4, Y;
  int idx[5];
  double flops[5];
  int nlab = 1;
};

Status heff_plan(const fpeps_tensor* T, const fpeps_tensor* L, const fpeps_tensor* B,
                 const fpeps_tensor* R, const fpeps_tensor* W, const fpeps_tensor* A,
                 const fpeps_opts* o, HeffPlan& hp) {
  if (!T || !L || !B || !R || !W || !A || !o) return fail(FPEPS_ERR_ARG, "null argument");
  if (o->precision != FPEPS_FP64) return fail(FPEPS_ERR_UNSUPPORTED, "precision: FPEPS_FP64");
  SymInfo sym;
  sym.kind = o->symmetry;
  sym.fermionic = o->fermionic != 0;
  sym.coef_seed = o->coef_seed;
  if (sym.kind < 0 || sym.kind > 2) return fail(FPEPS_ERR_ARG, "bad symmetry");
  hp.nlab = sym.kind == SYM_U1U1 ? 2 : 1;
  BT bT, bL, bB, bR, bW, bA;
  FP_TRY(tensor_to_bt(T, H_T, hp.nlab, bT));
  FP_TRY(tensor_to_bt(L, H_L, hp.nlab, bL));
  FP_TRY(tensor_to_bt(B, H_B, hp.nlab, bB));
  FP_TRY(tensor_to_bt(R, H_R, hp.nlab, bR));
  FP_TRY(tensor_to_bt(W, H_PEPO, hp.nlab, bW));
  FP_TRY(tensor_to_bt(A, H_KET, hp.nlab, bA));
  struct Step {
    const BT* X;
    const BT* S;
    const std::vector<int>* out;
    const std::vector<int>* key;
    int step;
  };
  BT* outs[5] = {&hp.X1, &hp.X2, &hp.X3, &hp.X4, &hp.Y};
  const Step steps[5] = {{&bT, &bL, &H_X1, &H_T, 11},
                         {&hp.X1, &bA, &H_X2, &H_X1, 12},
                         {&hp.X2, &bW, &H_X3, &H_X2, 13},
                         {&bB, &bR, &H_X4, &H_B, 14},
                         {&hp.X3, &hp.X4, &H_Y, &H_X3, 15}};
  std::string err;
  for (int s = 0; s < 5; ++s) {
    StepSpec sp;
    sp.step = steps[s].step;
    sp.m_is_x = true;
    sp.key_side = 0;
    sp.out_names = *steps[s].out;
    sp.key_order = *steps[s].key;
    StepResult r;
    if (!plan_step(*steps[s].X, *steps[s].S, sp, sym, hp.ps.pool, nullptr, r, err))
      return fail(FPEPS_ERR_SHAPE, "effective-operator step " + std::to_string(s + 1) + ": " + err);
    hp.flops[s] = r.plan.flops;
    hp.idx[s] = hp.ps.add(std::move(r.plan));
    *outs[s] = std::move(r.out);
  }
  return Status::ok();
}

// The output structure (bra-side legs, blocks as the last step made them)
// into ``y`` (capacity checked; required sizes in the report).
Status heff_out_struct(const HeffPlan& hp, fpeps_tensor* y, fpeps_report* rep) {
  const BT& Y = hp.Y;
  int need_sect = 0;
  for (auto& l : Y.cat) need_sect = std::max(need_sect, l->nsect());
  if (rep) {
    rep->required_sect = need_sect;
    rep->required_blocks = (int32_t)Y.blocks.size();
    rep->required_elem = Y.size;
  }
  if (need_sect > y->max_sect || (int64_t)Y.blocks.size() > y->max_blocks || Y.size > y->max_elem)
    return fail(FPEPS_ERR_CAPACITY, "output tensor capacity too small (see report)");
  if (!y->nsect || !y->dirs || !y->labels || !y->dims || !y->block_sect || !y->block_off)
    return fail(FPEPS_ERR_ARG, "output tensor has null arrays");
  const int nlab = hp.nlab;
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
  return Status::ok();
}

}  // namespace

Status heff_apply(fpeps_ctx_s* ctx, const fpeps_tensor* T, const fpeps_tensor* L,
                  const fpeps_tensor* B, const fpeps_tensor* R, const fpeps_tensor* W,
                  const fpeps_tensor* A, const fpeps_opts* o, fpeps_tensor* y,
                  fpeps_report* rep) {
  if (!y) return fail(FPEPS_ERR_ARG, "null argument");
  HeffPlan hp;
  FP_TRY(heff_plan(T, L, B, R, W, A, o, hp));
  FP_TRY(heff_out_struct(hp, y, rep));
  if (hp.Y.size > 0 && !y->data) return fail(FPEPS_ERR_ARG, "output tensor has null arrays");
  PlanSet& ps = hp.ps;
  const int* idx = hp.idx;
  FP_TRY(ps.upload(ctx, "heff"));
  EventPair evp;
  FP_HIP(evp.create());
  FP_HIP(hipEventRecord(evp.a, ctx->stream));
  double *x1 = nullptr, *x2 = nullptr, *x3 = nullptr, *x4 = nullptr;
  const int64_t s1 = std::max<int64_t>(hp.X1.size, 1), s2 = std::max<int64_t>(hp.X2.size, 1),
                s3 = std::max<int64_t>(hp.X3.size, 1), s4 = std::max<int64_t>(hp.X4.size, 1);
  FP_TRY(ctx->bufT("heff_x1", (size_t)s1, &x1));
  FP_TRY(ctx->bufT("heff_x2", (size_t)s2, &x2));
  FP_TRY(ctx->bufT("heff_x3", (size_t)s3, &x3));
  FP_TRY(ctx->bufT("heff_x4", (size_t)s4, &x4));
  FP_TRY(run_gemm(ctx, ps, idx[0], T->data, T->nelem, L->data, L->nelem, x1, s1));
  FP_TRY(run_gemm(ctx, ps, idx[1], x1, s1, A->data, A->nelem, x2, s2));
  FP_TRY(run_gemm(ctx, ps, idx[2], x2, s2, W->data, W->nelem, x3, s3));
  FP_TRY(run_gemm(ctx, ps, idx[3], B->data, B->nelem, R->data, R->nelem, x4, s4));
  if (hp.Y.size > 0) FP_TRY(run_gemm(ctx, ps, idx[4], x3, s3, x4, s4, y->data, hp.Y.size));
  FP_HIP(hipEventRecord(evp.b, ctx->stream));
  FP_HIP(hipEventSynchronize(evp.b));
  float ms = 0;
  FP_HIP(hipEventElapsedTime(&ms, evp.a, evp.b));
  if (rep) {
    double f = 0;
    for (double v : hp.flops) f += v;
    rep->alg_flops = f;
    rep->seconds = ms * 1e-3;
    rep->workspace_bytes = (double)ctx->ws_bytes;
  }
  return Status::ok();
}

}  // namespace fp

// ---------------------------------------------------------------------------
// The prepared operator: for repeated products with one environment (the
// Davidson iterations of a site), T L and B R do not depend on the vector
// and are contracted once; the three vector-dependent steps are captured as a
// HIP graph and replayed for every vector. Every buffer the graph touches
// (plan tables, X1..X4, the PEPO, the vector in and out, split-K parts) is
// the handle's own, under names no other call uses, so nothing else can move
// them while the handle lives.
// ---------------------------------------------------------------------------
struct fpeps_heff_s {
  fpeps_ctx_s* ctx = nullptr;
  fp::HeffPlan hp;
  std::string tag;                  // unique prefix of the handle's buffers
  uint64_t ws_gen = 0;              // the context's workspace generation
  double *x1 = nullptr, *x2 = nullptr, *x3 = nullptr, *x4 = nullptr;
  double *w = nullptr, *a_in = nullptr, *y_out = nullptr, *part = nullptr;
  int64_t s1 = 1, s2 = 1, s3 = 1, s4 = 1, w_size = 1, a_size = 1, y_size = 1;
  int64_t a_nelem = 0;              // elements of the prepared vector structure
  bool eager = false;               // FPEPS_FLAG_NO_GRAPH: launch, do not replay
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~fpeps_heff_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace fp {

namespace {
std::atomic<uint64_t> heff_ids{0};

// the three vector-dependent products, on the handle's buffers, on stream s
Status heff_vec_steps(fpeps_heff_s* h, hipStream_t s) {
  fpeps_ctx_s* ctx = h->ctx;
  const hipStream_t keep = ctx->stream;
  ctx->stream = s;
  const int* idx = h->hp.idx;
  Status st = run_gemm_any(ctx, h->hp.ps, idx[1], h->x1, nullptr, h->s1, h->a_in, false,
                           h->a_size, h->x2, false, h->s2, false, -1, h->part);
  if (st.good())
    st = run_gemm_any(ctx, h->hp.ps, idx[2], h->x2, nullptr, h->s2, h->w, false, h->w_size, h->x3,
                      false, h->s3, false, -1, h->part);
  if (st.good() && h->hp.Y.size > 0)
    st = run_gemm_any(ctx, h->hp.ps, idx[4], h->x3, nullptr, h->s3, h->x4, false, h->s4,
                      h->y_out, false, h->y_size, false, -1, h->part);
  ctx->stream = keep;
  return st;
}
}  // namespace

Status heff_prepare(fpeps_ctx_s* ctx, const fpeps_tensor* T, const fpeps_tensor* L,
                    const fpeps_tensor* B, const fpeps_tensor* R, const fpeps_tensor* W,
                    const fpeps_tensor* A, const fpeps_opts* o, fpeps_tensor* y,
                    fpeps_heff_s** out, fpeps_report* rep) {
  if (!y || !out) return fail(FPEPS_ERR_ARG, "null argument");
  *out = nullptr;
  std::unique_ptr<fpeps_heff_s> h(new fpeps_heff_s());
  h->ctx = ctx;
  FP_TRY(heff_plan(T, L, B, R, W, A, o, h->hp));
  FP_TRY(heff_out_struct(h->hp, y, rep));
  h->tag = "heffp" + std::to_string(heff_ids.fetch_add(1)) + "_";
  HeffPlan& hp = h->hp;
  FP_TRY(hp.ps.upload(ctx, h->tag + "plans"));
  h->s1 = std::max<int64_t>(hp.X1.size, 1);
  h->s2 = std::max<int64_t>(hp.X2.size, 1);
  h->s3 = std::max<int64_t>(hp.X3.size, 1);
  h->s4 = std::max<int64_t>(hp.X4.size, 1);
  h->w_size = std::max<int64_t>(W->nelem, 1);
  h->a_size = std::max<int64_t>(A->nelem, 1);
  h->a_nelem = A->nelem;
  h->y_size = std::max<int64_t>(hp.Y.size, 1);
  int64_t part = 1;
  for (const GemmPlan& g : hp.ps.plans) part = std::max<int64_t>(part, g.partial_size);
  FP_TRY(ctx->bufT(h->tag + "x1", (size_t)h->s1, &h->x1));
  FP_TRY(ctx->bufT(h->tag + "x2", (size_t)h->s2, &h->x2));
  FP_TRY(ctx->bufT(h->tag + "x3", (size_t)h->s3, &h->x3));
  FP_TRY(ctx->bufT(h->tag + "x4", (size_t)h->s4, &h->x4));
  FP_TRY(ctx->bufT(h->tag + "w", (size_t)h->w_size, &h->w));
  FP_TRY(ctx->bufT(h->tag + "a", (size_t)h->a_size, &h->a_in));
  FP_TRY(ctx->bufT(h->tag + "y", (size_t)h->y_size, &h->y_out));
  FP_TRY(ctx->bufT(h->tag + "part", (size_t)part, &h->part));
  FP_HIP(hipMemcpyAsync(h->w, W->data, W->nelem * sizeof(double), hipMemcpyDeviceToDevice,
                        ctx->stream));
  FP_HIP(hipMemcpyAsync(h->a_in, A->data, A->nelem * sizeof(double), hipMemcpyDeviceToDevice,
                        ctx->stream));
  // the vector-independent halves, once
  FP_TRY(run_gemm_any(ctx, hp.ps, hp.idx[0], T->data, nullptr, T->nelem, L->data, false, L->nelem,
                      h->x1, false, h->s1, false, -1, h->part));
  FP_TRY(run_gemm_any(ctx, hp.ps, hp.idx[3], B->data, nullptr, B->nelem, R->data, false, R->nelem,
                      h->x4, false, h->s4, false, -1, h->part));
  // one eager run of the vector steps (the product for A goes to y), then
  // the capture of the same launches on a stream of the handle's own
  FP_TRY(heff_vec_steps(h.get(), ctx->stream));
  if (hp.Y.size > 0) {
    if (!y->data) return fail(FPEPS_ERR_ARG, "output tensor has null arrays");
    FP_HIP(hipMemcpyAsync(y->data, h->y_out, hp.Y.size * sizeof(double), hipMemcpyDeviceToDevice,
                          ctx->stream));
  }
  FP_HIP(hipStreamSynchronize(ctx->stream));
  h->eager = (o->flags & FPEPS_FLAG_NO_GRAPH) != 0;
  if (!h->eager) {
    FP_HIP(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    FP_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    Status cs = heff_vec_steps(h.get(), h->cap);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(h->cap, &g);
    FP_TRY(cs);
    FP_HIP(ce);
    h->graph = g;
    FP_HIP(hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0));
  }
  h->ws_gen = ctx->ws_generation;
  if (rep) {
    rep->alg_flops = hp.flops[0] + hp.flops[3];
    rep->workspace_bytes = (double)ctx->ws_bytes;
  }
  *out = h.release();
  return Status::ok();
}

fpeps_ctx_s* heff_context(fpeps_heff_s* h) { return h->ctx; }

Status heff_release(fpeps_heff_s* h) {
  std::unique_ptr<fpeps_heff_s> own(h);
  // the graph's buffers go once no replay can still run
  if (h->ctx->ws_generation == h->ws_gen) FP_TRY(h->ctx->release_prefix(h->tag));
  return Status::ok();
}

Status heff_apply_prepared(fpeps_heff_s* h, const double* a, int64_t a_elems, double* y,
                           int64_t y_elems, fpeps_report* rep) {
  fpeps_ctx_s* ctx = h->ctx;
  if (!a || (h->hp.Y.size > 0 && !y)) return fail(FPEPS_ERR_ARG, "null argument");
  if (a_elems != h->a_nelem || y_elems < h->hp.Y.size)
    return fail(FPEPS_ERR_ARG, "vector or output size does not match the prepared structure");
  if (ctx->ws_generation != h->ws_gen)
    return fail(FPEPS_ERR_ARG, "the context's workspace was released since the operator was "
                               "prepared (fpeps_set_allocator); prepare it again");
  EventPair evp;
  FP_HIP(evp.create());
  FP_HIP(hipEventRecord(evp.a, ctx->stream));
  FP_HIP(hipMemcpyAsync(h->a_in, a, a_elems * sizeof(double), hipMemcpyDeviceToDevice,
                        ctx->stream));
  if (h->eager)
    FP_TRY(heff_vec_steps(h, ctx->stream));
  else
    FP_HIP(hipGraphLaunch(h->exec, ctx->stream));
  if (h->hp.Y.size > 0)
    FP_HIP(hipMemcpyAsync(y, h->y_out, h->hp.Y.size * sizeof(double), hipMemcpyDeviceToDevice,
                          ctx->stream));
  FP_HIP(hipEventRecord(evp.b, ctx->stream));
  FP_HIP(hipEventSynchronize(evp.b));
  float ms = 0;
  FP_HIP(hipEventElapsedTime(&ms, evp.a, evp.b));
  if (rep) {
    rep->alg_flops = h->hp.flops[1] + h->hp.flops[2] + h->hp.flops[4];
    rep->seconds = ms * 1e-3;
  }
  return Status::ok();
}

}  // namespace fp
