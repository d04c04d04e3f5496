// Site operator M_x: sector structure, sliced chain plans, application.
#include "site.hpp"

#include <algorithm>
#include <chrono>
#include <map>
#include <thread>

namespace fp {

const std::vector<int> ORDER_X[6] = {
    {N_b, N_rk, N_rw, N_rb, N_j},
    {N_a, N_tk, N_tw, N_tb, N_rk, N_rw, N_rb, N_j},
    {N_a, N_tw, N_tb, N_rw, N_rb, N_j, N_p, N_lk, N_dk},
    {N_a, N_tb, N_rb, N_j, N_lk, N_dk, N_q, N_lw, N_dw},
    {N_a, N_j, N_lk, N_dk, N_lw, N_dw, N_lb, N_db},
    {N_c, N_dk, N_dw, N_db, N_j},
};

// storage orders of the intermediates: the sketch column index j is
// innermost (stride 1) in all of them, and the free legs of each layer step
// form at most three runs contiguous in both its input and its output
static const std::vector<int> STORE_X1 = {N_a, N_tk, N_rk, N_tw, N_rw, N_tb, N_rb, N_j};
static const std::vector<int> STORE_X2 = {N_a, N_p, N_tw, N_rw, N_lk, N_dk, N_tb, N_rb, N_j};
static const std::vector<int> STORE_X3 = {N_a, N_q, N_lw, N_dw, N_lk, N_dk, N_tb, N_rb, N_j};
static const std::vector<int> STORE_X4 = {N_a, N_lw, N_dw, N_lk, N_dk, N_lb, N_db, N_j};

Status tensor_to_bt(const fpeps_tensor* t, const std::vector<int>& names, int nlab, BT& out,
                    bool flip_dirs) {
  if (!t) return fail(FPEPS_ERR_ARG, "null tensor");
  if (t->nlegs != (int)names.size())
    return fail(FPEPS_ERR_SHAPE, "tensor has " + std::to_string(t->nlegs) + " legs, expected " +
                                     std::to_string(names.size()));
  if (t->nlab != nlab) return fail(FPEPS_ERR_SHAPE, "label count differs from the symmetry's");
  if (!t->nsect || !t->dims || !t->labels || !t->dirs || (t->nblocks > 0 && (!t->block_sect || !t->block_off)))
    return fail(FPEPS_ERR_ARG, "null structure array");
  if (t->nblocks > 0 && !t->data) return fail(FPEPS_ERR_ARG, "null tensor data");
  out = BT();
  out.names = names;
  for (int l = 0; l < t->nlegs; ++l) {
    auto leg = std::make_shared<Leg>();
    leg->nlab = nlab;
    leg->dir = flip_dirs ? -t->dirs[l] : t->dirs[l];
    const int ns = t->nsect[l];
    if (ns <= 0 || ns > t->max_sect || ns > 65535)
      return fail(FPEPS_ERR_SHAPE, "bad sector count");
    for (int s = 0; s < ns; ++s) {
      for (int i = 0; i < nlab; ++i)
        leg->lab.push_back(t->labels[((int64_t)l * t->max_sect + s) * nlab + i]);
      const int d = t->dims[(int64_t)l * t->max_sect + s];
      if (d <= 0) return fail(FPEPS_ERR_SHAPE, "non-positive sector dimension");
      leg->dim.push_back(d);
    }
    out.cat.push_back(leg);
  }
  for (int b = 0; b < t->nblocks; ++b) {
    Block bk;
    for (int l = 0; l < t->nlegs; ++l) {
      const int s = t->block_sect[(int64_t)b * t->nlegs + l];
      if (s < 0 || s >= t->nsect[l]) return fail(FPEPS_ERR_SHAPE, "block sector out of range");
      bk.sect[l] = (uint16_t)s;
    }
    bk.base = t->block_off[b];
    set_rowmajor(out, bk);
    if (bk.base < 0 || bk.base + out.block_elems(bk) > t->nelem)
      return fail(FPEPS_ERR_SHAPE, "block outside the tensor data");
    out.blocks.push_back(bk);
  }
  out.size = t->nelem;
  return Status::ok();
}

Status SiteOp::init(const SymInfo& s, int nlab_, BT&& T_, BT&& ket_, BT&& W_, BT&& R_,
                    const SiteData& d) {
  sym = s;
  nlab = nlab_;
  T = std::move(T_);
  ket = std::move(ket_);
  W = std::move(W_);
  R = std::move(R_);
  dev = d;
  // the bra is the ket with reversed directions and its own leg names
  bra = ket;
  bra.names = {N_q, N_lb, N_rb, N_tb, N_db};
  for (auto& c : bra.cat) {
    auto l = std::make_shared<Leg>(*c);
    l->dir = -l->dir;
    c = l;
  }
  return Status::ok();
}

namespace {
std::vector<std::vector<int32_t>> col_labels(const SymInfo& sym, int nlab,
                                             const std::vector<const Leg*>& legs,
                                             const std::array<uint16_t, 4>& t) {
  std::vector<std::vector<int32_t>> out;
  if (sym.kind == SYM_NONE) {
    out.push_back(std::vector<int32_t>(nlab, 0));
  } else if (sym.kind == SYM_U1U1) {
    std::vector<int32_t> tot(nlab, 0);
    for (int i = 0; i < 4; ++i)
      for (int c = 0; c < nlab; ++c) tot[c] -= legs[i]->dir * legs[i]->label(t[i])[c];
    out.push_back(tot);
  } else {
    int s = 0, mx = 0;
    for (int i = 0; i < 4; ++i) {
      const int tj = legs[i]->label(t[i])[0];
      s += tj;
      mx = std::max(mx, tj);
    }
    for (int J = 0; J <= s; ++J) {
      const int tot = s + J;
      if (tot % 2 == 0 && 2 * std::max(mx, J) <= tot) out.push_back(std::vector<int32_t>{J});
    }
  }
  return out;
}

void sizes_by_sector(const BT& bt, int jpos, std::vector<int64_t>& acc) {
  for (const Block& b : bt.blocks) acc[b.sect[jpos]] += bt.block_elems(b);
}
}  // namespace

Status SiteOp::analyse(FwdAnalysis* fwdc) {
  std::string tkw;
  if (fwdc) tkw = structure_key_tkw();
  const bool reuse = fwdc && !fwdc->key.empty() && fwdc->key == tkw;
  int ns = 0;
  std::vector<int32_t> k1;
  std::vector<SliceCol> all;
  std::string err;
  BT X4;
  if (reuse) {
    sect = fwdc->sect;
    ns = (int)sect.size();
    unit_size.assign(ns, std::vector<int64_t>(8, 0));
    for (int J = 0; J < ns; ++J)
      for (int s = 0; s < 4; ++s) unit_size[J][s] = fwdc->unit[J][s];
    X4 = fwdc->x4;
    k1.assign(ns, 1);
    for (int J = 0; J < ns; ++J) all.push_back({J, 0, 1});
  } else {
    const int pb = T.pos(N_b), prk = ket.pos(N_rk), prw = W.pos(N_rw), prb = bra.pos(N_rb);
    std::vector<const Leg*> cl = {T.cat[pb].get(), ket.cat[prk].get(), W.cat[prw].get(),
                                  bra.cat[prb].get()};
    std::map<std::vector<int32_t>, Sector> by;
    std::array<uint16_t, 4> t{};
    for (t[0] = 0; t[0] < cl[0]->nsect(); ++t[0])
      for (t[1] = 0; t[1] < cl[1]->nsect(); ++t[1])
        for (t[2] = 0; t[2] < cl[2]->nsect(); ++t[2])
          for (t[3] = 0; t[3] < cl[3]->nsect(); ++t[3]) {
            int64_t d = 1;
            for (int i = 0; i < 4; ++i) d *= cl[i]->dim[t[i]];
            for (auto& J : col_labels(sym, nlab, cl, t)) {
              Sector& s = by[J];
              s.label = J;
              s.cols.push_back(t);
              s.crow.push_back(s.n);
              s.cdim.push_back(d);
              s.n += d;
            }
          }
    sect.clear();
    for (auto& kv : by) sect.push_back(std::move(kv.second));
    ns = (int)sect.size();
    if (ns == 0) return fail(FPEPS_ERR_SHAPE, "empty column space");

    // structure-only pass with one column per sector: the rows of Y_J and
    // the size of every intermediate per unit of width
    k1.assign(ns, 1);
    std::vector<int64_t> off(ns);
    int64_t tot = 0;
    for (int J = 0; J < ns; ++J) {
      off[J] = tot;
      tot += sect[J].n;
    }
    for (int J = 0; J < ns; ++J) all.push_back({J, 0, 1});
    BT X = omega_layout(all, k1, off, tot, false);
    TablePool dummy;
    const std::vector<int>* store[4] = {&STORE_X1, &STORE_X2, &STORE_X3, &STORE_X4};
    const BT* S[4] = {&T, &ket, &W, &bra};
    const bool mx[4] = {false, true, true, true};
    unit_size.assign(ns, std::vector<int64_t>(8, 0));
    for (int s = 0; s < 4; ++s) {
      StepSpec sp;
      sp.step = s + 1;
      sp.m_is_x = mx[s];
      sp.key_side = 0;
      sp.out_names = *store[s];
      sp.key_order = ORDER_X[s];
      sp.symbolic = true;
      StepResult r;
      if (!plan_step(X, *S[s], sp, sym, dummy, nullptr, r, err))
        return fail(FPEPS_ERR_SHAPE, "chain step " + std::to_string(s + 1) + ": " + err);
      X = std::move(r.out);
      std::vector<int64_t> acc(ns, 0);
      sizes_by_sector(X, X.pos(N_j), acc);
      for (int J = 0; J < ns; ++J) unit_size[J][s] = acc[J];
    }
    X4 = std::move(X);
    if (fwdc) {
      fwdc->key = std::move(tkw);
      fwdc->sect = sect;
      fwdc->unit.assign(ns, std::vector<int64_t>(4, 0));
      for (int J = 0; J < ns; ++J)
        for (int s = 0; s < 4; ++s) fwdc->unit[J][s] = unit_size[J][s];
      fwdc->x4 = X4;
    }
  }
  // the last forward step (the remainder) fixes the rows of every sector
  TablePool dummy;
  BT Y;
  {
    StepSpec sp;
    sp.step = 5;
    sp.m_is_x = false;
    sp.key_side = 0;
    sp.out_names = ORDER_X[5];
    sp.key_order = ORDER_X[4];
    sp.symbolic = true;
    StepResult r;
    if (!plan_step(X4, R, sp, sym, dummy, nullptr, r, err))
      return fail(FPEPS_ERR_SHAPE, "chain step 5: " + err);
    Y = std::move(r.out);
  }
  const BT* S[5] = {&T, &ket, &W, &bra, &R};
  // rows of every sector, lexicographic in (c, dk, dw, db)
  for (const Block& b : Y.blocks) {
    std::array<uint16_t, 4> r = {b.sect[0], b.sect[1], b.sect[2], b.sect[3]};
    sect[b.sect[4]].rows.push_back(r);
  }
  for (auto& s : sect) {
    std::sort(s.rows.begin(), s.rows.end());
    s.m = 0;
    for (auto& r : s.rows) {
      int64_t d = R.cat[R.pos(N_c)]->dim[r[0]] * (int64_t)ket.cat[ket.pos(N_dk)]->dim[r[1]] *
                  W.cat[W.pos(N_dw)]->dim[r[2]] * bra.cat[bra.pos(N_db)]->dim[r[3]];
      s.rrow.push_back(s.m);
      s.rdim.push_back(d);
      s.m += d;
    }
  }
  // backward structure from the row layout
  int64_t rtot = 0;
  std::vector<int64_t> roff(ns);
  for (int J = 0; J < ns; ++J) {
    roff[J] = rtot;
    rtot += sect[J].m;
  }
  BT Z = omega_layout(all, k1, roff, rtot, true);
  const std::vector<int>* bstore[5] = {&STORE_X4, &STORE_X3, &STORE_X2, &STORE_X1, &ORDER_X[0]};
  const bool bmx[5] = {false, true, true, true, false};
  const int bstep[5] = {5, 4, 3, 2, 1};
  for (int s = 0; s < 4; ++s) {
    StepSpec sp;
    sp.step = bstep[s];
    sp.m_is_x = bmx[s];
    sp.key_side = 1;
    sp.out_names = *bstore[s];
    sp.key_order = ORDER_X[bstep[s] - 1];
    sp.symbolic = true;
    StepResult r;
    if (!plan_step(Z, *S[bstep[s] - 1], sp, sym, dummy, nullptr, r, err))
      return fail(FPEPS_ERR_SHAPE, "transposed chain step " + std::to_string(bstep[s]) + ": " + err);
    Z = std::move(r.out);
    std::vector<int64_t> acc(ns, 0);
    sizes_by_sector(Z, Z.pos(N_j), acc);
    for (int J = 0; J < ns; ++J) unit_size[J][4 + s] = acc[J];
  }
  return Status::ok();
}

BT SiteOp::omega_layout(const std::vector<SliceCol>& cols, const std::vector<int32_t>& k,
                        const std::vector<int64_t>& off, int64_t total, bool rows) const {
  BT bt;
  auto jl = std::make_shared<Leg>();
  jl->nlab = nlab;
  jl->dir = -1;
  for (auto& c : cols) {
    for (int32_t v : sect[c.sect].label) jl->lab.push_back(v);
    jl->dim.push_back(c.j1 - c.j0);
  }
  if (!rows) {
    bt.names = {N_b, N_rk, N_rw, N_rb, N_j};
    auto f = [](const LegP& l) {
      auto m = std::make_shared<Leg>(*l);
      m->dir = -m->dir;
      return LegP(m);
    };
    bt.cat = {f(T.cat[T.pos(N_b)]), f(ket.cat[ket.pos(N_rk)]), f(W.cat[W.pos(N_rw)]),
              f(bra.cat[bra.pos(N_rb)]), jl};
  } else {
    bt.names = {N_c, N_dk, N_dw, N_db, N_j};
    bt.cat = {R.cat[R.pos(N_c)], ket.cat[ket.pos(N_dk)], W.cat[W.pos(N_dw)],
              bra.cat[bra.pos(N_db)], jl};
  }
  for (int si = 0; si < (int)cols.size(); ++si) {
    const SliceCol& c = cols[si];
    const Sector& s = sect[c.sect];
    const auto& tup = rows ? s.rows : s.cols;
    const auto& r0 = rows ? s.rrow : s.crow;
    const int64_t kj = k[c.sect];
    for (size_t t = 0; t < tup.size(); ++t) {
      Block b;
      for (int i = 0; i < 4; ++i) b.sect[i] = tup[t][i];
      b.sect[4] = (uint16_t)si;
      b.base = off[c.sect] + r0[t] * kj + c.j0;
      int64_t st = kj;
      b.stride[4] = 1;
      for (int i = 3; i >= 0; --i) {
        b.stride[i] = st;
        st *= bt.cat[i]->dim[tup[t][i]];
      }
      bt.blocks.push_back(b);
    }
  }
  bt.size = total;
  return bt;
}

Status SiteOp::plan(fpeps_ctx_s* ctx, const std::vector<int32_t>& k, int64_t budget, Plans& out,
                    bool with_bwd, bool f32) {
  FP_TRY(plan_host(k, budget, out, with_bwd, f32));
  return upload(ctx, out);
}

namespace {
void key_put(std::string& s, const void* p, size_t n) { s.append((const char*)p, n); }
void key_bt(std::string& s, const BT& bt) {
  const int64_t nn = (int64_t)bt.names.size(), nb = (int64_t)bt.blocks.size();
  key_put(s, &nn, sizeof nn);
  key_put(s, bt.names.data(), bt.names.size() * sizeof(int));
  for (const LegP& l : bt.cat) {
    const int64_t h[3] = {l->nlab, l->dir, (int64_t)l->dim.size()};
    key_put(s, h, sizeof h);
    key_put(s, l->lab.data(), l->lab.size() * sizeof(int32_t));
    key_put(s, l->dim.data(), l->dim.size() * sizeof(int32_t));
  }
  key_put(s, &nb, sizeof nb);
  for (const Block& b : bt.blocks) {
    key_put(s, b.sect.data(), nn * sizeof(uint16_t));
    key_put(s, &b.base, sizeof b.base);
    key_put(s, b.stride.data(), nn * sizeof(int64_t));
  }
  key_put(s, &bt.size, sizeof bt.size);
}
}  // namespace

std::string SiteOp::structure_key_tkw() const {
  std::string s;
  const int64_t h[4] = {sym.kind, sym.fermionic ? 1 : 0, (int64_t)sym.coef_seed, nlab};
  key_put(s, h, sizeof h);
  for (const BT* b : {&T, &ket, &W}) key_bt(s, *b);
  return s;
}

std::string SiteOp::structure_key() const {
  std::string s;
  const int64_t h[4] = {sym.kind, sym.fermionic ? 1 : 0, (int64_t)sym.coef_seed, nlab};
  key_put(s, h, sizeof h);
  for (const BT* b : {&T, &ket, &W, &bra, &R}) key_bt(s, *b);
  return s;
}

Status SiteOp::plan_host(const std::vector<int32_t>& k, int64_t budget, Plans& out,
                         bool with_bwd, bool f32) const {
  const int ns = (int)sect.size();
  if ((int)k.size() != ns) return fail(FPEPS_ERR_ARG, "width list does not match the sectors");
  out = Plans();
  out.f32 = f32;
  out.col_off.resize(ns);
  out.row_off.resize(ns);
  for (int J = 0; J < ns; ++J) {
    out.col_off[J] = out.col_total;
    out.row_off[J] = out.row_total;
    out.col_total += sect[J].n * (int64_t)k[J];
    out.row_total += sect[J].m * (int64_t)k[J];
  }
  // slices: whole sectors packed greedily; a sector larger than the budget
  // is split into column ranges. The budget counts FP64 elements also when
  // the intermediates are stored in FP32: a mixed-precision site applies the
  // same slices with FP64 intermediates too (its last range-finder product
  // and the projection).
  const double elem_budget = (double)budget / sizeof(double);
  // Slices are planned on host threads, one slice per thread: a site whose
  // whole chain fits the budget (many small sectors) is still packed into at
  // least MIN_SLICES slices of about equal work, so that its planning is
  // spread over the threads (results do not depend on the slicing).
  constexpr int MIN_SLICES = 16;
  double total_work = 0;
  for (int J = 0; J < ns; ++J) {
    if (k[J] <= 0 || sect[J].m == 0) continue;
    const auto& u = unit_size[J];
    total_work += ((double)std::max({u[0], u[2], u[5], u[7]}) +
                   (double)std::max({u[1], u[3], u[4], u[6]})) * k[J];
  }
  const double pack_cap = std::min(elem_budget, total_work / MIN_SLICES);
  std::vector<std::vector<SliceCol>> slices;
  std::vector<SliceCol> cur;
  double used = 0;
  for (int J = 0; J < ns; ++J) {
    if (k[J] <= 0 || sect[J].m == 0) continue;
    const auto& u = unit_size[J];
    const double per = (double)std::max({u[0], u[2], u[5], u[7]}) +
                       (double)std::max({u[1], u[3], u[4], u[6]});
    if (used + per * k[J] <= elem_budget && (cur.empty() || used + per * k[J] <= pack_cap)) {
      cur.push_back({J, 0, k[J]});
      used += per * k[J];
      continue;
    }
    if (!cur.empty()) {
      slices.push_back(cur);
      cur.clear();
      used = 0;
    }
    int w = per > 0 ? (int)std::max(1.0, std::floor(elem_budget / per)) : k[J];
    w = std::min(w, (int)k[J]);
    for (int j0 = 0; j0 < k[J]; j0 += w) {
      const int j1 = std::min((int)k[J], j0 + w);
      if (j1 - j0 == w && j1 < k[J]) {
        slices.push_back({{J, j0, j1}});
      } else {
        cur.push_back({J, j0, j1});
        used = per * (j1 - j0);
      }
    }
  }
  if (!cur.empty()) slices.push_back(cur);

  out.slices.resize(slices.size());
  for (size_t i = 0; i < slices.size(); ++i) out.slices[i].cols = slices[i];
  // slices are independent: plan them on host threads
  // tasks: the forward and the transposed chain of every slice
  const size_t ntask = slices.size() * (with_bwd ? 2 : 1);
  std::vector<Status> st(ntask);
  for (auto& sl : out.slices)
    for (int s = 0; s < 5; ++s) sl.bwd[s] = -1;
  {
    const unsigned hc = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>(ntask, std::min(16u, hc));
    auto work = [&](size_t t) {
      for (size_t i = t; i < ntask; i += nt)
        st[i] = plan_slice(k, out, out.slices[i % slices.size()], i >= slices.size());
    };
    std::vector<std::thread> th;
    for (size_t t = 1; t < nt; ++t) th.emplace_back(work, t);
    if (nt > 0) work(0);
    for (auto& x : th) x.join();
  }
  for (auto& e : st) FP_TRY(e);
  sum_plans(out);
  return Status::ok();
}

Status SiteOp::plan_bwd(const std::vector<int32_t>& k, Plans& out) const {
  const size_t ntask = out.slices.size();
  std::vector<Status> st(ntask);
  {
    const unsigned hc = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>(ntask, std::min(16u, hc));
    auto work = [&](size_t t) {
      for (size_t i = t; i < ntask; i += nt) st[i] = plan_slice(k, out, out.slices[i], true);
    };
    std::vector<std::thread> th;
    for (size_t t = 1; t < nt; ++t) th.emplace_back(work, t);
    if (nt > 0) work(0);
    for (auto& x : th) x.join();
  }
  for (auto& e : st) FP_TRY(e);
  return Status::ok();
}

void SiteOp::sum_plans(Plans& out) const {
  out.flops_fwd = out.flops_bwd = 0;
  out.ws1 = out.ws2 = 0;
  for (const Slice& sl : out.slices) {
    out.flops_fwd += sl.flops_fwd;
    out.flops_bwd += sl.flops_bwd;
    out.ws1 = std::max(out.ws1, std::max(sl.size1, sl.bsize1));
    out.ws2 = std::max(out.ws2, std::max(sl.size2, sl.bsize2));
  }
}

Status SiteOp::upload(fpeps_ctx_s* ctx, Plans& out, int which) const {
  // uploads through the pinned arena, asynchronous on the stream
  const auto up0 = std::chrono::steady_clock::now();
  FP_TRY(ctx->stage_begin());
  // one arena region per plan set, written on host threads, then one copy each
  std::vector<PlanSet*> sets;
  std::vector<std::string> tags;
  const bool up_f = (which & 1) != 0, up_b = (which & 2) != 0;
  for (size_t i = 0; i < out.slices.size(); ++i) {
    if (up_f) {
      sets.push_back(out.slices[i].ps.get());
      tags.push_back("site" + std::to_string(i) + "f");
    }
    if (up_b && out.slices[i].psb) {
      sets.push_back(out.slices[i].psb.get());
      tags.push_back("site" + std::to_string(i) + "b");
    }
  }
  std::vector<size_t> region(sets.size() + 1, 0);
  for (size_t i = 0; i < sets.size(); ++i) {
    if (!sets[i]->img.ready) FP_TRY(sets[i]->serialize());
    region[i + 1] = region[i] + (sets[i]->img.bytes + 255) / 256 * 256;
  }
  char* arena = nullptr;
  FP_TRY(ctx->stage_alloc(std::max<size_t>(region.back(), 1), &arena));
  {
    const unsigned hc = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>(sets.size(), std::min(16u, hc));
    auto work = [&](size_t t) {
      for (size_t i = t; i < sets.size(); i += nt) sets[i]->write_image(arena + region[i]);
    };
    std::vector<std::thread> th;
    for (size_t t = 1; t < nt; ++t) th.emplace_back(work, t);
    if (nt > 0) work(0);
    for (auto& x : th) x.join();
  }
  for (size_t i = 0; i < sets.size(); ++i) FP_TRY(sets[i]->bind(ctx, tags[i], arena + region[i]));
  for (size_t i = 0; i < out.slices.size(); ++i) {
    Slice& sl = out.slices[i];
    // layer sub-blocks scaled by the per-pair scalars (the bra shares the
    // ket's data)
    for (int s = 0; s < 5; ++s) {
      if (up_f && sl.fwd_rt[s]) {
        const bool w = s == 2;
        FP_TRY(sl.ps->pack(ctx, sl.fwd[s], w ? dev.W : dev.A, w ? dev.W_size : dev.A_size));
      }
      if (up_b && sl.psb && sl.bwd[s] >= 0 && sl.bwd_rt[s]) {
        const bool w = s == 2;   // bwd order: T5, T4, T3, T2, T1
        FP_TRY(sl.psb->pack(ctx, sl.bwd[s], w ? dev.W : dev.A, w ? dev.W_size : dev.A_size));
      }
    }
  }
  ctx->plan_up_bytes = (double)ctx->stage_used;
  ctx->stage_end();
  ctx->plan_up_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - up0).count();
  ctx->peak_ws = std::max(ctx->peak_ws,
                          (double)(out.ws1 + out.ws2) * sizeof(double));
  ctx->nslices = std::max(ctx->nslices, (int)out.slices.size());
  return Status::ok();
}

Status SiteOp::plan_slice(const std::vector<int32_t>& k, const Plans& pl, Slice& sl,
                          bool bwd) const {
  std::shared_ptr<PlanSet> own = std::make_shared<PlanSet>();
  if (bwd)
    sl.psb = own;
  else
    sl.ps = own;
  PlanSet& ps = *own;
  const std::vector<SliceCol>& sc = sl.cols;
  std::string err;
  const std::vector<int>* store[5] = {&STORE_X1, &STORE_X2, &STORE_X3, &STORE_X4, &ORDER_X[5]};
  const BT* S[5] = {&T, &ket, &W, &bra, &R};
  const bool mx[5] = {false, true, true, true, false};
  const std::vector<int>* bstore[5] = {&STORE_X4, &STORE_X3, &STORE_X2, &STORE_X1, &ORDER_X[0]};
  const int bstep[5] = {5, 4, 3, 2, 1};
  BT colL = omega_layout(sc, k, pl.col_off, pl.col_total, false);
  BT rowL = omega_layout(sc, k, pl.row_off, pl.row_total, true);
  BT X = colL;
  for (int s = 0; s < 5 && !bwd; ++s) {
    StepSpec sp;
    sp.step = s + 1;
    sp.m_is_x = mx[s];
    sp.key_side = 0;
    sp.out_names = *store[s];
    sp.key_order = ORDER_X[s];
    StepResult r;
    const bool layer = s >= 1 && s <= 3;
    if (layer) {
      RtPlan rp;
      if (!plan_step_rt(X, *S[s], sp, sym, ps.pool, r, rp, err))
        return fail(FPEPS_ERR_SHAPE, "chain step " + std::to_string(s + 1) + ": " + err);
      sl.flops_fwd += rp.flops;
      sl.fwd[s] = ps.add_rt(std::move(rp));
    } else {
      if (!plan_step(X, *S[s], sp, sym, ps.pool, s == 4 ? &rowL : nullptr, r, err))
        return fail(FPEPS_ERR_SHAPE, "chain step " + std::to_string(s + 1) + ": " + err);
      sl.flops_fwd += r.plan.flops;
      sl.fwd[s] = ps.add(std::move(r.plan));
    }
    sl.fwd_rt[s] = layer;
    if (s < 4) {
      if (s % 2 == 0)
        sl.size1 = std::max(sl.size1, r.out.size);
      else
        sl.size2 = std::max(sl.size2, r.out.size);
    }
    X = std::move(r.out);
  }
  if (bwd) {
    BT Z = rowL;
    for (int s = 0; s < 5; ++s) {
      StepSpec sp;
      sp.step = bstep[s];
      sp.m_is_x = mx[bstep[s] - 1];
      sp.key_side = 1;
      sp.out_names = *bstore[s];
      sp.key_order = ORDER_X[bstep[s] - 1];
      // M^T is the transpose of M on M's domain: the column tuples of each
      // sector (synthetic SU(2) scalars can reach others, which are dropped)
      sp.restrict_to_fixed = true;
      StepResult r;
      const bool layer = s >= 1 && s <= 3;
      if (layer) {
        RtPlan rp;
        if (!plan_step_rt(Z, *S[bstep[s] - 1], sp, sym, ps.pool, r, rp, err))
          return fail(FPEPS_ERR_SHAPE,
                      "transposed chain step " + std::to_string(bstep[s]) + ": " + err);
        sl.flops_bwd += rp.flops;
        sl.bwd[s] = ps.add_rt(std::move(rp));
      } else {
        if (!plan_step(Z, *S[bstep[s] - 1], sp, sym, ps.pool, s == 4 ? &colL : nullptr, r,
                       err))
          return fail(FPEPS_ERR_SHAPE,
                      "transposed chain step " + std::to_string(bstep[s]) + ": " + err);
        sl.flops_bwd += r.plan.flops;
        sl.bwd[s] = ps.add(std::move(r.plan));
      }
      sl.bwd_rt[s] = layer;
      // its own fields: the forward chain of this slice is planned on
      // another thread at the same time
      if (s < 4) {
        if (s % 2 == 0)
          sl.bsize2 = std::max(sl.bsize2, r.out.size);
        else
          sl.bsize1 = std::max(sl.bsize1, r.out.size);
      }
      Z = std::move(r.out);
    }
  }
  // the device image of this slice's plans, built here on the planning thread
  return own->serialize();
}

Status SiteOp::make_f32_operands(fpeps_ctx_s* ctx) {
  float *t = nullptr, *r = nullptr;
  FP_TRY(ctx->bufT("T32", (size_t)std::max<int64_t>(dev.T_size, 1), &t));
  FP_TRY(ctx->bufT("R32", (size_t)std::max<int64_t>(dev.R_size, 1), &r));
  FP_HIP(launch_to_f32(t, dev.T, dev.T_size, ctx->stream));
  FP_HIP(launch_to_f32(r, dev.R, dev.R_size, ctx->stream));
  dev.T32 = t;
  dev.R32 = r;
  return Status::ok();
}

Status SiteOp::apply(fpeps_ctx_s* ctx, const Plans& pl, bool transpose, const double* x, double* y,
                     bool f32) {
  if (f32 && (!dev.T32 || !dev.R32))
    return fail(FPEPS_ERR_ARG, "mixed-precision chain without FP32 operand copies");
  const size_t es = f32 ? sizeof(float) : sizeof(double);
  const int64_t s1 = std::max<int64_t>(pl.ws1, 1), s2 = std::max<int64_t>(pl.ws2, 1);
  // Slices are independent (disjoint sketch columns, disjoint outputs): they
  // are spread round-robin over the context's stream and up to
  // max_streams - 1 more, each with its own ping-pong intermediates, so the
  // GEMM steps of one slice can run beside the layer steps of the others.
  const int nst = ctx->multi_stream ? (int)std::min<size_t>(pl.slices.size(),
                                                           (size_t)std::max(1, ctx->max_streams))
                                   : 1;
  std::vector<std::array<void*, 2>> b((size_t)nst, std::array<void*, 2>{nullptr, nullptr});
  hipStream_t s0 = ctx->stream;
  std::vector<hipStream_t> sq(1, s0);
  if (nst > 1) {
    FP_TRY(ctx->ensure_streams(nst));
    for (int q = 1; q < nst; ++q) sq.push_back(ctx->xstreams[q - 1]);
  }
  for (int q = 0; q < nst; ++q) {
    const std::string sfx = q ? "_s" + std::to_string(q + 1) : std::string();
    FP_TRY(ctx->buf("chain1" + sfx, (size_t)s1 * es + 256, &b[q][0]));
    FP_TRY(ctx->buf("chain2" + sfx, (size_t)s2 * es + 256, &b[q][1]));
  }
  if (nst > 1) {
    // the other streams start after everything queued so far (x is ready)
    FP_HIP(hipEventRecord(ctx->ev_fork, s0));
    for (int q = 1; q < nst; ++q) FP_HIP(hipStreamWaitEvent(sq[q], ctx->ev_fork, 0));
  }
  ctx->peak_ws = std::max(ctx->peak_ws, (double)(s1 + s2) * (double)es * (double)nst);
  const bool f = f32;
  auto run_slice = [&](const Slice& sl, void* c1, void* c2) -> Status {
    // in mixed precision the FP64 masters T, R are replaced by their FP32
    // copies (FP32 MFMA); otherwise A32 is null and the FP64 kernel runs
    const double* T64 = f ? nullptr : dev.T;
    const double* R64 = f ? nullptr : dev.R;
    const float* T32 = f ? dev.T32 : nullptr;
    const float* R32 = f ? dev.R32 : nullptr;
    if (!transpose) {
      const PlanSet& ps = *sl.ps;
      FP_TRY(run_gemm_any(ctx, ps, sl.fwd[0], T64, T32, dev.T_size, x, false, pl.col_total, c1, f,
                          s1, true, 1));
      FP_TRY(run_rt(ctx, ps, sl.fwd[1], c1, s1, c2, s2, f, true, 2));
      FP_TRY(run_rt(ctx, ps, sl.fwd[2], c2, s2, c1, s1, f, true, 3));
      FP_TRY(run_rt(ctx, ps, sl.fwd[3], c1, s1, c2, s2, f, true, 4));
      FP_TRY(run_gemm_any(ctx, ps, sl.fwd[4], R64, R32, dev.R_size, c2, f, s2, y, false,
                          pl.row_total, true, 5));
    } else {
      if (sl.bwd[0] < 0 || !sl.psb) return fail(FPEPS_ERR_ARG, "transposed chain was not planned");
      const PlanSet& psb = *sl.psb;
      FP_TRY(run_gemm_any(ctx, psb, sl.bwd[0], R64, R32, dev.R_size, x, false, pl.row_total, c2, f,
                          s2, true, 15));
      FP_TRY(run_rt(ctx, psb, sl.bwd[1], c2, s2, c1, s1, f, true, 14));
      FP_TRY(run_rt(ctx, psb, sl.bwd[2], c1, s1, c2, s2, f, true, 13));
      FP_TRY(run_rt(ctx, psb, sl.bwd[3], c2, s2, c1, s1, f, true, 12));
      FP_TRY(run_gemm_any(ctx, psb, sl.bwd[4], T64, T32, dev.T_size, c1, f, s1, y, false,
                          pl.col_total, true, 11));
    }
    return Status::ok();
  };
  Status st = Status::ok();
  for (size_t i = 0; i < pl.slices.size() && st.good(); ++i) {
    const int q = (int)(i % (size_t)nst);
    ctx->stream = sq[q];
    st = run_slice(pl.slices[i], b[q][0], b[q][1]);
  }
  ctx->stream = s0;
  // the context's stream continues after all of them
  for (int q = 1; q < nst; ++q) {
    FP_HIP(hipEventRecord(ctx->xjoin[q - 1], sq[q]));
    FP_HIP(hipStreamWaitEvent(s0, ctx->xjoin[q - 1], 0));
  }
  return st;
}

}  // namespace fp
