// Host planner of the block-sparse contraction chain (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <climits>
#include <cstring>
#include <map>
#include <numeric>

namespace fp {

void set_rowmajor(const BT& bt, Block& b) {
  int64_t s = 1;
  for (int p = bt.nlegs() - 1; p >= 0; --p) {
    b.stride[p] = s;
    s *= bt.dim(b, p);
  }
}

uint64_t splitmix64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline int label_parity(int kind, const int32_t* lab) {
  if (kind == SYM_U1U1) return lab[1] & 1;
  if (kind == SYM_SU2) return lab[0] & 1;
  return 0;
}

double pair_alpha(const SymInfo& sym, int step, const std::vector<const int32_t*>& xlabs,
                  const std::vector<const int32_t*>& tlabs, const std::vector<bool>& xshared,
                  const std::vector<bool>& tshared, int nlab) {
  double a = 1.0;
  if (sym.kind == SYM_SU2) {
    const uint64_t golden = 0x9E3779B97F4A7C15ull;
    uint64_t h = sym.coef_seed;
    auto fold = [&](int64_t w) { h = splitmix64_mix(h + golden + (uint64_t)w); };
    fold(step);
    for (auto* l : xlabs)
      for (int i = 0; i < nlab; ++i) fold(l[i]);
    for (auto* l : tlabs)
      for (int i = 0; i < nlab; ++i) fold(l[i]);
    a = 2.0 * ((double)(h >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  }
  if (sym.fermionic) {
    int px = 0, pt = 0;
    for (size_t i = 0; i < xlabs.size(); ++i)
      if (!xshared[i]) px += label_parity(sym.kind, xlabs[i]);
    for (size_t i = 0; i < tlabs.size(); ++i)
      if (tshared[i]) pt += label_parity(sym.kind, tlabs[i]);
    if ((px * pt) & 1) a = -a;
  }
  return a;
}

int32_t TablePool::add(const std::vector<int32_t>& dims, const std::vector<int64_t>& strides,
                       bool* ok) {
  std::string key;
  key.resize(dims.size() * 12);
  char* w = key.data();
  for (size_t i = 0; i < dims.size(); ++i) {
    std::memcpy(w, &dims[i], 4);
    std::memcpy(w + 4, &strides[i], 8);
    w += 12;
  }
  auto it = index.find(key);
  if (it != index.end()) return it->second;
  int64_t n = 1;
  for (int d : dims) n *= d;
  if ((int64_t)data.size() + n > (int64_t)INT32_MAX) {
    *ok = false;
    return 0;
  }
  int32_t id = (int32_t)data.size();
  data.resize(data.size() + (size_t)n);
  // enumerate the fused index row-major over ``dims``
  std::vector<int32_t> idx(dims.size(), 0);
  int64_t off = 0;
  for (int64_t e = 0; e < n; ++e) {
    if (off > INT32_MAX || off < 0) {
      *ok = false;
      return 0;
    }
    data[(size_t)id + (size_t)e] = (int32_t)off;
    for (int d = (int)dims.size() - 1; d >= 0; --d) {
      if (++idx[d] < dims[d]) {
        off += strides[d];
        break;
      }
      off -= strides[d] * (int64_t)(dims[d] - 1);
      idx[d] = 0;
    }
  }
  index.emplace(std::move(key), id);
  return id;
}

namespace {

struct SectKey {
  std::array<uint16_t, MAXL> v{};
  uint8_t n = 0;
  bool operator==(const SectKey& o) const {
    return n == o.n && std::memcmp(v.data(), o.v.data(), n * sizeof(uint16_t)) == 0;
  }
  bool operator<(const SectKey& o) const {
    for (int i = 0; i < n && i < o.n; ++i)
      if (v[i] != o.v[i]) return v[i] < o.v[i];
    return n < o.n;
  }
};
struct SectKeyHash {
  size_t operator()(const SectKey& k) const {
    uint64_t h = 1469598103934665603ull;
    for (int i = 0; i < k.n; ++i) h = (h ^ k.v[i]) * 1099511628211ull;
    return (size_t)h;
  }
};

struct TabRef {
  int32_t id;
  int64_t maxoff;
};

TabRef make_table(TablePool& pool, const BT& bt, const Block& b, const std::vector<int>& pos,
                  bool* ok) {
  std::vector<int32_t> dims;
  std::vector<int64_t> strides;
  int64_t mx = 0;
  for (int p : pos) {
    int d = bt.dim(b, p);
    dims.push_back(d);
    strides.push_back(b.stride[p]);
    mx += (int64_t)(d - 1) * b.stride[p];
  }
  if (pos.empty()) {
    dims.push_back(1);
    strides.push_back(0);
  }
  return {pool.add(dims, strides, ok), mx};
}

int64_t prod_dims(const BT& bt, const Block& b, const std::vector<int>& pos) {
  int64_t n = 1;
  for (int p : pos) n *= bt.dim(b, p);
  return n;
}

}  // namespace

void choose_tile(const std::vector<std::pair<int64_t, int64_t>>& mn, int* mt, int* nt) {
  static const int cand[][2] = {{64, 64}, {128, 32}, {32, 128}, {256, 16}, {16, 256}};
  double best = -1;
  int bi = 0;
  for (int c = 0; c < 5; ++c) {
    double padded = 0, useful = 0;
    for (auto& p : mn) {
      int64_t M = p.first, N = p.second;
      padded += (double)((M + cand[c][0] - 1) / cand[c][0] * cand[c][0]) *
                (double)((N + cand[c][1] - 1) / cand[c][1] * cand[c][1]);
      useful += (double)M * (double)N;
    }
    double eff = padded > 0 ? useful / padded : 1.0;
    // prefer the square tile unless another is clearly better
    if (c == 0) eff *= 1.15;
    if (eff > best) {
      best = eff;
      bi = c;
    }
  }
  *mt = cand[bi][0];
  *nt = cand[bi][1];
}

bool plan_step(const BT& X, const BT& S, const StepSpec& spec, const SymInfo& sym,
               TablePool& pool, const BT* fixed_out, StepResult& res, std::string& err) {
  // shared legs in X order
  std::vector<int> xs, ss, xfree, sfree;
  for (int p = 0; p < X.nlegs(); ++p) {
    int q = S.pos(X.names[p]);
    if (q >= 0) {
      xs.push_back(p);
      ss.push_back(q);
    } else {
      xfree.push_back(p);
    }
  }
  for (int q = 0; q < S.nlegs(); ++q)
    if (X.pos(S.names[q]) < 0) sfree.push_back(q);
  for (size_t i = 0; i < xs.size(); ++i) {
    if (!X.cat[xs[i]]->same_sectors(*S.cat[ss[i]])) {
      err = "contracted legs carry different sectors";
      return false;
    }
  }
  // output leg sources
  const int no = (int)spec.out_names.size();
  if (no != (int)(xfree.size() + sfree.size())) {
    err = "output leg count mismatch";
    return false;
  }
  std::vector<int> src_side(no), src_pos(no);
  for (int o = 0; o < no; ++o) {
    int n = spec.out_names[o];
    int p = X.pos(n), q = S.pos(n);
    if (p >= 0 && q < 0) {
      src_side[o] = 0;
      src_pos[o] = p;
    } else if (q >= 0 && p < 0) {
      src_side[o] = 1;
      src_pos[o] = q;
    } else {
      err = "output leg is not a free leg";
      return false;
    }
  }
  BT& out = res.out;
  out = BT();
  out.names = spec.out_names;
  for (int o = 0; o < no; ++o) out.cat.push_back(src_side[o] ? S.cat[src_pos[o]] : X.cat[src_pos[o]]);

  // group S blocks by their contracted sectors
  std::unordered_map<SectKey, std::vector<int>, SectKeyHash> groups;
  groups.reserve(S.blocks.size() * 2 + 1);
  for (int sb = 0; sb < (int)S.blocks.size(); ++sb) {
    SectKey k;
    k.n = (uint8_t)ss.size();
    for (size_t i = 0; i < ss.size(); ++i) k.v[i] = S.blocks[sb].sect[ss[i]];
    groups[k].push_back(sb);
  }
  // enumerate pairs
  std::unordered_map<SectKey, int, SectKeyHash> out_index;
  std::vector<SectKey> out_keys;
  if (fixed_out) {
    if (fixed_out->names != spec.out_names) {
      err = "fixed output layout has a different leg order";
      return false;
    }
    out = *fixed_out;
    for (int ob = 0; ob < (int)out.blocks.size(); ++ob) {
      SectKey k;
      k.n = (uint8_t)no;
      for (int o = 0; o < no; ++o) k.v[o] = out.blocks[ob].sect[o];
      out_index.emplace(k, ob);
      out_keys.push_back(k);
    }
  }
  struct P3 {
    int xb, sb, ob;
  };
  std::vector<P3> trip;
  for (int xb = 0; xb < (int)X.blocks.size(); ++xb) {
    SectKey k;
    k.n = (uint8_t)xs.size();
    for (size_t i = 0; i < xs.size(); ++i) k.v[i] = X.blocks[xb].sect[xs[i]];
    auto g = groups.find(k);
    if (g == groups.end()) continue;
    for (int sb : g->second) {
      SectKey ok;
      ok.n = (uint8_t)no;
      for (int o = 0; o < no; ++o)
        ok.v[o] = src_side[o] ? S.blocks[sb].sect[src_pos[o]] : X.blocks[xb].sect[src_pos[o]];
      auto it = out_index.find(ok);
      int ob;
      if (it == out_index.end()) {
        if (fixed_out) {
          if (spec.restrict_to_fixed) continue;
          err = "a block pair produces a block outside the fixed output layout";
          return false;
        }
        ob = (int)out_keys.size();
        out_index.emplace(ok, ob);
        out_keys.push_back(ok);
      } else {
        ob = it->second;
      }
      trip.push_back({xb, sb, ob});
    }
  }
  // assign output blocks (sorted by sector tuple) when not fixed
  std::vector<int> remap(out_keys.size());
  if (!fixed_out) {
    std::vector<int> order(out_keys.size());
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return out_keys[a] < out_keys[b]; });
    out.blocks.resize(order.size());
    int64_t off = 0;
    for (size_t i = 0; i < order.size(); ++i) {
      remap[order[i]] = (int)i;
      Block& b = out.blocks[i];
      for (int o = 0; o < no; ++o) b.sect[o] = out_keys[order[i]].v[o];
      b.base = off;
      set_rowmajor(out, b);
      off += out.block_elems(b);
    }
    out.size = off;
  } else {
    std::iota(remap.begin(), remap.end(), 0);
  }
  for (auto& t : trip) t.ob = remap[t.ob];
  if (spec.symbolic) return true;
  std::stable_sort(trip.begin(), trip.end(), [](const P3& a, const P3& b) { return a.ob < b.ob; });

  // operand roles
  const BT& A = spec.m_is_x ? X : S;
  const BT& B = spec.m_is_x ? S : X;
  const std::vector<int>& afree = spec.m_is_x ? xfree : sfree;
  const std::vector<int>& bfree = spec.m_is_x ? sfree : xfree;
  const std::vector<int>& ak = spec.m_is_x ? xs : ss;
  const std::vector<int>& bk = spec.m_is_x ? ss : xs;
  // positions in the output of the M and N legs
  std::vector<int> cm, cn;
  for (int p : afree) cm.push_back(out.pos(A.names[p]));
  for (int p : bfree) cn.push_back(out.pos(B.names[p]));

  // key tensor for alpha
  const BT& KT = spec.key_side == 0 ? X : out;
  std::vector<int> kpos;
  std::vector<bool> kshared;
  for (int n : spec.key_order) {
    int p = KT.pos(n);
    if (p < 0) {
      err = "key order names a leg the keyed tensor lacks";
      return false;
    }
    kpos.push_back(p);
    kshared.push_back(S.pos(n) >= 0);
  }
  std::vector<bool> sshared(S.nlegs());
  for (int q = 0; q < S.nlegs(); ++q) sshared[q] = KT.pos(S.names[q]) >= 0;
  const int nlab = S.cat.empty() ? 1 : S.cat[0]->nlab;

  // tables and pairs
  GemmPlan& plan = res.plan;
  plan = GemmPlan();
  std::vector<std::pair<int64_t, int64_t>> mn;
  mn.reserve(out.blocks.size());
  for (auto& b : out.blocks) mn.emplace_back(prod_dims(out, b, cm), prod_dims(out, b, cn));
  choose_tile(mn, &plan.mt, &plan.nt);
  bool ok = true;
  std::vector<int> pstart(out.blocks.size() + 1, 0);
  {
    size_t t = 0;
    for (size_t ob = 0; ob < out.blocks.size(); ++ob) {
      pstart[ob] = (int)t;
      while (t < trip.size() && trip[t].ob == (int)ob) ++t;
    }
    pstart[out.blocks.size()] = (int)trip.size();
  }
  plan.pairs.reserve(trip.size());
  std::vector<const int32_t*> xl(kpos.size()), tl(S.nlegs());
  for (auto& t : trip) {
    const Block& xbk = X.blocks[t.xb];
    const Block& sbk = S.blocks[t.sb];
    const Block& abk = spec.m_is_x ? xbk : sbk;
    const Block& bbk = spec.m_is_x ? sbk : xbk;
    TabRef tam = make_table(pool, A, abk, afree, &ok);
    TabRef tak = make_table(pool, A, abk, ak, &ok);
    TabRef tbk = make_table(pool, B, bbk, bk, &ok);
    TabRef tbn = make_table(pool, B, bbk, bfree, &ok);
    GemmPair gp;
    gp.a_off = abk.base;
    gp.b_off = bbk.base;
    gp.K = (int32_t)prod_dims(A, abk, ak);
    gp.tam = tam.id;
    gp.tak = tak.id;
    gp.tbk = tbk.id;
    gp.tbn = tbn.id;
    gp.flags = 0;
    if (!ak.empty() && abk.stride[ak.back()] == 1) gp.flags |= 1;
    if (!bfree.empty() && bbk.stride[bfree.back()] == 1) gp.flags |= 2;
    // alpha keyed by the sketch-side block
    const Block& kb = spec.key_side == 0 ? xbk : out.blocks[t.ob];
    for (size_t i = 0; i < kpos.size(); ++i) xl[i] = KT.cat[kpos[i]]->label(kb.sect[kpos[i]]);
    for (int q = 0; q < S.nlegs(); ++q) tl[q] = S.cat[q]->label(sbk.sect[q]);
    gp.alpha = pair_alpha(sym, spec.step, xl, tl, kshared, sshared, nlab);
    plan.a_extent = std::max(plan.a_extent, gp.a_off + tam.maxoff + tak.maxoff + 1);
    plan.b_extent = std::max(plan.b_extent, gp.b_off + tbk.maxoff + tbn.maxoff + 1);
    int64_t M = prod_dims(A, abk, afree), N = prod_dims(B, bbk, bfree);
    plan.flops += 2.0 * (double)M * (double)N * (double)gp.K;
    plan.pairs.push_back(gp);
  }
  // jobs: one per output tile
  for (size_t ob = 0; ob < out.blocks.size(); ++ob) {
    const Block& cb = out.blocks[ob];
    int64_t M = prod_dims(out, cb, cm), N = prod_dims(out, cb, cn);
    if (M > INT32_MAX || N > INT32_MAX) {
      err = "block too large";
      return false;
    }
    TabRef tcm = make_table(pool, out, cb, cm, &ok);
    TabRef tcn = make_table(pool, out, cb, cn, &ok);
    plan.c_extent = std::max(plan.c_extent, cb.base + tcm.maxoff + tcn.maxoff + 1);
    for (int64_t m0 = 0; m0 < M; m0 += plan.mt)
      for (int64_t n0 = 0; n0 < N; n0 += plan.nt) {
        GemmJob j;
        j.c_off = cb.base;
        j.M = (int32_t)M;
        j.N = (int32_t)N;
        j.m0 = (int32_t)m0;
        j.n0 = (int32_t)n0;
        j.tcm = tcm.id;
        j.tcn = tcn.id;
        j.p0 = pstart[ob];
        j.p1 = pstart[ob + 1];
        j.k0 = 0;
        j.k1 = INT32_MAX;
        plan.jobs.push_back(j);
      }
  }
  if (!ok) {
    err = "offset table overflow (block or pool exceeds 2^31 elements)";
    return false;
  }
  return true;
}

bool plan_dense(const std::vector<DenseOp>& ops, TablePool& pool, int mt, int nt, int ksplit,
                GemmPlan& plan, std::string& err) {
  plan = GemmPlan();
  plan.mt = mt;
  plan.nt = nt;
  bool ok = true;
  auto tab = [&](int32_t n, int64_t s) -> TabRef {
    std::vector<int32_t> d{std::max(n, 1)};
    std::vector<int64_t> st{s};
    return {pool.add(d, st, &ok), (int64_t)(std::max(n, 1) - 1) * s};
  };
  for (const DenseOp& op : ops) {
    if (op.M <= 0 || op.N <= 0) continue;
    TabRef tam = tab(op.M, op.a_rs), tak = tab(op.K, op.a_cs);
    TabRef tbk = tab(op.K, op.b_rs), tbn = tab(op.N, op.b_cs);
    GemmPair gp;
    gp.a_off = op.a_off;
    gp.b_off = op.b_off;
    gp.K = op.K;
    gp.tam = tam.id;
    gp.tak = tak.id;
    gp.tbk = tbk.id;
    gp.tbn = tbn.id;
    gp.flags = (op.a_cs == 1 ? 1 : 0) | (op.b_cs == 1 ? 2 : 0);
    gp.alpha = op.alpha;
    plan.a_extent = std::max(plan.a_extent, op.a_off + tam.maxoff + tak.maxoff + 1);
    plan.b_extent = std::max(plan.b_extent, op.b_off + tbk.maxoff + tbn.maxoff + 1);
    plan.flops += 2.0 * op.M * (double)op.N * (double)op.K;
    int pidx = (int)plan.pairs.size();
    plan.pairs.push_back(gp);
    const int ks = op.ksplit > 0 ? op.ksplit : ksplit;
    const int nchunk = ks > 1 ? ks : 1;
    int chunk = ks > 1 ? ((op.K + ks - 1) / ks + 15) / 16 * 16 : op.K;
    for (int c = 0; c < nchunk; ++c) {
      int k0 = std::min(op.K, c * chunk), k1 = std::min(op.K, (c + 1) * chunk);
      TabRef tcm, tcn;
      int64_t coff;
      if (ks > 1) {
        tcm = tab(op.M, op.N);
        tcn = tab(op.N, 1);
        coff = op.c_off + (int64_t)c * op.M * op.N;
      } else {
        tcm = tab(op.M, op.c_rs);
        tcn = tab(op.N, op.c_cs);
        coff = op.c_off;
      }
      plan.c_extent = std::max(plan.c_extent, coff + tcm.maxoff + tcn.maxoff + 1);
      for (int m0 = 0; m0 < op.M; m0 += mt)
        for (int n0 = 0; n0 < op.N; n0 += nt) {
          GemmJob j;
          j.c_off = coff;
          j.M = op.M;
          j.N = op.N;
          j.m0 = m0;
          j.n0 = n0;
          j.tcm = tcm.id;
          j.tcn = tcn.id;
          j.p0 = pidx;
          j.p1 = pidx + 1;
          j.k0 = ks > 1 ? k0 : 0;
          j.k1 = ks > 1 ? k1 : INT32_MAX;
          plan.jobs.push_back(j);
        }
    }
  }
  if (!ok) {
    err = "offset table overflow";
    return false;
  }
  return true;
}

}  // namespace fp
