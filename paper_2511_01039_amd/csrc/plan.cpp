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

// The scalar is split in two halves: the sketch-side half (the hash state
// after the step and the X labels, and the parity of X's free legs) depends
// only on the keyed block, so a plan computes it once per block.
struct AlphaHead {
  uint64_t h;
  int px;
};

static AlphaHead alpha_head(const SymInfo& sym, int step, const int32_t* const* xlabs, int nx,
                            const char* xshared, int nlab) {
  AlphaHead a{sym.coef_seed, 0};
  if (sym.kind == SYM_SU2) {
    a.h = splitmix64_mix(a.h + 0x9E3779B97F4A7C15ull + (uint64_t)(int64_t)step);
    for (int j = 0; j < nx; ++j)
      for (int i = 0; i < nlab; ++i)
        a.h = splitmix64_mix(a.h + 0x9E3779B97F4A7C15ull + (uint64_t)(int64_t)xlabs[j][i]);
  }
  if (sym.fermionic)
    for (int i = 0; i < nx; ++i)
      if (!xshared[i]) a.px += label_parity(sym.kind, xlabs[i]);
  return a;
}

static double alpha_tail(const SymInfo& sym, AlphaHead a, const int32_t* const* tlabs, int nt,
                         const char* tshared, int nlab) {
  double v = 1.0;
  if (sym.kind == SYM_SU2) {
    uint64_t h = a.h;
    for (int j = 0; j < nt; ++j)
      for (int i = 0; i < nlab; ++i)
        h = splitmix64_mix(h + 0x9E3779B97F4A7C15ull + (uint64_t)(int64_t)tlabs[j][i]);
    v = 2.0 * ((double)(h >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  }
  if (sym.fermionic) {
    int pt = 0;
    for (int i = 0; i < nt; ++i)
      if (tshared[i]) pt += label_parity(sym.kind, tlabs[i]);
    if ((a.px * pt) & 1) v = -v;
  }
  return v;
}

double pair_alpha(const SymInfo& sym, int step, const int32_t* const* xlabs, int nx,
                  const int32_t* const* tlabs, int nt, const char* xshared, const char* tshared,
                  int nlab) {
  return alpha_tail(sym, alpha_head(sym, step, xlabs, nx, xshared, nlab), tlabs, nt, tshared, nlab);
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

int32_t TablePool::add_raw(const std::vector<int32_t>& v, bool* ok) {
  std::string key(v.size() * 4 + 1, '\0');
  key[0] = 'r';
  std::memcpy(&key[1], v.data(), v.size() * 4);
  auto it = index.find(key);
  if (it != index.end()) return it->second;
  if ((int64_t)data.size() + (int64_t)v.size() > (int64_t)INT32_MAX) {
    *ok = false;
    return 0;
  }
  int32_t id = (int32_t)data.size();
  data.insert(data.end(), v.begin(), v.end());
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
  int32_t lin = 0;   // > 0: entry i is i * lin
};

// Stride s when the offsets of legs ``dims``/``strides`` (last fastest) are
// i * s for the row-major index i, else 0. Legs of dimension 1 do not count.
int32_t linear_stride(const std::vector<int32_t>& dims, const std::vector<int64_t>& strides) {
  int64_t s = 0, run = 0;
  for (int i = (int)dims.size() - 1; i >= 0; --i) {
    if (dims[i] <= 1) continue;
    if (run == 0) {
      s = strides[i];
      if (s <= 0) return 0;
      run = s * dims[i];
    } else {
      if (strides[i] != run) return 0;
      run *= dims[i];
    }
  }
  if (run == 0) return 1;   // every leg has dimension 1: one entry, 0
  return s <= INT32_MAX ? (int32_t)s : 0;
}

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
  TabRef t{pool.add(dims, strides, ok), mx};
  t.lin = linear_stride(dims, strides);
  return t;
}

TabRef make_table_dense(TablePool& pool, int32_t n, int64_t stride, bool* ok) {
  std::vector<int32_t> d{std::max(n, 1)};
  std::vector<int64_t> st{stride};
  TabRef t{pool.add(d, st, ok), (int64_t)(std::max(n, 1) - 1) * stride};
  t.lin = linear_stride(d, st);
  return t;
}

int64_t prod_dims(const BT& bt, const Block& b, const std::vector<int>& pos) {
  int64_t n = 1;
  for (int p : pos) n *= bt.dim(b, p);
  return n;
}

}  // namespace

namespace {
const int TILE_CAND[][2] = {{128, 128}, {128, 64}, {64, 128}, {64, 64},
                            {128, 32},  {32, 128}, {256, 16}, {16, 256}};
constexpr int NTILE = sizeof(TILE_CAND) / sizeof(TILE_CAND[0]);

// padding efficiency of every tile: useful / padded products, weighted by
// the contracted extent of each output block
void tile_efficiency(const std::vector<std::pair<int64_t, int64_t>>& mn,
                     const std::vector<int64_t>& ktot, double* eff, double* best) {
  *best = 0;
  for (int c = 0; c < NTILE; ++c) {
    double padded = 0, useful = 0;
    for (size_t i = 0; i < mn.size(); ++i) {
      const int64_t M = mn[i].first, N = mn[i].second;
      const double w = (double)std::max<int64_t>(ktot[i], 1);
      padded += w * (double)((M + TILE_CAND[c][0] - 1) / TILE_CAND[c][0] * TILE_CAND[c][0]) *
                (double)((N + TILE_CAND[c][1] - 1) / TILE_CAND[c][1] * TILE_CAND[c][1]);
      useful += w * (double)M * (double)N;
    }
    eff[c] = padded > 0 ? useful / padded : 1.0;
    *best = std::max(*best, eff[c]);
  }
}
}  // namespace

bool valid_tile(int mt, int nt) {
  for (int c = 0; c < NTILE; ++c)
    if (TILE_CAND[c][0] == mt && TILE_CAND[c][1] == nt) return true;
  return false;
}

void choose_tile(const std::vector<std::pair<int64_t, int64_t>>& mn,
                 const std::vector<int64_t>& ktot, int* mt, int* nt) {
  double eff[NTILE], best = 0;
  tile_efficiency(mn, ktot, eff, &best);
  // the largest tile (most reuse per loaded element) among those within 15%
  // of the best padding efficiency; candidates are ordered by preference
  for (int c = 0; c < NTILE; ++c)
    if (eff[c] >= 0.85 * best) {
      *mt = TILE_CAND[c][0];
      *nt = TILE_CAND[c][1];
      return;
    }
  *mt = 64;
  *nt = 64;
}

std::vector<std::array<int, 2>> tile_candidates(const std::vector<std::pair<int64_t, int64_t>>& mn,
                                                const std::vector<int64_t>& ktot, int max_n) {
  std::vector<std::array<int, 2>> out;
  int mt = 64, nt = 64;
  choose_tile(mn, ktot, &mt, &nt);
  out.push_back({mt, nt});
  double eff[NTILE], best = 0;
  tile_efficiency(mn, ktot, eff, &best);
  std::vector<int> order;
  for (int c = 0; c < NTILE; ++c)
    if (eff[c] >= 0.7 * best && !(TILE_CAND[c][0] == mt && TILE_CAND[c][1] == nt))
      order.push_back(c);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return eff[a] > eff[b]; });
  for (int c : order) {
    if ((int)out.size() >= max_n) break;
    out.push_back({TILE_CAND[c][0], TILE_CAND[c][1]});
  }
  return out;
}

namespace {

struct P3 {
  int xb, sb, ob;
};

// Pair enumeration shared by both plan forms: contracted/free legs, the
// output structure, and every (X block, S block, output block) triple,
// sorted by output block.
struct StepEnum {
  std::vector<int> xs, ss, xfree, sfree;
  std::vector<P3> trip;
  // per-pair scalar keys
  std::vector<int> kpos;
  std::vector<char> kshared, sshared;
  int nlab = 1;
  // sketch-side halves of the pair scalar, per keyed block (filled lazily)
  std::vector<AlphaHead> head;
  std::vector<char> head_set;
};

bool enumerate_step(const BT& X, const BT& S, const StepSpec& spec, const BT* fixed_out, BT& out,
                    StepEnum& E, std::string& err) {
  std::vector<int>&xs = E.xs, &ss = E.ss, &xfree = E.xfree, &sfree = E.sfree;
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
  std::vector<P3>& trip = E.trip;
  // Output sector tuples packed in mixed radix (first leg most significant)
  // when they fit 64 bits: numeric order is then the tuple order, and the X
  // and S parts of a key are computed once per block and OR-ed per pair.
  int shift[MAXL] = {0};
  int tbits = 0;
  for (int o = no - 1; o >= 0; --o) {
    int b = 0;
    while ((1ll << b) < (int64_t)out.cat[o]->nsect()) ++b;
    shift[o] = tbits;
    tbits += b;
  }
  std::vector<int> remap;
  if (!fixed_out && tbits <= 64) {
    std::vector<uint64_t> xpart(X.blocks.size(), 0), spart(S.blocks.size(), 0);
    for (int o = 0; o < no; ++o) {
      if (src_side[o])
        for (size_t b = 0; b < S.blocks.size(); ++b)
          spart[b] |= (uint64_t)S.blocks[b].sect[src_pos[o]] << shift[o];
      else
        for (size_t b = 0; b < X.blocks.size(); ++b)
          xpart[b] |= (uint64_t)X.blocks[b].sect[src_pos[o]] << shift[o];
    }
    // open-addressing index of the packed keys (value -1: empty slot)
    std::vector<uint64_t> hkey(1024);
    std::vector<int32_t> hval(1024, -1);
    uint64_t hmask = 1023;
    std::vector<uint64_t> keys;
    auto hslot = [&](uint64_t k) {
      uint64_t h = k * 0x9E3779B97F4A7C15ull;
      uint64_t i = (h ^ (h >> 29)) & hmask;
      while (hval[i] >= 0 && hkey[i] != k) i = (i + 1) & hmask;
      return i;
    };
    for (int xb = 0; xb < (int)X.blocks.size(); ++xb) {
      SectKey k;
      k.n = (uint8_t)xs.size();
      for (size_t i = 0; i < xs.size(); ++i) k.v[i] = X.blocks[xb].sect[xs[i]];
      auto g = groups.find(k);
      if (g == groups.end()) continue;
      for (int sb : g->second) {
        const uint64_t key = xpart[xb] | spart[sb];
        uint64_t i = hslot(key);
        if (hval[i] < 0) {
          if (2 * (keys.size() + 1) > hkey.size()) {
            std::vector<uint64_t> ok2(hkey.size() * 2);
            std::vector<int32_t> ov2(hkey.size() * 2, -1);
            hkey.swap(ok2);
            hval.swap(ov2);
            hmask = hkey.size() - 1;
            for (size_t j = 0; j < ok2.size(); ++j)
              if (ov2[j] >= 0) {
                const uint64_t q = hslot(ok2[j]);
                hkey[q] = ok2[j];
                hval[q] = ov2[j];
              }
            i = hslot(key);
          }
          hkey[i] = key;
          hval[i] = (int32_t)keys.size();
          keys.push_back(key);
        }
        if (!spec.symbolic) trip.push_back({xb, sb, hval[i]});
      }
    }
    std::vector<std::pair<uint64_t, int>> order(keys.size());
    for (size_t i = 0; i < keys.size(); ++i) order[i] = {keys[i], (int)i};
    std::sort(order.begin(), order.end());
    remap.resize(keys.size());
    out.blocks.resize(order.size());
    int64_t off = 0;
    for (size_t i = 0; i < order.size(); ++i) {
      remap[order[i].second] = (int)i;
      Block& b = out.blocks[i];
      for (int o = 0; o < no; ++o) {
        const int nb = (o == 0 ? tbits : shift[o - 1]) - shift[o];
        b.sect[o] = (uint16_t)((order[i].first >> shift[o]) & ((nb >= 64 ? 0ull : (1ull << nb)) - 1ull));
      }
      b.base = off;
      set_rowmajor(out, b);
      off += out.block_elems(b);
    }
    out.size = off;
  } else {
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
    // output blocks sorted by sector tuple when not fixed
    remap.assign(out_keys.size(), 0);
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
  }
  if (spec.symbolic) return true;
  // triples ordered by output block, in enumeration order within a block
  // (a counting sort)
  {
    std::vector<int64_t> start(out.blocks.size() + 1, 0);
    for (auto& t : trip) {
      t.ob = remap[t.ob];
      ++start[t.ob + 1];
    }
    for (size_t b = 0; b < out.blocks.size(); ++b) start[b + 1] += start[b];
    std::vector<P3> sorted(trip.size());
    for (const P3& t : trip) sorted[start[t.ob]++] = t;
    trip.swap(sorted);
  }

  // keys of the per-pair scalar
  if (spec.key_order.size() > 2 * MAXL) {
    err = "key order too long";
    return false;
  }
  const BT& KT = spec.key_side == 0 ? X : out;
  for (int n : spec.key_order) {
    int p = KT.pos(n);
    if (p < 0) {
      err = "key order names a leg the keyed tensor lacks";
      return false;
    }
    E.kpos.push_back(p);
    E.kshared.push_back(S.pos(n) >= 0);
  }
  E.sshared.resize(S.nlegs());
  for (int q = 0; q < S.nlegs(); ++q) E.sshared[q] = KT.pos(S.names[q]) >= 0;
  E.nlab = S.cat.empty() ? 1 : S.cat[0]->nlab;
  return true;
}

double trip_alpha(StepEnum& E, const BT& X, const BT& S, const BT& out, const StepSpec& spec,
                  const SymInfo& sym, const P3& t) {
  if (sym.kind != SYM_SU2 && !sym.fermionic) return 1.0;
  const BT& KT = spec.key_side == 0 ? X : out;
  const int kbi = spec.key_side == 0 ? t.xb : t.ob;
  if (E.head.empty()) {
    E.head.resize(KT.blocks.size());
    E.head_set.assign(KT.blocks.size(), 0);
  }
  if (!E.head_set[kbi]) {
    const Block& kb = KT.blocks[kbi];
    const int nx = (int)E.kpos.size();
    const int32_t* xl[2 * MAXL];
    for (int i = 0; i < nx; ++i) xl[i] = KT.cat[E.kpos[i]]->label(kb.sect[E.kpos[i]]);
    E.head[kbi] = alpha_head(sym, spec.step, xl, nx, E.kshared.data(), E.nlab);
    E.head_set[kbi] = 1;
  }
  const Block& sbk = S.blocks[t.sb];
  const int nt = S.nlegs();
  const int32_t* tl[MAXL];
  for (int q = 0; q < nt; ++q) tl[q] = S.cat[q]->label(sbk.sect[q]);
  return alpha_tail(sym, E.head[kbi], tl, nt, E.sshared.data(), E.nlab);
}

}  // namespace

bool plan_step(const BT& X, const BT& S, const StepSpec& spec, const SymInfo& sym,
               TablePool& pool, const BT* fixed_out, StepResult& res, std::string& err) {
  StepEnum E;
  BT& out = res.out;
  if (!enumerate_step(X, S, spec, fixed_out, out, E, err)) return false;
  if (spec.symbolic) return true;
  const std::vector<P3>& trip = E.trip;

  // operand roles
  const BT& A = spec.m_is_x ? X : S;
  const BT& B = spec.m_is_x ? S : X;
  const std::vector<int>& afree = spec.m_is_x ? E.xfree : E.sfree;
  const std::vector<int>& bfree = spec.m_is_x ? E.sfree : E.xfree;
  const std::vector<int>& ak = spec.m_is_x ? E.xs : E.ss;
  const std::vector<int>& bk = spec.m_is_x ? E.ss : E.xs;
  // positions in the output of the M and N legs
  std::vector<int> cm, cn;
  for (int p : afree) cm.push_back(out.pos(A.names[p]));
  for (int p : bfree) cn.push_back(out.pos(B.names[p]));

  // tables and pairs
  GemmPlan& plan = res.plan;
  plan = GemmPlan();
  std::vector<std::pair<int64_t, int64_t>> mn;
  mn.reserve(out.blocks.size());
  for (auto& b : out.blocks) mn.emplace_back(prod_dims(out, b, cm), prod_dims(out, b, cn));
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
  std::vector<int64_t> ktot(out.blocks.size(), 0);
  for (size_t ob = 0; ob < out.blocks.size(); ++ob)
    for (int t = pstart[ob]; t < pstart[ob + 1]; ++t)
      ktot[ob] += prod_dims(A, spec.m_is_x ? X.blocks[trip[t].xb] : S.blocks[trip[t].sb], ak);
  {
    // signature: step, operand roles, and every output block's M, N and
    // contracted extent in order
    uint64_t h = splitmix64_mix(0x9e3779b97f4a7c15ull ^ (uint64_t)spec.step);
    h = splitmix64_mix(h ^ (spec.m_is_x ? 1u : 2u) ^ ((uint64_t)mn.size() << 8));
    for (size_t ob = 0; ob < mn.size(); ++ob) {
      h = splitmix64_mix(h ^ (uint64_t)mn[ob].first);
      h = splitmix64_mix(h ^ (uint64_t)mn[ob].second);
      h = splitmix64_mix(h ^ (uint64_t)ktot[ob]);
    }
    plan.sig = h;
    const std::array<int16_t, 2>* tuned = nullptr;
    if (sym.tune) {
      auto it = sym.tune->tiles.find(h);
      if (it != sym.tune->tiles.end() && valid_tile(it->second[0], it->second[1]))
        tuned = &it->second;
    }
    if (tuned) {
      plan.mt = (*tuned)[0];
      plan.nt = (*tuned)[1];
    } else if (sym.tile_rank > 0) {
      const auto c = tile_candidates(mn, ktot, sym.tile_rank + 1);
      const auto& t = c[std::min<size_t>((size_t)sym.tile_rank, c.size() - 1)];
      plan.mt = t[0];
      plan.nt = t[1];
    } else {
      choose_tile(mn, ktot, &plan.mt, &plan.nt);
    }
  }
  plan.pairs.reserve(trip.size());
  // tables depend only on the block: built once per block
  std::vector<TabRef> c_am(A.blocks.size(), TabRef{-1, 0}), c_ak(A.blocks.size(), TabRef{-1, 0});
  std::vector<TabRef> c_bk(B.blocks.size(), TabRef{-1, 0}), c_bn(B.blocks.size(), TabRef{-1, 0});
  auto cached = [&](std::vector<TabRef>& c, int i, const BT& bt, const std::vector<int>& pos) {
    if (c[i].id < 0) c[i] = make_table(pool, bt, bt.blocks[i], pos, &ok);
    return c[i];
  };
  for (auto& t : trip) {
    const Block& xbk = X.blocks[t.xb];
    const Block& sbk = S.blocks[t.sb];
    const Block& abk = spec.m_is_x ? xbk : sbk;
    const Block& bbk = spec.m_is_x ? sbk : xbk;
    const int ai = spec.m_is_x ? t.xb : t.sb, bi = spec.m_is_x ? t.sb : t.xb;
    TabRef tam = cached(c_am, ai, A, afree);
    TabRef tak = cached(c_ak, ai, A, ak);
    TabRef tbk = cached(c_bk, bi, B, bk);
    TabRef tbn = cached(c_bn, bi, B, bfree);
    GemmPair gp;
    gp.a_off = abk.base;
    gp.b_off = bbk.base;
    gp.K = (int32_t)prod_dims(A, abk, ak);
    gp.tam = tam.id;
    gp.tak = tak.id;
    gp.tbk = tbk.id;
    gp.tbn = tbn.id;
    gp.sam = tam.lin;
    gp.sak = tak.lin;
    gp.sbk = tbk.lin;
    gp.sbn = tbn.lin;
    gp.flags = 0;
    if (!ak.empty() && abk.stride[ak.back()] == 1) gp.flags |= 1;
    if (!bfree.empty() && bbk.stride[bfree.back()] == 1) gp.flags |= 2;
    gp.alpha = trip_alpha(E, X, S, out, spec, sym, t);
    plan.a_extent = std::max(plan.a_extent, gp.a_off + tam.maxoff + tak.maxoff + 1);
    plan.b_extent = std::max(plan.b_extent, gp.b_off + tbk.maxoff + tbn.maxoff + 1);
    int64_t M = prod_dims(A, abk, afree), N = prod_dims(B, bbk, bfree);
    plan.flops += 2.0 * (double)M * (double)N * (double)gp.K;
    plan.pairs.push_back(gp);
  }
  {
    std::vector<char> ua(A.blocks.size(), 0), ub(B.blocks.size(), 0);
    for (const P3& t : trip) {
      ua[spec.m_is_x ? t.xb : t.sb] = 1;
      ub[spec.m_is_x ? t.sb : t.xb] = 1;
    }
    double e = 0;
    for (size_t b = 0; b < A.blocks.size(); ++b)
      if (ua[b]) e += (double)A.block_elems(A.blocks[b]);
    for (size_t b = 0; b < B.blocks.size(); ++b)
      if (ub[b]) e += (double)B.block_elems(B.blocks[b]);
    for (const Block& b : out.blocks) e += (double)out.block_elems(b);
    plan.bytes = 8.0 * e;
  }
  // jobs: one per output tile and split part. Launches with too few tiles
  // for the chip split the pair list of long-K blocks into parts (pair
  // boundaries, or K ranges of a single pair) summed by a reduction.
  int64_t ntiles = 0;
  for (size_t ob = 0; ob < out.blocks.size(); ++ob)
    ntiles += (mn[ob].first + plan.mt - 1) / plan.mt * ((mn[ob].second + plan.nt - 1) / plan.nt);
  constexpr int64_t TARGET_JOBS = 2048, MIN_PART_K = 256, MAX_SPLIT = 16;
  int64_t want = ntiles > 0 ? (TARGET_JOBS + ntiles - 1) / ntiles : 1;
  want = std::min<int64_t>(want, MAX_SPLIT);
  bool split = false;
  if (want > 1)
    for (size_t ob = 0; ob < out.blocks.size(); ++ob)
      if (ktot[ob] >= 2 * MIN_PART_K) split = true;
  for (size_t ob = 0; ob < out.blocks.size(); ++ob) {
    const Block& cb = out.blocks[ob];
    int64_t M = mn[ob].first, N = mn[ob].second;
    if (M > INT32_MAX || N > INT32_MAX || (split && M * N > INT32_MAX)) {
      err = "block too large";
      return false;
    }
    TabRef tcm = make_table(pool, out, cb, cm, &ok);
    TabRef tcn = make_table(pool, out, cb, cn, &ok);
    plan.c_extent = std::max(plan.c_extent, cb.base + tcm.maxoff + tcn.maxoff + 1);
    // parts: (p0, p1, k0, k1)
    struct Part {
      int p0, p1, k0, k1;
    };
    std::vector<Part> parts;
    const int p0 = pstart[ob], p1 = pstart[ob + 1];
    const int64_t nparts = split ? std::max<int64_t>(1, std::min(want, ktot[ob] / MIN_PART_K)) : 1;
    if (nparts <= 1 || p1 - p0 == 0) {
      parts.push_back({p0, p1, 0, INT32_MAX});
    } else if (p1 - p0 == 1) {
      const int K = plan.pairs[p0].K;
      int chunk = (int)((K + nparts - 1) / nparts);
      chunk = (chunk + 15) / 16 * 16;
      for (int k0 = 0; k0 < K; k0 += chunk) parts.push_back({p0, p1, k0, std::min(K, k0 + chunk)});
    } else {
      // contiguous pair ranges with about ktot / nparts contracted extent each
      const double per = (double)ktot[ob] / (double)nparts;
      double acc = 0;
      int start = p0;
      for (int t = p0; t < p1; ++t) {
        acc += plan.pairs[t].K;
        if ((acc >= per * (double)(parts.size() + 1) || t == p1 - 1) && t + 1 > start) {
          parts.push_back({start, t + 1, 0, INT32_MAX});
          start = t + 1;
        }
      }
    }
    int32_t pm = 0, pn = 0;
    int64_t p_off = 0;
    if (split) {
      TabRef rm = make_table_dense(pool, (int32_t)M, N, &ok);
      TabRef rn = make_table_dense(pool, (int32_t)N, 1, &ok);
      pm = rm.id;
      pn = rn.id;
      p_off = plan.partial_size;
      ReduceTab rd;
      rd.c_off = cb.base;
      rd.p_off = p_off;
      rd.tcm = tcm.id;
      rd.tcn = tcn.id;
      rd.M = (int32_t)M;
      rd.N = (int32_t)N;
      rd.nsplit = (int32_t)parts.size();
      rd.pad = 0;
      plan.reduces.push_back(rd);
      plan.partial_size += (int64_t)parts.size() * M * N;
      plan.max_red_mn = std::max(plan.max_red_mn, M * N);
    }
    for (size_t q = 0; q < parts.size(); ++q)
      for (int64_t m0 = 0; m0 < M; m0 += plan.mt)
        for (int64_t n0 = 0; n0 < N; n0 += plan.nt) {
          GemmJob j;
          j.c_off = split ? p_off + (int64_t)q * M * N : cb.base;
          j.M = (int32_t)M;
          j.N = (int32_t)N;
          j.m0 = (int32_t)m0;
          j.n0 = (int32_t)n0;
          j.tcm = split ? pm : tcm.id;
          j.tcn = split ? pn : tcn.id;
          j.p0 = parts[q].p0;
          j.p1 = parts[q].p1;
          j.k0 = parts[q].k0;
          j.k1 = parts[q].k1;
          plan.jobs.push_back(j);
        }
  }
  if (!ok) {
    err = "offset table overflow (block or pool exceeds 2^31 elements)";
    return false;
  }
  return true;
}

bool plan_step_rt(const BT& X, const BT& S, const StepSpec& spec, const SymInfo& sym,
                  TablePool& pool, StepResult& res, RtPlan& rt, std::string& err) {
  StepEnum E;
  BT& out = res.out;
  rt = RtPlan();
  if (!enumerate_step(X, S, spec, nullptr, out, E, err)) return false;
  if (spec.symbolic) return true;
  const std::vector<P3>& trip = E.trip;
  // levels: runs of X's free legs adjacent, in the same order, in X and in
  // the output
  std::vector<int> opos;
  for (int p : E.xfree) opos.push_back(out.pos(X.names[p]));
  std::vector<std::vector<int>> lev;   // X positions per level
  for (size_t i = 0; i < E.xfree.size(); ++i) {
    if (i > 0 && E.xfree[i] == E.xfree[i - 1] + 1 && opos[i] == opos[i - 1] + 1)
      lev.back().push_back((int)i);
    else
      lev.push_back({(int)i});
  }
  const int nlev = (int)lev.size();
  if (nlev > RT_MAXLEV) {
    err = "layer step needs " + std::to_string(nlev) + " row levels (at most " +
          std::to_string(RT_MAXLEV) + ")";
    return false;
  }
  const int pad = RT_MAXLEV - nlev;
  // per-level dims and strides of a block (legs of a level are contiguous
  // row-major inside the block: the level stride is its last leg's)
  auto level_geom = [&](const BT& bt, const Block& b, const std::vector<int>& pos_of,
                        int32_t* md, int32_t* st) -> bool {
    for (int l = 0; l < RT_MAXLEV; ++l) {
      md[l] = 1;
      st[l] = 0;
    }
    for (int l = 0; l < nlev; ++l) {
      int64_t d = 1;
      for (size_t u = 0; u < lev[l].size(); ++u) {
        const int p = pos_of[lev[l][u]];
        if (u > 0) {
          const int pp = pos_of[lev[l][u - 1]];
          if (b.stride[pp] != b.stride[p] * bt.dim(b, p)) return false;
        }
        d *= bt.dim(b, p);
      }
      const int64_t s = b.stride[pos_of[lev[l].back()]];
      if (d > INT32_MAX || s > INT32_MAX) return false;
      md[pad + l] = (int32_t)d;
      st[pad + l] = (int32_t)s;
    }
    return true;
  };
  // per-block caches of the small tables
  std::vector<TabRef> c_xk(X.blocks.size(), TabRef{-1, 0}), c_sk(S.blocks.size(), TabRef{-1, 0});
  std::vector<std::vector<int32_t>> c_sn(S.blocks.size());
  std::map<std::pair<int, int64_t>, int32_t> c_snt;
  std::vector<int> opos_by_i(E.xfree.size());
  for (size_t i = 0; i < E.xfree.size(); ++i) opos_by_i[i] = opos[i];
  std::vector<int> xpos_by_i = E.xfree;
  // S legs: contracted (in X's contracted order) and free (S order)
  bool ok = true;
  // output N legs, in S order, located in the output
  std::vector<int> onpos;
  for (int q : E.sfree) onpos.push_back(out.pos(S.names[q]));

  // groups: output blocks with equal sectors on X's free legs
  const std::vector<int>& xkey_pos = opos;   // output positions of X's free legs
  std::map<std::vector<uint16_t>, std::vector<int>> gmap;
  for (int ob = 0; ob < (int)out.blocks.size(); ++ob) {
    std::vector<uint16_t> k;
    for (int p : xkey_pos) k.push_back(out.blocks[ob].sect[p]);
    gmap[k].push_back(ob);
  }
  std::vector<int> pstart(out.blocks.size() + 1, 0);
  {
    size_t t = 0;
    for (size_t ob = 0; ob < out.blocks.size(); ++ob) {
      pstart[ob] = (int)t;
      while (t < trip.size() && trip[t].ob == (int)ob) ++t;
    }
    pstart[out.blocks.size()] = (int)trip.size();
  }
  int64_t tiles = 0;
  std::vector<double> palpha;
  for (auto& kv : gmap) {
    const int ob0 = kv.second.front();
    const Block& cb0 = out.blocks[ob0];
    RtGroup g;
    int32_t st_dummy[RT_MAXLEV];
    if (!level_geom(out, cb0, opos_by_i, g.md, st_dummy)) {
      err = "output block rows are not level-contiguous";
      return false;
    }
    int64_t M = 1;
    for (int l = 0; l < RT_MAXLEV; ++l) M *= g.md[l];
    if (M > INT32_MAX) {
      err = "layer step group too large";
      return false;
    }
    g.M = (int32_t)M;
    for (int l = 0; l < RT_MAXLEV; ++l)
      g.mg[l] = g.md[l] > 1 ? UINT64_MAX / (uint64_t)g.md[l] + 1 : 0;
    g.tile0 = (int32_t)tiles;
    g.o0 = (int32_t)rt.outs.size();
    g.k0 = (int32_t)rt.kblks.size();
    // the group's distinct X blocks, each with its staged column offset
    std::map<int, int32_t> kmap;   // X block -> RtKblk index
    int32_t ktot = 0;
    for (int ob : kv.second)
      for (int pi = pstart[ob]; pi < pstart[ob + 1]; ++pi) {
        const int xbi = trip[pi].xb;
        if (kmap.count(xbi)) continue;
        const Block& xb = X.blocks[xbi];
        RtKblk kb;
        int32_t mdx[RT_MAXLEV];
        if (!level_geom(X, xb, xpos_by_i, mdx, kb.xs)) {
          err = "input block rows are not level-contiguous";
          return false;
        }
        for (int l = 0; l < RT_MAXLEV; ++l)
          if (mdx[l] != g.md[l]) {
            err = "row levels differ between input and output block";
            return false;
          }
        kb.xbase = xb.base;
        const int64_t Kb = prod_dims(X, xb, E.xs);
        if (Kb > INT32_MAX / 2) {
          err = "contracted extent too large";
          return false;
        }
        kb.Kb = (int32_t)Kb;
        if (c_xk[xbi].id < 0) c_xk[xbi] = make_table(pool, X, xb, E.xs, &ok);
        kb.xktab = c_xk[xbi].id;
        int64_t xrow = 0;
        for (int l = 0; l < RT_MAXLEV; ++l) xrow += (int64_t)(g.md[l] - 1) * kb.xs[l];
        rt.x_extent = std::max(rt.x_extent, xb.base + xrow + c_xk[xbi].maxoff + 1);
        kb.koff = ktot;
        kb.pad = 0;
        ktot += kb.Kb;
        kmap.emplace(xbi, (int32_t)rt.kblks.size());
        rt.kblks.push_back(kb);
      }
    g.k1 = (int32_t)rt.kblks.size();
    g.ktot = ktot;
    g.c0 = (int32_t)rt.cols.size();
    // two rows per lane (see RT_PAIR_LDS) when the chunks at RT_NC columns
    // already fill the four waves
    bool pair_rows = false;
    {
      int64_t have = 0;
      for (int ob : kv.second) have += (prod_dims(out, out.blocks[ob], onpos) + RT_NC - 1) / RT_NC;
      pair_rows = have >= 4 && M >= 128 && (int64_t)128 * ktot * 8 <= RT_PAIR_LDS;
    }
    const int ncmax = pair_rows ? RT_NC2 : RT_NC;
    for (int ob : kv.second) {
      const Block& cb = out.blocks[ob];
      RtOut base_o;
      int32_t md2[RT_MAXLEV];
      if (!level_geom(out, cb, opos_by_i, md2, base_o.ms)) {
        err = "output block rows are not level-contiguous";
        return false;
      }
      base_o.base = cb.base;
      const int64_t Nb = prod_dims(out, cb, onpos);
      // all N offsets of the block, then chunked
      std::vector<int32_t> noff;
      {
        std::vector<int32_t> dims;
        std::vector<int64_t> strides;
        for (int p : onpos) {
          dims.push_back(out.dim(cb, p));
          strides.push_back(cb.stride[p]);
        }
        std::vector<int32_t> idx(dims.size(), 0);
        int64_t off = 0;
        for (int64_t e = 0; e < Nb; ++e) {
          noff.push_back((int32_t)off);
          for (int d = (int)dims.size() - 1; d >= 0; --d) {
            if (++idx[d] < dims[d]) {
              off += strides[d];
              break;
            }
            off -= strides[d] * (int64_t)(dims[d] - 1);
            idx[d] = 0;
          }
        }
      }
      int64_t rowmax = 0;
      for (int l = 0; l < RT_MAXLEV; ++l) rowmax += (int64_t)(g.md[l] - 1) * base_o.ms[l];
      int32_t nmax = 0;
      for (int32_t v : noff) nmax = std::max(nmax, v);
      rt.c_extent = std::max(rt.c_extent, cb.base + rowmax + nmax + 1);
      // equal chunks of at most RT_NC columns (18 -> 9 + 9, not 16 + 2):
      // every chunk re-reads the row's inputs
      const int64_t nchunks = (Nb + ncmax - 1) / ncmax;
      const int64_t cw = (Nb + nchunks - 1) / nchunks;
      // the pair scalars of this block, shared by its chunks
      palpha.resize((size_t)(pstart[ob + 1] - pstart[ob]));
      for (int pi = pstart[ob]; pi < pstart[ob + 1]; ++pi)
        palpha[pi - pstart[ob]] = trip_alpha(E, X, S, out, spec, sym, trip[pi]);
      for (int64_t n0 = 0; n0 < Nb; n0 += cw) {
        const int nc = (int)std::min<int64_t>(cw, Nb - n0);
        RtOut o = base_o;
        o.nc = nc;
        o.ntab = pool.add_raw(std::vector<int32_t>(noff.begin() + n0, noff.begin() + n0 + nc), &ok);
        o.p0 = (int32_t)rt.pairs.size();
        for (int pi = pstart[ob]; pi < pstart[ob + 1]; ++pi) {
          const P3& t = trip[pi];
          const Block& sb = S.blocks[t.sb];
          RtPair pr;
          const int32_t kbi = kmap.at(t.xb);
          pr.kblk = kbi;
          pr.koff = rt.kblks[kbi].koff;
          pr.Kb = rt.kblks[kbi].Kb;
          pr.pad = 0;
          const int64_t Kb = pr.Kb;
          pr.pk = rt.pack_size;
          RtPack pk;
          pk.dst = rt.pack_size;
          pk.sbase = sb.base;
          pk.Kb = pr.Kb;
          pk.nc = nc;
          if (c_sk[t.sb].id < 0) c_sk[t.sb] = make_table(pool, S, sb, E.ss, &ok);
          const int64_t skmax = c_sk[t.sb].maxoff;
          pk.sktab = c_sk[t.sb].id;
          // layer block N offsets (all Nb), then this chunk's table
          std::vector<int32_t>& all = c_sn[t.sb];
          if (all.empty()) {
            std::vector<int32_t> dims;
            std::vector<int64_t> strides;
            for (int q : E.sfree) {
              dims.push_back(S.dim(sb, q));
              strides.push_back(sb.stride[q]);
            }
            std::vector<int32_t> idx(dims.size(), 0);
            int64_t off = 0;
            for (int64_t e = 0; e < Nb; ++e) {
              all.push_back((int32_t)off);
              for (int d = (int)dims.size() - 1; d >= 0; --d) {
                if (++idx[d] < dims[d]) {
                  off += strides[d];
                  break;
                }
                off -= strides[d] * (int64_t)(dims[d] - 1);
                idx[d] = 0;
              }
            }
          }
          int32_t snmax = 0;
          for (int64_t e = n0; e < n0 + nc; ++e) snmax = std::max(snmax, all[e]);
          rt.s_extent = std::max(rt.s_extent, sb.base + skmax + snmax + 1);
          // keyed by the chunk's first column and its width (a block may be
          // chunked differently in another group)
          auto key = std::make_pair(t.sb, n0 * (RT_NC + 1) + nc);
          auto it = c_snt.find(key);
          if (it == c_snt.end())
            it = c_snt.emplace(key, pool.add_raw(std::vector<int32_t>(all.begin() + n0,
                                                                        all.begin() + n0 + nc),
                                                 &ok)).first;
          pk.sntab = it->second;
          pk.alpha = palpha[pi - pstart[ob]];
          rt.pack_size += Kb * nc;
          rt.packs.push_back(pk);
          rt.pairs.push_back(pr);
          rt.flops += 2.0 * (double)M * (double)Kb * (double)nc;
          rt.x_loads += (double)M * (double)Kb;
        }
        o.p1 = (int32_t)rt.pairs.size();
        rt.outs.push_back(o);
      }
    }
    g.o1 = (int32_t)rt.outs.size();
    // rows per workgroup: four waves share the chunks of 64 rows when there
    // are enough chunks, else take 128 or 256 rows; staged when the X rows
    // fit the LDS budget
    const int nch = g.o1 - g.o0;
    int rows = nch >= 4 ? 64 : (nch >= 2 ? 128 : 256);
    while (rows > 64 && (int64_t)rows * ktot * 8 > RT_LDS_BYTES) rows /= 2;
    if (pair_rows) rows = 128;
    g.rows = rows;
    g.staged = (int64_t)rows * ktot * 8 <= RT_LDS_BYTES ? (pair_rows ? 2 : 1) : 0;
    if (g.staged) {
      for (int b = g.k0; b < g.k1; ++b) {
        const RtKblk& K = rt.kblks[b];
        const int32_t* kt = pool.data.data() + K.xktab;
        for (int k = 0; k < K.Kb; ++k) {
          RtCol c;
          c.xbase = K.xbase + kt[k];
          for (int l = 0; l < RT_MAXLEV; ++l) c.xs[l] = K.xs[l];
          rt.cols.push_back(c);
        }
      }
    }
    if (g.staged) rt.lds_bytes = std::max<int32_t>(rt.lds_bytes, rows * ktot * 8);
    rt.groups.push_back(g);
    tiles += (M + rows - 1) / rows;
    if (tiles > INT32_MAX) {
      err = "layer step has too many row tiles";
      return false;
    }
  }
  // order the groups by LDS class and renumber their tiles; every class is
  // one launch
  {
    auto cls = [](const RtGroup& g) {
      if (!g.staged) return 0;
      const int64_t b = (int64_t)g.rows * g.ktot * 8;
      return b <= 16 * 1024 ? 1 : (b <= 32 * 1024 ? 2 : 3);
    };
    std::vector<RtGroup> sorted;
    sorted.reserve(rt.groups.size());
    for (int c = 0; c < RT_NCLASS; ++c)
      for (const RtGroup& g : rt.groups)
        if (cls(g) == c) sorted.push_back(g);
    rt.groups.swap(sorted);
    int64_t t = 0;
    rt.nlaunch = 0;
    for (int c = 0; c < RT_NCLASS; ++c) {
      const int64_t t0 = t;
      int32_t lds = 0;
      double lf = 0, lb = 0;
      for (size_t gi = 0; gi < rt.groups.size(); ++gi) {
        RtGroup& g = rt.groups[gi];
        if (cls(g) != c) continue;
        // algorithmic work of the group: its rows of every X block read
        // once, its output chunks written once, 2 M Kb nc per pair
        for (int b = g.k0; b < g.k1; ++b) lb += 8.0 * g.M * rt.kblks[b].Kb;
        for (int o = g.o0; o < g.o1; ++o) {
          lb += 8.0 * g.M * rt.outs[o].nc;
          for (int p = rt.outs[o].p0; p < rt.outs[o].p1; ++p)
            lf += 2.0 * g.M * rt.pairs[p].Kb * rt.outs[o].nc;
        }
        g.tile0 = (int32_t)t;
        const int64_t nt = ((int64_t)g.M + g.rows - 1) / g.rows;
        t += nt;
        if (g.staged) lds = std::max<int32_t>(lds, g.rows * g.ktot * 8);
      }
      if (t > t0) {
        rt.l_tile0[rt.nlaunch] = (int32_t)t0;
        rt.l_ntiles[rt.nlaunch] = (int32_t)(t - t0);
        rt.l_lds[rt.nlaunch] = lds;
        rt.l_flops[rt.nlaunch] = lf;
        rt.l_bytes[rt.nlaunch] = lb;
        ++rt.nlaunch;
      }
    }
    if (t != tiles) {
      err = "layer step tile count mismatch";
      return false;
    }
  }
  rt.ntiles = (int32_t)tiles;
  {
    std::vector<char> used(X.blocks.size(), 0);
    for (const P3& t : trip) used[t.xb] = 1;
    double xe = 0;
    for (size_t b = 0; b < X.blocks.size(); ++b)
      if (used[b]) xe += (double)X.block_elems(X.blocks[b]);
    rt.bytes = 8.0 * (xe + (double)out.size);
  }
  if (!ok) {
    err = "offset table overflow";
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
    TabRef t{pool.add(d, st, &ok), (int64_t)(std::max(n, 1) - 1) * s};
    t.lin = linear_stride(d, st);
    return t;
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
    gp.sam = tam.lin;
    gp.sak = tak.lin;
    gp.sbk = tbk.lin;
    gp.sbn = tbn.lin;
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
