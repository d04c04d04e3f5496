// Host check of the block-pair planner (csrc/plan.cpp), built with address
// and undefined-behaviour sanitizers by tests/test_planner_sanitized.py.
//
// Random block-sparse tensors (random sector counts, dimensions and block
// subsets) are contracted over a shared leg, as a GEMM step and as a
// row-thread layer step. Every offset that a device kernel would form from
// the plan is replayed here: for GEMM plans each A, B and C (or partial)
// element a job touches, and each reduction; for layer plans each staged
// column, X element, packed layer value, layer element and output element
// of every row of every group. All of them must fall inside the buffers,
// every output element must be written exactly once, and the flop counts
// must equal 2 m n k over the block pairs. A table the plan marks as a
// row-major run (offset computed as i * stride, not read) must hold exactly
// those values. Exit status 0 when every check holds.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../paper_2511_01039_amd/csrc/plan.hpp"

using namespace fp;

namespace {

int failures = 0;
long linear_pairs = 0;
#define CHECK(c)                                                                    \
  do {                                                                              \
    if (!(c)) {                                                                     \
      if (failures < 20) std::fprintf(stderr, "check failed (line %d): %s\n", __LINE__, #c); \
      ++failures;                                                                   \
    }                                                                               \
  } while (0)

LegP make_leg(std::mt19937& g, int nsect, int maxdim) {
  auto l = std::make_shared<Leg>();
  l->nlab = 1;
  for (int s = 0; s < nsect; ++s) {
    l->lab.push_back(s);
    l->dim.push_back(1 + (int)(g() % (unsigned)maxdim));
  }
  return l;
}

// A tensor on the given legs holding a random subset of its sector tuples,
// blocks row-major and packed in tuple order.
BT make_bt(std::mt19937& g, const std::vector<int>& names, const std::vector<LegP>& legs,
           double density) {
  BT t;
  t.names = names;
  t.cat = legs;
  std::vector<int> idx(names.size(), 0);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  int64_t off = 0;
  while (true) {
    if (u(g) < density) {
      Block b;
      for (size_t p = 0; p < names.size(); ++p) b.sect[p] = (uint16_t)idx[p];
      b.base = off;
      set_rowmajor(t, b);
      off += t.block_elems(b);
      t.blocks.push_back(b);
    }
    size_t p = names.size();
    bool done = true;
    while (p > 0) {
      --p;
      if (++idx[p] < legs[p]->nsect()) {
        done = false;
        break;
      }
      idx[p] = 0;
    }
    if (done) {
      t.size = off;
      return t;
    }
  }
}

struct Tabs {
  const TablePool& pool;
  int32_t at(int32_t id, int64_t i) const {
    CHECK(id >= 0 && (size_t)id + (size_t)i < pool.data.size());
    if (id < 0 || (size_t)id + (size_t)i >= pool.data.size()) return 0;
    return pool.data[(size_t)id + (size_t)i];
  }
};

// GEMM step: X[a, b, j] S[b, c] -> out[a, c, j], M = (a, j), K = b, N = c.
void check_gemm(const BT& X, const BT& S, const StepResult& r, const TablePool& pool) {
  const GemmPlan& p = r.plan;
  const Tabs T{pool};
  CHECK(p.a_extent <= X.size && p.b_extent <= S.size && p.c_extent <= r.out.size);
  CHECK(p.mt > 0 && p.nt > 0);
  const bool split = p.partial_size > 0;
  std::vector<int> wc((size_t)std::max<int64_t>(r.out.size, 1), 0);
  std::vector<int> wp((size_t)std::max<int64_t>(p.partial_size, 1), 0);
  double flops = 0;
  std::vector<char> seen(p.pairs.size(), 0);
  for (const GemmJob& j : p.jobs) {
    CHECK(j.p0 >= 0 && j.p0 <= j.p1 && j.p1 <= (int)p.pairs.size());
    CHECK(j.m0 >= 0 && j.m0 < j.M && j.n0 >= 0 && j.n0 < j.N);
    const int m1 = std::min(j.M, j.m0 + p.mt), n1 = std::min(j.N, j.n0 + p.nt);
    for (int q = j.p0; q < j.p1 && q < (int)p.pairs.size(); ++q) {
      const GemmPair& pr = p.pairs[q];
      const int k0 = std::max(0, j.k0), k1 = std::min(j.k1, pr.K);
      CHECK(k0 <= k1);
      int64_t amax = 0, bmax = 0, amin = INT64_MAX, bmin = INT64_MAX;
      int32_t tm = 0, tk = 0, tn = 0, tb = 0;
      for (int m = j.m0; m < m1; ++m) tm = std::max(tm, T.at(pr.tam, m));
      for (int n = j.n0; n < n1; ++n) tn = std::max(tn, T.at(pr.tbn, n));
      for (int k = k0; k < k1; ++k) {
        tk = std::max(tk, T.at(pr.tak, k));
        tb = std::max(tb, T.at(pr.tbk, k));
        CHECK(T.at(pr.tak, k) >= 0 && T.at(pr.tbk, k) >= 0);
      }
      // a table flagged as a row-major run must equal i * stride
      auto linear_ok = [&](int32_t id, int32_t s, int n) {
        if (s <= 0) return true;
        for (int i = 0; i < n; ++i)
          if (T.at(id, i) != (int64_t)i * s) return false;
        return true;
      };
      CHECK(linear_ok(pr.tam, pr.sam, j.M) && linear_ok(pr.tak, pr.sak, pr.K));
      CHECK(linear_ok(pr.tbk, pr.sbk, pr.K) && linear_ok(pr.tbn, pr.sbn, j.N));
      if (pr.sam > 0 || pr.sak > 0 || pr.sbk > 0 || pr.sbn > 0) ++linear_pairs;
      amax = pr.a_off + tm + tk;
      bmax = pr.b_off + tb + tn;
      amin = pr.a_off;
      bmin = pr.b_off;
      if (k1 > k0) {
        CHECK(amin >= 0 && amax < X.size && amax < p.a_extent);
        CHECK(bmin >= 0 && bmax < S.size && bmax < p.b_extent);
      }
      if (!seen[q]) {
        seen[q] = 1;
        flops += 2.0 * j.M * (double)j.N * pr.K;
      }
    }
    for (int m = j.m0; m < m1; ++m)
      for (int n = j.n0; n < n1; ++n) {
        const int64_t c = j.c_off + T.at(j.tcm, m) + T.at(j.tcn, n);
        if (split) {
          CHECK(c >= 0 && c < p.partial_size);
          if (c >= 0 && c < p.partial_size) ++wp[(size_t)c];
        } else {
          CHECK(c >= 0 && c < r.out.size);
          if (c >= 0 && c < r.out.size) ++wc[(size_t)c];
        }
      }
  }
  for (const ReduceTab& rd : p.reduces) {
    CHECK((int64_t)rd.M * rd.N <= p.max_red_mn && rd.nsplit >= 1);
    for (int m = 0; m < rd.M; ++m)
      for (int n = 0; n < rd.N; ++n) {
        const int64_t c = rd.c_off + T.at(rd.tcm, m) + T.at(rd.tcn, n);
        CHECK(c >= 0 && c < r.out.size);
        if (c >= 0 && c < r.out.size) ++wc[(size_t)c];
        for (int s = 0; s < rd.nsplit; ++s) {
          const int64_t e = rd.p_off + (int64_t)s * rd.M * rd.N + (int64_t)m * rd.N + n;
          CHECK(e >= 0 && e < p.partial_size);
        }
      }
  }
  CHECK(std::fabs(flops - p.flops) <= 1e-9 * std::max(1.0, p.flops));
  for (const Block& b : r.out.blocks)
    for (int64_t e = 0; e < r.out.block_elems(b); ++e) CHECK(wc[(size_t)(b.base + e)] == 1);
  if (split)
    for (int64_t e = 0; e < p.partial_size; ++e) CHECK(wp[(size_t)e] == 1);
}

// Layer step: X[a, k, j] S[k, p] -> out[a, p, j], rows (a, j) in levels.
void check_rt(const BT& X, const BT& S, const StepResult& r, const RtPlan& rt,
              const TablePool& pool) {
  const Tabs T{pool};
  const BT& out = r.out;
  CHECK(rt.x_extent <= X.size && rt.s_extent <= S.size && rt.c_extent <= out.size);
  std::vector<int> wc((size_t)std::max<int64_t>(out.size, 1), 0);
  double flops = 0;
  int64_t tiles = 0;
  for (const RtGroup& g : rt.groups) {
    CHECK(g.o0 >= 0 && g.o0 <= g.o1 && g.o1 <= (int)rt.outs.size());
    CHECK(g.k0 >= 0 && g.k0 <= g.k1 && g.k1 <= (int)rt.kblks.size());
    CHECK(g.rows == 64 || g.rows == 128 || g.rows == 256);
    CHECK(g.M >= 1);
    int64_t mprod = 1;
    for (int l = 0; l < RT_MAXLEV; ++l) {
      CHECK(g.md[l] >= 1);
      mprod *= g.md[l];
    }
    CHECK(mprod == g.M);
    if (g.staged) {
      CHECK(g.c0 >= 0 && g.c0 + g.ktot <= (int)rt.cols.size());
      CHECK((int64_t)g.rows * g.ktot * 8 <= RT_LDS_BYTES);
    }
    tiles += (g.M + g.rows - 1) / g.rows;
    for (int64_t m = 0; m < g.M; ++m) {
      // level indices by plain division, and by the multiply-high
      // constants the kernel divides with
      int32_t idx[RT_MAXLEV];
      uint64_t rr = (uint64_t)m;
      for (int l = RT_MAXLEV - 1; l >= 0; --l) {
        idx[l] = (int32_t)(rr % (uint64_t)g.md[l]);
        if (g.md[l] > 1) {
          const uint64_t q = (uint64_t)(((unsigned __int128)rr * g.mg[l]) >> 64);
          CHECK(q == rr / (uint64_t)g.md[l]);
        }
        rr /= (uint64_t)g.md[l];
      }
      if (g.staged)
        for (int c = g.c0; c < g.c0 + g.ktot && c < (int)rt.cols.size(); ++c) {
          int64_t xo = rt.cols[c].xbase;
          for (int l = 0; l < RT_MAXLEV; ++l) xo += (int64_t)idx[l] * rt.cols[c].xs[l];
          CHECK(xo >= 0 && xo < X.size);
        }
      for (int o = g.o0; o < g.o1 && o < (int)rt.outs.size(); ++o) {
        const RtOut& O = rt.outs[o];
        CHECK(O.nc >= 1 && O.nc <= RT_NC);
        CHECK(O.p0 >= 0 && O.p0 <= O.p1 && O.p1 <= (int)rt.pairs.size());
        int64_t oo = O.base;
        for (int l = 0; l < RT_MAXLEV; ++l) oo += (int64_t)idx[l] * O.ms[l];
        for (int c = 0; c < O.nc; ++c) {
          const int64_t e = oo + T.at(O.ntab, c);
          CHECK(e >= 0 && e < out.size);
          if (e >= 0 && e < out.size) ++wc[(size_t)e];
        }
        for (int q = O.p0; q < O.p1 && q < (int)rt.pairs.size(); ++q) {
          const RtPair& P = rt.pairs[q];
          CHECK(P.kblk >= g.k0 && P.kblk < g.k1);
          if (P.kblk < 0 || P.kblk >= (int)rt.kblks.size()) continue;
          const RtKblk& K = rt.kblks[P.kblk];
          CHECK(P.Kb == K.Kb && P.koff == K.koff);
          CHECK(P.pk >= 0 && P.pk + (int64_t)P.Kb * O.nc <= rt.pack_size);
          if (g.staged) CHECK(K.koff >= 0 && K.koff + K.Kb <= g.ktot);
          int64_t xo = K.xbase;
          for (int l = 0; l < RT_MAXLEV; ++l) xo += (int64_t)idx[l] * K.xs[l];
          for (int k = 0; k < K.Kb; ++k) {
            const int64_t e = xo + T.at(K.xktab, k);
            CHECK(e >= 0 && e < X.size);
          }
          if (m == 0) flops += 2.0 * g.M * (double)P.Kb * O.nc;
        }
      }
    }
  }
  CHECK(tiles == rt.ntiles);
  CHECK(std::fabs(flops - rt.flops) <= 1e-9 * std::max(1.0, rt.flops));
  CHECK(rt.packs.size() == rt.pairs.size());
  for (const RtPack& P : rt.packs) {
    CHECK(P.dst >= 0 && P.dst + (int64_t)P.Kb * P.nc <= rt.pack_size);
    for (int k = 0; k < P.Kb; ++k)
      for (int c = 0; c < P.nc; ++c) {
        const int64_t e = P.sbase + T.at(P.sktab, k) + T.at(P.sntab, c);
        CHECK(e >= 0 && e < S.size);
      }
  }
  for (const Block& b : out.blocks)
    for (int64_t e = 0; e < out.block_elems(b); ++e) CHECK(wc[(size_t)(b.base + e)] == 1);
}

}  // namespace

int main(int argc, char** argv) {
  const int cases = argc > 1 ? std::atoi(argv[1]) : 60;
  std::mt19937 g(20251101u);
  int plans = 0, splits = 0, rt_plans = 0, staged = 0, refused = 0;
  std::string last_err;
  for (int c = 0; c < cases; ++c) {
    const bool big_k = c % 4 == 3;   // long contracted legs: split-K plans
    LegP la = make_leg(g, 1 + g() % 5, 48), lb = make_leg(g, 1 + g() % 5, big_k ? 400 : 40),
         lj = make_leg(g, 1 + g() % 3, 12), lc = make_leg(g, 1 + g() % 4, 24);
    const double dens = 0.4 + 0.6 * (double)(g() % 100) / 100.0;
    SymInfo sym;
    if (c % 3 == 1) {
      sym.kind = SYM_SU2;
      sym.coef_seed = 7 + (uint64_t)c;
    }
    {
      BT X = make_bt(g, {N_a, N_b, N_j}, {la, lb, lj}, dens);
      BT S = make_bt(g, {N_b, N_c}, {lb, lc}, dens);
      StepSpec sp;
      sp.step = 1 + c % 5;
      sp.m_is_x = true;
      sp.out_names = {N_a, N_c, N_j};
      sp.key_order = {N_a, N_b, N_j};
      TablePool pool;
      StepResult r;
      std::string err;
      if (plan_step(X, S, sp, sym, pool, nullptr, r, err)) {
        ++plans;
        if (r.plan.partial_size > 0) ++splits;
        check_gemm(X, S, r, pool);
      } else {
        ++refused;
        last_err = err;
      }
    }
    {
      LegP lk = make_leg(g, 1 + g() % 3, 4), lp = make_leg(g, 1 + g() % 3, 10);
      BT X = make_bt(g, {N_a, N_tk, N_j}, {la, lk, lj}, dens);
      BT S = make_bt(g, {N_tk, N_p}, {lk, lp}, 1.0);
      StepSpec sp;
      sp.step = 2;
      sp.m_is_x = true;
      sp.out_names = {N_a, N_p, N_j};
      sp.key_order = {N_a, N_tk, N_j};
      TablePool pool;
      StepResult r;
      RtPlan rt;
      std::string err;
      if (plan_step_rt(X, S, sp, sym, pool, r, rt, err)) {
        ++rt_plans;
        for (const RtGroup& gr : rt.groups) staged += gr.staged ? 1 : 0;
        check_rt(X, S, r, rt, pool);
      } else {
        ++refused;
        last_err = err;
      }
    }
  }
  std::printf("planned %d GEMM steps (%d split-K, %ld pair visits with computed offsets), "
              "%d layer steps (%d staged groups); %d refused%s%s; %d failed checks\n",
              plans, splits, linear_pairs, rt_plans, staged, refused, refused ? ": " : "",
              last_err.c_str(), failures);
  return failures == 0 && refused == 0 && plans > 0 && rt_plans > 0 && splits > 0 &&
                 linear_pairs > 0
             ? 0
             : 1;
}
