// Layer steps of the chain (ket, PEPO and bra contracted into the
// sketch-side intermediate, and their transposes). Intermediates are stored
// in FP64 or FP32; every product and sum is FP64.
//
// These products have a huge row count (environment x sketch indices) and
// tiny contracted/column extents (a few virtual or physical indices), so
// they are bound by HBM traffic, not by arithmetic. A workgroup takes 64,
// 128 or 256 consecutive rows of one row group (fixed sectors on the free
// legs of X). It first copies those rows of every X block of the group into
// LDS, so each input element is read from HBM once (re-reading it from
// global memory per output chunk thrashes L2); then each lane owns one row
// and the four waves split the output chunks. A chunk's NC accumulators
// are multiplied against the packed, scalar-scaled layer sub-block
// (wave-uniform addresses, served by the scalar data path), and every
// output value is written once. Rows are numbered with the sketch column
// index innermost, which is stride-1 in every intermediate, so loads and
// stores of a wave are contiguous runs. Groups whose X rows do not fit the
// LDS budget read X directly.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fp {

// Plan data (groups, chunks, pairs, tables, packed layer blocks) is never
// written by the kernel: reading it through the constant address space lets
// wave-uniform loads use the scalar unit (s_load) even after the LDS barrier.
#define FP_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ const FP_CONST T* as_const(const T* p) {
  return (const FP_CONST T*)p;
}
// field-wise copies out of the constant address space
__device__ __forceinline__ RtGroup ld(const FP_CONST RtGroup* p) {
  RtGroup g;
#pragma unroll
  for (int l = 0; l < RT_MAXLEV; ++l) g.mg[l] = p->mg[l];
  g.tile0 = p->tile0;
  g.M = p->M;
#pragma unroll
  for (int l = 0; l < RT_MAXLEV; ++l) g.md[l] = p->md[l];
  g.o0 = p->o0;
  g.o1 = p->o1;
  g.k0 = p->k0;
  g.k1 = p->k1;
  g.rows = p->rows;
  g.staged = p->staged;
  g.ktot = p->ktot;
  g.c0 = p->c0;
  return g;
}
__device__ __forceinline__ RtOut ld(const FP_CONST RtOut* p) {
  RtOut o;
  o.base = p->base;
#pragma unroll
  for (int l = 0; l < RT_MAXLEV; ++l) o.ms[l] = p->ms[l];
  o.nc = p->nc;
  o.ntab = p->ntab;
  o.p0 = p->p0;
  o.p1 = p->p1;
  return o;
}
__device__ __forceinline__ RtKblk ld(const FP_CONST RtKblk* p) {
  RtKblk k;
  k.xbase = p->xbase;
#pragma unroll
  for (int l = 0; l < RT_MAXLEV; ++l) k.xs[l] = p->xs[l];
  k.Kb = p->Kb;
  k.xktab = p->xktab;
  k.koff = p->koff;
  k.pad = 0;
  return k;
}
__device__ __forceinline__ RtCol ld(const FP_CONST RtCol* p) {
  RtCol c;
  c.xbase = p->xbase;
#pragma unroll
  for (int l = 0; l < RT_MAXLEV; ++l) c.xs[l] = p->xs[l];
  return c;
}
__device__ __forceinline__ RtPair ld(const FP_CONST RtPair* p) {
  RtPair r;
  r.pk = p->pk;
  r.kblk = p->kblk;
  r.koff = p->koff;
  r.Kb = p->Kb;
  r.pad = 0;
  return r;
}

// Accumulate one output chunk (NC columns) of row r of the tile and store it.
// Staged groups read X from LDS: the tile's rows are split into 64-row
// sub-blocks, and staged column c of row r is at
// lds[((r / 64) * ktot + c) * 64 + r % 64], so a wave reads 64 consecutive
// doubles per column and successive columns sit at fixed byte offsets
// (immediate offsets of ds_read). Unstaged groups read X from global memory
// through the X block's level strides and contracted-offset table.
template <int NC, bool STAGED, class T>
__device__ __forceinline__ void rt_chunk(const T* __restrict__ X,
                                         const FP_CONST double* PK, T* __restrict__ Y,
                                         const T* __restrict__ lds, int rows, int r,
                                         const RtOut& O, const FP_CONST RtPair* pairs,
                                         const FP_CONST RtKblk* kblks,
                                         const FP_CONST int32_t* tab,
                                         const int32_t (&idx)[RT_MAXLEV], bool live) {
  double acc[NC];
#pragma unroll
  for (int n = 0; n < NC; ++n) acc[n] = 0.0;
  for (int p = O.p0; p < O.p1; ++p) {
    const RtPair P = ld(pairs + p);
    const FP_CONST double* bp = PK + P.pk;
    const int Kb = P.Kb;
    if (STAGED) {
      const T* lp = lds + P.koff * 64;
      int k = 0;
      for (; k + 4 <= Kb; k += 4) {
        const double a0 = (double)lp[(k + 0) * 64], a1 = (double)lp[(k + 1) * 64];
        const double a2 = (double)lp[(k + 2) * 64], a3 = (double)lp[(k + 3) * 64];
        const FP_CONST double* b = bp + k * NC;
#pragma unroll
        for (int n = 0; n < NC; ++n) {
          acc[n] = fma(a0, b[n], acc[n]);
          acc[n] = fma(a1, b[NC + n], acc[n]);
          acc[n] = fma(a2, b[2 * NC + n], acc[n]);
          acc[n] = fma(a3, b[3 * NC + n], acc[n]);
        }
      }
      for (; k < Kb; ++k) {
        const double a = (double)lp[k * 64];
        const FP_CONST double* b = bp + k * NC;
#pragma unroll
        for (int n = 0; n < NC; ++n) acc[n] = fma(a, b[n], acc[n]);
      }
    } else {
      const RtKblk K = ld(kblks + P.kblk);
      int32_t xo = 0;
#pragma unroll
      for (int l = 0; l < RT_MAXLEV; ++l) xo += idx[l] * K.xs[l];
      const T* xp = X + K.xbase + xo;
      const FP_CONST int32_t* kt = tab + K.xktab;
      int k = 0;
      for (; k + 4 <= Kb; k += 4) {
        const double a0 = (double)xp[kt[k]], a1 = (double)xp[kt[k + 1]];
        const double a2 = (double)xp[kt[k + 2]], a3 = (double)xp[kt[k + 3]];
        const FP_CONST double* b = bp + k * NC;
#pragma unroll
        for (int n = 0; n < NC; ++n) {
          acc[n] = fma(a0, b[n], acc[n]);
          acc[n] = fma(a1, b[NC + n], acc[n]);
          acc[n] = fma(a2, b[2 * NC + n], acc[n]);
          acc[n] = fma(a3, b[3 * NC + n], acc[n]);
        }
      }
      for (; k < Kb; ++k) {
        const double a = (double)xp[kt[k]];
        const FP_CONST double* b = bp + k * NC;
#pragma unroll
        for (int n = 0; n < NC; ++n) acc[n] = fma(a, b[n], acc[n]);
      }
    }
  }
  if (live) {
    int32_t oo = 0;
#pragma unroll
    for (int l = 0; l < RT_MAXLEV; ++l) oo += idx[l] * O.ms[l];
    T* yp = Y + O.base + oo;
    const FP_CONST int32_t* nt = tab + O.ntab;
#pragma unroll
    for (int n = 0; n < NC; ++n) yp[nt[n]] = (T)acc[n];
  }
}

template <bool STAGED, class T>
__device__ __forceinline__ void rt_chunks(const T* __restrict__ X,
                                          const FP_CONST double* PK, T* __restrict__ Y,
                                          const T* __restrict__ lds, int rows, int r,
                                          const RtGroup& G, int o_first, int o_step,
                                          const FP_CONST RtOut* outs,
                                          const FP_CONST RtPair* pairs,
                                          const FP_CONST RtKblk* kblks,
                                          const FP_CONST int32_t* tab,
                                          const int32_t (&idx)[RT_MAXLEV], bool live) {
  for (int o = G.o0 + o_first; o < G.o1; o += o_step) {
    const RtOut O = ld(outs + o);
    switch (O.nc) {
#define FP_RT_CASE(n)                                                                    \
  case n:                                                                                \
    rt_chunk<n, STAGED, T>(X, PK, Y, lds, rows, r, O, pairs, kblks, tab, idx, live); \
    break;
      FP_RT_CASE(1) FP_RT_CASE(2) FP_RT_CASE(3) FP_RT_CASE(4) FP_RT_CASE(5) FP_RT_CASE(6)
      FP_RT_CASE(7) FP_RT_CASE(8) FP_RT_CASE(9) FP_RT_CASE(10) FP_RT_CASE(11) FP_RT_CASE(12)
      FP_RT_CASE(13) FP_RT_CASE(14) FP_RT_CASE(15) FP_RT_CASE(16)
#undef FP_RT_CASE
      default:
        break;
    }
  }
}

// One chunk (NC <= RT_NC2 columns) for the two rows of a lane in a two-row
// tile: row a in sub-block 0 and row b = a + 64 in sub-block 1; every packed
// layer value feeds both products.
template <int NC, class T>
__device__ __forceinline__ void rt_chunk2(const FP_CONST double* PK, T* __restrict__ Y,
                                          const T* __restrict__ la, const T* __restrict__ lb,
                                          const RtOut& O, const FP_CONST RtPair* pairs,
                                          const FP_CONST int32_t* tab,
                                          const int32_t (&ia)[RT_MAXLEV],
                                          const int32_t (&ib)[RT_MAXLEV], bool live_a,
                                          bool live_b) {
  double acc_a[NC], acc_b[NC];
#pragma unroll
  for (int n = 0; n < NC; ++n) acc_a[n] = acc_b[n] = 0.0;
  for (int p = O.p0; p < O.p1; ++p) {
    const RtPair P = ld(pairs + p);
    const FP_CONST double* bp = PK + P.pk;
    const int Kb = P.Kb;
    const T* pa = la + P.koff * 64;
    const T* pb = lb + P.koff * 64;
    constexpr int KU = NC > 4 ? 4 : 8;
    int k = 0;
    for (; k + KU <= Kb; k += KU) {
      double xa[KU], xb[KU];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        xa[u] = (double)pa[(k + u) * 64];
        xb[u] = (double)pb[(k + u) * 64];
      }
      const FP_CONST double* b = bp + k * NC;
#pragma unroll
      for (int u = 0; u < KU; ++u)
#pragma unroll
        for (int n = 0; n < NC; ++n) {
          acc_a[n] = fma(xa[u], b[u * NC + n], acc_a[n]);
          acc_b[n] = fma(xb[u], b[u * NC + n], acc_b[n]);
        }
    }
    for (; k < Kb; ++k) {
      const double xa = (double)pa[k * 64], xb = (double)pb[k * 64];
      const FP_CONST double* b = bp + k * NC;
#pragma unroll
      for (int n = 0; n < NC; ++n) {
        acc_a[n] = fma(xa, b[n], acc_a[n]);
        acc_b[n] = fma(xb, b[n], acc_b[n]);
      }
    }
  }
  const FP_CONST int32_t* nt = tab + O.ntab;
  if (live_a) {
    int32_t oo = 0;
#pragma unroll
    for (int l = 0; l < RT_MAXLEV; ++l) oo += ia[l] * O.ms[l];
    T* yp = Y + O.base + oo;
#pragma unroll
    for (int n = 0; n < NC; ++n) yp[nt[n]] = (T)acc_a[n];
  }
  if (live_b) {
    int32_t oo = 0;
#pragma unroll
    for (int l = 0; l < RT_MAXLEV; ++l) oo += ib[l] * O.ms[l];
    T* yp = Y + O.base + oo;
#pragma unroll
    for (int n = 0; n < NC; ++n) yp[nt[n]] = (T)acc_b[n];
  }
}

// Level indices of row m (m < 2^31): division by the level dims through
// their multiply-high constants (no integer division instructions).
__device__ __forceinline__ void row_levels(const RtGroup& G, int m, int32_t (&idx)[RT_MAXLEV]) {
  uint32_t r = (uint32_t)m;
#pragma unroll
  for (int l = RT_MAXLEV - 1; l >= 0; --l) {
    if (G.md[l] == 1) {
      idx[l] = 0;
      continue;
    }
    const uint32_t q = (uint32_t)__umul64hi((uint64_t)r, G.mg[l]);
    idx[l] = (int32_t)(r - q * (uint32_t)G.md[l]);
    r = q;
  }
}

// Loads each thread keeps in flight while staging X rows into LDS (16
// measured 1% faster over the layer steps of a row than 8).
constexpr int RT_STAGE_BATCH = 16;

template <class T>
__global__ __launch_bounds__(RT_THREADS) void k_rt_f64(
    const T* __restrict__ X, const double* __restrict__ PK_, T* __restrict__ Y,
    const RtGroup* __restrict__ groups_, const int32_t* __restrict__ tile_group,
    const RtOut* __restrict__ outs_,
    const RtKblk* __restrict__ kblks_, const RtCol* __restrict__ cols_,
    const RtPair* __restrict__ pairs_, const int32_t* __restrict__ tab_, int tile_base, int swz) {
  extern __shared__ double lds_raw[];
  T* lds = (T*)lds_raw;
  const FP_CONST RtGroup* groups = as_const(groups_);
  const FP_CONST RtOut* outs = as_const(outs_);
  const FP_CONST RtKblk* kblks = as_const(kblks_);
  const FP_CONST RtCol* cols = as_const(cols_);
  const FP_CONST RtPair* pairs = as_const(pairs_);
  const FP_CONST int32_t* tab = as_const(tab_);
  const FP_CONST double* PK = as_const(PK_);
  const int wg = tile_base + xcd_swizzle((int)blockIdx.x, (int)gridDim.x, swz);
  const RtGroup G = ld(groups + as_const(tile_group)[wg]);
  const int rows = G.rows;                    // 64, 128 or 256
  const int m0 = (wg - G.tile0) * rows;
  const int tid = threadIdx.x;
  // thread tid stages and computes the same tile row r = tid % rows
  // (= (wave % (rows/64)) * 64 + lane); rows past the group end repeat row
  // M-1 (in bounds, never stored)
  const int lrows = 31 - __builtin_clz(rows);  // rows is a power of two
  const int r = tid & (rows - 1);
  const int m = m0 + r;
  const bool live = m < G.M;
  int32_t idx[RT_MAXLEV];
  row_levels(G, live ? m : G.M - 1, idx);
  if (G.staged) {
    // stage the staged columns slot, slot + nslot, ... (slot = tid / rows
    // is uniform per wave), RT_STAGE_BATCH loads in flight per batch
    const int nslot = RT_THREADS >> lrows;
    const int slot = __builtin_amdgcn_readfirstlane(tid >> lrows);
    const FP_CONST RtCol* gc = cols + G.c0;
    T* lst = lds + (r >> 6) * G.ktot * 64 + (r & 63);
    constexpr int SB = RT_STAGE_BATCH;
    for (int c0 = slot; c0 < G.ktot; c0 += SB * nslot) {
      // descriptors of the batch first (clamped: always valid), then the
      // loads, then the LDS writes
      RtCol C[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) C[u] = ld(gc + min(c0 + u * nslot, G.ktot - 1));
      double v[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        int32_t xo = 0;
#pragma unroll
        for (int l = 0; l < RT_MAXLEV; ++l) xo += idx[l] * C[u].xs[l];
        v[u] = (double)X[C[u].xbase + xo];
      }
#pragma unroll
      for (int u = 0; u < SB; ++u) {
        const int c = c0 + u * nslot;
        if (c < G.ktot) lst[c * 64] = (T)v[u];
      }
    }
    __syncthreads();
  }
  // compute: wave w owns tile rows (w % (rows/64)) * 64 + lane and the
  // output chunks o0 + w / (rows/64), stepping by 4 / (rows/64); the wave
  // index is uniform per wave: say so, so that the chunk loop and
  // everything it loads stay scalar
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (G.staged == 2) {
    // two-row tile (128 rows): lane rows m0 + lane and m0 + 64 + lane (rows
    // past the group end repeat row M - 1, never stored); wave w takes
    // chunks o0 + w, o0 + w + 4, ...
    const int lane = tid & 63;
    const int ma = m0 + lane, mb = m0 + 64 + lane;
    const bool live_a = ma < G.M, live_b = mb < G.M;
    int32_t ia[RT_MAXLEV], ib[RT_MAXLEV];
    row_levels(G, live_a ? ma : G.M - 1, ia);
    row_levels(G, live_b ? mb : G.M - 1, ib);
    const T* la = lds + lane;
    const T* lb = lds + G.ktot * 64 + lane;
    for (int o = G.o0 + wave; o < G.o1; o += 4) {
      const RtOut O = ld(outs + o);
      switch (O.nc) {
#define FP_RT2_CASE(n)                                                                   \
  case n:                                                                                \
    rt_chunk2<n, T>(PK, Y, la, lb, O, pairs, tab, ia, ib, live_a, live_b);               \
    break;
        FP_RT2_CASE(1) FP_RT2_CASE(2) FP_RT2_CASE(3) FP_RT2_CASE(4) FP_RT2_CASE(5)
        FP_RT2_CASE(6) FP_RT2_CASE(7) FP_RT2_CASE(8)
#undef FP_RT2_CASE
        default:
          break;
      }
    }
    return;
  }
  const int lsub = lrows - 6;                  // log2(rows / 64)
  const int o_first = wave >> lsub, o_step = 4 >> lsub;
  // this lane's row inside the staged tile: sub-block r / 64, lane r % 64
  const T* lrow = lds + (r >> 6) * G.ktot * 64 + (r & 63);
  if (G.staged)
    rt_chunks<true, T>(X, PK, Y, lrow, rows, r, G, o_first, o_step, outs, pairs, kblks, tab, idx,
                    live);
  else
    rt_chunks<false, T>(X, PK, Y, lrow, rows, r, G, o_first, o_step, outs, pairs, kblks, tab, idx,
                     live);
}

__global__ void k_tile_group(const RtGroup* __restrict__ groups, int g_first,
                             int32_t* __restrict__ tile_group) {
  const int g = g_first + (int)blockIdx.x;
  const RtGroup G = groups[g];
  const int nt = (G.M + G.rows - 1) / G.rows;
  for (int i = threadIdx.x; i < nt; i += blockDim.x) tile_group[G.tile0 + i] = g;
}

hipError_t launch_tile_group(const RtGroup* groups, int g_first, int ngroups, int32_t* tile_group,
                             hipStream_t s) {
  if (ngroups <= 0) return hipSuccess;
  k_tile_group<<<dim3(ngroups), dim3(256), 0, s>>>(groups, g_first, tile_group);
  return hipGetLastError();
}

__global__ void k_rt_pack(const RtPack* __restrict__ packs, const double* __restrict__ S,
                          const int32_t* __restrict__ tab, double* __restrict__ PK) {
  const RtPack P = packs[blockIdx.x];
  const int n = P.Kb * P.nc;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int k = e / P.nc, c = e % P.nc;
    PK[P.dst + e] = P.alpha * S[P.sbase + tab[P.sktab + k] + tab[P.sntab + c]];
  }
}

// One contiguous range of tiles per XCD: neighbouring tiles of a row group
// share its plan data and packed layer blocks in that XCD's L2.
constexpr int LAYER_XCD_RUN = 0;

hipError_t launch_rt_f64(const DevRt& r, int c, const void* X, bool f32, const double* PK,
                         void* Y, const int32_t* tab, hipStream_t s) {
  if (c < 0 || c >= r.nlaunch || r.ngroups <= 0) return hipErrorInvalidValue;
  if (r.l_lds[c] < 0 || r.l_lds[c] > RT_LDS_BYTES || r.l_ntiles[c] <= 0) return hipErrorInvalidValue;
  // the plan sizes LDS for double; FP32 staging takes half
  if (f32)
    k_rt_f64<float><<<dim3(r.l_ntiles[c]), dim3(RT_THREADS), (size_t)r.l_lds[c] / 2, s>>>(
        (const float*)X, PK, (float*)Y, r.groups, r.tile_group, r.outs, r.kblks, r.cols, r.pairs,
        tab, r.l_tile0[c], LAYER_XCD_RUN);
  else
    k_rt_f64<double><<<dim3(r.l_ntiles[c]), dim3(RT_THREADS), (size_t)r.l_lds[c], s>>>(
        (const double*)X, PK, (double*)Y, r.groups, r.tile_group, r.outs, r.kblks, r.cols,
        r.pairs, tab, r.l_tile0[c], LAYER_XCD_RUN);
  return hipGetLastError();
}

hipError_t launch_rt_pack(const DevRt& r, const double* S, const int32_t* tab, double* PK,
                          hipStream_t s) {
  if (r.npacks <= 0) return hipSuccess;
  k_rt_pack<<<dim3(r.npacks), dim3(64), 0, s>>>(r.packs, S, tab, PK);
  return hipGetLastError();
}

}  // namespace fp
