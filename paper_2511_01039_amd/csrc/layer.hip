// Layer steps of the chain (ket, PEPO and bra contracted into the
// sketch-side intermediate, and their transposes), FP64.
//
// These products have a huge row count (environment x sketch indices) and
// tiny contracted/column extents (a few virtual or physical indices), so
// they are bound by HBM traffic, not by arithmetic. One thread owns one row
// of one row group (fixed sectors on the free legs of X): it reads each of
// its input values once per column chunk, multiplies them into NC
// register accumulators against the packed, scalar-scaled layer sub-block
// (wave-uniform addresses, served by the scalar data path), and writes
// every output value once. Rows are numbered with the sketch column index
// innermost, which is stride-1 in every intermediate, so loads and stores
// of a wave are contiguous runs.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fp {

template <int NC>
__device__ __forceinline__ void rt_chunk(const double* __restrict__ X,
                                         const double* __restrict__ PK, double* __restrict__ Y,
                                         const RtOut& O, const RtPair* __restrict__ pairs,
                                         const int32_t* __restrict__ tab,
                                         const int32_t (&idx)[RT_MAXLEV], bool live) {
  double acc[NC];
#pragma unroll
  for (int n = 0; n < NC; ++n) acc[n] = 0.0;
  for (int p = O.p0; p < O.p1; ++p) {
    const RtPair P = pairs[p];
    int32_t xo = 0;
#pragma unroll
    for (int l = 0; l < RT_MAXLEV; ++l) xo += idx[l] * P.xs[l];
    const double* xp = X + P.xbase + xo;
    const int32_t* kt = tab + P.xktab;
    const double* bp = PK + P.pk;
    const int Kb = P.Kb;
    // eight independent loads in flight per batch (Kb is wave-uniform, so
    // the guards are scalar branches)
    for (int k0 = 0; k0 < Kb; k0 += 8) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = (k0 + u < Kb) ? xp[kt[k0 + u]] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (k0 + u < Kb) {
          const double* b = bp + (k0 + u) * NC;
#pragma unroll
          for (int n = 0; n < NC; ++n) acc[n] = fma(a[u], b[n], acc[n]);
        }
      }
    }
  }
  if (live) {
    int32_t oo = 0;
#pragma unroll
    for (int l = 0; l < RT_MAXLEV; ++l) oo += idx[l] * O.ms[l];
    double* yp = Y + O.base + oo;
    const int32_t* nt = tab + O.ntab;
#pragma unroll
    for (int n = 0; n < NC; ++n) yp[nt[n]] = acc[n];
  }
}

__global__ __launch_bounds__(RT_ROWS) void k_rt_f64(const double* __restrict__ X,
                                                    const double* __restrict__ PK,
                                                    double* __restrict__ Y,
                                                    const RtGroup* __restrict__ groups,
                                                    int ngroups, const RtOut* __restrict__ outs,
                                                    const RtPair* __restrict__ pairs,
                                                    const int32_t* __restrict__ tab) {
  const int wg = blockIdx.x;
  int lo = 0, hi = ngroups - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (groups[mid].tile0 <= wg)
      lo = mid;
    else
      hi = mid - 1;
  }
  const RtGroup G = groups[lo];
  const int m = (wg - G.tile0) * RT_ROWS + (int)threadIdx.x;
  const bool live = m < G.M;
  // rows past the group end compute row M-1 (in bounds) and store nothing
  int r = live ? m : G.M - 1;
  int32_t idx[RT_MAXLEV];
#pragma unroll
  for (int l = RT_MAXLEV - 1; l >= 0; --l) {
    const int d = G.md[l];
    idx[l] = r % d;
    r /= d;
  }
  for (int o = G.o0; o < G.o1; ++o) {
    const RtOut O = outs[o];
    switch (O.nc) {
#define FP_RT_CASE(n) \
  case n:             \
    rt_chunk<n>(X, PK, Y, O, pairs, tab, idx, live); \
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

__global__ void k_rt_pack(const RtPack* __restrict__ packs, const double* __restrict__ S,
                          const int32_t* __restrict__ tab, double* __restrict__ PK) {
  const RtPack P = packs[blockIdx.x];
  const int n = P.Kb * P.nc;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int k = e / P.nc, c = e % P.nc;
    PK[P.dst + e] = P.alpha * S[P.sbase + tab[P.sktab + k] + tab[P.sntab + c]];
  }
}

hipError_t launch_rt_f64(const DevRt& r, const double* X, const double* PK, double* Y,
                         const int32_t* tab, hipStream_t s) {
  if (r.ntiles <= 0 || r.ngroups <= 0) return hipSuccess;
  k_rt_f64<<<dim3(r.ntiles), dim3(RT_ROWS), 0, s>>>(X, PK, Y, r.groups, r.ngroups, r.outs,
                                                   r.pairs, tab);
  return hipGetLastError();
}

hipError_t launch_rt_pack(const DevRt& r, const double* S, const int32_t* tab, double* PK,
                          hipStream_t s) {
  if (r.npacks <= 0) return hipSuccess;
  k_rt_pack<<<dim3(r.npacks), dim3(64), 0, s>>>(r.packs, S, tab, PK);
  return hipGetLastError();
}

}  // namespace fp
