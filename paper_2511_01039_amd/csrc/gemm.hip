// Grouped, table-addressed GEMM on FP64 MFMA (gfx950).
//
// One workgroup owns one output tile of one output block and accumulates,
// in registers, every block pair that contributes to it (the disjoint
// output slices of Sec. 3 need no atomics). Operand elements are addressed
// through per-pair offset tables, so any leg permutation of a block is read
// in place: A(m, k) = A[a_off + tam[m] + tak[k]], B(k, n) likewise, and the
// tile is written to C[c_off + tcm[m] + tcn[n]].
//
// Tiles are staged through LDS (KT = 16 deep); each of the four waves runs
// v_mfma_f64_16x16x4f64 on its sub-tile. Register layout of that
// instruction (checked on the device): A[i][k] in lane i + 16k, B[k][j] in
// lane j + 16k, result register r of lane l holds D[4r + l/16][l % 16].
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fp {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int MT, int NT, int WM, int WN>
__global__ __launch_bounds__(256) void k_gemm_f64(const double* __restrict__ A,
                                                  const double* __restrict__ B,
                                                  double* __restrict__ C,
                                                  const GemmJob* __restrict__ jobs,
                                                  const GemmPair* __restrict__ pairs,
                                                  const int32_t* __restrict__ tab) {
  constexpr int KT = 16;
  constexpr int WTM = MT / WM, WTN = NT / WN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  static_assert(WM * WN == 4, "four waves");
  static_assert(FM >= 1 && FN >= 1, "wave tile at least 16x16");
  __shared__ double sA[KT][MT + 1];
  __shared__ double sB[KT][NT + 1];

  const GemmJob job = jobs[blockIdx.x];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int lrow = lane & 15, lk = lane >> 4;

  d4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  for (int p = job.p0; p < job.p1; ++p) {
    const GemmPair pr = pairs[p];
    const int kbeg = job.k0 > 0 ? job.k0 : 0;
    const int kend = job.k1 < pr.K ? job.k1 : pr.K;
    const double* Ab = A + pr.a_off;
    const double* Bb = B + pr.b_off;
    const int32_t* tam = tab + pr.tam;
    const int32_t* tak = tab + pr.tak;
    const int32_t* tbk = tab + pr.tbk;
    const int32_t* tbn = tab + pr.tbn;
    const bool a_kfast = pr.flags & 1;
    const bool b_nfast = pr.flags & 2;
    for (int kb = kbeg; kb < kend; kb += KT) {
#pragma unroll
      for (int i = 0; i < (MT * KT) / 256; ++i) {
        const int e = tid + i * 256;
        int mm, kk;
        if (a_kfast) {
          kk = e % KT;
          mm = e / KT;
        } else {
          mm = e % MT;
          kk = e / MT;
        }
        const int m = job.m0 + mm, k = kb + kk;
        double v = 0.0;
        if (m < job.M && k < kend) v = Ab[(int64_t)tam[m] + tak[k]];
        sA[kk][mm] = v * pr.alpha;
      }
#pragma unroll
      for (int i = 0; i < (NT * KT) / 256; ++i) {
        const int e = tid + i * 256;
        int nn, kk;
        if (b_nfast) {
          nn = e % NT;
          kk = e / NT;
        } else {
          kk = e % KT;
          nn = e / KT;
        }
        const int n = job.n0 + nn, k = kb + kk;
        double v = 0.0;
        if (n < job.N && k < kend) v = Bb[(int64_t)tbk[k] + tbn[n]];
        sB[kk][nn] = v;
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < KT; kk += 4) {
        double a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = sA[kk + lk][wm * WTM + i * 16 + lrow];
#pragma unroll
        for (int j = 0; j < FN; ++j) b[j] = sB[kk + lk][wn * WTN + j * 16 + lrow];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      __syncthreads();
    }
  }

  const int32_t* tcm = tab + job.tcm;
  const int32_t* tcn = tab + job.tcn;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = job.m0 + wm * WTM + i * 16 + 4 * r + lk;
        const int n = job.n0 + wn * WTN + j * 16 + lrow;
        if (m < job.M && n < job.N) C[job.c_off + (int64_t)tcm[m] + tcn[n]] = acc[i][j][r];
      }
}

hipError_t launch_gemm_f64(const DevGemm& g, const double* A, const double* B, double* C,
                           const int32_t* tables, hipStream_t s) {
  if (g.njobs <= 0) return hipSuccess;
  dim3 grid(g.njobs), block(256);
  if (g.mt == 64 && g.nt == 64)
    k_gemm_f64<64, 64, 2, 2><<<grid, block, 0, s>>>(A, B, C, g.jobs, g.pairs, tables);
  else if (g.mt == 128 && g.nt == 32)
    k_gemm_f64<128, 32, 4, 1><<<grid, block, 0, s>>>(A, B, C, g.jobs, g.pairs, tables);
  else if (g.mt == 32 && g.nt == 128)
    k_gemm_f64<32, 128, 1, 4><<<grid, block, 0, s>>>(A, B, C, g.jobs, g.pairs, tables);
  else if (g.mt == 256 && g.nt == 16)
    k_gemm_f64<256, 16, 4, 1><<<grid, block, 0, s>>>(A, B, C, g.jobs, g.pairs, tables);
  else if (g.mt == 16 && g.nt == 256)
    k_gemm_f64<16, 256, 1, 4><<<grid, block, 0, s>>>(A, B, C, g.jobs, g.pairs, tables);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

__global__ void k_reduce_partials(const ReduceDesc* __restrict__ d, double* __restrict__ C,
                                  const double* __restrict__ P) {
  const ReduceDesc r = d[blockIdx.y];
  const int64_t mn = (int64_t)r.M * r.N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mn;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int q = 0; q < r.nsplit; ++q) s += P[r.p_off + (int64_t)q * mn + e];
    const int64_t m = e / r.N, n = e % r.N;
    C[r.c_off + m * r.c_rs + n * r.c_cs] = s;
  }
}

hipError_t launch_reduce_partials(const ReduceDesc* d, int nd, int max_mn, double* C,
                                  const double* P, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  int bx = (max_mn + 255) / 256;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  k_reduce_partials<<<dim3(bx, nd), 256, 0, s>>>(d, C, P);
  return hipGetLastError();
}

}  // namespace fp
