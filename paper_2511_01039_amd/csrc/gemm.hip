// Grouped, table-addressed GEMM on FP64 MFMA (gfx950).
//
// One workgroup owns one output tile of one output block and accumulates,
// in registers, every block pair that contributes to it (the disjoint
// output slices of Sec. 3 need no atomics). Operand elements are addressed
// through per-pair offset tables, so any leg permutation of a block is read
// in place: A(m, k) = A[a_off + tam[m] + tak[k]], B(k, n) likewise, and the
// tile is written to C[c_off + tcm[m] + tcn[n]].
//
// Tiles are staged through LDS (KT = 16 deep, double-buffered); each of the
// four waves runs v_mfma_f64_16x16x4f64 (FP64) or v_mfma_f32_16x16x4f32
// (FP32 operands, FP32 accumulation inside each 16-deep K tile, the tiles
// summed in FP64) on its sub-tile. Register layouts
// (checked on the device): A[i][k] in lane i + 16k, B[k][j] in lane j + 16k;
// result register r of lane l holds D[4r + l/16][l % 16] for the FP64
// instruction and D[4(l/16) + r][l % 16] for the FP32 one.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace fp {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// The matrix instruction of each compute type.
template <class TM>
struct Mfma;
template <>
struct Mfma<double> {
  typedef d4 acc;
  static __device__ __forceinline__ acc zero() { return d4{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the 16 x 16 result held by register r of a lane in lane group lk
  static __device__ __forceinline__ int row(int r, int lk) { return 4 * r + lk; }
};
template <>
struct Mfma<float> {
  typedef f4 acc;
  static __device__ __forceinline__ acc zero() { return f4{0.0f, 0.0f, 0.0f, 0.0f}; }
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int lk) { return 4 * lk + r; }
};

// Position of one K tile in a job's sequence of (pair, K range) tiles.
struct TileCursor {
  int p;    // pair index
  int kb;   // first K of the tile
};

template <int MT, int NT, int KT, class TM>
struct TileRegs {
  TM a[(MT * KT) / 256];
  TM b[(NT * KT) / 256];
  TM alpha;
  uint32_t valid;   // bit i: a[i] in range; bit NA + i: b[i] in range
  bool akf, bnf;
};

template <int MT, int NT, int KT, class TA, class TB, class TM>
__device__ __forceinline__ void load_tile(const TA* __restrict__ A,
                                          const TB* __restrict__ B,
                                          const GemmPair* __restrict__ pairs,
                                          const int32_t* __restrict__ tab, const GemmJob& job,
                                          const TileCursor& t, int tid,
                                          TileRegs<MT, NT, KT, TM>& r) {
  const GemmPair pr = pairs[t.p];
  const int kend = job.k1 < pr.K ? job.k1 : pr.K;
  const TA* Ab = A + pr.a_off;
  const TB* Bb = B + pr.b_off;
  const int32_t* tam = tab + pr.tam;
  const int32_t* tak = tab + pr.tak;
  const int32_t* tbk = tab + pr.tbk;
  const int32_t* tbn = tab + pr.tbn;
  r.akf = pr.flags & 1;
  r.bnf = pr.flags & 2;
  // branch-free: indices are clamped into the block (always a valid
  // address), every table and data load of the tile is issued before any is
  // used, and out-of-range elements are zeroed when the tile is stored to LDS
  // (after the current tile's products, so the loads stay in flight meanwhile).
  // Element i of a thread is e = tid + 256 i of the tile. With A contiguous
  // along K (akf) it is (m, k) = (e / KT, e % KT), else (e % MT, e / MT); as
  // MT, KT and 256 / KT divide 256, one of the two indices is the same for
  // all i, and its table entry is loaded once. B likewise. A table that is a
  // row-major run (stride s > 0 in the pair) is not read at all: entry i is
  // i * s.
  constexpr int NA = (MT * KT) / 256, NB = (NT * KT) / 256;
  static_assert(NA + NB <= 32, "validity mask");
  static_assert(256 % MT == 0 && 256 % NT == 0 && 256 % KT == 0, "tile divides 256");
  int32_t oa[NA], ob[NB];
  uint32_t valid = 0;
  if (r.akf) {
    const int k = t.kb + tid % KT, kc = min(k, kend - 1);
    const int32_t ok = pr.sak > 0 ? kc * pr.sak : tak[kc];
    const bool kv = k < kend;
    int mc[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int m = job.m0 + tid / KT + i * (256 / KT);
      valid |= (m < job.M && kv) ? (1u << i) : 0u;
      mc[i] = min(m, job.M - 1);
    }
    if (pr.sam > 0) {
#pragma unroll
      for (int i = 0; i < NA; ++i) oa[i] = mc[i] * pr.sam + ok;
    } else {
#pragma unroll
      for (int i = 0; i < NA; ++i) oa[i] = tam[mc[i]] + ok;
    }
  } else {
    const int m = job.m0 + tid % MT, mc = min(m, job.M - 1);
    const int32_t om = pr.sam > 0 ? mc * pr.sam : tam[mc];
    const bool mv = m < job.M;
    int kc[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int k = t.kb + tid / MT + i * (256 / MT);
      valid |= (mv && k < kend) ? (1u << i) : 0u;
      kc[i] = min(k, kend - 1);
    }
    if (pr.sak > 0) {
#pragma unroll
      for (int i = 0; i < NA; ++i) oa[i] = om + kc[i] * pr.sak;
    } else {
#pragma unroll
      for (int i = 0; i < NA; ++i) oa[i] = om + tak[kc[i]];
    }
  }
  if (r.bnf) {
    const int n = job.n0 + tid % NT, nc = min(n, job.N - 1);
    const int32_t on = pr.sbn > 0 ? nc * pr.sbn : tbn[nc];
    const bool nv = n < job.N;
    int kc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int k = t.kb + tid / NT + i * (256 / NT);
      valid |= (nv && k < kend) ? (1u << (NA + i)) : 0u;
      kc[i] = min(k, kend - 1);
    }
    if (pr.sbk > 0) {
#pragma unroll
      for (int i = 0; i < NB; ++i) ob[i] = kc[i] * pr.sbk + on;
    } else {
#pragma unroll
      for (int i = 0; i < NB; ++i) ob[i] = tbk[kc[i]] + on;
    }
  } else {
    const int k = t.kb + tid % KT, kc = min(k, kend - 1);
    const int32_t ok = pr.sbk > 0 ? kc * pr.sbk : tbk[kc];
    const bool kv = k < kend;
    int nc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int n = job.n0 + tid / KT + i * (256 / KT);
      valid |= (n < job.N && kv) ? (1u << (NA + i)) : 0u;
      nc[i] = min(n, job.N - 1);
    }
    if (pr.sbn > 0) {
#pragma unroll
      for (int i = 0; i < NB; ++i) ob[i] = ok + nc[i] * pr.sbn;
    } else {
#pragma unroll
      for (int i = 0; i < NB; ++i) ob[i] = ok + tbn[nc[i]];
    }
  }
#pragma unroll
  for (int i = 0; i < NA; ++i) r.a[i] = (TM)Ab[oa[i]];
#pragma unroll
  for (int i = 0; i < NB; ++i) r.b[i] = (TM)Bb[ob[i]];
  r.alpha = (TM)pr.alpha;
  r.valid = valid;
}

template <int MT, int NT, int KT, class TM>
__device__ __forceinline__ void store_tile(TM (*sA)[MT + 1], TM (*sB)[NT + 1], int tid,
                                           const TileRegs<MT, NT, KT, TM>& r) {
  constexpr int NA = (MT * KT) / 256;
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int e = tid + i * 256;
    const int mm = r.akf ? e / KT : e % MT;
    const int kk = r.akf ? e % KT : e / MT;
    sA[kk][mm] = (r.valid >> i) & 1u ? r.a[i] * r.alpha : (TM)0;
  }
#pragma unroll
  for (int i = 0; i < (NT * KT) / 256; ++i) {
    const int e = tid + i * 256;
    const int nn = r.bnf ? e % NT : e / KT;
    const int kk = r.bnf ? e / NT : e % KT;
    sB[kk][nn] = (r.valid >> (NA + i)) & 1u ? r.b[i] : (TM)0;
  }
}

// Next tile of the job; false at the end.
__device__ __forceinline__ bool next_tile(const GemmPair* __restrict__ pairs, const GemmJob& job,
                                          TileCursor& t, int KT) {
  const int kend = job.k1 < pairs[t.p].K ? job.k1 : pairs[t.p].K;
  t.kb += KT;
  if (t.kb < kend) return true;
  for (++t.p; t.p < job.p1; ++t.p) {
    t.kb = job.k0 > 0 ? job.k0 : 0;
    const int ke = job.k1 < pairs[t.p].K ? job.k1 : pairs[t.p].K;
    if (t.kb < ke) return true;
  }
  return false;
}

// One workgroup (four waves, WM x WN) per output tile; K tiles are
// prefetched into registers while the previous tile is multiplied out of
// LDS (double-buffered, one barrier per tile). TM is the compute type (the
// MFMA operand and accumulator type).
template <int MT, int NT, int WM, int WN, class TA, class TB, class TC, class TM>
__device__ __forceinline__ void gemm_tile(const TA* __restrict__ A, const TB* __restrict__ B,
                                          TC* __restrict__ C, const GemmJob* __restrict__ jobs,
                                          const GemmPair* __restrict__ pairs,
                                          const int32_t* __restrict__ tab, int swz,
                                          TM (*sA)[16][MT + 1], TM (*sB)[16][NT + 1]) {
  constexpr int KT = 16;
  constexpr int WTM = MT / WM, WTN = NT / WN;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  static_assert(WM * WN == 4, "four waves");
  static_assert(FM >= 1 && FN >= 1, "wave tile at least 16x16");
  static_assert((MT * KT) % 256 == 0 && (NT * KT) % 256 == 0, "tile loads cover 256 threads");
  typedef Mfma<TM> MF;

  const GemmJob job = jobs[xcd_swizzle((int)blockIdx.x, (int)gridDim.x, swz)];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int lrow = lane & 15, lk = lane >> 4;

  typename MF::acc acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = MF::zero();
  // FP32 MFMA: each 16-deep K tile accumulates in FP32 on the matrix core,
  // the tiles are summed in FP64 (the rounding of the sum then does not grow
  // with the contracted length)
  constexpr bool kSplit = sizeof(TM) == 4;
  d4 acc64[kSplit ? FM : 1][kSplit ? FN : 1];
  if constexpr (kSplit) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc64[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  }

  // first tile of the job (jobs without any tile write zeros)
  TileCursor cur{job.p0, job.k0 > 0 ? job.k0 : 0};
  bool have = false;
  for (; cur.p < job.p1; ++cur.p) {
    const int ke = job.k1 < pairs[cur.p].K ? job.k1 : pairs[cur.p].K;
    if (cur.kb < ke) {
      have = true;
      break;
    }
    cur.kb = job.k0 > 0 ? job.k0 : 0;
  }
  if (have) {
    TileRegs<MT, NT, KT, TM> regs;
    load_tile<MT, NT, KT, TA, TB, TM>(A, B, pairs, tab, job, cur, tid, regs);
    store_tile<MT, NT, KT, TM>(sA[0], sB[0], tid, regs);
    __syncthreads();
    int buf = 0;
    while (true) {
      const bool more = next_tile(pairs, job, cur, KT);
      if (more) load_tile<MT, NT, KT, TA, TB, TM>(A, B, pairs, tab, job, cur, tid, regs);
#pragma unroll
      for (int kk = 0; kk < KT; kk += 4) {
        TM a[FM], b[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) a[i] = sA[buf][kk + lk][wm * WTM + i * 16 + lrow];
#pragma unroll
        for (int j = 0; j < FN; ++j) b[j] = sB[buf][kk + lk][wn * WTN + j * 16 + lrow];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[i][j] = MF::run(a[i], b[j], acc[i][j]);
      }
      if constexpr (kSplit) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
            acc[i][j] = MF::zero();
          }
      }
      if (!more) break;
      store_tile<MT, NT, KT, TM>(sA[buf ^ 1], sB[buf ^ 1], tid, regs);
      __syncthreads();
      buf ^= 1;
    }
  }

  // epilogue: the thread's FM*4 row offsets and FN column offsets are
  // loaded once (clamped, branch-free); the stores are predicated
  const int32_t* tcm = tab + job.tcm;
  const int32_t* tcn = tab + job.tcn;
  int32_t om[FM][4], on[FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = job.m0 + wm * WTM + i * 16 + MF::row(r, lk);
      om[i][r] = tcm[min(m, job.M - 1)];
    }
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int n = job.n0 + wn * WTN + j * 16 + lrow;
    on[j] = tcn[min(n, job.N - 1)];
  }
  TC* Cb = C + job.c_off;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = job.m0 + wm * WTM + i * 16 + MF::row(r, lk);
        const int n = job.n0 + wn * WTN + j * 16 + lrow;
        if (m < job.M && n < job.N) {
          if constexpr (kSplit)
            Cb[(int64_t)om[i][r] + on[j]] = (TC)acc64[i][j][r];
          else
            Cb[(int64_t)om[i][r] + on[j]] = (TC)acc[i][j][r];
        }
      }
}

template <int MT, int NT, int WM, int WN, class TB, class TC>
__global__ __launch_bounds__(256, 2) void k_gemm_f64(const double* __restrict__ A,
                                                  const TB* __restrict__ B,
                                                  TC* __restrict__ C,
                                                  const GemmJob* __restrict__ jobs,
                                                  const GemmPair* __restrict__ pairs,
                                                  const int32_t* __restrict__ tab, int swz) {
  __shared__ double sA[2][16][MT + 1];
  __shared__ double sB[2][16][NT + 1];
  gemm_tile<MT, NT, WM, WN, double, TB, TC, double>(A, B, C, jobs, pairs, tab, swz, sA, sB);
}

// FP32 operands (A an FP32 copy), FP32 MFMA, FP32 accumulation.
template <int MT, int NT, int WM, int WN, class TB, class TC>
__global__ __launch_bounds__(256, 2) void k_gemm_f32(const float* __restrict__ A,
                                                  const TB* __restrict__ B,
                                                  TC* __restrict__ C,
                                                  const GemmJob* __restrict__ jobs,
                                                  const GemmPair* __restrict__ pairs,
                                                  const int32_t* __restrict__ tab, int swz) {
  __shared__ float sA[2][16][MT + 1];
  __shared__ float sB[2][16][NT + 1];
  gemm_tile<MT, NT, WM, WN, float, TB, TC, float>(A, B, C, jobs, pairs, tab, swz, sA, sB);
}

// Runs of 4 consecutive jobs per XCD: larger runs (or one contiguous range
// per XCD) leave long-K split blocks on a few XCDs and unbalance the launch.
constexpr int GEMM_XCD_RUN = 4;

template <class TB, class TC>
static hipError_t launch_typed(const DevGemm& g, const double* A, const TB* B, TC* C,
                               const int32_t* tables, hipStream_t s) {
  dim3 grid(g.njobs), block(256);
#define FP_GEMM_TILE(mt_, nt_, wm_, wn_)                                                 \
  if (g.mt == mt_ && g.nt == nt_) {                                                      \
    k_gemm_f64<mt_, nt_, wm_, wn_, TB, TC>                                               \
        <<<grid, block, 0, s>>>(A, B, C, g.jobs, g.pairs, tables, GEMM_XCD_RUN); \
    return hipGetLastError();                                                            \
  }
  FP_GEMM_TILE(128, 128, 2, 2)
  FP_GEMM_TILE(128, 64, 2, 2)
  FP_GEMM_TILE(64, 128, 2, 2)
  FP_GEMM_TILE(64, 64, 2, 2)
  FP_GEMM_TILE(128, 32, 4, 1)
  FP_GEMM_TILE(32, 128, 1, 4)
  FP_GEMM_TILE(256, 16, 4, 1)
  FP_GEMM_TILE(16, 256, 1, 4)
#undef FP_GEMM_TILE
  return hipErrorInvalidValue;
}

template <class TB, class TC>
static hipError_t launch_typed_f32(const DevGemm& g, const float* A, const TB* B, TC* C,
                                   const int32_t* tables, hipStream_t s) {
  dim3 grid(g.njobs), block(256);
#define FP_GEMM_TILE(mt_, nt_, wm_, wn_)                                                 \
  if (g.mt == mt_ && g.nt == nt_) {                                                      \
    k_gemm_f32<mt_, nt_, wm_, wn_, TB, TC>                                               \
        <<<grid, block, 0, s>>>(A, B, C, g.jobs, g.pairs, tables, GEMM_XCD_RUN); \
    return hipGetLastError();                                                            \
  }
  FP_GEMM_TILE(128, 128, 2, 2)
  FP_GEMM_TILE(128, 64, 2, 2)
  FP_GEMM_TILE(64, 128, 2, 2)
  FP_GEMM_TILE(64, 64, 2, 2)
  FP_GEMM_TILE(128, 32, 4, 1)
  FP_GEMM_TILE(32, 128, 1, 4)
  FP_GEMM_TILE(256, 16, 4, 1)
  FP_GEMM_TILE(16, 256, 1, 4)
#undef FP_GEMM_TILE
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_f32(const DevGemm& g, const float* A, const void* B, bool b_f32, void* C,
                           bool c_f32, const int32_t* tables, hipStream_t s) {
  if (g.njobs <= 0) return hipSuccess;
  if (b_f32 && !c_f32)
    return launch_typed_f32<float, double>(g, A, (const float*)B, (double*)C, tables, s);
  if (!b_f32 && c_f32)
    return launch_typed_f32<double, float>(g, A, (const double*)B, (float*)C, tables, s);
  if (!b_f32 && !c_f32)
    return launch_typed_f32<double, double>(g, A, (const double*)B, (double*)C, tables, s);
  return launch_typed_f32<float, float>(g, A, (const float*)B, (float*)C, tables, s);
}

// FP64 -> FP32 copy (round to nearest)
__global__ void k_to_f32(float* __restrict__ dst, const double* __restrict__ src, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

hipError_t launch_to_f32(float* dst, const double* src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  k_to_f32<<<(unsigned)nb, 256, 0, s>>>(dst, src, n);
  return hipGetLastError();
}

hipError_t launch_gemm_f64(const DevGemm& g, const double* A, const double* B, double* C,
                           const int32_t* tables, hipStream_t s) {
  if (g.njobs <= 0) return hipSuccess;
  return launch_typed<double, double>(g, A, B, C, tables, s);
}

hipError_t launch_gemm_mixed(const DevGemm& g, const double* A, const void* B, bool b_f32,
                             void* C, bool c_f32, const int32_t* tables, hipStream_t s) {
  if (g.njobs <= 0) return hipSuccess;
  if (!b_f32 && !c_f32)
    return launch_typed<double, double>(g, A, (const double*)B, (double*)C, tables, s);
  if (!b_f32 && c_f32)
    return launch_typed<double, float>(g, A, (const double*)B, (float*)C, tables, s);
  if (b_f32 && !c_f32)
    return launch_typed<float, double>(g, A, (const float*)B, (double*)C, tables, s);
  return hipErrorInvalidValue;
}

// Sum of the split parts of table-addressed output blocks:
// C[c_off + tcm[m] + tcn[n]] = sum_q P[p_off + q M N + m N + n].
template <class TC>
__global__ void k_reduce_tab(const ReduceTab* __restrict__ d, TC* __restrict__ C,
                             const double* __restrict__ P, const int32_t* __restrict__ tab) {
  const ReduceTab r = d[blockIdx.y];
  const int64_t mn = (int64_t)r.M * r.N;
  const int32_t* tcm = tab + r.tcm;
  const int32_t* tcn = tab + r.tcn;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < mn;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int q = 0; q < r.nsplit; ++q) s += P[r.p_off + (int64_t)q * mn + e];
    const int m = (int)(e / r.N), n = (int)(e % r.N);
    C[r.c_off + (int64_t)tcm[m] + tcn[n]] = (TC)s;
  }
}

hipError_t launch_reduce_tab(const ReduceTab* d, int nd, int64_t max_mn, void* C, bool c_f32,
                             const double* P, const int32_t* tab, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  int64_t bx = (max_mn + 255) / 256;
  if (bx > 256) bx = 256;
  if (bx < 1) bx = 1;
  if (c_f32)
    k_reduce_tab<float><<<dim3((unsigned)bx, nd), 256, 0, s>>>(d, (float*)C, P, tab);
  else
    k_reduce_tab<double><<<dim3((unsigned)bx, nd), 256, 0, s>>>(d, (double*)C, P, tab);
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
