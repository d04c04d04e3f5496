// Device kernel launchers (implemented in gemm.hip and linalg.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace fp {

// Workgroups of a launch are dispatched round-robin over the 8 XCDs, each
// with its own L2. Block b runs job xcd_swizzle(b, n, c): runs of c
// consecutive jobs (which share operand panels) go to one XCD, and the runs
// are dealt round-robin over the XCDs (c = 0: one contiguous range per XCD).
// Bijective on [0, n): the first whole rounds are permuted, the tail is
// unchanged.
__device__ __forceinline__ int xcd_swizzle(int b, int n, int c) {
  if (c <= 0) {
    const int per = n >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
  }
  const int round = 8 * c;
  if (b >= (n / round) * round) return b;
  const int slot = b >> 3;   // position of b in its XCD's sequence
  return (slot / c) * round + (b & 7) * c + (slot % c);
}

// A GEMM plan resident on the device.
struct DevGemm {
  const GemmJob* jobs = nullptr;
  const GemmPair* pairs = nullptr;
  int njobs = 0;
  int mt = 64, nt = 64;
  const ReduceTab* reduces = nullptr;   // split-K parts (see GemmPlan)
  int nred = 0;
};

// C[job tiles] = sum over pairs alpha * A(tables) * B(tables), FP64 MFMA.
hipError_t launch_gemm_f64(const DevGemm& g, const double* A, const double* B, double* C,
                           const int32_t* tables, hipStream_t s);
// The same with an FP32 copy of A, B and C in FP32 or FP64, on FP32 MFMA with
// FP32 accumulation per 16-deep K tile, the tiles summed in FP64 (B rounded to
// FP32 when loaded, C rounded from FP64).
hipError_t launch_gemm_f32(const DevGemm& g, const float* A, const void* B, bool b_f32, void* C,
                           bool c_f32, const int32_t* tables, hipStream_t s);
// dst[i] = (float)src[i]
hipError_t launch_to_f32(float* dst, const double* src, int64_t n, hipStream_t s);

// A row-thread layer-step plan resident on the device.
struct DevRt {
  const RtGroup* groups = nullptr;
  const int32_t* tile_group = nullptr;   // group of every workgroup (filled on the device)
  const RtOut* outs = nullptr;
  const RtKblk* kblks = nullptr;
  const RtCol* cols = nullptr;
  const RtPair* pairs = nullptr;
  const RtPack* packs = nullptr;
  int ngroups = 0, ntiles = 0, npacks = 0;
  int lds_bytes = 0;
  int nlaunch = 0;                     // one launch per LDS class
  int l_tile0[RT_NCLASS] = {0}, l_ntiles[RT_NCLASS] = {0}, l_lds[RT_NCLASS] = {0};
};
// Y[rows of the groups of LDS class launch c] = X rows times the packed
// layer sub-blocks PK (one launch of the plan's nlaunch).
// X and Y are double, or float when ``f32`` (FP32 storage, FP64 arithmetic).
hipError_t launch_rt_f64(const DevRt& r, int c, const void* X, bool f32, const double* PK,
                         void* Y, const int32_t* tab, hipStream_t s);
// PK[dst + k nc + c] = alpha S[sbase + sk[k] + sn[c]] for every pack entry.
// tile_group[tile0 + i] = g_first + g for every group g of groups[g_first ..
// g_first + ngroups) and its tiles i < ceil(M / rows): the group of every
// workgroup, written on the device instead of being uploaded.
hipError_t launch_tile_group(const RtGroup* groups, int g_first, int ngroups, int32_t* tile_group,
                             hipStream_t s);
hipError_t launch_rt_pack(const DevRt& r, const double* S, const int32_t* tab, double* PK,
                          hipStream_t s);

// The same with FP32 storage of B or C (loads widen to FP64, stores round
// the FP64 accumulators once): (B f64, C f32) or (B f32, C f64).
hipError_t launch_gemm_mixed(const DevGemm& g, const double* A, const void* B, bool b_f32,
                             void* C, bool c_f32, const int32_t* tables, hipStream_t s);

// Sum of the split parts of table-addressed output blocks (see GemmPlan).
hipError_t launch_reduce_tab(const ReduceTab* d, int nd, int64_t max_mn, void* C, bool c_f32,
                             const double* P, const int32_t* tab, hipStream_t s);

// Sum of split-K partials: C(m, n) = sum_s P[p_off + s*M*N + m*N + n].
struct ReduceDesc {
  int64_t c_off, c_rs, c_cs, p_off;
  int32_t M, N, nsplit, pad;
};
hipError_t launch_reduce_partials(const ReduceDesc* d, int nd, int max_mn, double* C,
                                  const double* P, hipStream_t s);

// Gaussian sketch: out[off + e] for e < nelem from Philox4x32-10 with
// counter (e >> 1, c1, c2, c3) and key (seed lo, seed hi), Box-Muller.
struct GaussDesc {
  int64_t off, nelem;
  uint32_t c1, c2, c3, pad;
};
hipError_t launch_gaussian(const GaussDesc* d, int nd, int64_t max_elem, double* out,
                           uint64_t seed, hipStream_t s);

// Cholesky with shift and triangular inverse per matrix (one workgroup each).
struct SmallDesc {
  int64_t a_off;    // k x k input (overwritten)
  int64_t b_off;    // k x k output
  int64_t c_off;    // k output values (eigenvalues)
  int32_t k;
  int32_t rows;     // rows of the tall matrix whose Gram this is (shift size)
  double shift;     // relative shift (0: none)
};
hipError_t launch_chol_inv(const SmallDesc* d, int nd, double* buf, int* status, hipStream_t s);

// Symmetric Jacobi eigensolver per matrix: A (k x k) -> eigenvalues
// descending at c_off, eigenvectors as columns of the k x k matrix at b_off.
// ``rel``: stop by the relative rule |a_pq| <= k eps sqrt(a_pp a_qq) for
// every pair (each eigenvalue resolved to its own size on a Gram matrix of
// nearly orthogonal columns); otherwise by the off-diagonal norm.
// status |= 4 when 40 sweeps do not converge. One workgroup per matrix;
// k <= JACOBI_MAX_K.
constexpr int JACOBI_MAX_K = 2048;
hipError_t launch_jacobi_eig(const SmallDesc* d, int nd, int max_k, double* buf, int* status,
                             hipStream_t s, bool rel = false);
// Multi-workgroup versions for widths beyond one workgroup's LDS (dense.hip).
// Blocked shifted Cholesky and inverse: the contract of launch_chol_inv;
// zf: nd ints of scratch.
hipError_t launch_chol_inv_blocked(const SmallDesc* d, int nd, int max_k, double* buf, int* zf,
                                   int* status, hipStream_t s);
// Block Jacobi eigensolver: the contract of launch_jacobi_eig with the
// absolute rule (rel = false) and no size limit, to absolute accuracy (a few
// k eps |A|; eigenvectors orthogonal to about 1e-13), driven by the host:
// flags (2 nd + 1 ints, zeroed by the caller) and work (bj_work_doubles) are
// scratch; launch_bj_init, then launch_bj_sweep until flags[2 nd] (matrices
// not converged) reads 0, then launch_bj_finish.
size_t bj_work_doubles(int nd, int max_k);
hipError_t launch_bj_init(const SmallDesc* d, int nd, int max_k, double* buf, int* flags,
                          double* work, hipStream_t s);
hipError_t launch_bj_sweep(const SmallDesc* d, int nd, int max_k, double* buf, int* flags,
                           double* work, hipStream_t s);
hipError_t launch_bj_finish(const SmallDesc* d, int nd, int max_k, double* buf, double* work,
                            hipStream_t s);
// SVQB scaling: column i of the k x k eigenvector matrix at b_off times
// 1/sqrt(lambda_i) (eigenvalues at c_off, descending), or zero when
// lambda_i <= tau * lambda_0.
hipError_t launch_svqb_scale(const SmallDesc* d, int nd, double* buf, double tau, hipStream_t s);

// Global truncation over sectors: eigenvalues (descending per sector) at
// lam_off[i] with k[i] entries; keeps the ``chi`` largest sqrt(lam).
struct CutOut {
  double total2;      // sum of all s^2
  double kept2;       // sum of kept s^2
  double s_last;      // smallest kept s
  double s_next;      // largest cut s (or -1)
};
// One cut per group: group g ranks the values of sectors [s0, s0 + ns) of
// the lists (lam_off, k), ``total`` values in all, keeps ranks < chi, and
// writes kept[s0 ..] and out[g]. One workgroup per group.
// Values at or below ``floor`` times the group's largest are never kept.
struct CutGroup {
  int32_t s0, ns, total, pad;
  double floor;
};
hipError_t launch_cut(const CutGroup* groups, int ngroups, int max_ns, int max_total,
                      const int64_t* lam_off, const int32_t* k, int chi,
                      const double* buf, int32_t* kept, CutOut* out, hipStream_t s);

// Canonical signs of a truncated factorisation: column c of U (m x ncol,
// row-major at u_off) is flipped together with row c of R (ncol x n at
// r_off) so that the column's leading entry is positive: the first row whose
// magnitude is within a relative 1e-5 of the column's largest. One
// workgroup per (matrix, column).
struct SignDesc {
  int64_t u_off, r_off;
  int32_t m, ncol, n, col0;   // col0: first global column index of this matrix
};
hipError_t launch_sign_fix(const SignDesc* d, int nd, int total_cols, const int32_t* col_desc,
                           double* U, double* R, hipStream_t s);

// One sector's block in the per-sector helpers of the bond expansion.
struct SectDesc {
  int64_t off_a, off_b, off_out;
  int32_t rows, cols, cols_b, s0;
};
// out = in with row i of each sector scaled by sc[s0 + i] (rows x cols blocks)
hipError_t launch_row_scale(const SectDesc* d, int nd, int64_t max_elems, const double* in,
                            double* out, const double* sc, hipStream_t s);
// out = [A | B] per sector: rows x cols and rows x cols_b into rows x (cols + cols_b)
hipError_t launch_merge_cols(const SectDesc* d, int nd, int64_t max_elems, const double* A,
                             const double* B, double* out, hipStream_t s);
// out = [A ; B^T] per sector: A rows x cols, B cols x cols_b (row-major) into
// (rows + cols_b) x cols
hipError_t launch_stack_rows_t(const SectDesc* d, int nd, int64_t max_elems, const double* A,
                               const double* B, double* out, hipStream_t s);

// sum of squares of x[0..n) into *out (deterministic two-pass reduction).
hipError_t launch_sumsq(const double* x, int64_t n, double* partial, double* out, hipStream_t s);
hipError_t launch_scale(double* x, int64_t n, double a, hipStream_t s);
hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s);
hipError_t launch_fill_int(int* x, int64_t n, int v, hipStream_t s);
// x[i] += y[i]
hipError_t launch_add(double* x, const double* y, int64_t n, hipStream_t s);
// 1 in *flag if any x is not finite
hipError_t launch_check_finite(const double* x, int64_t n, int* flag, hipStream_t s);

}  // namespace fp
