// Multi-workgroup versions of the k x k factorisations of the randomized SVD
// (Sec. 4; Halko et al. 2011, Example 1.6) for sketch widths beyond what one
// workgroup's LDS holds: the shifted Cholesky factor with its triangular
// inverse (CholeskyQR) and the symmetric Jacobi eigensolver (core
// factorisation, SVQB). Each works on a batch of matrices described by
// SmallDesc, one grid dimension per matrix, and spreads every matrix over
// many workgroups: 64 x 64 tiles staged in LDS, FP64 throughout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels.hpp"

namespace fp {

namespace {

constexpr int TB = 64;        // tile edge of the blocked Cholesky and inverse
constexpr int TP = TB + 1;    // padded LDS row (no bank conflicts on columns)
constexpr int JB = 32;        // block edge of the block Jacobi (sub-problems <= 64)
constexpr int JS = 2 * JB;    // largest sub-problem
constexpr int JP = JS + 1;
// per (matrix, pair) record of the block Jacobi: rotation (JS x JS) and a
// flag (rotated or not)
constexpr int JREC = JS * JS + 1;
constexpr double EPS = 2.220446049250313e-16;

__device__ inline int imin(int a, int b) { return a < b ? a : b; }

}  // namespace

// ---------------------------------------------------------------------------
// Blocked shifted Cholesky A + s I = R^T R and X = R^{-1} (the arithmetic of
// k_chol_inv rearranged by 64 x 64 tiles, right-looking; Golub & Van Loan,
// Alg. 4.2.10). R overwrites the upper triangle of A; X (upper triangular,
// zeros below) is written at b_off.
// ---------------------------------------------------------------------------

// Trace, shift, zero test; clears the blocks of X below the block diagonal.
// zf[m] = 1 marks an exactly zero matrix (X = 0, nothing else to do).
__global__ __launch_bounds__(256) void k_bchol_prep(const SmallDesc* __restrict__ d,
                                                    double* __restrict__ buf,
                                                    int* __restrict__ zf,
                                                    int* __restrict__ status) {
  const SmallDesc g = d[blockIdx.x];
  const int k = g.k;
  double* A = buf + g.a_off;
  double* X = buf + g.b_off;
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double red[256];
  __shared__ double sh_shift;
  double t = 0.0;
  for (int i = tid; i < k; i += nt) t += A[(int64_t)i * k + i];
  red[tid] = t;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const bool zero = !(red[0] > 0.0);
  if (tid == 0) zf[blockIdx.x] = zero ? 1 : 0;
  if (zero) {
    for (int64_t e = tid; e < (int64_t)k * k; e += nt) X[e] = 0.0;
    return;
  }
  for (int64_t e = tid; e < (int64_t)k * k; e += nt) {
    const int i = (int)(e / k), j = (int)(e % k);
    if (i / TB > j / TB) X[e] = 0.0;
  }
  if (g.shift > 0.0) {
    if (tid == 0) {
      sh_shift = g.shift * ((double)g.rows * k + (double)k * (k + 1)) * (0.5 * EPS) * red[0];
      if (sh_shift > 0.0) atomicOr(status, 2);
    }
    __syncthreads();
    for (int i = tid; i < k; i += nt) A[(int64_t)i * k + i] += sh_shift;
  }
}

// Diagonal tile j0: unblocked Cholesky in LDS and its inverse, written to the
// diagonal tile of X.
__global__ __launch_bounds__(256) void k_bchol_diag(const SmallDesc* __restrict__ d,
                                                    double* __restrict__ buf,
                                                    const int* __restrict__ zf,
                                                    int* __restrict__ status, int j0) {
  const SmallDesc g = d[blockIdx.x];
  const int k = g.k;
  if (zf[blockIdx.x] || j0 >= k) return;
  double* A = buf + g.a_off;
  double* X = buf + g.b_off;
  const int bs = imin(TB, k - j0);
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double R[TB * TP];
  __shared__ double Xd[TB * TP];
  for (int e = tid; e < bs * bs; e += nt) {
    const int i = e / bs, j = e % bs;
    R[i * TP + j] = (j >= i) ? A[(int64_t)(j0 + i) * k + j0 + j] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < bs; ++j) {
    double djj = R[j * TP + j];
    if (!(djj > 0.0)) {
      if (tid == 0) {
        atomicOr(status, 1);
        if (status[1 + blockIdx.x] == 0) status[1 + blockIdx.x] = j0 + j + 1;
      }
      djj = 1e-300;
    }
    const double rjj = sqrt(djj);
    __syncthreads();
    if (tid == 0) R[j * TP + j] = rjj;
    for (int l = j + 1 + tid; l < bs; l += nt) R[j * TP + l] /= rjj;
    __syncthreads();
    const int w = bs - j - 1;
    for (int e = tid; e < w * w; e += nt) {
      const int i = j + 1 + e / w, l = j + 1 + e % w;
      if (l >= i) R[i * TP + l] -= R[j * TP + i] * R[j * TP + l];
    }
    __syncthreads();
  }
  // inverse of the tile: column c by back substitution
  for (int c = tid; c < bs; c += nt) {
    for (int i = bs - 1; i > c; --i) Xd[i * TP + c] = 0.0;
    Xd[c * TP + c] = 1.0 / R[c * TP + c];
    for (int i = c - 1; i >= 0; --i) {
      double s = 0.0;
      for (int l = i + 1; l <= c; ++l) s += R[i * TP + l] * Xd[l * TP + c];
      Xd[i * TP + c] = -s / R[i * TP + i];
    }
  }
  __syncthreads();
  for (int e = tid; e < bs * bs; e += nt) {
    const int i = e / bs, j = e % bs;
    if (j >= i) A[(int64_t)(j0 + i) * k + j0 + j] = R[i * TP + j];
    X[(int64_t)(j0 + i) * k + j0 + j] = Xd[i * TP + j];
  }
}

// Panel right of tile j0: R(j0 rows, c0 + 64 bx ..) = R_jj^{-T} A(same).
__global__ __launch_bounds__(256) void k_bchol_panel(const SmallDesc* __restrict__ d,
                                                     double* __restrict__ buf,
                                                     const int* __restrict__ zf, int j0) {
  const SmallDesc g = d[blockIdx.y];
  const int k = g.k;
  const int c0 = j0 + TB + TB * blockIdx.x;
  if (zf[blockIdx.y] || c0 >= k) return;
  double* A = buf + g.a_off;
  const double* X = buf + g.b_off;
  const int bs = imin(TB, k - j0), cw = imin(TB, k - c0);
  const int tid = threadIdx.x;
  __shared__ double Xd[TB * TP];
  __shared__ double T[TB * TP];
  for (int e = tid; e < TB * TB; e += 256) {
    const int i = e / TB, j = e % TB;
    Xd[i * TP + j] = (i < bs && j < bs) ? X[(int64_t)(j0 + i) * k + j0 + j] : 0.0;
    T[i * TP + j] = (i < bs && j < cw) ? A[(int64_t)(j0 + i) * k + c0 + j] : 0.0;
  }
  __syncthreads();
  // thread: column c = tid % 64, rows r = tid / 64 + 4 t
  const int c = tid & 63;
  double acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = 0.0;
  for (int l = 0; l < bs; ++l) {
    const double tv = T[l * TP + c];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int r = (tid >> 6) + 4 * t;
      if (l <= r) acc[t] += Xd[l * TP + r] * tv;
    }
  }
  if (c < cw) {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int r = (tid >> 6) + 4 * t;
      if (r < bs) A[(int64_t)(j0 + r) * k + c0 + c] = acc[t];
    }
  }
}

// Trailing update A(I, J) -= R(j0, I)^T R(j0, J) over upper tile pairs I <= J
// of the part right of and below tile j0.
__global__ __launch_bounds__(256) void k_bchol_trail(const SmallDesc* __restrict__ d,
                                                     double* __restrict__ buf,
                                                     const int* __restrict__ zf, int j0) {
  const SmallDesc g = d[blockIdx.y];
  const int k = g.k;
  const int base = j0 + TB;
  if (zf[blockIdx.y] || base >= k) return;
  const int nt = (k - base + TB - 1) / TB;
  // linear index -> (I, J), I <= J, row by row
  int rem = blockIdx.x, I = 0;
  while (I < nt && rem >= nt - I) {
    rem -= nt - I;
    ++I;
  }
  if (I >= nt) return;
  const int J = I + rem;
  double* A = buf + g.a_off;
  const int bs = imin(TB, k - j0);
  const int r0 = base + TB * I, c0 = base + TB * J;
  const int rw = imin(TB, k - r0), cw = imin(TB, k - c0);
  const int tid = threadIdx.x;
  __shared__ double P[TB * TP];
  __shared__ double Q[TB * TP];
  for (int e = tid; e < TB * TB; e += 256) {
    const int l = e / TB, j = e % TB;
    P[l * TP + j] = (l < bs && j < rw) ? A[(int64_t)(j0 + l) * k + r0 + j] : 0.0;
    Q[l * TP + j] = (l < bs && j < cw) ? A[(int64_t)(j0 + l) * k + c0 + j] : 0.0;
  }
  __syncthreads();
  const int c = tid & 63;
  double acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = 0.0;
  for (int l = 0; l < bs; ++l) {
    const double qv = Q[l * TP + c];
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] += P[l * TP + (tid >> 6) + 4 * t] * qv;
  }
  if (c < cw) {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int r = (tid >> 6) + 4 * t;
      if (r < rw) A[(int64_t)(r0 + r) * k + c0 + c] -= acc[t];
    }
  }
}

// Off-diagonal tiles of X at block distance dd: X_ij = -X_ii sum_{i<l<=j}
// R_il X_lj (from R X = I), j = i + dd; tiles of smaller distance are done.
__global__ __launch_bounds__(256) void k_bchol_trinv(const SmallDesc* __restrict__ d,
                                                     double* __restrict__ buf,
                                                     const int* __restrict__ zf, int dd) {
  const SmallDesc g = d[blockIdx.y];
  const int k = g.k;
  const int nb = (k + TB - 1) / TB;
  const int ib = blockIdx.x, jb = ib + dd;
  if (zf[blockIdx.y] || jb >= nb) return;
  const double* A = buf + g.a_off;
  double* X = buf + g.b_off;
  const int r0 = TB * ib, c0 = TB * jb;
  const int rw = imin(TB, k - r0), cw = imin(TB, k - c0);
  const int tid = threadIdx.x;
  __shared__ double Ra[TB * TP];
  __shared__ double Xb[TB * TP];
  const int c = tid & 63;
  double acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = 0.0;
  for (int lb = ib + 1; lb <= jb; ++lb) {
    const int l0 = TB * lb, lw = imin(TB, k - l0);
    __syncthreads();
    for (int e = tid; e < TB * TB; e += 256) {
      const int i = e / TB, j = e % TB;
      // Ra stored transposed: Ra[t][r] = R(r0 + r, l0 + t)
      Ra[j * TP + i] = (i < rw && j < lw) ? A[(int64_t)(r0 + i) * k + l0 + j] : 0.0;
      Xb[i * TP + j] = (i < lw && j < cw) ? X[(int64_t)(l0 + i) * k + c0 + j] : 0.0;
    }
    __syncthreads();
    for (int t = 0; t < lw; ++t) {
      const double xv = Xb[t * TP + c];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] += Ra[t * TP + (tid >> 6) + 4 * u] * xv;
    }
  }
  __syncthreads();
  // T into Xb, X_ii (transposed) into Ra
  for (int e = tid; e < TB * TB; e += 256) {
    const int i = e / TB, j = e % TB;
    Ra[j * TP + i] = (i < rw && j < rw) ? X[(int64_t)(r0 + i) * k + r0 + j] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) Xb[((tid >> 6) + 4 * u) * TP + c] = acc[u];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 16; ++u) acc[u] = 0.0;
  for (int t = 0; t < rw; ++t) {
    const double tv = Xb[t * TP + c];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] += Ra[t * TP + (tid >> 6) + 4 * u] * tv;
  }
  if (c < cw) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = (tid >> 6) + 4 * u;
      if (r < rw) X[(int64_t)(r0 + r) * k + c0 + c] = -acc[u];
    }
  }
}

hipError_t launch_chol_inv_blocked(const SmallDesc* d, int nd, int max_k, double* buf, int* zf,
                                   int* status, hipStream_t s) {
  if (nd <= 0 || max_k <= 0) return hipSuccess;
  k_bchol_prep<<<nd, 256, 0, s>>>(d, buf, zf, status);
  const int nb = (max_k + TB - 1) / TB;
  for (int jb = 0; jb < nb; ++jb) {
    const int j0 = TB * jb;
    k_bchol_diag<<<nd, 256, 0, s>>>(d, buf, zf, status, j0);
    if (j0 + TB < max_k) {
      const int nt = (max_k - j0 - TB + TB - 1) / TB;
      k_bchol_panel<<<dim3(nt, nd), 256, 0, s>>>(d, buf, zf, j0);
      k_bchol_trail<<<dim3(nt * (nt + 1) / 2, nd), 256, 0, s>>>(d, buf, zf, j0);
    }
  }
  for (int dd = 1; dd < nb; ++dd) k_bchol_trinv<<<dim3(nb - dd, nd), 256, 0, s>>>(d, buf, zf, dd);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block Jacobi eigensolver for a symmetric k x k matrix A (in place at a_off)
// with eigenvectors V at b_off and eigenvalues (descending) at c_off. The
// index range is cut into blocks of 32; a sweep pairs every two blocks once
// (round-robin); in one round the pairs are disjoint, so each workgroup
// runs one cyclic Jacobi sweep over its pair's principal sub-matrix (at most
// 64 x 64, in LDS) and the accumulated rotation W is applied to the block
// rows, then to the block columns of A and V by many workgroups (Golub & Van
// Loan, Sec. 8.5.4). Applying W, whose entries carry absolute rounding errors of order
// eps, adds noise of order eps |A| to every row it touches, so this solver
// gives absolute accuracy only (eigenvalues to a few k eps |A|, V orthogonal
// to about 1e-13): a pair is rotated while |a_pq| > max(k, 64) eps a_max,
// a_max the largest diagonal entry of the input, which stays above that
// noise; a matrix is done after a sweep without rotations. (Relative
// accuracy, the rule of Demmel & Veselic, needs single plane rotations.)
// Work per matrix m: flags[2m] done, flags[2m + 1] rotations this sweep,
// flags[2 nd] matrices not done; dmax[m]; rec: JREC doubles per pair.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bj_init(const SmallDesc* __restrict__ d,
                                                 double* __restrict__ buf,
                                                 int* __restrict__ flags,
                                                 double* __restrict__ dmax, int nd) {
  const SmallDesc g = d[blockIdx.y];
  const int k = g.k;
  double* V = buf + g.b_off;
  const double* A = buf + g.a_off;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)k * k;
       e += (int64_t)gridDim.x * blockDim.x)
    V[e] = (e / k == e % k) ? 1.0 : 0.0;
  if (blockIdx.x == 0) {
    __shared__ double red[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < k; i += 256) m = fmax(m, fabs(A[(int64_t)i * k + i]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      dmax[blockIdx.y] = red[0];
      flags[2 * blockIdx.y] = k <= 1 ? 1 : 0;
      flags[2 * blockIdx.y + 1] = 0;
      if (k > 1) atomicAdd(&flags[2 * nd], 1);
    }
  }
}

namespace {
// pair i of round rnd among nbp (even) blocks, circle method
__device__ inline void bj_pair(int i, int rnd, int nbp, int* P, int* Q) {
  auto player = [&](int t) { return t == 0 ? 0 : ((t - 1 + rnd) % (nbp - 1)) + 1; };
  int p = player(i), q = player(nbp - 1 - i);
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
  *P = p;
  *Q = q;
}
// global index of sub-problem index i for blocks P (size sp) and Q
__device__ inline int bj_index(int i, int P, int Q, int sp) {
  return i < sp ? JB * P + i : JB * Q + (i - sp);
}
}  // namespace

__global__ __launch_bounds__(256) void k_bj_solve(const SmallDesc* __restrict__ d,
                                                  const double* __restrict__ buf,
                                                  int* __restrict__ flags,
                                                  const double* __restrict__ dmax,
                                                  double* __restrict__ rec, int npmax, int rnd) {
  const int m = blockIdx.y;
  const SmallDesc g = d[m];
  const int k = g.k;
  const int nb = (k + JB - 1) / JB, nbp = nb + (nb & 1);
  double* out = rec + ((int64_t)m * npmax + blockIdx.x) * JREC;
  if (flags[2 * m] || (int)blockIdx.x >= nbp / 2) return;
  int P, Q;
  bj_pair(blockIdx.x, rnd, nbp, &P, &Q);
  const int tid = threadIdx.x;
  if (Q >= nb) {
    if (tid == 0) out[JS * JS] = 0.0;
    return;
  }
  const int sp = imin(JB, k - JB * P), sq = imin(JB, k - JB * Q), s = sp + sq;
  const double* A = buf + g.a_off;
  // the sub-matrix padded to JS x JS with zeros (padding never rotates)
  __shared__ double S[JS * JP];
  __shared__ double W[JS * JP];
  __shared__ double cs[JS / 2], sn[JS / 2];
  __shared__ int pi[JS / 2], qi[JS / 2];
  __shared__ int nrot;
  for (int e = tid; e < JS * JS; e += 256) {
    const int i = e >> 6, j = e & 63;
    double v = 0.0;
    if (i < s && j < s) {
      const int gi = bj_index(i, P, Q, sp), gj = bj_index(j, P, Q, sp);
      v = gi <= gj ? A[(int64_t)gi * k + gj] : A[(int64_t)gj * k + gi];
    }
    S[i * JP + j] = v;
    W[i * JP + j] = (i == j) ? 1.0 : 0.0;
  }
  if (tid == 0) nrot = 0;
  const double tol = (double)(k > 64 ? k : 64) * EPS * dmax[m];
  __syncthreads();
  // one cyclic sweep over the sub-matrix (round-robin over JS indices);
  // each round's rotations are disjoint, so J^T S J is applied block by
  // block: every 2 x 2 block (row pair a, column pair b) from its own four
  // entries, rows first, then columns
  for (int r = 0; r < JS - 1; ++r) {
    if (tid < JS / 2) {
      int p, q;
      {
        auto player = [&](int t) { return t == 0 ? 0 : ((t - 1 + r) % (JS - 1)) + 1; };
        p = player(tid);
        q = player(JS - 1 - tid);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
      }
      double c = 1.0, sv = 0.0;
      if (q < s) {
        const double apq = S[p * JP + q], app = S[p * JP + p], aqq = S[q * JP + q];
        if (fabs(apq) > tol) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double t = fabs(tau) > 1e150
                               ? 0.5 / tau
                               : (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + t * t);
          sv = t * c;
          if (sv != 0.0) atomicAdd(&nrot, 1);
        }
      }
      cs[tid] = c;
      sn[tid] = sv;
      pi[tid] = p;
      qi[tid] = q;
    }
    __syncthreads();
    for (int e = tid; e < (JS / 2) * (JS / 2); e += 256) {
      const int a = e >> 5, b = e & 31;
      const double sa = sn[a], sb = sn[b];
      if (sa == 0.0 && sb == 0.0) continue;
      const double ca = cs[a], cb = cs[b];
      const int pa = pi[a], qa = qi[a], pb = pi[b], qb = qi[b];
      const double x00 = S[pa * JP + pb], x01 = S[pa * JP + qb];
      const double x10 = S[qa * JP + pb], x11 = S[qa * JP + qb];
      const double r00 = ca * x00 - sa * x10, r01 = ca * x01 - sa * x11;
      const double r10 = sa * x00 + ca * x10, r11 = sa * x01 + ca * x11;
      S[pa * JP + pb] = cb * r00 - sb * r01;
      S[pa * JP + qb] = sb * r00 + cb * r01;
      S[qa * JP + pb] = cb * r10 - sb * r11;
      S[qa * JP + qb] = sb * r10 + cb * r11;
    }
    for (int e = tid; e < (JS / 2) * JS; e += 256) {
      const int i = e >> 6, row = e & 63;
      const double sv = sn[i];
      if (sv == 0.0) continue;
      const double c = cs[i];
      const int p = pi[i], q = qi[i];
      const double wp = W[row * JP + p], wq = W[row * JP + q];
      W[row * JP + p] = c * wp - sv * wq;
      W[row * JP + q] = sv * wp + c * wq;
    }
    __syncthreads();
  }
  for (int e = tid; e < s * s; e += 256) out[(e / s) * JS + (e % s)] = W[(e / s) * JP + (e % s)];
  if (tid == 0) {
    out[JS * JS] = nrot > 0 ? 1.0 : 0.0;
    if (nrot > 0) atomicAdd(&flags[2 * m + 1], 1);
  }
}

// Block rows P, Q of A <- W^T (rows), column tile 64 bx.
__global__ __launch_bounds__(256) void k_bj_rows(const SmallDesc* __restrict__ d,
                                                 double* __restrict__ buf,
                                                 const int* __restrict__ flags,
                                                 const double* __restrict__ rec, int npmax,
                                                 int rnd) {
  const int m = blockIdx.z, pr = blockIdx.y;
  const SmallDesc g = d[m];
  const int k = g.k;
  const int nb = (k + JB - 1) / JB, nbp = nb + (nb & 1);
  const int c0 = 64 * blockIdx.x;
  if (flags[2 * m] || pr >= nbp / 2 || c0 >= k) return;
  int P, Q;
  bj_pair(pr, rnd, nbp, &P, &Q);
  if (Q >= nb) return;
  const double* W = rec + ((int64_t)m * npmax + pr) * JREC;
  if (W[JS * JS] == 0.0) return;
  const int sp = imin(JB, k - JB * P), sq = imin(JB, k - JB * Q), s = sp + sq;
  const int cw = imin(64, k - c0);
  double* A = buf + g.a_off;
  __shared__ double Ws[JS * JP];
  __shared__ double X[JS * JP];
  const int tid = threadIdx.x;
  for (int e = tid; e < JS * 64; e += 256) {
    const int i = e / 64, j = e % 64;
    Ws[i * JP + j] = (i < s && j < s) ? W[i * JS + j] : 0.0;
    X[i * JP + j] = (i < s && j < cw) ? A[(int64_t)bj_index(i, P, Q, sp) * k + c0 + j] : 0.0;
  }
  __syncthreads();
  const int c = tid & 63;
  double acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = 0.0;
  for (int l = 0; l < s; ++l) {
    const double xv = X[l * JP + c];
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] += Ws[l * JP + (tid >> 6) + 4 * t] * xv;
  }
  if (c < cw) {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int r = (tid >> 6) + 4 * t;
      if (r < s) A[(int64_t)bj_index(r, P, Q, sp) * k + c0 + c] = acc[t];
    }
  }
}

// Block columns P, Q of A (z even) or V (z odd) <- (columns) W, row tile
// 64 bx.
__global__ __launch_bounds__(256) void k_bj_cols(const SmallDesc* __restrict__ d,
                                                 double* __restrict__ buf,
                                                 const int* __restrict__ flags,
                                                 const double* __restrict__ rec, int npmax,
                                                 int rnd) {
  const int m = blockIdx.z >> 1, isV = blockIdx.z & 1, pr = blockIdx.y;
  const SmallDesc g = d[m];
  const int k = g.k;
  const int nb = (k + JB - 1) / JB, nbp = nb + (nb & 1);
  const int r0 = 64 * blockIdx.x;
  if (flags[2 * m] || pr >= nbp / 2 || r0 >= k) return;
  int P, Q;
  bj_pair(pr, rnd, nbp, &P, &Q);
  if (Q >= nb) return;
  const double* W = rec + ((int64_t)m * npmax + pr) * JREC;
  if (W[JS * JS] == 0.0) return;
  const int sp = imin(JB, k - JB * P), sq = imin(JB, k - JB * Q), s = sp + sq;
  const int rw = imin(64, k - r0);
  double* M = buf + (isV ? g.b_off : g.a_off);
  __shared__ double Ws[JS * JP];
  __shared__ double Y[JS * JP];   // Y[l][r] = M(r0 + r, index l)
  const int tid = threadIdx.x;
  for (int e = tid; e < JS * 64; e += 256) {
    const int i = e / 64, j = e % 64;
    Ws[i * JP + j] = (i < s && j < s) ? W[i * JS + j] : 0.0;
  }
  for (int e = tid; e < 64 * JS; e += 256) {
    const int r = e / JS, l = e % JS;
    Y[l * JP + r] = (r < rw && l < s) ? M[(int64_t)(r0 + r) * k + bj_index(l, P, Q, sp)] : 0.0;
  }
  __syncthreads();
  // thread: row r = tid % 64, sub-columns c = tid / 64 + 4 t
  const int r = tid & 63;
  double acc[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) acc[t] = 0.0;
  for (int l = 0; l < s; ++l) {
    const double yv = Y[l * JP + r];
#pragma unroll
    for (int t = 0; t < 16; ++t) acc[t] += yv * Ws[l * JP + (tid >> 6) + 4 * t];
  }
  if (r < rw) {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int c = (tid >> 6) + 4 * t;
      if (c < s) M[(int64_t)(r0 + r) * k + bj_index(c, P, Q, sp)] = acc[t];
    }
  }
}

// Sweep bookkeeping: a matrix whose sweep rotated nothing is done.
__global__ void k_bj_sweep_end(int* __restrict__ flags, int nd) {
  for (int m = threadIdx.x; m < nd; m += blockDim.x) {
    if (!flags[2 * m] && flags[2 * m + 1] == 0) {
      flags[2 * m] = 1;
      atomicSub(&flags[2 * nd], 1);
    }
    flags[2 * m + 1] = 0;
  }
}

// Eigenvalues descending (ties by index) to c_off; rank of each column.
__global__ __launch_bounds__(1024) void k_bj_rank(const SmallDesc* __restrict__ d,
                                                  double* __restrict__ buf,
                                                  int* __restrict__ rank, int max_k) {
  const SmallDesc g = d[blockIdx.x];
  const int k = g.k;
  const double* A = buf + g.a_off;
  double* lam = buf + g.c_off;
  int* rk = rank + (int64_t)blockIdx.x * max_k;
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const double li = A[(int64_t)i * k + i];
    int r = 0;
    for (int j = 0; j < k; ++j) {
      const double lj = A[(int64_t)j * k + j];
      if (lj > li || (lj == li && j < i)) ++r;
    }
    lam[r] = li;
    rk[i] = r;
  }
}

// A <- V with columns permuted by rank (A is free after the eigenvalues).
__global__ __launch_bounds__(256) void k_bj_permute(const SmallDesc* __restrict__ d,
                                                    double* __restrict__ buf,
                                                    const int* __restrict__ rank, int max_k) {
  const SmallDesc g = d[blockIdx.y];
  const int k = g.k;
  double* A = buf + g.a_off;
  const double* V = buf + g.b_off;
  const int* rk = rank + (int64_t)blockIdx.y * max_k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)k * k;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e / k), col = (int)(e % k);
    A[(int64_t)row * k + rk[col]] = V[e];
  }
}

__global__ __launch_bounds__(256) void k_bj_copy(const SmallDesc* __restrict__ d,
                                                 double* __restrict__ buf) {
  const SmallDesc g = d[blockIdx.y];
  const int k = g.k;
  const double* A = buf + g.a_off;
  double* V = buf + g.b_off;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)k * k;
       e += (int64_t)gridDim.x * blockDim.x)
    V[e] = A[e];
}

int bj_pairs_max(int max_k) {
  const int nb = (max_k + JB - 1) / JB;
  return (nb + (nb & 1)) / 2;
}

size_t bj_work_doubles(int nd, int max_k) {
  const size_t rec = (size_t)nd * bj_pairs_max(max_k) * JREC;
  const size_t rank = ((size_t)nd * max_k + 1) / 2 + 1;   // ints, in doubles
  return rec + nd + (rank > 0 ? rank : 1);
}

hipError_t launch_bj_init(const SmallDesc* d, int nd, int max_k, double* buf, int* flags,
                          double* work, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  double* dmax = work + (size_t)nd * bj_pairs_max(max_k) * JREC;
  int gx = (int)std::min<int64_t>(((int64_t)max_k * max_k + 255) / 256, 64);
  k_bj_init<<<dim3(std::max(gx, 1), nd), 256, 0, s>>>(d, buf, flags, dmax, nd);
  return hipGetLastError();
}

hipError_t launch_bj_sweep(const SmallDesc* d, int nd, int max_k, double* buf, int* flags,
                           double* work, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  const int npmax = bj_pairs_max(max_k);
  const int nb = (max_k + JB - 1) / JB, nbp = nb + (nb & 1);
  double* rec = work;
  const double* dmax = work + (size_t)nd * npmax * JREC;
  const int tiles = (max_k + 63) / 64;
  for (int rnd = 0; rnd < nbp - 1; ++rnd) {
    k_bj_solve<<<dim3(npmax, nd), 256, 0, s>>>(d, buf, flags, dmax, rec, npmax, rnd);
    k_bj_rows<<<dim3(tiles, npmax, nd), 256, 0, s>>>(d, buf, flags, rec, npmax, rnd);
    k_bj_cols<<<dim3(tiles, npmax, 2 * nd), 256, 0, s>>>(d, buf, flags, rec, npmax, rnd);
  }
  k_bj_sweep_end<<<1, 256, 0, s>>>(flags, nd);
  return hipGetLastError();
}

hipError_t launch_bj_finish(const SmallDesc* d, int nd, int max_k, double* buf, double* work,
                            hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  int* rank = (int*)(work + (size_t)nd * bj_pairs_max(max_k) * JREC + nd);
  k_bj_rank<<<nd, 1024, 0, s>>>(d, buf, rank, max_k);
  int gx = (int)std::min<int64_t>(((int64_t)max_k * max_k + 255) / 256, 256);
  k_bj_permute<<<dim3(std::max(gx, 1), nd), 256, 0, s>>>(d, buf, rank, max_k);
  k_bj_copy<<<dim3(std::max(gx, 1), nd), 256, 0, s>>>(d, buf);
  return hipGetLastError();
}

}  // namespace fp
