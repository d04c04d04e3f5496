// Small dense kernels of the randomized SVD (Sec. 4; Halko et al. 2011,
// Example 1.6) on gfx950: Gaussian sketch, shifted Cholesky with triangular
// inverse (the k x k part of CholeskyQR), symmetric Jacobi eigensolver for
// the k x k core factorisation, the global truncation and norms. All
// arithmetic here is FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "kernels.hpp"

namespace fp {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and Box-Muller.
// ---------------------------------------------------------------------------
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__global__ void k_gaussian(const GaussDesc* __restrict__ d, double* __restrict__ out,
                           uint64_t seed) {
  const GaussDesc g = d[blockIdx.y];
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < g.nelem;
       e += (int64_t)gridDim.x * blockDim.x) {
    uint32_t c[4] = {(uint32_t)(e >> 1), g.c1, g.c2, g.c3};
    philox4x32_10(c, k0, k1);
    const double sc = 1.0 / 9007199254740992.0;
    const double u1 = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6)) * sc;
    const double u2 = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6)) * sc;
    const double rad = sqrt(-2.0 * log(1.0 - u1));
    const double ang = 2.0 * M_PI * u2;
    out[g.off + e] = (e & 1) ? rad * sin(ang) : rad * cos(ang);
  }
}

hipError_t launch_gaussian(const GaussDesc* d, int nd, int64_t max_elem, double* out,
                           uint64_t seed, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  int64_t bx = (max_elem + 255) / 256;
  if (bx > 2048) bx = 2048;
  if (bx < 1) bx = 1;
  k_gaussian<<<dim3((unsigned)bx, nd), 256, 0, s>>>(d, out, seed);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shifted Cholesky A + s I = R^T R (R upper) and X = R^{-1}, one workgroup per
// matrix. The shift (shifted CholeskyQR, Fukaya et al., SIAM J. Sci. Comput.
// 42 (2020) A477) is s = shift * (rows*k + k*(k+1)) * eps * trace(A).
// status[0] |= 1 on a non-positive pivot, |= 2 when a shift was applied;
// status[1 + i] = 1 + first failing pivot of matrix i (0: none).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_chol_inv(const SmallDesc* __restrict__ d,
                                                  double* __restrict__ buf,
                                                  int* __restrict__ status) {
  const SmallDesc g = d[blockIdx.x];
  const int k = g.k;
  double* A = buf + g.a_off;
  double* X = buf + g.b_off;
  const int tid = threadIdx.x, nt = blockDim.x;
  __shared__ double red[256];
  __shared__ double sh_shift;
  {
    double t = 0.0;
    for (int i = tid; i < k; i += nt) t += A[(int64_t)i * k + i];
    red[tid] = t;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
  }
  // an exactly zero block (a sector the operator maps to zero) has an empty
  // range: X = 0 makes its Q zero, and no breakdown is reported
  if (!(red[0] > 0.0)) {
    for (int64_t e = tid; e < (int64_t)k * k; e += nt) X[e] = 0.0;
    return;
  }
  if (g.shift > 0.0) {
    if (tid == 0) {
      const double eps = 1.1102230246251565e-16;
      sh_shift = g.shift * ((double)g.rows * k + (double)k * (k + 1)) * eps * red[0];
      if (sh_shift > 0.0) atomicOr(status, 2);
    }
    __syncthreads();
    for (int i = tid; i < k; i += nt) A[(int64_t)i * k + i] += sh_shift;
    __syncthreads();
  }
  for (int j = 0; j < k; ++j) {
    double djj = A[(int64_t)j * k + j];
    if (!(djj > 0.0)) {
      if (tid == 0) {
        atomicOr(status, 1);
        if (status[1 + blockIdx.x] == 0) status[1 + blockIdx.x] = j + 1;
      }
      djj = 1e-300;
    }
    const double rjj = sqrt(djj);
    __syncthreads();
    if (tid == 0) A[(int64_t)j * k + j] = rjj;
    for (int l = j + 1 + tid; l < k; l += nt) A[(int64_t)j * k + l] /= rjj;
    __syncthreads();
    const int w = k - j - 1;
    for (int64_t e = tid; e < (int64_t)w * w; e += nt) {
      const int i = j + 1 + (int)(e / w), l = j + 1 + (int)(e % w);
      if (l >= i) A[(int64_t)i * k + l] -= A[(int64_t)j * k + i] * A[(int64_t)j * k + l];
    }
    __syncthreads();
  }
  // X = R^{-1}: column c by back substitution
  for (int c = tid; c < k; c += nt) {
    for (int i = k - 1; i > c; --i) X[(int64_t)i * k + c] = 0.0;
    X[(int64_t)c * k + c] = 1.0 / A[(int64_t)c * k + c];
    for (int i = c - 1; i >= 0; --i) {
      double s = 0.0;
      for (int l = i + 1; l <= c; ++l) s += A[(int64_t)i * k + l] * X[(int64_t)l * k + c];
      X[(int64_t)i * k + c] = -s / A[(int64_t)i * k + i];
    }
  }
}

hipError_t launch_chol_inv(const SmallDesc* d, int nd, double* buf, int* status, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  k_chol_inv<<<nd, 256, 0, s>>>(d, buf, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi for a symmetric k x k matrix (Golub & Van Loan, Sec. 8.5),
// parallel ordering by the round-robin (circle) schedule: every round
// rotates k/2 disjoint pairs, first all row pairs then all column pairs.
// With LDS, the matrix being rotated lives in LDS (a copy; the k x k input in
// global memory is left as it was), otherwise in place in global memory.
// Same arithmetic in the same order either way.
// Two stopping rules: the off-diagonal Frobenius norm below 1e-15 of the
// diagonal's (REL false), or (REL true) the rule of Demmel & Veselic (SIAM
// J. Matrix Anal. Appl. 13 (1992) 1204): a pair is rotated only while
// |a_pq| > k eps sqrt(a_pp a_qq), and the iteration stops after a sweep
// without rotations. On a Gram matrix whose columns are nearly orthogonal
// the relative rule resolves every eigenvalue to its own size, not to the
// largest one's. It stops at eigenvalues of eps^2 times the largest
// diagonal entry (singular values of eps times the largest): pairs with
// |a_pq| <= eps^2 a_max are left, which moves no singular value by more than
// about eps times the largest, and without this floor the rule never holds
// among null directions whose entries are rounding noise.
// ---------------------------------------------------------------------------
// LDS scratch in doubles for pair capacity ``npc`` (>= kp/2 of every
// matrix): rotation cosines and sines, pair indices (ints, two per double),
// and a 1024-entry reduction.
__host__ __device__ constexpr int jac_scratch(int npc) { return 3 * npc + 1024; }

template <bool LDS, bool REL>
__global__ __launch_bounds__(1024) void k_jacobi(const SmallDesc* __restrict__ d,
                                                 double* __restrict__ buf,
                                                 int* __restrict__ status, int npc) {
  const SmallDesc g = d[blockIdx.x];
  const int k = g.k;
  double* V = buf + g.b_off;
  double* lam = buf + g.c_off;
  const int tid = threadIdx.x, nt = blockDim.x;
  extern __shared__ double sm[];
  double* cs = sm;                   // [npc]
  double* sn = sm + npc;             // [npc]
  int* pp = (int*)(sm + 2 * npc);    // [npc]
  int* qq = pp + npc;                // [npc]
  double* red = sm + 3 * npc;        // [1024]
  double* A = LDS ? sm + jac_scratch(npc) : buf + g.a_off;   // [k * k]
  __shared__ int done;
  __shared__ int nrot;
  const double rel_tol = (double)k * 2.220446049250313e-16;
  const int kp = k + (k & 1);
  const int npair = kp / 2;
  if (LDS) {
    const double* Ag = buf + g.a_off;
    for (int64_t e = tid; e < (int64_t)k * k; e += nt) A[e] = Ag[e];
  }
  __shared__ double abs_floor;
  if (REL) {
    __syncthreads();
    double mx = 0.0;
    for (int i = tid; i < k; i += nt) mx = fmax(mx, fabs(A[(int64_t)i * k + i]));
    red[tid] = mx;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
      __syncthreads();
    }
    if (tid == 0) abs_floor = 4.930380657631324e-32 * red[0];   // eps^2 a_max
    __syncthreads();
  }
  // V = I
  for (int64_t e = tid; e < (int64_t)k * k; e += nt) V[e] = (e / k == e % k) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (REL) {
      if (tid == 0) nrot = 0;
      __syncthreads();
    } else {
    // convergence test: off-diagonal vs diagonal Frobenius norms
    double off = 0.0, dia = 0.0;
    for (int64_t e = tid; e < (int64_t)k * k; e += nt) {
      const double v = A[e];
      if (e / k == e % k)
        dia += v * v;
      else
        off += v * v;
    }
    red[tid] = off;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double offsum = red[0];
    __syncthreads();
    red[tid] = dia;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) done = (offsum <= 1e-30 * red[0]) || (offsum == 0.0);
    __syncthreads();
    if (done) break;
    }
    for (int rnd = 0; rnd < kp - 1; ++rnd) {
      for (int i = tid; i < npair; i += nt) {
        // circle method: position 0 fixed, others rotate by rnd
        auto player = [&](int t) { return t == 0 ? 0 : ((t - 1 + rnd) % (kp - 1)) + 1; };
        int p = player(i), q = player(kp - 1 - i);
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        double c = 1.0, s = 0.0;
        if (q < k) {
          const double apq = A[(int64_t)p * k + q];
          const double app = A[(int64_t)p * k + p], aqq = A[(int64_t)q * k + q];
          const bool rot = REL ? fabs(apq) > rel_tol * sqrt(fabs(app * aqq)) &&
                                     fabs(apq) > abs_floor
                               : (apq != 0.0 && fabs(apq) > 1e-300);
          if (rot) {
            const double tau = (aqq - app) / (2.0 * apq);
            // t = sign(tau) / (|tau| + sqrt(1 + tau^2)), ~ 1 / (2 tau) for large |tau|
            const double t = fabs(tau) > 1e150
                                 ? 0.5 / tau
                                 : (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            if (REL && s != 0.0) atomicAdd(&nrot, 1);
          }
        }
        cs[i] = c;
        sn[i] = s;
        pp[i] = p;
        qq[i] = q < k ? q : -1;
      }
      __syncthreads();
      // rows p, q <- J^T A
      for (int64_t e = tid; e < (int64_t)npair * k; e += nt) {
        const int i = (int)(e / k), col = (int)(e % k);
        const int q = qq[i];
        if (q < 0 || sn[i] == 0.0) continue;
        const int p = pp[i];
        const double c = cs[i], s = sn[i];
        const double ap = A[(int64_t)p * k + col], aq = A[(int64_t)q * k + col];
        A[(int64_t)p * k + col] = c * ap - s * aq;
        A[(int64_t)q * k + col] = s * ap + c * aq;
      }
      __syncthreads();
      // columns p, q <- A J, and V <- V J
      for (int64_t e = tid; e < (int64_t)npair * k; e += nt) {
        const int i = (int)(e / k), row = (int)(e % k);
        const int q = qq[i];
        if (q < 0 || sn[i] == 0.0) continue;
        const int p = pp[i];
        const double c = cs[i], s = sn[i];
        const double ap = A[(int64_t)row * k + p], aq = A[(int64_t)row * k + q];
        A[(int64_t)row * k + p] = c * ap - s * aq;
        A[(int64_t)row * k + q] = s * ap + c * aq;
        const double vp = V[(int64_t)row * k + p], vq = V[(int64_t)row * k + q];
        V[(int64_t)row * k + p] = c * vp - s * vq;
        V[(int64_t)row * k + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    if (REL) {
      __syncthreads();
      if (nrot == 0) break;
    }
    if (sweep == 39 && tid == 0) atomicOr(status, 4);
  }
  // sort eigenvalues descending (ties by index) and permute columns of V
  // into the k x k storage of A (A is no longer needed).
  for (int i = tid; i < k; i += nt) {
    const double li = A[(int64_t)i * k + i];
    int rank = 0;
    for (int j = 0; j < k; ++j) {
      const double lj = A[(int64_t)j * k + j];
      if (lj > li || (lj == li && j < i)) ++rank;
    }
    lam[rank] = li;
    pp[i] = rank;  // reuse: pp and qq together hold 2 npc >= k ints
  }
  __syncthreads();
  // copy V into A with permuted columns, then back into V
  for (int64_t e = tid; e < (int64_t)k * k; e += nt) {
    const int row = (int)(e / k), col = (int)(e % k);
    A[(int64_t)row * k + pp[col]] = V[e];
  }
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)k * k; e += nt) V[e] = A[e];
}

hipError_t launch_jacobi_eig(const SmallDesc* d, int nd, int max_k, double* buf, int* status,
                             hipStream_t s, bool rel) {
  if (nd <= 0) return hipSuccess;
  if (max_k > JACOBI_MAX_K || max_k < 0) return hipErrorInvalidValue;
  const int npc = std::max((max_k + 1) / 2, 1);
  // the matrix in LDS when it fits beside the scratch in 64 KiB
  const size_t scratch = (size_t)jac_scratch(npc) * sizeof(double);
  const size_t mat = (size_t)max_k * max_k * sizeof(double);
  const bool lds = scratch + mat <= 64 * 1024;
  if (lds && rel)
    k_jacobi<true, true><<<nd, 1024, scratch + mat, s>>>(d, buf, status, npc);
  else if (lds)
    k_jacobi<true, false><<<nd, 1024, scratch + mat, s>>>(d, buf, status, npc);
  else if (rel)
    k_jacobi<false, true><<<nd, 1024, scratch, s>>>(d, buf, status, npc);
  else
    k_jacobi<false, false><<<nd, 1024, scratch, s>>>(d, buf, status, npc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Global cut of one group (one workgroup each): rank every sqrt(lambda) among
// the group's sectors (descending, ties by sector then position) and keep
// ranks < chi.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_cut(const CutGroup* __restrict__ groups,
                                              const int64_t* __restrict__ lam_off_all,
                                              const int32_t* __restrict__ kk_all, int chi,
                                              const double* __restrict__ buf,
                                              int32_t* __restrict__ kept_all,
                                              CutOut* __restrict__ outs) {
  extern __shared__ double sm[];
  const CutGroup G = groups[blockIdx.x];
  const int64_t* lam_off = lam_off_all + G.s0;
  const int32_t* kk = kk_all + G.s0;
  int32_t* kept = kept_all + G.s0;
  CutOut* out = outs + blockIdx.x;
  const int nsect = G.ns, total = G.total;
  double* sig = sm;                               // [total]
  int* sec = (int*)(sm + total);                  // [total]
  int* pos = sec + total;                         // [total]
  __shared__ int kcount[1024];
  __shared__ double red1[1024], red2[1024];
  __shared__ double s_last, s_next, s_max;
  __shared__ int n_above;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < nsect; i += nt) kcount[i] = 0;
  if (tid == 0) {
    int e = 0;
    double mx = 0.0;
    for (int si = 0; si < nsect; ++si)
      for (int j = 0; j < kk[si]; ++j) {
        const double l = buf[lam_off[si] + j];
        sig[e] = l > 0.0 ? sqrt(l) : 0.0;
        mx = fmax(mx, sig[e]);
        sec[e] = si;
        pos[e] = j;
        ++e;
      }
    s_last = -1.0;
    s_next = -1.0;
    s_max = mx;
    n_above = 0;
  }
  __syncthreads();
  // values at or below floor * max are never kept
  {
    int c = 0;
    for (int i = tid; i < total; i += nt) c += sig[i] > G.floor * s_max ? 1 : 0;
    atomicAdd(&n_above, c);
  }
  __syncthreads();
  const int nkeep = chi < n_above ? chi : n_above;
  double t2 = 0.0, k2 = 0.0;
  for (int i = tid; i < total; i += nt) {
    const double si = sig[i];
    int rank = 0;
    for (int j = 0; j < total; ++j) {
      const double sj = sig[j];
      if (sj > si || (sj == si && (sec[j] < sec[i] || (sec[j] == sec[i] && pos[j] < pos[i]))))
        ++rank;
    }
    t2 += si * si;
    if (rank < nkeep) {
      atomicAdd(&kcount[sec[i]], 1);
      k2 += si * si;
    }
    if (rank == nkeep - 1) s_last = si;
    if (rank == nkeep) s_next = si;
  }
  red1[tid] = t2;
  red2[tid] = k2;
  __syncthreads();
  for (int w = nt / 2; w > 0; w >>= 1) {
    if (tid < w) {
      red1[tid] += red1[tid + w];
      red2[tid] += red2[tid + w];
    }
    __syncthreads();
  }
  for (int i = tid; i < nsect; i += nt) kept[i] = kcount[i];
  if (tid == 0) {
    out->total2 = red1[0];
    out->kept2 = red2[0];
    out->s_last = s_last;
    out->s_next = s_next;
  }
}

hipError_t launch_cut(const CutGroup* groups, int ngroups, int max_ns, int max_total,
                      const int64_t* lam_off, const int32_t* k, int chi,
                      const double* buf, int32_t* kept, CutOut* out, hipStream_t s) {
  if (ngroups <= 0) return hipSuccess;
  if (max_ns > 1024) return hipErrorInvalidValue;
  const size_t shm = (size_t)max_total * (sizeof(double) + 2 * sizeof(int));
  if (shm > 96 * 1024) return hipErrorInvalidValue;
  k_cut<<<dim3(ngroups), 1024, shm, s>>>(groups, lam_off, k, chi, buf, kept, out);
  return hipGetLastError();
}

// SVQB scaling (Stathopoulos & Wu, SIAM J. Sci. Comput. 23 (2002) 2165):
// column i of the k x k eigenvector matrix at b_off is multiplied by
// 1/sqrt(lambda_i), or set to zero when lambda_i <= tau * lambda_0.
__global__ void k_svqb_scale(const SmallDesc* __restrict__ d, double* __restrict__ buf, double tau) {
  const SmallDesc g = d[blockIdx.x];
  const int k = g.k;
  double* V = buf + g.b_off;
  const double* lam = buf + g.c_off;
  const double l0 = lam[0];
  for (int64_t e = threadIdx.x; e < (int64_t)k * k; e += blockDim.x) {
    const int col = (int)(e % k);
    const double l = lam[col];
    V[e] *= (l > tau * l0 && l > 0.0) ? 1.0 / sqrt(l) : 0.0;
  }
}

hipError_t launch_svqb_scale(const SmallDesc* d, int nd, double* buf, double tau, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  k_svqb_scale<<<nd, 256, 0, s>>>(d, buf, tau);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// canonical column signs
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sign_fix(const SignDesc* __restrict__ d,
                                                  const int32_t* __restrict__ col_desc,
                                                  double* __restrict__ U, double* __restrict__ R) {
  const SignDesc g = d[col_desc[blockIdx.x]];
  const int c = blockIdx.x - g.col0;
  __shared__ double bv[256];
  __shared__ int bi[256];
  // pass 1: largest magnitude of the column
  double best = 0.0;
  for (int i = threadIdx.x; i < g.m; i += blockDim.x)
    best = fmax(best, fabs(U[g.u_off + (int64_t)i * g.ncol + c]));
  bv[threadIdx.x] = best;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) bv[threadIdx.x] = fmax(bv[threadIdx.x], bv[threadIdx.x + w]);
    __syncthreads();
  }
  const double thr = bv[0] * (1.0 - 1e-5);
  // pass 2: first row whose magnitude reaches the threshold
  int first = 0x7fffffff;
  for (int i = threadIdx.x; i < g.m; i += blockDim.x)
    if (fabs(U[g.u_off + (int64_t)i * g.ncol + c]) >= thr) {
      first = i;
      break;
    }
  bi[threadIdx.x] = first;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) bi[threadIdx.x] = min(bi[threadIdx.x], bi[threadIdx.x + w]);
    __syncthreads();
  }
  const int imax = bi[0];
  if (imax >= g.m) return;
  const bool flip = U[g.u_off + (int64_t)imax * g.ncol + c] < 0.0;
  __syncthreads();
  if (!flip) return;
  for (int i = threadIdx.x; i < g.m; i += blockDim.x) U[g.u_off + (int64_t)i * g.ncol + c] *= -1.0;
  if (R)
    for (int j = threadIdx.x; j < g.n; j += blockDim.x) R[g.r_off + (int64_t)c * g.n + j] *= -1.0;
}

hipError_t launch_sign_fix(const SignDesc* d, int nd, int total_cols, const int32_t* col_desc,
                           double* U, double* R, hipStream_t s) {
  if (nd <= 0 || total_cols <= 0) return hipSuccess;
  k_sign_fix<<<total_cols, 256, 0, s>>>(d, col_desc, U, R);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-sector helpers of the bond expansion
// ---------------------------------------------------------------------------
// out[o + i n + j] = in[o + i n + j] * sc[s0 + i] for the rows of every
// sector (row-major rows x n blocks)
__global__ void k_row_scale(const SectDesc* __restrict__ d, const double* __restrict__ in,
                            double* __restrict__ out, const double* __restrict__ sc) {
  const SectDesc g = d[blockIdx.y];
  const int64_t tot = (int64_t)g.rows * g.cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x)
    out[g.off_out + e] = in[g.off_a + e] * sc[g.s0 + e / g.cols];
}

hipError_t launch_row_scale(const SectDesc* d, int nd, int64_t max_elems, const double* in,
                            double* out, const double* sc, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  int64_t bx = (max_elems + 255) / 256;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  k_row_scale<<<dim3((unsigned)bx, nd), 256, 0, s>>>(d, in, out, sc);
  return hipGetLastError();
}

// Columns side by side: out (rows x (ca + cb)) = [A (rows x ca) | B (rows x cb)]
__global__ void k_merge_cols(const SectDesc* __restrict__ d, const double* __restrict__ A,
                             const double* __restrict__ B, double* __restrict__ out) {
  const SectDesc g = d[blockIdx.y];
  const int c = g.cols + g.cols_b;
  const int64_t tot = (int64_t)g.rows * c;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / c;
    const int j = (int)(e % c);
    out[g.off_out + e] = j < g.cols ? A[g.off_a + r * g.cols + j]
                                    : B[g.off_b + r * g.cols_b + (j - g.cols)];
  }
}

hipError_t launch_merge_cols(const SectDesc* d, int nd, int64_t max_elems, const double* A,
                             const double* B, double* out, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  int64_t bx = (max_elems + 255) / 256;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  k_merge_cols<<<dim3((unsigned)bx, nd), 256, 0, s>>>(d, A, B, out);
  return hipGetLastError();
}

// Rows one after the other, B transposed: out ((ra + cb) x n) = [A (ra x n) ;
// B^T], B given as n x cb (row-major)
__global__ void k_stack_rows_t(const SectDesc* __restrict__ d, const double* __restrict__ A,
                               const double* __restrict__ B, double* __restrict__ out) {
  const SectDesc g = d[blockIdx.y];
  const int n = g.cols;
  const int64_t tot = (int64_t)(g.rows + g.cols_b) * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n;
    const int j = (int)(e % n);
    out[g.off_out + e] = r < g.rows ? A[g.off_a + r * n + j]
                                    : B[g.off_b + (int64_t)j * g.cols_b + (r - g.rows)];
  }
}

hipError_t launch_stack_rows_t(const SectDesc* d, int nd, int64_t max_elems, const double* A,
                               const double* B, double* out, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  int64_t bx = (max_elems + 255) / 256;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  k_stack_rows_t<<<dim3((unsigned)bx, nd), 256, 0, s>>>(d, A, B, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reductions and elementwise helpers
// ---------------------------------------------------------------------------
__global__ void k_sumsq_partial(const double* __restrict__ x, int64_t n,
                                double* __restrict__ partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    s += x[e] * x[e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_sum_final(const double* __restrict__ partial, int n, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_sumsq(const double* x, int64_t n, double* partial, double* out, hipStream_t s) {
  const int nb = 512;
  k_sumsq_partial<<<nb, 256, 0, s>>>(x, n, partial);
  k_sum_final<<<1, 256, 0, s>>>(partial, nb, out);
  return hipGetLastError();
}

__global__ void k_scale(double* __restrict__ x, int64_t n, double a) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] *= a;
}

hipError_t launch_scale(double* x, int64_t n, double a, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  k_scale<<<(unsigned)nb, 256, 0, s>>>(x, n, a);
  return hipGetLastError();
}

__global__ void k_fill(double* __restrict__ x, int64_t n, double v) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = v;
}

hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  k_fill<<<(unsigned)nb, 256, 0, s>>>(x, n, v);
  return hipGetLastError();
}

__global__ void k_fill_int(int* __restrict__ x, int64_t n, int v) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] = v;
}

hipError_t launch_fill_int(int* x, int64_t n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  k_fill_int<<<(unsigned)nb, 256, 0, s>>>(x, n, v);
  return hipGetLastError();
}

__global__ void k_add(double* __restrict__ x, const double* __restrict__ y, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[e] += y[e];
}

hipError_t launch_add(double* x, const double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  k_add<<<(unsigned)nb, 256, 0, s>>>(x, y, n);
  return hipGetLastError();
}

__global__ void k_check_finite(const double* __restrict__ x, int64_t n, int* __restrict__ flag) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(x[e])) {
      atomicOr(flag, 1);
      return;
    }
}

hipError_t launch_check_finite(const double* x, int64_t n, int* flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  k_check_finite<<<(unsigned)nb, 256, 0, s>>>(x, n, flag);
  return hipGetLastError();
}

}  // namespace fp
