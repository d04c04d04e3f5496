// Randomized SVD driver, row absorption, explicit-matrix rSVD / CBE and the
// overlap of two environments (see driver.cpp).
#pragma once

#include <functional>
#include <vector>

#include "core.hpp"
#include "site.hpp"

namespace fp {

// An operator given as independent sectors with per-sector row/column
// counts m, n. ``prepare`` receives the sketch widths before the first
// application; ``apply`` maps per-sector n_J x k_J matrices (concatenated in
// sector order) to m_J x k_J ones, or back when transposed.
struct RsvdIO {
  std::vector<int64_t> m, n;
  std::vector<int64_t> width_m, width_n;   // sizes deciding the widths (default m, n)
  std::vector<uint32_t> c1;                // sketch counter word per sector
  uint32_t c2 = 0, c3 = 0;
  // independent truncation problems in one batch: group of every sector
  // (empty: one group), its own widths and cut; c2v (if set) replaces c2 per
  // sector
  std::vector<int32_t> grp;
  std::vector<uint32_t> c2v;
  // guess of each sector's kept count (-1: none; empty: none), e.g. the
  // previous site's kept count for the same sector label
  std::vector<int32_t> hint;
  std::function<Status(const std::vector<int32_t>&)> prepare;
  // apply(transpose, final, x, y): y = M x or M^T x; ``final`` marks the
  // last range-finder product (it fixes Q) and the projection B^T = M^T Q
  // (FP64 intermediates in mixed precision; the earlier range-finder
  // products tolerate FP32 intermediates, their rounding being damped by
  // the later multiplications)
  std::function<Status(bool, bool, const double*, double*)> apply;
};

struct RsvdOut {
  std::vector<int32_t> k, kept;
  std::vector<int64_t> row_off, col_off, small_off, lam_off;
  int64_t S = 0;
  double* Q = nullptr;       // row layout
  double* Bt = nullptr;      // column layout, B^T = M^T Q
  double* small = nullptr;   // [G | U~ (k x k per sector) | eigenvalues | V0]
  std::vector<double> lam;   // eigenvalues of B B^T, per sector descending
  CutOut cut{};                // group 0 (the only one of a single problem)
  std::vector<CutOut> cuts;    // every group
  uint32_t fallbacks = 0;
  // widths and kept counts of every factorisation pass (a pass with a
  // saturated sector is followed by one with that sector widened)
  std::vector<std::vector<int32_t>> pass_k, pass_kept;
};

Status rsvd_run(fpeps_ctx_s* ctx, RsvdIO& io, int chi, int p, int q, uint64_t seed, RsvdOut& out,
                double sv_cut);
Status rsvd_factors(fpeps_ctx_s* ctx, const RsvdIO& io, const RsvdOut& r,
                    const std::vector<int64_t>& uoff, double* Uout, int64_t u_size,
                    const std::vector<int64_t>& roff, double* Rout, int64_t r_size);
Status absorb_row(fpeps_ctx_s* ctx, int L, const fpeps_tensor* env_in, const fpeps_tensor* ket,
                  const fpeps_tensor* pepo, const fpeps_opts* o, fpeps_tensor* env_out,
                  double* log_norm, fpeps_report* rep);
Status make_site(fpeps_ctx_s* ctx, const fpeps_tensor* R, const fpeps_tensor* T,
                 const fpeps_tensor* A, const fpeps_tensor* W, const fpeps_opts* o, SiteOp& op);
Status explicit_rsvd(fpeps_ctx_s* ctx, int nmat, const int64_t* m, const int64_t* n,
                     const double* const* A, const fpeps_opts* o, double* const* U_out,
                     double* const* R_out, int32_t* kept, double* sigma, fpeps_report* rep,
                     const int32_t* r, const double* const* U, const double* const* V, bool cbe,
                     const int32_t* group = nullptr);
Status overlap(fpeps_ctx_s* ctx, int L, const fpeps_tensor* top, const fpeps_tensor* bot,
               double log_norm, int32_t* sign, double* log_abs);
Status axpy_inplace(fpeps_ctx_s* ctx, double* x, const double* y, int64_t n);
// y = H_eff A (heff.cpp)
Status heff_apply(fpeps_ctx_s* ctx, const fpeps_tensor* T, const fpeps_tensor* L,
                  const fpeps_tensor* B, const fpeps_tensor* R, const fpeps_tensor* W,
                  const fpeps_tensor* A, const fpeps_opts* o, fpeps_tensor* y,
                  fpeps_report* rep);
// The prepared effective operator (T L and B R once, the vector-dependent
// steps as a replayed HIP graph); ``y`` receives the output structure and
// the product for A.
Status heff_prepare(fpeps_ctx_s* ctx, const fpeps_tensor* T, const fpeps_tensor* L,
                    const fpeps_tensor* B, const fpeps_tensor* R, const fpeps_tensor* W,
                    const fpeps_tensor* A, const fpeps_opts* o, fpeps_tensor* y,
                    fpeps_heff_s** out, fpeps_report* rep);
Status heff_apply_prepared(fpeps_heff_s* h, const double* a, int64_t a_elems, double* y,
                           int64_t y_elems, fpeps_report* rep);
fpeps_ctx_s* heff_context(fpeps_heff_s* h);
// frees the handle and its device buffers
Status heff_release(fpeps_heff_s* h);

// Autotuner (tune.cpp): measures slice budgets and GEMM tiles on the row,
// keeps the table in the context, and returns the row absorbed with it.
Status autotune_absorb(fpeps_ctx_s* ctx, int L, const fpeps_tensor* env_in,
                       const fpeps_tensor* ket, const fpeps_tensor* pepo, const fpeps_opts* o,
                       int ncand, fpeps_tensor* env_out, double* log_norm, fpeps_report* rep);
Status tune_save(fpeps_ctx_s* ctx, const char* path);
Status tune_load(fpeps_ctx_s* ctx, const char* path);
Status tune_clear(fpeps_ctx_s* ctx);
Status tune_info(fpeps_ctx_s* ctx, int32_t* entries, int64_t* slice_budget);

// Bytes of the file-scope device array behind fpeps_expect_noalloc.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
// The array's device address on ``device`` (that device current), looked up
// once per device.
Status scratch_init(int device);
// overlap() with every workspace buffer in that array (no allocation)
Status overlap_noalloc(fpeps_ctx_s* ctx, int L, const fpeps_tensor* top, const fpeps_tensor* bot,
                       double log_norm, int32_t* sign, double* log_abs);

}  // namespace fp
