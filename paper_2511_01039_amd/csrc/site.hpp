// The implicit site operator M_x of one zip-up step and its transpose, as a
// chain of planned block-sparse contractions (Sec. 3 contraction pattern
// 2(a), applied layer by layer; Sec. 4 matrix A).
#pragma once

#include <array>
#include <memory>
#include <string>
#include <vector>

#include "core.hpp"

namespace fp {

struct Sector {
  std::vector<int32_t> label;                     // nlab ints
  std::vector<std::array<uint16_t, 4>> cols;      // (b, rk, rw, rb) sector tuples
  std::vector<int64_t> crow;                      // first row of each tuple in the n x k matrix
  std::vector<int64_t> cdim;                      // rows of each tuple
  int64_t n = 0;
  std::vector<std::array<uint16_t, 4>> rows;      // (c, dk, dw, db) tuples
  std::vector<int64_t> rrow, rdim;
  int64_t m = 0;
};

struct SliceCol {
  int sect;      // sector ordinal
  int j0, j1;    // column range of that sector
};

// Device tensors of one site (all double, caller or library memory).
struct SiteData {
  const double* T = nullptr;
  const double* A = nullptr;
  const double* W = nullptr;
  const double* R = nullptr;
  int64_t T_size = 0, A_size = 0, W_size = 0, R_size = 0;
  // FP32 copies of T and R (mixed precision: the environment and remainder
  // products of the earlier range-finder applications run on FP32 MFMA)
  const float* T32 = nullptr;
  const float* R32 = nullptr;
};

// The part of a site's structure analysis that depends only on T, the ket
// and the PEPO (not on the remainder): the column sectors, and the forward
// chain up to X4 at unit width. Interior sites of a row share it.
struct FwdAnalysis {
  std::string key;                              // structure of T, ket and W
  std::vector<Sector> sect;                     // column sectors (rows empty)
  std::vector<std::vector<int64_t>> unit;       // [sector][X1..X4 elements per unit width]
  BT x4;                                        // X4 structure at unit width
};

class SiteOp {
 public:
  SymInfo sym;
  int nlab = 1;
  BT T, ket, W, bra, R;
  SiteData dev;
  std::vector<Sector> sect;
  std::vector<std::vector<int64_t>> unit_size;  // [sector][8]: elements per unit width of X1..X4, Z4..Z1

  // Build legs/blocks. R is the remainder [c, a, lk, lw, lb].
  Status init(const SymInfo& s, int nlab_, BT&& T_, BT&& ket_, BT&& W_, BT&& R_,
              const SiteData& d);
  // Sector structure (columns, rows via a structure-only forward pass).
  // ``fwd``, when given, holds the remainder-independent part of a previous
  // site's analysis: it is reused when that site's T, ket and W structure
  // equals this one's, and replaced otherwise.
  Status analyse(FwdAnalysis* fwd = nullptr);
  // Everything the analysis and the plans depend on, serialised: symmetry,
  // and the legs, block sectors, offsets and strides of T, ket, W, bra and
  // R (not their data). Two sites with equal keys have equal sectors, and
  // equal plans for equal widths.
  std::string structure_key() const;
  // the same for T, ket and W only (the bra is the ket)
  std::string structure_key_tkw() const;

  // Plans of M (fwd) and M^T (bwd) for per-sector widths k, sliced so that
  // the chain intermediates of one slice fit ``budget`` bytes.
  struct Slice {
    std::shared_ptr<PlanSet> ps;   // this slice's forward plans (planned independently)
    std::shared_ptr<PlanSet> psb;  // and its transposed-chain plans
    double flops_fwd = 0, flops_bwd = 0;
    std::vector<SliceCol> cols;
    int fwd[5], bwd[5];       // plan indices in the PlanSet (GEMM or row-thread list)
    bool fwd_rt[5] = {false, false, false, false, false};
    bool bwd_rt[5] = {false, false, false, false, false};
    int64_t size1 = 0, size2 = 0;    // ping-pong intermediate sizes (elements), forward
    int64_t bsize1 = 0, bsize2 = 0;  // and transposed chain
  };
  struct Plans {
    std::vector<Slice> slices;
    std::vector<int64_t> col_off, row_off;   // per sector offsets for width k
    int64_t col_total = 0, row_total = 0;
    int64_t ws1 = 0, ws2 = 0;   // elements of the two ping-pong intermediates
    double flops_fwd = 0, flops_bwd = 0;
    bool f32 = false;           // FP32 operands: steps 1 and 5 on FP32 MFMA, FP32 intermediates
  };
  Status plan(fpeps_ctx_s* ctx, const std::vector<int32_t>& k, int64_t budget, Plans& out,
              bool with_bwd = true, bool f32 = false);
  // the two halves of plan(): host planning (no device work), and the upload
  // of the plans with this site's packed layer blocks (plans of another site
  // with the same structure key can be uploaded for this one)
  Status plan_host(const std::vector<int32_t>& k, int64_t budget, Plans& out, bool with_bwd,
                   bool f32) const;
  // the transposed-chain plans of every slice of ``out`` (planned by
  // plan_host without them). Thread safe against apply() of the forward
  // chain: it writes only the transposed fields of the slices. Call
  // sum_plans() afterwards, on the thread that uses ``out``.
  Status plan_bwd(const std::vector<int32_t>& k, Plans& out) const;
  // totals of ``out`` (flops, intermediate sizes) from its slices
  void sum_plans(Plans& out) const;
  // which: 1 the forward plans, 2 the transposed ones, 3 both
  Status upload(fpeps_ctx_s* ctx, Plans& pl, int which = 3) const;
  // y = M x (transpose = false) or M^T x, per-sector matrices at the offsets
  // of ``pl`` (x: col layout for M, row layout for M^T). ``f32`` stores the
  // chain intermediates of this application in FP32 and runs its
  // environment and remainder products on FP32 MFMA (FP32 accumulation per K
  // tile, tiles summed in FP64)
  // (make_f32_operands first); the layer steps keep FP64 arithmetic.
  Status apply(fpeps_ctx_s* ctx, const Plans& pl, bool transpose, const double* x, double* y,
               bool f32);
  // FP32 copies of T and R in the context's workspace (for apply with f32)
  Status make_f32_operands(fpeps_ctx_s* ctx);

 private:
  BT omega_layout(const std::vector<SliceCol>& cols, const std::vector<int32_t>& k,
                  const std::vector<int64_t>& off, int64_t total, bool rows) const;
  // forward (bwd = false) or transposed chain plans of one slice (host only,
  // thread safe; the two directions write different fields of the slice)
  Status plan_slice(const std::vector<int32_t>& k, const Plans& pl, Slice& sl, bool bwd) const;
};

// Convert an fpeps_tensor into a planner BT with the given leg names.
Status tensor_to_bt(const fpeps_tensor* t, const std::vector<int>& names, int nlab, BT& out,
                    bool flip_dirs = false);

// Canonical leg orders of the chain intermediates (the keys of the per-pair
// scalars): X0 = Omega, X1 .. X4, Y.
extern const std::vector<int> ORDER_X[6];

}  // namespace fp
