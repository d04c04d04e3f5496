// The network value of two environments with no device allocation: every
// workspace buffer of the contraction (partial environments, intermediates,
// reductions, GEMM plans) is carved out of one file-scope device array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "driver.hpp"

namespace fp {

// One per device, held until the process ends.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex scratch_mu;
void* scratch_dev[64] = {nullptr};   // device address of ``scratch`` per device
}  // namespace

// With ``device`` current: the device address of the array (host code may
// not use its name as an address).
Status scratch_init(int device) {
  if (device < 0 || device >= 64) return fail(FPEPS_ERR_ARG, "device id");
  std::lock_guard<std::mutex> g(scratch_mu);
  if (scratch_dev[device]) return Status::ok();
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(FPEPS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  scratch_dev[device] = p;
  return Status::ok();
}

Status overlap_noalloc(fpeps_ctx_s* ctx, int L, const fpeps_tensor* top, const fpeps_tensor* bot,
                       double log_norm, int32_t* sign, double* log_abs) {
  FP_TRY(scratch_init(ctx->device));
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> g(scratch_mu);
    base = scratch_dev[ctx->device];
  }
  // the arena is the whole array; it is left as the call leaves it
  ctx->arena_begin((char*)base, NOALLOC_SCRATCH_BYTES);
  Status st = overlap(ctx, L, top, bot, log_norm, sign, log_abs);
  ctx->arena_end();
  if (!st.good() && st.code == FPEPS_ERR_CAPACITY)
    return fail(FPEPS_ERR_CAPACITY, st.msg);
  return st;
}

}  // namespace fp
