// Context, workspace and plan upload.
#include "core.hpp"

#include <algorithm>
#include <cstring>

fpeps_ctx_s::~fpeps_ctx_s() {
  if (!bufs.empty() || !evpool.empty()) (void)hipDeviceSynchronize();
  for (auto e : evpool) (void)hipEventDestroy(e);
  for (auto& kv : bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
}

fp::Status fpeps_ctx_s::buf(const std::string& name, size_t bytes, void** out) {
  fp::DevBuf& b = bufs[name];
  if (b.bytes < bytes) {
    if (b.p) {
      FP_HIP(hipStreamSynchronize(stream));
      FP_HIP(hipFree(b.p));
      b.p = nullptr;
      b.bytes = 0;
    }
    size_t want = std::max(bytes, (size_t)4096);
    want = (want + 4095) / 4096 * 4096;
    if (hipMalloc(&b.p, want) != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      return fp::fail(FPEPS_ERR_NOMEM, "device allocation of " + std::to_string(want) +
                                           " bytes failed (" + name + ")");
    }
    b.bytes = want;
  }
  *out = b.p;
  return fp::Status::ok();
}

fp::Status fpeps_ctx_s::upload(const std::string& name, const void* host, size_t bytes,
                               void** dev) {
  FP_TRY(buf(name, bytes, dev));
  if (bytes) {
    // the previous contents may still be read by queued kernels
    FP_HIP(hipStreamSynchronize(stream));
    FP_HIP(hipMemcpy(*dev, host, bytes, hipMemcpyHostToDevice));
  }
  return fp::Status::ok();
}

fp::Status fpeps_ctx_s::sync() {
  FP_HIP(hipStreamSynchronize(stream));
  if (time_kernels && evused) return harvest_timing();
  return fp::Status::ok();
}

fp::Status fpeps_ctx_s::timed_events(hipEvent_t* a, hipEvent_t* b) {
  while (evpool.size() < evused + 2) {
    hipEvent_t e;
    FP_HIP(hipEventCreate(&e));
    evpool.push_back(e);
  }
  *a = evpool[evused];
  *b = evpool[evused + 1];
  evused += 2;
  return fp::Status::ok();
}

fp::Status fpeps_ctx_s::harvest_timing() {
  for (size_t i = 0; i + 1 < evused; i += 2) {
    float ms = 0;
    FP_HIP(hipEventElapsedTime(&ms, evpool[i], evpool[i + 1]));
    kt_seconds += ms * 1e-3;
    kt_flops += evflops[i / 2];
    ++kt_launches;
  }
  evused = 0;
  evflops.clear();
  return fp::Status::ok();
}

namespace fp {

Status PlanSet::upload(fpeps_ctx_s* ctx, const std::string& tag) {
  std::vector<GemmJob> jobs;
  std::vector<GemmPair> pairs;
  std::vector<std::pair<size_t, size_t>> range;
  for (auto& p : plans) {
    const int32_t base = (int32_t)pairs.size();
    const size_t j0 = jobs.size();
    for (auto j : p.jobs) {
      j.p0 += base;
      j.p1 += base;
      jobs.push_back(j);
    }
    pairs.insert(pairs.end(), p.pairs.begin(), p.pairs.end());
    range.emplace_back(j0, p.jobs.size());
  }
  if (pairs.size() > (size_t)INT32_MAX || jobs.size() > (size_t)INT32_MAX)
    return fail(FPEPS_ERR_UNSUPPORTED, "plan too large");
  void *dj = nullptr, *dp = nullptr, *dt = nullptr;
  FP_TRY(ctx->upload(tag + "_jobs", jobs.data(), jobs.size() * sizeof(GemmJob), &dj));
  FP_TRY(ctx->upload(tag + "_pairs", pairs.data(), pairs.size() * sizeof(GemmPair), &dp));
  FP_TRY(ctx->upload(tag + "_tab", pool.data.data(), pool.data.size() * sizeof(int32_t), &dt));
  dtab = (int32_t*)dt;
  dev.clear();
  for (size_t i = 0; i < plans.size(); ++i) {
    DevGemm g;
    g.jobs = (const GemmJob*)dj + range[i].first;
    g.pairs = (const GemmPair*)dp;
    g.njobs = (int)range[i].second;
    g.mt = plans[i].mt;
    g.nt = plans[i].nt;
    dev.push_back(g);
  }
  return Status::ok();
}

Status run_gemm(fpeps_ctx_s* ctx, const PlanSet& ps, int idx, const double* A, int64_t a_size,
                const double* B, int64_t b_size, double* C, int64_t c_size, bool timed) {
  const GemmPlan& p = ps.plans[idx];
  if (p.jobs.empty()) return Status::ok();
  // every table-addressed access must stay inside its buffer
  if (p.a_extent > a_size || p.b_extent > b_size || p.c_extent > c_size)
    return fail(FPEPS_ERR_SHAPE, "plan reaches outside a buffer (a " + std::to_string(p.a_extent) +
                                     "/" + std::to_string(a_size) + ", b " +
                                     std::to_string(p.b_extent) + "/" + std::to_string(b_size) +
                                     ", c " + std::to_string(p.c_extent) + "/" +
                                     std::to_string(c_size) + ")");
  if (!A || !B || !C) return fail(FPEPS_ERR_ARG, "null operand buffer");
  if (timed && ctx->time_kernels) {
    hipEvent_t a, b;
    FP_TRY(ctx->timed_events(&a, &b));
    ctx->evflops.push_back(p.flops);
    FP_HIP(hipEventRecord(a, ctx->stream));
    FP_HIP(launch_gemm_f64(ps.dev[idx], A, B, C, ps.dtab, ctx->stream));
    FP_HIP(hipEventRecord(b, ctx->stream));
    return Status::ok();
  }
  FP_HIP(launch_gemm_f64(ps.dev[idx], A, B, C, ps.dtab, ctx->stream));
  return Status::ok();
}

}  // namespace fp
