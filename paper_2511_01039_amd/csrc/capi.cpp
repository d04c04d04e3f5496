// extern "C" entry points (include/fpeps.h). No exception crosses the ABI.
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "driver.hpp"

namespace {

fpeps_status finish(fpeps_ctx ctx, const fp::Status& s) {
  if (ctx) ctx->err = s.good() ? std::string() : s.msg;
  return s.code;
}

template <class F>
fpeps_status guarded(fpeps_ctx ctx, F&& f) {
  if (!ctx) return FPEPS_ERR_ARG;
  try {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return finish(ctx, fp::fail(FPEPS_ERR_HIP, hipGetErrorString(e)));
    return finish(ctx, f());
  } catch (const std::bad_alloc&) {
    return finish(ctx, fp::fail(FPEPS_ERR_NOMEM, "host allocation failed"));
  } catch (const std::exception& ex) {
    return finish(ctx, fp::fail(FPEPS_ERR_ARG, std::string("internal error: ") + ex.what()));
  } catch (...) {
    return finish(ctx, fp::fail(FPEPS_ERR_ARG, "internal error"));
  }
}

}  // namespace

extern "C" {

const char* fpeps_version(void) { return "fpeps-gfx950 0.1 (fp64)"; }

fpeps_status fpeps_create(fpeps_ctx* out, int32_t device, void* stream) {
  if (!out) return FPEPS_ERR_ARG;
  *out = nullptr;
  try {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
      (void)hipGetLastError();
      return FPEPS_ERR_NODEVICE;
    }
    if (device < 0 || device >= n) return FPEPS_ERR_NODEVICE;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return FPEPS_ERR_NODEVICE;
    if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0) return FPEPS_ERR_NODEVICE;
    if (hipSetDevice(device) != hipSuccess) return FPEPS_ERR_HIP;
    // device address of the no-allocation scratch array, once per device
    if (!fp::scratch_init(device).good()) return FPEPS_ERR_HIP;
    fpeps_ctx c = new fpeps_ctx_s();
    c->device = device;
    c->stream = (hipStream_t)stream;
    *out = c;
    return FPEPS_OK;
  } catch (...) {
    return FPEPS_ERR_NOMEM;
  }
}

fpeps_status fpeps_destroy(fpeps_ctx ctx) {
  if (!ctx) return FPEPS_ERR_ARG;
  (void)hipSetDevice(ctx->device);
  delete ctx;
  return FPEPS_OK;
}

fpeps_status fpeps_set_stream(fpeps_ctx ctx, void* stream) {
  if (!ctx) return FPEPS_ERR_ARG;
  ctx->stream = (hipStream_t)stream;
  return FPEPS_OK;
}

const char* fpeps_last_error(fpeps_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

fpeps_status fpeps_set_allocator(fpeps_ctx ctx, void* (*alloc)(size_t, void*),
                                 void (*free_)(void*, void*), void* user) {
  return guarded(ctx, [&]() -> fp::Status {
    if ((alloc == nullptr) != (free_ == nullptr))
      return fp::fail(FPEPS_ERR_ARG, "give both allocator functions or neither");
    // buffers from the previous allocator go back to it first
    FP_TRY(ctx->release_workspace());
    ctx->alloc_fn = alloc;
    ctx->free_fn = free_;
    ctx->alloc_user = alloc ? user : nullptr;
    return fp::Status::ok();
  });
}

fpeps_status fpeps_env_absorb(fpeps_ctx ctx, int32_t L, const fpeps_tensor* env_in,
                              const fpeps_tensor* ket, const fpeps_tensor* pepo,
                              const fpeps_opts* opts, fpeps_tensor* env_out, double* log_norm,
                              fpeps_report* report) {
  return guarded(ctx, [&] {
    if (report) std::memset(report, 0, sizeof(*report));
    return fp::absorb_row(ctx, L, env_in, ket, pepo, opts, env_out, log_norm, report);
  });
}

fpeps_status fpeps_autotune_absorb(fpeps_ctx ctx, int32_t L, const fpeps_tensor* env_in,
                                   const fpeps_tensor* ket, const fpeps_tensor* pepo,
                                   const fpeps_opts* opts, int32_t tile_candidates,
                                   fpeps_tensor* env_out, double* log_norm,
                                   fpeps_report* report) {
  return guarded(ctx, [&] {
    if (report) std::memset(report, 0, sizeof(*report));
    return fp::autotune_absorb(ctx, L, env_in, ket, pepo, opts, tile_candidates, env_out,
                               log_norm, report);
  });
}

fpeps_status fpeps_tune_save(fpeps_ctx ctx, const char* path) {
  return guarded(ctx, [&] { return fp::tune_save(ctx, path); });
}

fpeps_status fpeps_tune_load(fpeps_ctx ctx, const char* path) {
  return guarded(ctx, [&] { return fp::tune_load(ctx, path); });
}

fpeps_status fpeps_tune_clear(fpeps_ctx ctx) {
  return guarded(ctx, [&] { return fp::tune_clear(ctx); });
}

fpeps_status fpeps_tune_info(fpeps_ctx ctx, int32_t* entries, int64_t* slice_budget) {
  return guarded(ctx, [&] { return fp::tune_info(ctx, entries, slice_budget); });
}

fpeps_status fpeps_absorb_diag(fpeps_ctx ctx, int32_t site, int32_t capacity, double* sigma,
                               int32_t* sector, int32_t* count, int32_t* nsectors,
                               int32_t* kept) {
  if (!ctx) return FPEPS_ERR_ARG;
  if (site < 0 || site >= (int)ctx->diag.size() || !count || !nsectors)
    return finish(ctx, fp::fail(FPEPS_ERR_ARG, "no diagnostics for this site"));
  const fp::SiteDiag& d = ctx->diag[site];
  *count = (int32_t)d.sigma.size();
  *nsectors = (int32_t)d.kept.size();
  if ((int)d.sigma.size() > capacity || (int)d.kept.size() > capacity)
    return finish(ctx, fp::fail(FPEPS_ERR_CAPACITY, "diagnostic capacity too small"));
  for (size_t i = 0; i < d.sigma.size(); ++i) {
    if (sigma) sigma[i] = d.sigma[i];
    if (sector) sector[i] = d.sector[i];
  }
  if (kept)
    for (size_t i = 0; i < d.kept.size(); ++i) kept[i] = d.kept[i];
  return finish(ctx, fp::Status::ok());
}

fpeps_status fpeps_site_shape(fpeps_ctx ctx, const fpeps_tensor* R, const fpeps_tensor* T,
                              const fpeps_tensor* A, const fpeps_tensor* W,
                              const fpeps_opts* opts, int32_t capacity, int32_t* nsect,
                              int32_t* labels, int64_t* m, int64_t* n) {
  return guarded(ctx, [&]() -> fp::Status {
    if (!nsect) return fp::fail(FPEPS_ERR_ARG, "null nsect");
    fp::SiteOp op;
    FP_TRY(fp::make_site(ctx, R, T, A, W, opts, op));
    const int ns = (int)op.sect.size();
    *nsect = ns;
    if (ns > capacity) return fp::fail(FPEPS_ERR_CAPACITY, "sector capacity too small");
    for (int J = 0; J < ns; ++J) {
      if (m) m[J] = op.sect[J].m;
      if (n) n[J] = op.sect[J].n;
      if (labels)
        for (int i = 0; i < op.nlab; ++i) labels[J * op.nlab + i] = op.sect[J].label[i];
    }
    return fp::Status::ok();
  });
}

fpeps_status fpeps_site_apply(fpeps_ctx ctx, const fpeps_tensor* R, const fpeps_tensor* T,
                              const fpeps_tensor* A, const fpeps_tensor* W,
                              const fpeps_opts* opts, int32_t transpose, const int32_t* k,
                              const double* x_in, double* y_out, fpeps_report* report) {
  return guarded(ctx, [&]() -> fp::Status {
    if (!k || !x_in || !y_out) return fp::fail(FPEPS_ERR_ARG, "null argument");
    if (opts->precision != FPEPS_FP64 && opts->precision != FPEPS_FP32)
      return fp::fail(FPEPS_ERR_UNSUPPORTED, "precision: FPEPS_FP64 or FPEPS_FP32");
    if (report) std::memset(report, 0, sizeof(*report));
    fp::SiteOp op;
    FP_TRY(fp::make_site(ctx, R, T, A, W, opts, op));
    std::vector<int32_t> kk(k, k + op.sect.size());
    for (int v : kk)
      if (v < 0) return fp::fail(FPEPS_ERR_ARG, "negative width");
    fp::SiteOp::Plans pl;
    // one budget for the chain intermediates of all streams: up to
    // max_streams slices are live at once, each within its share
    const int64_t budget =
        std::max<int64_t>(1, ctx->total_budget(opts) / std::max(1, ctx->max_streams));
    ctx->peak_ws = 0;
    ctx->nslices = 0;
    FP_TRY(op.plan(ctx, kk, budget, pl, transpose != 0, opts->precision == FPEPS_FP32));
    if (opts->precision == FPEPS_FP32) FP_TRY(op.make_f32_operands(ctx));
    fp::EventPair evp;
    FP_HIP(evp.create());
    hipEvent_t e0 = evp.a, e1 = evp.b;
    FP_HIP(hipEventRecord(e0, ctx->stream));
    ctx->multi_stream = (opts->flags & FPEPS_FLAG_ONE_STREAM) == 0;
    FP_TRY(op.apply(ctx, pl, transpose != 0, x_in, y_out, opts->precision == FPEPS_FP32));
    FP_HIP(hipEventRecord(e1, ctx->stream));
    FP_HIP(hipEventSynchronize(e1));
    float ms = 0;
    FP_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (report) {
      report->alg_flops = transpose ? pl.flops_bwd : pl.flops_fwd;
      report->seconds = ms * 1e-3;
      report->peak_workspace = ctx->peak_ws;
      report->workspace_bytes = (double)ctx->ws_bytes;
      report->nslices = ctx->nslices;
    }
    return fp::Status::ok();
  });
}

fpeps_status fpeps_rsvd_truncate(fpeps_ctx ctx, int32_t nmat, const int64_t* m, const int64_t* n,
                                 const double* const* A, const fpeps_opts* opts,
                                 double* const* U_out, double* const* R_out, int32_t* kept,
                                 double* sigma, fpeps_report* report) {
  return guarded(ctx, [&] {
    if (report) std::memset(report, 0, sizeof(*report));
    return fp::explicit_rsvd(ctx, nmat, m, n, A, opts, U_out, R_out, kept, sigma, report,
                             nullptr, nullptr, nullptr, false);
  });
}

fpeps_status fpeps_rsvd_truncate_grouped(fpeps_ctx ctx, int32_t nmat, const int64_t* m,
                                         const int64_t* n, const double* const* A,
                                         const int32_t* group, const fpeps_opts* opts,
                                         double* const* U_out, double* const* R_out,
                                         int32_t* kept, double* sigma, fpeps_report* report) {
  return guarded(ctx, [&] {
    if (report) std::memset(report, 0, sizeof(*report));
    if (!group) return fp::fail(FPEPS_ERR_ARG, "null group list");
    return fp::explicit_rsvd(ctx, nmat, m, n, A, opts, U_out, R_out, kept, sigma, report,
                             nullptr, nullptr, nullptr, false, group);
  });
}

fpeps_status fpeps_cbe_expand_grouped(fpeps_ctx ctx, int32_t nmat, const int64_t* m,
                                      const int64_t* n, const double* const* A,
                                      const int32_t* group, const int32_t* r,
                                      const double* const* U, const double* const* V,
                                      const fpeps_opts* opts, double* const* Q_out,
                                      int32_t* kept, double* sigma, fpeps_report* report) {
  return guarded(ctx, [&] {
    if (report) std::memset(report, 0, sizeof(*report));
    if (!group) return fp::fail(FPEPS_ERR_ARG, "null group list");
    return fp::explicit_rsvd(ctx, nmat, m, n, A, opts, Q_out, nullptr, kept, sigma, report, r,
                             U, V, true, group);
  });
}

fpeps_status fpeps_cbe_expand(fpeps_ctx ctx, int32_t nmat, const int64_t* m, const int64_t* n,
                              const double* const* A, const int32_t* r, const double* const* U,
                              const double* const* V, const fpeps_opts* opts,
                              double* const* Q_out, int32_t* kept, double* sigma,
                              fpeps_report* report) {
  return guarded(ctx, [&] {
    if (report) std::memset(report, 0, sizeof(*report));
    return fp::explicit_rsvd(ctx, nmat, m, n, A, opts, Q_out, nullptr, kept, sigma, report, r,
                             U, V, true);
  });
}

fpeps_status fpeps_expect(fpeps_ctx ctx, int32_t L, const fpeps_tensor* top,
                          const fpeps_tensor* bottom, double log_norm_top,
                          double log_norm_bottom, int32_t* sign, double* log_abs) {
  return guarded(ctx, [&] {
    return fp::overlap(ctx, L, top, bottom, log_norm_top + log_norm_bottom, sign, log_abs);
  });
}

fpeps_status fpeps_heff_apply(fpeps_ctx ctx, const fpeps_tensor* T, const fpeps_tensor* L,
                              const fpeps_tensor* B, const fpeps_tensor* R, const fpeps_tensor* W,
                              const fpeps_tensor* A, const fpeps_opts* opts, fpeps_tensor* y_out,
                              fpeps_report* report) {
  return guarded(ctx, [&] {
    if (report) std::memset(report, 0, sizeof(*report));
    return fp::heff_apply(ctx, T, L, B, R, W, A, opts, y_out, report);
  });
}

fpeps_status fpeps_heff_prepare(fpeps_ctx ctx, const fpeps_tensor* T, const fpeps_tensor* L,
                                const fpeps_tensor* B, const fpeps_tensor* R,
                                const fpeps_tensor* W, const fpeps_tensor* A,
                                const fpeps_opts* opts, fpeps_tensor* y_out, fpeps_heff* op,
                                fpeps_report* report) {
  return guarded(ctx, [&] {
    if (report) std::memset(report, 0, sizeof(*report));
    return fp::heff_prepare(ctx, T, L, B, R, W, A, opts, y_out, op, report);
  });
}

fpeps_status fpeps_heff_apply_prepared(fpeps_heff op, const double* a, int64_t a_elems,
                                       double* y, int64_t y_elems, fpeps_report* report) {
  if (!op) return FPEPS_ERR_ARG;
  return guarded(fp::heff_context(op), [&] {
    if (report) std::memset(report, 0, sizeof(*report));
    return fp::heff_apply_prepared(op, a, a_elems, y, y_elems, report);
  });
}

fpeps_status fpeps_heff_release(fpeps_heff op) {
  if (!op) return FPEPS_ERR_ARG;
  return guarded(fp::heff_context(op), [&] { return fp::heff_release(op); });
}

fpeps_status fpeps_expect_noalloc(fpeps_ctx ctx, int32_t L, const fpeps_tensor* top,
                                  const fpeps_tensor* bottom, double log_norm_top,
                                  double log_norm_bottom, int32_t* sign, double* log_abs) {
  return guarded(ctx, [&] {
    return fp::overlap_noalloc(ctx, L, top, bottom, log_norm_top + log_norm_bottom, sign,
                               log_abs);
  });
}

}  // extern "C"
