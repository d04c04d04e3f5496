// Context, workspace and plan upload.
#include "core.hpp"

#include <algorithm>
#include <cstring>

fpeps_ctx_s::~fpeps_ctx_s() {
  if (!bufs.empty() || !evpool.empty() || stage) (void)hipDeviceSynchronize();
  for (auto e : evpool) (void)hipEventDestroy(e);
  for (auto& kv : bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  if (stage) (void)hipHostFree(stage);
}

fp::Status fpeps_ctx_s::stage_begin() {
  FP_HIP(hipStreamSynchronize(stream));
  stage_used = 0;
  stage_async = true;
  return fp::Status::ok();
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
  if (stage_async && bytes) {
    const size_t need = (bytes + 255) / 256 * 256;
    if (stage_used + need > stage_cap) {
      // every copy issued from the arena so far must finish before it is
      // replaced
      FP_HIP(hipStreamSynchronize(stream));
      const size_t cap = std::max({2 * stage_cap, need, (size_t)64 << 20});
      if (stage) FP_HIP(hipHostFree(stage));
      stage = nullptr;
      stage_cap = 0;
      if (hipHostMalloc((void**)&stage, cap, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        stage = nullptr;
        return fp::fail(FPEPS_ERR_NOMEM, "pinned staging allocation failed");
      }
      stage_cap = cap;
      stage_used = 0;
    }
    std::memcpy(stage + stage_used, host, bytes);
    FP_HIP(hipMemcpyAsync(*dev, stage + stage_used, bytes, hipMemcpyHostToDevice, stream));
    stage_used += need;
    return fp::Status::ok();
  }
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
    auto& b = kt_by_label[evlabel[i / 2]];
    b[0] += ms * 1e-3;
    b[1] += evflops[i / 2];
    b[2] += 1;
    b[3] += evbytes[i / 2];
    b[4] += evshape[i / 2][0];
    b[5] += evshape[i / 2][1];
  }
  evused = 0;
  evflops.clear();
  evlabel.clear();
  evbytes.clear();
  evshape.clear();
  return fp::Status::ok();
}

namespace fp {

Status PlanSet::upload(fpeps_ctx_s* ctx, const std::string& tag) {
  std::vector<GemmJob> jobs;
  std::vector<GemmPair> pairs;
  std::vector<ReduceTab> reds;
  std::vector<size_t> red0;
  std::vector<std::pair<size_t, size_t>> range;
  for (auto& p : plans) {
    red0.push_back(reds.size());
    reds.insert(reds.end(), p.reduces.begin(), p.reduces.end());
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
  // row-thread plans, concatenated with rebased ranges
  std::vector<RtGroup> rg;
  std::vector<int32_t> rtg;
  std::vector<size_t> rtg0;
  std::vector<RtOut> ro;
  std::vector<RtKblk> rb;
  std::vector<RtCol> rc;
  std::vector<RtPair> rp;
  std::vector<RtPack> rk;
  struct R4 {
    size_t g, o, b, c, p, k;
  };
  std::vector<R4> rr;
  pack_off.clear();
  pack_total = 0;
  for (auto& r : rts) {
    R4 b{rg.size(), ro.size(), rb.size(), rc.size(), rp.size(), rk.size()};
    rr.push_back(b);
    pack_off.push_back(pack_total);
    rtg0.push_back(rtg.size());
    for (int32_t t : r.tile_group) rtg.push_back(t + (int32_t)b.g);
    for (auto g : r.groups) {
      g.o0 += (int32_t)b.o;
      g.o1 += (int32_t)b.o;
      g.k0 += (int32_t)b.b;
      g.k1 += (int32_t)b.b;
      g.c0 += (int32_t)b.c;
      rg.push_back(g);
    }
    rb.insert(rb.end(), r.kblks.begin(), r.kblks.end());
    rc.insert(rc.end(), r.cols.begin(), r.cols.end());
    for (auto o : r.outs) {
      o.p0 += (int32_t)b.p;
      o.p1 += (int32_t)b.p;
      ro.push_back(o);
    }
    for (auto p : r.pairs) {
      p.pk += pack_total;
      p.kblk += (int32_t)b.b;
      rp.push_back(p);
    }
    for (auto k : r.packs) {
      k.dst += pack_total;
      rk.push_back(k);
    }
    pack_total += r.pack_size;
    if (ro.size() > (size_t)INT32_MAX || rp.size() > (size_t)INT32_MAX ||
        rk.size() > (size_t)INT32_MAX || rb.size() > (size_t)INT32_MAX ||
        rc.size() > (size_t)INT32_MAX)
      return fail(FPEPS_ERR_UNSUPPORTED, "layer plan too large");
  }
  void *dj = nullptr, *dp = nullptr, *dt = nullptr;
  FP_TRY(ctx->upload(tag + "_jobs", jobs.data(), jobs.size() * sizeof(GemmJob), &dj));
  FP_TRY(ctx->upload(tag + "_pairs", pairs.data(), pairs.size() * sizeof(GemmPair), &dp));
  FP_TRY(ctx->upload(tag + "_tab", pool.data.data(), pool.data.size() * sizeof(int32_t), &dt));
  dtab = (int32_t*)dt;
  void* dr = nullptr;
  FP_TRY(ctx->upload(tag + "_red", reds.data(), reds.size() * sizeof(ReduceTab), &dr));
  void *dg = nullptr, *dO = nullptr, *dP = nullptr, *dK = nullptr, *dpk = nullptr, *dB = nullptr;
  FP_TRY(ctx->upload(tag + "_rtg", rg.data(), rg.size() * sizeof(RtGroup), &dg));
  void* dTG = nullptr;
  FP_TRY(ctx->upload(tag + "_rttg", rtg.data(), rtg.size() * sizeof(int32_t), &dTG));
  FP_TRY(ctx->upload(tag + "_rtb", rb.data(), rb.size() * sizeof(RtKblk), &dB));
  void* dC = nullptr;
  FP_TRY(ctx->upload(tag + "_rtc", rc.data(), rc.size() * sizeof(RtCol), &dC));
  FP_TRY(ctx->upload(tag + "_rto", ro.data(), ro.size() * sizeof(RtOut), &dO));
  FP_TRY(ctx->upload(tag + "_rtp", rp.data(), rp.size() * sizeof(RtPair), &dP));
  FP_TRY(ctx->upload(tag + "_rtk", rk.data(), rk.size() * sizeof(RtPack), &dK));
  FP_TRY(ctx->buf(tag + "_pack", (size_t)std::max<int64_t>(pack_total, 1) * sizeof(double), &dpk));
  dpack = (double*)dpk;
  this->tag = tag;
  drt.clear();
  for (size_t i = 0; i < rts.size(); ++i) {
    DevRt d;
    d.groups = (const RtGroup*)dg;
    d.tile_group = (const int32_t*)dTG + rtg0[i];
    d.outs = (const RtOut*)dO;
    d.kblks = (const RtKblk*)dB;
    d.cols = (const RtCol*)dC;
    d.pairs = (const RtPair*)dP;
    d.lds_bytes = rts[i].lds_bytes;
    d.nlaunch = rts[i].nlaunch;
    for (int c = 0; c < RT_NCLASS; ++c) {
      d.l_tile0[c] = rts[i].l_tile0[c];
      d.l_ntiles[c] = rts[i].l_ntiles[c];
      d.l_lds[c] = rts[i].l_lds[c];
    }
    d.packs = (const RtPack*)dK + rr[i].k;
    d.ngroups = (int)rts[i].groups.size();
    d.ntiles = rts[i].ntiles;
    d.npacks = (int)rts[i].packs.size();
    drt.push_back(d);
  }
  dev.clear();
  for (size_t i = 0; i < plans.size(); ++i) {
    DevGemm g;
    g.jobs = (const GemmJob*)dj + range[i].first;
    g.pairs = (const GemmPair*)dp;
    g.njobs = (int)range[i].second;
    g.mt = plans[i].mt;
    g.nt = plans[i].nt;
    g.reduces = (const ReduceTab*)dr + red0[i];
    g.nred = (int)plans[i].reduces.size();
    dev.push_back(g);
  }
  return Status::ok();
}

Status PlanSet::pack(fpeps_ctx_s* ctx, int idx, const double* S, int64_t s_size) {
  const RtPlan& r = rts[idx];
  if (r.packs.empty()) return Status::ok();
  if (r.s_extent > s_size)
    return fail(FPEPS_ERR_SHAPE, "layer pack reaches outside the layer tensor");
  if (!S || !dpack) return fail(FPEPS_ERR_ARG, "null layer tensor");
  FP_HIP(launch_rt_pack(drt[idx], S, dtab, dpack, ctx->stream));
  return Status::ok();
}

Status run_rt(fpeps_ctx_s* ctx, const PlanSet& ps, int idx, const void* X, int64_t x_size,
              void* Y, int64_t y_size, bool f32, bool timed, int label) {
  const RtPlan& p = ps.rts[idx];
  if (p.ntiles == 0) return Status::ok();
  if (p.x_extent > x_size || p.c_extent > y_size)
    return fail(FPEPS_ERR_SHAPE, "layer plan reaches outside a buffer (x " +
                                     std::to_string(p.x_extent) + "/" + std::to_string(x_size) +
                                     ", y " + std::to_string(p.c_extent) + "/" +
                                     std::to_string(y_size) + ")");
  if (!X || !Y) return fail(FPEPS_ERR_ARG, "null operand buffer");
  const DevRt& d = ps.drt[idx];
  for (int c = 0; c < d.nlaunch; ++c) {
    if (timed && ctx->time_kernels) {
      hipEvent_t a, b;
      FP_TRY(ctx->timed_events(&a, &b));
      ctx->evflops.push_back(p.l_flops[c]);
      // at verbose level 2 every launch class of a step is kept apart
      ctx->evlabel.push_back(ctx->verbose >= 2 ? label + 100 * (c + 1) : label);
      ctx->evbytes.push_back(f32 ? 0.5 * p.l_bytes[c] : p.l_bytes[c]);
      ctx->evshape.push_back({(double)p.l_ntiles[c], (double)p.l_lds[c]});
      FP_HIP(hipEventRecord(a, ctx->stream));
      FP_HIP(launch_rt_f64(d, c, X, f32, ps.dpack, Y, ps.dtab, ctx->stream));
      FP_HIP(hipEventRecord(b, ctx->stream));
    } else {
      FP_HIP(launch_rt_f64(d, c, X, f32, ps.dpack, Y, ps.dtab, ctx->stream));
    }
  }
  return Status::ok();
}

Status run_gemm(fpeps_ctx_s* ctx, const PlanSet& ps, int idx, const double* A, int64_t a_size,
                const double* B, int64_t b_size, double* C, int64_t c_size, bool timed,
                int label) {
  return run_gemm_mixed(ctx, ps, idx, A, a_size, B, false, b_size, C, false, c_size, timed, label);
}

Status run_gemm_mixed(fpeps_ctx_s* ctx, const PlanSet& ps, int idx, const double* A,
                      int64_t a_size, const void* B, bool b_f32, int64_t b_size, void* C,
                      bool c_f32, int64_t c_size, bool timed, int label) {
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
  if (b_f32 && c_f32) return fail(FPEPS_ERR_UNSUPPORTED, "GEMM with both B and C in FP32");
  // split-K parts are summed in FP64 and rounded once into C
  double* part = nullptr;
  if (p.partial_size > 0) FP_TRY(ctx->bufT("gemm_part", (size_t)p.partial_size, &part));
  hipEvent_t ea = nullptr, eb = nullptr;
  const bool tk = timed && ctx->time_kernels;
  if (tk) {
    FP_TRY(ctx->timed_events(&ea, &eb));
    ctx->evflops.push_back(p.flops);
    ctx->evlabel.push_back(label);
    ctx->evbytes.push_back(p.bytes);
    ctx->evshape.push_back({0.0, 0.0});
    FP_HIP(hipEventRecord(ea, ctx->stream));
  }
  if (part) {
    FP_HIP(launch_gemm_mixed(ps.dev[idx], A, B, b_f32, part, false, ps.dtab, ctx->stream));
    FP_HIP(launch_reduce_tab(ps.dev[idx].reduces, ps.dev[idx].nred, p.max_red_mn, C, c_f32, part,
                             ps.dtab, ctx->stream));
  } else {
    FP_HIP(launch_gemm_mixed(ps.dev[idx], A, B, b_f32, C, c_f32, ps.dtab, ctx->stream));
  }
  if (tk) FP_HIP(hipEventRecord(eb, ctx->stream));
  return Status::ok();
}

}  // namespace fp
