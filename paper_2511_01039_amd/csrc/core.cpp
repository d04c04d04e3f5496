// Context, workspace and plan upload.
#include "core.hpp"

#include <algorithm>
#include <chrono>
#include <cstring>

fpeps_ctx_s::~fpeps_ctx_s() {
  if (!bufs.empty() || !evpool.empty() || stage || !xstreams.empty()) (void)hipDeviceSynchronize();
  for (auto e : evpool) (void)hipEventDestroy(e);
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  for (auto e : xjoin) (void)hipEventDestroy(e);
  for (auto x : xstreams) (void)hipStreamDestroy(x);
  for (auto& kv : bufs)
    if (kv.second.p) dev_free(kv.second.p);
  if (stage) (void)hipHostFree(stage);
}

void* fpeps_ctx_s::dev_alloc(size_t bytes) {
  if (alloc_fn) return alloc_fn(bytes, alloc_user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void fpeps_ctx_s::dev_free(void* p) {
  if (!p) return;
  if (free_fn)
    free_fn(p, alloc_user);
  else
    (void)hipFree(p);
}

fp::Status fpeps_ctx_s::release_workspace() {
  if (bufs.empty()) return fp::Status::ok();
  FP_HIP(hipDeviceSynchronize());
  for (auto& kv : bufs)
    if (kv.second.p) dev_free(kv.second.p);
  bufs.clear();
  ws_bytes = 0;
  ++ws_generation;
  return fp::Status::ok();
}

fp::Status fpeps_ctx_s::release_prefix(const std::string& prefix) {
  FP_HIP(hipStreamSynchronize(stream));
  for (auto it = bufs.begin(); it != bufs.end();) {
    if (it->first.compare(0, prefix.size(), prefix) == 0) {
      if (it->second.p) {
        dev_free(it->second.p);
        ws_bytes -= std::min(ws_bytes, it->second.bytes);
      }
      it = bufs.erase(it);
    } else {
      ++it;
    }
  }
  return fp::Status::ok();
}

void fpeps_ctx_s::release_later(std::shared_ptr<void> p) {
  if (!p) return;
  reaping.erase(std::remove_if(reaping.begin(), reaping.end(),
                               [](std::future<void>& f) {
                                 return f.wait_for(std::chrono::seconds(0)) ==
                                        std::future_status::ready;
                               }),
                reaping.end());
  try {
    reaping.push_back(std::async(std::launch::async, [q = std::move(p)]() mutable { q.reset(); }));
  } catch (...) {
    // no helper thread: the captured reference is dropped here instead
  }
}

fp::Status fpeps_ctx_s::ensure_streams(int n) {
  if (!ev_fork) FP_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
  while ((int)xstreams.size() < n - 1) {
    hipStream_t x = nullptr;
    hipEvent_t e = nullptr;
    FP_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    xstreams.push_back(x);
    FP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    xjoin.push_back(e);
  }
  return fp::Status::ok();
}

int fpeps_ctx_s::stream_index(hipStream_t s) const {
  for (size_t i = 0; i < xstreams.size(); ++i)
    if (xstreams[i] == s) return (int)i + 1;
  return 0;
}

fp::Status fpeps_ctx_s::stage_begin() {
  FP_HIP(hipStreamSynchronize(stream));
  stage_used = 0;
  stage_async = true;
  return fp::Status::ok();
}

fp::Status fpeps_ctx_s::buf(const std::string& name, size_t bytes, void** out) {
  if (arena_base) {
    fp::DevBuf& a = arena_bufs[name];
    if (a.bytes < bytes) {
      const size_t want = (std::max(bytes, (size_t)256) + 255) / 256 * 256;
      if (arena_used + want > arena_cap)
        return fp::fail(FPEPS_ERR_CAPACITY,
                        "the no-allocation scratch of " + std::to_string(arena_cap >> 20) +
                            " MiB is too small for this problem (" + name + ": needs " +
                            std::to_string(arena_used + want) + " bytes in all)");
      a.p = arena_base + arena_used;
      a.bytes = want;
      arena_used += want;
    }
    *out = a.p;
    return fp::Status::ok();
  }
  fp::DevBuf& b = bufs[name];
  if (b.bytes < bytes) {
    if (b.p) {
      // every stream of the context joins the context's stream before a
      // call returns, so its work on the old buffer is done after this
      FP_HIP(hipStreamSynchronize(stream));
      dev_free(b.p);
      ws_bytes -= b.bytes;
      b.p = nullptr;
      b.bytes = 0;
    }
    size_t want = std::max(bytes, (size_t)4096);
    want = (want + 4095) / 4096 * 4096;
    b.p = dev_alloc(want);
    if (!b.p)
      return fp::fail(FPEPS_ERR_NOMEM, "device allocation of " + std::to_string(want) +
                                           " bytes failed (" + name + ")");
    b.bytes = want;
    ws_bytes += want;
    ws_peak = std::max(ws_peak, ws_bytes);
  }
  *out = b.p;
  return fp::Status::ok();
}

fp::Status fpeps_ctx_s::stage_alloc(size_t bytes, char** host) {
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
  *host = stage + stage_used;
  stage_used += need;
  return fp::Status::ok();
}

fp::Status fpeps_ctx_s::upload_region(const std::string& name, const char* host, size_t bytes,
                                      void** dev) {
  FP_TRY(buf(name, bytes, dev));
  if (!bytes) return fp::Status::ok();
  if (stage_async) {
    FP_HIP(hipMemcpyAsync(*dev, host, bytes, hipMemcpyHostToDevice, stream));
  } else {
    // the previous contents may still be read by queued kernels
    FP_HIP(hipStreamSynchronize(stream));
    FP_HIP(hipMemcpy(*dev, host, bytes, hipMemcpyHostToDevice));
  }
  return fp::Status::ok();
}

fp::Status fpeps_ctx_s::upload(const std::string& name, const void* host, size_t bytes,
                               void** dev) {
  if (stage_async && bytes) {
    char* h = nullptr;
    FP_TRY(stage_alloc(bytes, &h));
    std::memcpy(h, host, bytes);
    return upload_region(name, h, bytes, dev);
  }
  return upload_region(name, (const char*)host, bytes, dev);
}

int64_t fpeps_ctx_s::default_budget() {
  if (mem_total == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      tot = 0;
    }
    mem_total = tot > 0 ? tot : ((size_t)64 << 30) * 2;   // unknown: 64 GiB below
  }
  const int64_t cap = (int64_t)128 << 30;
  return std::min<int64_t>(cap, (int64_t)(0.45 * (double)mem_total));
}

int64_t fpeps_ctx_s::total_budget(const fpeps_opts* o) {
  if (o && o->slice_budget > 0) return o->slice_budget;
  if (tune && tune->slice_budget > 0) return tune->slice_budget;
  return default_budget();
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
    if (tune_record && evsig[i / 2]) {
      auto& t = tune_log[evsig[i / 2]][evtile[i / 2]];
      t[0] += ms * 1e-3;
      t[1] += 1;
    }
  }
  evused = 0;
  evflops.clear();
  evlabel.clear();
  evbytes.clear();
  evshape.clear();
  evsig.clear();
  evtile.clear();
  return fp::Status::ok();
}

namespace fp {

Status PlanSet::serialize() {
  Image m;
  for (auto& p : plans) {
    m.red0.push_back(m.reds.size());
    m.reds.insert(m.reds.end(), p.reduces.begin(), p.reduces.end());
    const int32_t base = (int32_t)m.pairs.size();
    const size_t j0 = m.jobs.size();
    for (auto j : p.jobs) {
      j.p0 += base;
      j.p1 += base;
      m.jobs.push_back(j);
    }
    m.pairs.insert(m.pairs.end(), p.pairs.begin(), p.pairs.end());
    m.range.emplace_back(j0, p.jobs.size());
  }
  if (m.pairs.size() > (size_t)INT32_MAX || m.jobs.size() > (size_t)INT32_MAX)
    return fail(FPEPS_ERR_UNSUPPORTED, "plan too large");
  // row-thread plans, concatenated with rebased ranges
  pack_off.clear();
  pack_total = 0;
  for (auto& r : rts) {
    const size_t g0 = m.rg.size(), o0 = m.ro.size(), b0 = m.rb.size(), c0 = m.rc.size(),
                 p0 = m.rp.size();
    m.rk0.push_back(m.rk.size());
    pack_off.push_back(pack_total);
    m.rg0.push_back(g0);
    m.rtg0.push_back(m.ntiles);
    m.ntiles += (size_t)r.ntiles;
    for (auto g : r.groups) {
      g.o0 += (int32_t)o0;
      g.o1 += (int32_t)o0;
      g.k0 += (int32_t)b0;
      g.k1 += (int32_t)b0;
      g.c0 += (int32_t)c0;
      m.rg.push_back(g);
    }
    m.rb.insert(m.rb.end(), r.kblks.begin(), r.kblks.end());
    m.rc.insert(m.rc.end(), r.cols.begin(), r.cols.end());
    for (auto o : r.outs) {
      o.p0 += (int32_t)p0;
      o.p1 += (int32_t)p0;
      m.ro.push_back(o);
    }
    for (auto pr : r.pairs) {
      pr.pk += pack_total;
      pr.kblk += (int32_t)b0;
      m.rp.push_back(pr);
    }
    for (auto k : r.packs) {
      k.dst += pack_total;
      m.rk.push_back(k);
    }
    pack_total += r.pack_size;
    if (m.rg.size() > (size_t)INT32_MAX || m.ro.size() > (size_t)INT32_MAX ||
        m.rp.size() > (size_t)INT32_MAX ||
        m.rk.size() > (size_t)INT32_MAX || m.rb.size() > (size_t)INT32_MAX ||
        m.rc.size() > (size_t)INT32_MAX)
      return fail(FPEPS_ERR_UNSUPPORTED, "layer plan too large");
  }
  // one device image: every array 256-byte aligned
  const size_t sz[10] = {m.jobs.size() * sizeof(GemmJob),   m.pairs.size() * sizeof(GemmPair),
                         pool.data.size() * sizeof(int32_t), m.reds.size() * sizeof(ReduceTab),
                         m.rg.size() * sizeof(RtGroup),      m.rb.size() * sizeof(RtKblk),
                         m.rc.size() * sizeof(RtCol),        m.ro.size() * sizeof(RtOut),
                         m.rp.size() * sizeof(RtPair),       m.rk.size() * sizeof(RtPack)};
  size_t o = 0;
  for (int i = 0; i < 10; ++i) {
    m.off[i] = o;
    o += (sz[i] + 255) / 256 * 256;
  }
  m.bytes = o;
  m.ready = true;
  img = std::move(m);
  return Status::ok();
}

void PlanSet::write_image(char* dst) const {
  const Image& m = img;
  const void* src[10] = {m.jobs.data(), m.pairs.data(), pool.data.data(), m.reds.data(),
                         m.rg.data(),   m.rb.data(),    m.rc.data(),       m.ro.data(),
                         m.rp.data(),   m.rk.data()};
  for (int i = 0; i < 10; ++i) {
    const size_t n = (i + 1 < 10 ? m.off[i + 1] : m.bytes) - m.off[i];
    if (n == 0) continue;
    // the array's own size; the rest of its aligned slot is padding
    size_t len = 0;
    switch (i) {
      case 0: len = m.jobs.size() * sizeof(GemmJob); break;
      case 1: len = m.pairs.size() * sizeof(GemmPair); break;
      case 2: len = pool.data.size() * sizeof(int32_t); break;
      case 3: len = m.reds.size() * sizeof(ReduceTab); break;
      case 4: len = m.rg.size() * sizeof(RtGroup); break;
      case 5: len = m.rb.size() * sizeof(RtKblk); break;
      case 6: len = m.rc.size() * sizeof(RtCol); break;
      case 7: len = m.ro.size() * sizeof(RtOut); break;
      case 8: len = m.rp.size() * sizeof(RtPair); break;
      default: len = m.rk.size() * sizeof(RtPack); break;
    }
    if (len) std::memcpy(dst + m.off[i], src[i], len);
  }
}

Status PlanSet::upload(fpeps_ctx_s* ctx, const std::string& tag) {
  if (!img.ready) FP_TRY(serialize());
  if (ctx->stage_async) {
    char* h = nullptr;
    FP_TRY(ctx->stage_alloc(img.bytes, &h));
    write_image(h);
    return bind(ctx, tag, h);
  }
  std::vector<char> h(std::max<size_t>(img.bytes, 1));
  write_image(h.data());
  return bind(ctx, tag, h.data());
}

Status PlanSet::bind(fpeps_ctx_s* ctx, const std::string& tag, const char* host) {
  if (!img.ready) return fail(FPEPS_ERR_ARG, "plan image was not built");
  const Image& m = img;
  void* dimg = nullptr;
  FP_TRY(ctx->upload_region(tag + "_img", host, m.bytes, &dimg));
  char* base = (char*)dimg;
  void* dj = base + m.off[0];
  void* dp = base + m.off[1];
  dtab = (int32_t*)(base + m.off[2]);
  void* dr = base + m.off[3];
  void* dg = base + m.off[4];
  void* dB = base + m.off[5];
  void* dC = base + m.off[6];
  void* dO = base + m.off[7];
  void* dP = base + m.off[8];
  void* dK = base + m.off[9];
  void* dpk = nullptr;
  // the group of every workgroup: written on the device from the groups
  void* dTG = nullptr;
  FP_TRY(ctx->buf(tag + "_rttg", std::max<size_t>(m.ntiles, 1) * sizeof(int32_t), &dTG));
  for (size_t i = 0; i < rts.size(); ++i)
    FP_HIP(launch_tile_group((const RtGroup*)dg, (int)m.rg0[i], (int)rts[i].groups.size(),
                             (int32_t*)dTG + m.rtg0[i], ctx->stream));
  FP_TRY(ctx->buf(tag + "_pack", (size_t)std::max<int64_t>(pack_total, 1) * sizeof(double), &dpk));
  dpack = (double*)dpk;
  this->tag = tag;
  drt.clear();
  for (size_t i = 0; i < rts.size(); ++i) {
    DevRt d;
    d.groups = (const RtGroup*)dg;
    d.tile_group = (const int32_t*)dTG + m.rtg0[i];
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
    d.packs = (const RtPack*)dK + m.rk0[i];
    d.ngroups = (int)rts[i].groups.size();
    d.ntiles = rts[i].ntiles;
    d.npacks = (int)rts[i].packs.size();
    drt.push_back(d);
  }
  dev.clear();
  for (size_t i = 0; i < plans.size(); ++i) {
    DevGemm g;
    g.jobs = (const GemmJob*)dj + m.range[i].first;
    g.pairs = (const GemmPair*)dp;
    g.njobs = (int)m.range[i].second;
    g.mt = plans[i].mt;
    g.nt = plans[i].nt;
    g.reduces = (const ReduceTab*)dr + m.red0[i];
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
      ctx->evsig.push_back(0);
      ctx->evtile.push_back({0, 0});
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
  return run_gemm_any(ctx, ps, idx, A, nullptr, a_size, B, b_f32, b_size, C, c_f32, c_size, timed,
                      label);
}

Status run_gemm_f32(fpeps_ctx_s* ctx, const PlanSet& ps, int idx, const float* A, int64_t a_size,
                    const void* B, bool b_f32, int64_t b_size, void* C, bool c_f32, int64_t c_size,
                    bool timed, int label) {
  return run_gemm_any(ctx, ps, idx, nullptr, A, a_size, B, b_f32, b_size, C, c_f32, c_size, timed,
                      label);
}

Status run_gemm_any(fpeps_ctx_s* ctx, const PlanSet& ps, int idx, const double* A,
                    const float* A32, int64_t a_size, const void* B, bool b_f32, int64_t b_size,
                    void* C, bool c_f32, int64_t c_size, bool timed, int label,
                    double* part_buf) {
  const GemmPlan& p = ps.plans[idx];
  if (p.jobs.empty()) return Status::ok();
  // every table-addressed access must stay inside its buffer
  if (p.a_extent > a_size || p.b_extent > b_size || p.c_extent > c_size)
    return fail(FPEPS_ERR_SHAPE, "plan reaches outside a buffer (a " + std::to_string(p.a_extent) +
                                     "/" + std::to_string(a_size) + ", b " +
                                     std::to_string(p.b_extent) + "/" + std::to_string(b_size) +
                                     ", c " + std::to_string(p.c_extent) + "/" +
                                     std::to_string(c_size) + ")");
  if ((!A && !A32) || !B || !C) return fail(FPEPS_ERR_ARG, "null operand buffer");
  if (A && b_f32 && c_f32) return fail(FPEPS_ERR_UNSUPPORTED, "FP64 GEMM with B and C in FP32");
  // split-K parts are summed in FP64 and rounded once into C
  double* part = nullptr;
  if (p.partial_size > 0 && part_buf) {
    part = part_buf;
  } else if (p.partial_size > 0) {
    // each stream has its own partial buffer (slices on several streams
    // overlap)
    const int si = ctx->stream_index(ctx->stream);
    FP_TRY(ctx->bufT(si ? "gemm_part" + std::to_string(si + 1) : std::string("gemm_part"),
                     (size_t)p.partial_size, &part));
  }
  hipEvent_t ea = nullptr, eb = nullptr;
  const bool tk = timed && ctx->time_kernels;
  if (tk) {
    FP_TRY(ctx->timed_events(&ea, &eb));
    ctx->evflops.push_back(p.flops);
    ctx->evlabel.push_back(label);
    ctx->evbytes.push_back(p.bytes);
    ctx->evshape.push_back({0.0, 0.0});
    ctx->evsig.push_back(p.sig);
    ctx->evtile.push_back({p.mt, p.nt});
    FP_HIP(hipEventRecord(ea, ctx->stream));
  }
  if (part) {
    if (A)
      FP_HIP(launch_gemm_mixed(ps.dev[idx], A, B, b_f32, part, false, ps.dtab, ctx->stream));
    else
      FP_HIP(launch_gemm_f32(ps.dev[idx], A32, B, b_f32, part, false, ps.dtab, ctx->stream));
    FP_HIP(launch_reduce_tab(ps.dev[idx].reduces, ps.dev[idx].nred, p.max_red_mn, C, c_f32, part,
                             ps.dtab, ctx->stream));
  } else if (A) {
    FP_HIP(launch_gemm_mixed(ps.dev[idx], A, B, b_f32, C, c_f32, ps.dtab, ctx->stream));
  } else {
    FP_HIP(launch_gemm_f32(ps.dev[idx], A32, B, b_f32, C, c_f32, ps.dtab, ctx->stream));
  }
  if (tk) FP_HIP(hipEventRecord(eb, ctx->stream));
  return Status::ok();
}

}  // namespace fp
