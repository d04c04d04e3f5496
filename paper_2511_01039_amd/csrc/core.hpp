// Context, device workspace and shared helpers of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <array>
#include <future>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/fpeps.h"
#include "kernels.hpp"
#include "plan.hpp"

namespace fp {

struct Status {
  fpeps_status code = FPEPS_OK;
  std::string msg;
  static Status ok() { return Status(); }
  bool good() const { return code == FPEPS_OK; }
};
inline Status fail(fpeps_status c, const std::string& m) {
  Status s;
  s.code = c;
  s.msg = m;
  return s;
}

#define FP_HIP(call)                                                                 \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::fp::fail(FPEPS_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define FP_TRY(expr)            \
  do {                          \
    ::fp::Status s_ = (expr);   \
    if (!s_.good()) return s_;  \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Per-site diagnostics of the last absorption.
struct SiteDiag {
  std::vector<double> sigma;     // all sectors, descending within a sector
  std::vector<int32_t> sector;   // sector ordinal of each value
  std::vector<int32_t> kept;     // per sector
  std::vector<int64_t> m, n;
  std::vector<int32_t> k;
  std::vector<int32_t> cbe;      // bond expansion per sector (empty: none)
};

}  // namespace fp

struct fpeps_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  // extra streams for the slices of a site (default priority; created on
  // first use): slice i runs on stream i % n, stream 0 being the context's.
  // One fork event orders them after the context's stream, and one join
  // event each orders the context's stream after them.
  std::vector<hipStream_t> xstreams;
  std::vector<hipEvent_t> xjoin;
  hipEvent_t ev_fork = nullptr;
  bool multi_stream = true;   // cleared by FPEPS_FLAG_ONE_STREAM (then one stream)
  int max_streams = 4;       // streams the slices of a site are spread over
  fp::Status ensure_streams(int n);   // n - 1 extra streams
  // 0 for the context's stream, i for xstreams[i - 1]
  int stream_index(hipStream_t s) const;
  std::string err;
  std::map<std::string, fp::DevBuf> bufs;
  // device memory of the workspace: the caller's allocator when set
  // (fpeps_set_allocator), else hipMalloc / hipFree
  void* (*alloc_fn)(size_t, void*) = nullptr;
  void (*free_fn)(void*, void*) = nullptr;
  void* alloc_user = nullptr;
  void* dev_alloc(size_t bytes);
  void dev_free(void* p);
  // frees every workspace buffer (waits for the device first)
  fp::Status release_workspace();
  // frees the workspace buffers whose names start with ``prefix`` (waits
  // for the context's stream first)
  fp::Status release_prefix(const std::string& prefix);
  size_t ws_bytes = 0;   // workspace bytes held now
  uint64_t ws_generation = 0;   // counts release_workspace() calls
  size_t ws_peak = 0;    // and at most since the last reset (a call's start)
  // Arena mode (fpeps_expect_noalloc): between arena_begin and arena_end,
  // buf() carves named regions out of [base, base + cap) with a bump
  // pointer instead of allocating; a request beyond it fails with
  // FPEPS_ERR_CAPACITY. Nothing is freed.
  char* arena_base = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  std::map<std::string, fp::DevBuf> arena_bufs;
  void arena_begin(char* base, size_t cap) {
    arena_base = base;
    arena_cap = cap;
    arena_used = 0;
    arena_bufs.clear();
  }
  void arena_end() {
    arena_base = nullptr;
    arena_cap = arena_used = 0;
    arena_bufs.clear();
  }
  std::vector<fp::SiteDiag> diag;
  double peak_ws = 0;
  int nslices = 0;
  // per-launch timing of the chain GEMM kernel (FPEPS_FLAG_TIME_KERNELS)
  bool time_kernels = false;
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  std::vector<double> evflops;
  std::vector<int> evlabel;
  std::vector<double> evbytes;
  std::vector<std::array<double, 2>> evshape;  // layer launches: tiles, LDS bytes
  // label -> {seconds, flops, launches, algorithmic bytes, tiles, LDS bytes}
  std::map<int, std::array<double, 6>> kt_by_label;
  // autotuning: the tuned table the planner consults (absent until a tuning
  // run or a load), the candidate rank forced during tuning runs, and the
  // measured seconds per GEMM signature and tile of those runs
  std::shared_ptr<fp::TuneTable> tune;
  int tile_rank = -1;
  bool tune_record = false;
  std::vector<uint64_t> evsig;   // per timed launch: GEMM signature (0: not a GEMM)
  std::vector<std::array<int, 2>> evtile;
  // signature -> tile -> {seconds, launches}
  std::map<uint64_t, std::map<std::array<int, 2>, std::array<double, 2>>> tune_log;
  // Bytes of chain intermediates the slices of a call may hold at once (all
  // streams): the caller's opts->slice_budget, else the tuned budget, else
  // default_budget().
  int64_t total_budget(const fpeps_opts* o);
  // min(128 GiB, 45% of the device's memory): larger slices mean fewer,
  // larger launches (a config-4 row: 64 GiB 13.6 s, 96 GiB 12.9 s, 128 GiB
  // 12.7 s), and the rest of the memory stays for the caller and the
  // remaining workspace
  int64_t default_budget();
  size_t mem_total = 0;   // device memory in bytes (queried once)
  // the SymInfo fields the planner takes from the context
  void tune_into(fp::SymInfo& s) const {
    s.tune = tune.get();
    s.tile_rank = tile_rank;
  }
  double kt_seconds = 0, kt_flops = 0;
  long kt_launches = 0;
  int verbose = 0;  // FPEPS_VERBOSE: 1 per site and step, 2 also per layer launch class
  // pinned staging arena for plan uploads (asynchronous host-to-device
  // copies between stage_begin and stage_end; stage_begin waits for the
  // stream, so the arena is never overwritten while a copy reads it)
  char* stage = nullptr;
  size_t stage_cap = 0, stage_used = 0;
  double plan_up_bytes = 0, plan_up_seconds = 0;   // last plan upload (diagnostics)
  bool stage_async = false;
  fp::Status stage_begin();
  void stage_end() { stage_async = false; }
  // ``bytes`` of the arena for the caller to fill (grows it, after waiting
  // for every copy issued from it, when it is too small)
  fp::Status stage_alloc(size_t bytes, char** host);
  // device buffer ``name`` filled from ``host`` (an arena region: an
  // asynchronous copy between stage_begin and stage_end, else a blocking one)
  fp::Status upload_region(const std::string& name, const char* host, size_t bytes, void** dev);

  // Host objects dropped on helper threads: the plan sets of a site take
  // milliseconds to free, which would otherwise leave the device idle
  // between sites. Finished releases are pruned on the next call; the rest
  // are waited for when the context is destroyed.
  std::vector<std::future<void>> reaping;
  void release_later(std::shared_ptr<void> p);

  ~fpeps_ctx_s();
  // device buffer ``name`` of at least ``bytes`` (grown, contents lost on growth)
  fp::Status buf(const std::string& name, size_t bytes, void** out);
  template <class T>
  fp::Status bufT(const std::string& name, size_t count, T** out) {
    void* p = nullptr;
    fp::Status s = buf(name, count * sizeof(T) + 256, &p);
    *out = (T*)p;
    return s;
  }
  fp::Status upload(const std::string& name, const void* host, size_t bytes, void** dev);
  fp::Status sync();
  // events bracketing one timed launch (pairs from the pool)
  fp::Status timed_events(hipEvent_t* a, hipEvent_t* b);
  // after a synchronisation: fold the recorded durations into kt_*
  fp::Status harvest_timing();
};

namespace fp {

// A set of GEMM plans uploaded together (one table pool).
struct PlanSet {
  TablePool pool;
  std::vector<GemmPlan> plans;
  std::vector<DevGemm> dev;
  std::vector<RtPlan> rts;
  std::vector<DevRt> drt;
  std::vector<int64_t> pack_off;   // per row-thread plan, into the pack buffer
  int64_t pack_total = 0;
  double* dpack = nullptr;
  int32_t* dtab = nullptr;
  std::string tag;
  // Host image of all plans of the set, concatenated with rebased ranges.
  // serialize() builds it (host only, safe on a planning thread); upload()
  // copies it to the device (building it first if needed). It is kept, so
  // the same plans can be uploaded again for another site.
  struct Image {
    std::vector<GemmJob> jobs;
    std::vector<GemmPair> pairs;
    std::vector<ReduceTab> reds;
    std::vector<size_t> red0;
    std::vector<std::pair<size_t, size_t>> range;
    std::vector<RtGroup> rg;
    std::vector<size_t> rg0;     // first group of every row-thread plan
    std::vector<size_t> rtg0;    // first tile of every row-thread plan
    size_t ntiles = 0;
    std::vector<RtOut> ro;
    std::vector<RtKblk> rb;
    std::vector<RtCol> rc;
    std::vector<RtPair> rp;
    std::vector<RtPack> rk;
    std::vector<size_t> rk0;
    // byte offsets of the arrays in the single device image, and its size
    size_t off[10] = {0};
    size_t bytes = 0;
    bool ready = false;
  } img;
  Status serialize();
  // host half of the upload: the image (serialize() first), written at dst
  // (img.bytes bytes); safe on any thread
  void write_image(char* dst) const;
  // device half: copies the image from ``host`` and sets the device views
  Status bind(fpeps_ctx_s* ctx, const std::string& tag, const char* host);
  Status upload(fpeps_ctx_s* ctx, const std::string& tag);
  int add(GemmPlan&& p) {
    plans.push_back(std::move(p));
    return (int)plans.size() - 1;
  }
  int add_rt(RtPlan&& p) {
    rts.push_back(std::move(p));
    return (int)rts.size() - 1;
  }
  // fill the packed layer sub-blocks of row-thread plan ``idx`` from S
  Status pack(fpeps_ctx_s* ctx, int idx, const double* S, int64_t s_size);
};

Status run_gemm(fpeps_ctx_s* ctx, const PlanSet& ps, int idx, const double* A, int64_t a_size,
                const double* B, int64_t b_size, double* C, int64_t c_size, bool timed = false,
                int label = 0);
// B or C in FP32 (sizes in elements; see launch_gemm_mixed)
Status run_gemm_mixed(fpeps_ctx_s* ctx, const PlanSet& ps, int idx, const double* A,
                      int64_t a_size, const void* B, bool b_f32, int64_t b_size, void* C,
                      bool c_f32, int64_t c_size, bool timed = false, int label = 0);
// The same on FP32 MFMA (FP32 accumulation per 16-deep K tile, tiles summed in
// FP64): A an FP32 copy, B and C in
// FP32 or FP64
Status run_gemm_f32(fpeps_ctx_s* ctx, const PlanSet& ps, int idx, const float* A, int64_t a_size,
                    const void* B, bool b_f32, int64_t b_size, void* C, bool c_f32, int64_t c_size,
                    bool timed = false, int label = 0);
// exactly one of A (FP64) and A32 (FP32) is given; ``part`` (at least the
// plan's partial_size doubles) replaces the context's split-K buffer
Status run_gemm_any(fpeps_ctx_s* ctx, const PlanSet& ps, int idx, const double* A,
                    const float* A32, int64_t a_size, const void* B, bool b_f32, int64_t b_size,
                    void* C, bool c_f32, int64_t c_size, bool timed, int label,
                    double* part = nullptr);
Status run_rt(fpeps_ctx_s* ctx, const PlanSet& ps, int idx, const void* X, int64_t x_size,
              void* Y, int64_t y_size, bool f32, bool timed = false, int label = 0);

// Two timing events released on every return path.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() = default;
  EventPair(const EventPair&) = delete;
  EventPair& operator=(const EventPair&) = delete;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  hipError_t create() {
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) {
      a = nullptr;
      return e;
    }
    e = hipEventCreate(&b);
    if (e != hipSuccess) b = nullptr;
    return e;
  }
};

}  // namespace fp
