// Autotuner of the row absorption: GEMM tile shapes per step signature and
// the slice budget, chosen by measurement on the caller's own row.
//
// The slices of Sec. 3 bound the chain intermediates; how large they may be
// (the budget) trades fewer, larger launches against overlap of slices on
// the library's streams. Every grouped GEMM step can run with any of the
// kernel's tile shapes; the planner's padding model ranks them. Both choices
// are measured here:
//   1. the row is absorbed once per slice-budget candidate (32 and 64 GiB
//      and the library's default, on the library's streams, with the
//      model's tiles) and the fastest budget is kept;
//   2. at that budget the row is absorbed once per tile rank (one stream,
//      every GEMM launch timed by HIP events; rank r makes every step use
//      the r-th tile of the model's ranking), and each step signature keeps
//      the tile with the smallest mean launch time.
// The table is the context's: later absorptions (and site products) whose
// steps have a tuned signature use its tile, and with slice_budget = 0 its
// budget. Step signatures hash the step's output block sizes, so a table
// applies to rows of the same block structure and widths.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "driver.hpp"

namespace fp {

Status autotune_absorb(fpeps_ctx_s* ctx, int L, const fpeps_tensor* env_in,
                       const fpeps_tensor* ket, const fpeps_tensor* pepo, const fpeps_opts* o,
                       int ncand, fpeps_tensor* env_out, double* log_norm, fpeps_report* rep) {
  if (!o || !log_norm) return fail(FPEPS_ERR_ARG, "null argument");
  if (ncand < 1 || ncand > 4) return fail(FPEPS_ERR_ARG, "tile candidates: 1 to 4");
  const double ln0 = *log_norm;
  // on failure the context keeps the table it had
  struct Restore {
    fpeps_ctx_s* c;
    std::shared_ptr<TuneTable> prev;
    bool done = false;
    ~Restore() {
      c->tile_rank = -1;
      c->tune_record = false;
      c->tune_log.clear();
      if (!done) c->tune = prev;
    }
  } restore{ctx, ctx->tune};
  ctx->tune.reset();   // the measurement runs use the model's ranking
  // every run fills the report afresh (some of its fields add up)
  auto run = [&](const fpeps_opts* oo, double* ln) {
    if (rep) std::memset(rep, 0, sizeof(*rep));
    return absorb_row(ctx, L, env_in, ket, pepo, oo, env_out, ln, rep);
  };
  auto tab = std::make_shared<TuneTable>();
  // 1. slice budget (only when the caller leaves it to the library)
  if (o->slice_budget <= 0) {
    // 32 and 64 GiB, and the default (128 GiB on a 288 GB device); none above it
    const int64_t dflt = ctx->default_budget();
    std::vector<int64_t> cand;
    for (int64_t b : {(int64_t)32 << 30, (int64_t)64 << 30})
      if (b < dflt) cand.push_back(b);
    cand.push_back(dflt);
    double best = std::numeric_limits<double>::infinity();
    int64_t best_b = 0;
    for (int64_t b : cand) {
      fpeps_opts u = *o;
      u.slice_budget = b;
      u.flags &= ~(uint32_t)FPEPS_FLAG_TIME_KERNELS;
      double ln = ln0;
      FP_TRY(run(&u, &ln));
      const double t = rep ? rep->seconds : 0.0;
      if (!rep || t < best) {
        best = t;
        best_b = b;
      }
      if (!rep) break;   // nothing to compare without a report
    }
    tab->slice_budget = best_b;
  }
  // 2. tiles, at the chosen budget
  fpeps_opts t = *o;
  t.flags |= FPEPS_FLAG_ONE_STREAM | FPEPS_FLAG_TIME_KERNELS;
  if (t.slice_budget <= 0) t.slice_budget = tab->slice_budget;
  ctx->tune_log.clear();
  ctx->tune_record = true;
  std::map<uint64_t, std::map<std::array<int, 2>, std::array<double, 2>>> acc;
  for (int r = 0; r < ncand; ++r) {
    ctx->tile_rank = r;
    double ln = ln0;
    FP_TRY(run(&t, &ln));
    // the log holds this run's seconds and launches per (signature, tile)
    for (auto& sv : ctx->tune_log)
      for (auto& tv : sv.second) {
        auto& a = acc[sv.first][tv.first];
        a[0] += tv.second[0];
        a[1] += tv.second[1];
      }
    ctx->tune_log.clear();
  }
  ctx->tile_rank = -1;
  ctx->tune_record = false;
  for (auto& sv : acc) {
    double best = std::numeric_limits<double>::infinity();
    std::array<int, 2> bt{0, 0};
    for (auto& tv : sv.second) {
      const double mean = tv.second[0] / std::max(1.0, tv.second[1]);
      if (mean < best) {
        best = mean;
        bt = tv.first;
      }
    }
    if (valid_tile(bt[0], bt[1])) tab->tiles[sv.first] = {(int16_t)bt[0], (int16_t)bt[1]};
  }
  // the result: the row with the tuned choices (the caller's flags)
  ctx->tune = tab;
  restore.done = true;
  return run(o, log_norm);
}

Status tune_save(fpeps_ctx_s* ctx, const char* path) {
  if (!path) return fail(FPEPS_ERR_ARG, "null path");
  if (!ctx->tune) return fail(FPEPS_ERR_ARG, "the context has no tuned table");
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(FPEPS_ERR_ARG, std::string("cannot write ") + path);
  std::fprintf(f, "fpeps-tune 1\nslice_budget %lld\n", (long long)ctx->tune->slice_budget);
  for (auto& kv : ctx->tune->tiles)
    std::fprintf(f, "%016llx %d %d\n", (unsigned long long)kv.first, kv.second[0], kv.second[1]);
  const bool ok = std::fclose(f) == 0;
  return ok ? Status::ok() : fail(FPEPS_ERR_ARG, std::string("cannot write ") + path);
}

// Text format: lines starting with '#' are comments; then "fpeps-tune 1",
// "slice_budget <bytes>", and one "<signature hex> <mt> <nt>" line per step.
Status tune_load(fpeps_ctx_s* ctx, const char* path) {
  if (!path) return fail(FPEPS_ERR_ARG, "null path");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(FPEPS_ERR_ARG, std::string("cannot read ") + path);
  auto tab = std::make_shared<TuneTable>();
  std::vector<std::string> lines;
  char buf[512];
  while (std::fgets(buf, sizeof buf, f)) {
    std::string l(buf);
    while (!l.empty() && (l.back() == '\n' || l.back() == '\r' || l.back() == ' ')) l.pop_back();
    if (l.empty() || l[0] == '#') continue;
    lines.push_back(l);
  }
  std::fclose(f);
  char magic[32] = {0};
  int version = 0;
  long long budget = -1;
  bool ok = lines.size() >= 2 && std::sscanf(lines[0].c_str(), "%31s %d", magic, &version) == 2 &&
            std::strcmp(magic, "fpeps-tune") == 0 && version == 1 &&
            std::sscanf(lines[1].c_str(), "slice_budget %lld", &budget) == 1 && budget >= 0;
  for (size_t i = 2; ok && i < lines.size(); ++i) {
    unsigned long long sig = 0;
    int mt = 0, nt = 0;
    char extra = 0;
    if (std::sscanf(lines[i].c_str(), "%llx %d %d %c", &sig, &mt, &nt, &extra) != 3 ||
        !valid_tile(mt, nt))
      ok = false;
    else
      tab->tiles[(uint64_t)sig] = {(int16_t)mt, (int16_t)nt};
  }
  if (!ok) return fail(FPEPS_ERR_ARG, std::string("not a tuned table: ") + path);
  tab->slice_budget = budget;
  ctx->tune = tab;
  return Status::ok();
}

Status tune_clear(fpeps_ctx_s* ctx) {
  ctx->tune.reset();
  return Status::ok();
}

Status tune_info(fpeps_ctx_s* ctx, int32_t* entries, int64_t* slice_budget) {
  if (entries) *entries = ctx->tune ? (int32_t)ctx->tune->tiles.size() : -1;
  if (slice_budget) *slice_budget = ctx->tune ? ctx->tune->slice_budget : 0;
  return Status::ok();
}

}  // namespace fp
