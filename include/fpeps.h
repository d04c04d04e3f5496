/*
 * fpeps.h -- C ABI of the MI355X (gfx950) library for the boundary-MPS row
 * absorption of finite PEPS-PEPO networks (Scheb, "Improved contraction of
 * finite projected entangled pair states", arXiv:2511.01039).
 *
 * What the calls compute
 *   fpeps_env_absorb     one row (ket, PEPO, bra = ket) absorbed into a
 *                        boundary MPS (Sec. 2: bundles of D w D legs are
 *                        compressed to a bond chi), each bond truncated by
 *                        the randomized SVD of Sec. 4 (Halko et al. 2011,
 *                        Example 1.6), optionally expanded by controlled bond
 *                        expansion (Sec. 4, Figs. 3-5).
 *   fpeps_site_shape /   the implicit site operator M_x (the (chi D w D) x
 *   fpeps_site_apply     (chi D w D) matrix A of Sec. 4, never formed) and its
 *                        transpose applied to blocks of vectors; the chain of
 *                        block-sparse contractions of Sec. 3.
 *   fpeps_rsvd_truncate  randomized SVD of explicit matrices with one
 *                        truncation over the whole batch (Sec. 4).
 *   fpeps_cbe_expand     truncated complement (CBE) of explicit matrices:
 *                        the most weighty directions of (1 - U U^T) A
 *                        (1 - V^T V), projectors split as in Fig. 5(b)-(g).
 *   fpeps_expect         network value of a top and a bottom environment
 *                        (the sandwich of Fig. 1 once environments exist).
 *   fpeps_heff_apply     the effective single-site operator of the Davidson
 *                        step applied to a PEPS tensor (Fig. 2(b)).
 *
 * Conventions (all calls)
 *   - Tensor data is double precision, on the device of the context, owned
 *     by the caller. Structure arrays (legs, blocks) are host memory owned
 *     by the caller. The library never frees caller memory; it keeps only
 *     its own workspace (device, grown on demand, freed by fpeps_destroy).
 *   - Block-sparse layout: a tensor has nlegs legs; leg l has nsect[l]
 *     sectors with nlab integer labels and a dimension each. A block is the
 *     dense sub-array of one sector tuple, stored row-major (last leg
 *     fastest) at data[block_off[i]]. Blocks may appear in any order but must
 *     not overlap.
 *   - Leg orders: ket A[p, l, r, u, d]; PEPO W[q, p, l, r, u, d] (q bra-side,
 *     p ket-side physical leg); environment site T[a, k, w, b', b] (left bond,
 *     the downward ket, PEPO and bra legs, right bond). A bottom environment
 *     uses the same order with the bundle legs facing up.
 *   - Symmetry: FPEPS_SYM_NONE (any sector tuple may be present),
 *     FPEPS_SYM_U1U1 (labels (dn, 2Sz); flux sum_l dir_l q_l = 0),
 *     FPEPS_SYM_SU2 (labels (2j); synthetic reduced tensors whose block
 *     pairs carry a recoupling scalar, see fpeps_opts.coef_seed).
 *   - Asynchrony: calls run on the context's HIP stream. Calls that return
 *     host values (reports, kept counts, fpeps_expect) synchronise it.
 *   - Errors: every call returns fpeps_status; no exception or abort crosses
 *     the ABI. fpeps_last_error(ctx) returns a message for the last failure.
 *     On error, output buffers hold unspecified values.
 */
#ifndef FPEPS_H
#define FPEPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fpeps_ctx_s* fpeps_ctx;

typedef enum {
  FPEPS_OK = 0,
  FPEPS_ERR_ARG = -1,         /* null pointer, bad enum, negative size */
  FPEPS_ERR_SHAPE = -2,       /* legs that must match do not, bad block */
  FPEPS_ERR_SYMMETRY = -3,    /* block violating the symmetry rule */
  FPEPS_ERR_NOMEM = -4,       /* device allocation failed */
  FPEPS_ERR_HIP = -5,         /* a HIP runtime call failed */
  FPEPS_ERR_NUMERIC = -6,     /* NaN / Inf met, or a factorisation broke down */
  FPEPS_ERR_CAPACITY = -7,    /* an output buffer is too small; see report */
  FPEPS_ERR_UNSUPPORTED = -8, /* valid request the library does not implement */
  FPEPS_ERR_NODEVICE = -9     /* no usable gfx950 device */
} fpeps_status;

typedef enum {
  FPEPS_FP64 = 0,     /* every product and intermediate in double precision */
  FPEPS_FP32 = 1,     /* mixed: in the range finder's sketch and power
                         iterations, except its last product, the
                         environment and remainder contractions (chain steps
                         1 and 5 and their transposes) run on FP32 MFMA with
                         FP32 accumulation inside each 16-deep K tile (the
                         tiles summed in FP64) from FP32 copies of T and R, and
                         the chain intermediates (X1..X4 and their
                         transposes) are stored in FP32 (the layer steps
                         read and write FP32 and accumulate in FP64). The
                         last range-finder product, the projection
                         B = Q^T M, orthonormalisation, core factorisation,
                         cut and norms are FP64. Available in
                         fpeps_env_absorb and fpeps_site_apply (which applies
                         the chain in this mixed form). */
  FPEPS_BF16X3 = 2    /* reserved (FPEPS_ERR_UNSUPPORTED) */
} fpeps_precision;

typedef enum {
  FPEPS_SYM_NONE = 0,
  FPEPS_SYM_U1U1 = 1,
  FPEPS_SYM_SU2 = 2
} fpeps_symmetry;

/* Block-sparse tensor (input and output).
 * Input: the library reads every field except the capacities.
 * Output: the caller sets the capacities and the array pointers; the library
 * fills nlegs, nsect, dirs, labels, dims, nblocks, block_sect, block_off,
 * nelem and data. If a capacity is too small the call fails with
 * FPEPS_ERR_CAPACITY and the report (when given) holds the required sizes. */
typedef struct {
  int32_t nlegs;
  int32_t nlab;          /* labels per sector (1 or 2) */
  int32_t max_sect;      /* row stride of labels/dims: sectors per leg */
  int32_t* nsect;        /* host [nlegs] */
  int32_t* dirs;         /* host [nlegs], +1 or -1 */
  int32_t* labels;       /* host [nlegs * max_sect * nlab]; leg l, sector s at (l*max_sect+s)*nlab */
  int32_t* dims;         /* host [nlegs * max_sect] */
  int32_t nblocks;
  int32_t max_blocks;    /* output capacity (blocks) */
  int32_t* block_sect;   /* host [nblocks * nlegs] (capacity max_blocks * nlegs) */
  int64_t* block_off;    /* host [nblocks] element offsets into data */
  double* data;          /* device */
  int64_t nelem;         /* elements used */
  int64_t max_elem;      /* output capacity (elements) */
} fpeps_tensor;

typedef struct {
  int32_t chi;            /* bond kept after truncation (multiplets for SU(2)) */
  int32_t oversample;     /* p: first sketch width k_J = min(m_J, n_J, h_J + p), h_J the
                             previous site's kept count of the sector's label (absorption)
                             or ceil(chi m_J / sum m); widened while saturated (see
                             fpeps_report.rsvd_passes) */
  int32_t power_iters;    /* q: subspace iterations */
  int32_t cbe_extra;      /* directions added by CBE per bond (0: none) */
  uint64_t seed;          /* Philox4x32-10 key of the Gaussian sketch */
  int32_t row;            /* row index, part of the sketch counter */
  int32_t precision;      /* fpeps_precision */
  int32_t symmetry;       /* fpeps_symmetry */
  int32_t fermionic;      /* 1: parity sign on every contracted block pair */
  uint64_t coef_seed;     /* SU(2): key of the synthetic recoupling scalars */
  int64_t slice_budget;   /* bytes of chain intermediates live at once, over all streams
                             (0: a budget tuned by fpeps_autotune_absorb, else the smaller
                             of 128 GiB and 45% of the device's memory). The slices of a
                             site are spread round-robin over four streams, so every
                             slice is sized for a quarter of it (also with
                             FPEPS_FLAG_ONE_STREAM, so that the slicing does not depend
                             on the streams) */
  uint32_t flags;         /* FPEPS_FLAG_* */
  int32_t tag;            /* explicit-matrix calls: counter word c2 of the sketch */
  double sv_cut;          /* singular values <= sv_cut * largest are never kept. <= 0: the
                             rank floor eps * max_J max(m_J, n_J) (eps = 2^-52, the rank
                             tolerance of Numerical Recipes Sec. 2.6): values below it are
                             not resolved by a backward-stable factorisation */
} fpeps_opts;

#define FPEPS_FLAG_NO_GRAPH 1u      /* fpeps_heff_prepare: capture no HIP graph;
                                       fpeps_heff_apply_prepared then launches the
                                       three products itself (same kernels, same
                                       results). No other call captures graphs */
#define FPEPS_FLAG_CHECK_FINITE 2u  /* scan inputs for NaN/Inf first */
#define FPEPS_FLAG_TIME_KERNELS 4u  /* time every chain launch with HIP events */
#define FPEPS_FLAG_ONE_STREAM 8u    /* run every slice on the context's stream (one set of
                                       chain intermediates; no overlap of slices) */

typedef struct {
  double alg_flops;        /* algorithmic flop count (block-pair GEMMs + factorisations) */
  double seconds;          /* device time of the call (HIP events) */
  double discarded_weight; /* largest per-site sum(s^2 cut)/sum(s^2) */
  double min_rel_gap;      /* smallest (s_kept_last - s_cut_first)/s_kept_last */
  double log_norm;         /* sum of log of the norms divided out */
  double peak_workspace;   /* bytes of chain intermediates live at once (all streams) */
  int32_t kept_total;      /* sum of kept values over sites / matrices */
  int32_t nslices;         /* chain slices used (largest site) */
  uint32_t fallbacks;      /* bit 0: an orthonormalisation needed more than one shifted
                              CholeskyQR pass (rank-deficient or very ill-conditioned
                              sketch); bit 1: a Jacobi eigen-decomposition stopped at its
                              40-sweep limit; bit 2: a sketch was exactly rank-deficient
                              and finished by SVQB (its null directions are zero columns) */
  int32_t required_blocks; /* on FPEPS_ERR_CAPACITY: blocks needed */
  int64_t required_elem;   /* on FPEPS_ERR_CAPACITY: elements needed */
  int32_t required_sect;   /* on FPEPS_ERR_CAPACITY: sectors per leg needed */
  int32_t kernel_launches; /* FPEPS_FLAG_TIME_KERNELS: chain launches timed */
  double kernel_seconds;   /* FPEPS_FLAG_TIME_KERNELS: sum of their durations (HIP events) */
  double kernel_flops;     /* algorithmic flops (2 m n k over block pairs) of those launches */
  /* the same split by kernel class (FPEPS_FLAG_TIME_KERNELS):
   * layer steps = ket, PEPO and bra contractions and their transposes
   * (HBM bound; bytes = distinct input blocks read once + output written once),
   * contractions = environment site and remainder products (MFMA) */
  int32_t layer_launches;
  double layer_seconds;
  double layer_flops;
  double layer_bytes;
  int32_t gemm_launches;
  double gemm_seconds;
  double gemm_flops;
  double gemm_bytes;
  /* fpeps_env_absorb: sites whose analysis and plans were those of the
     previous site (equal block structure of T, A, W and the remainder, equal
     sketch widths); they are uploaded again with the site's own layer data. */
  int32_t plan_reuses;
  /* factorisation passes (summed over the sites of an absorption): a pass
     whose cut kept more than k_J - p/2 values of a sector its sketch does not
     cover is repeated with that sector's width raised to
     min(m_J, n_J, 2 k_J + p) */
  int32_t rsvd_passes;
  double workspace_bytes;  /* device workspace the context holds at the end of the call
                              (every buffer; freed by fpeps_destroy or a new allocator) */
  double alg_bytes;        /* fpeps_env_absorb: algorithmic HBM bytes, every chain
                              application reading T, R, the ket and the PEPO once and
                              writing its output once (intermediates not counted) */
} fpeps_report;

/* Context: one per host thread. ``stream`` is a hipStream_t (NULL: default
 * stream). Fails with FPEPS_ERR_NODEVICE when ``device`` is not a gfx950. */
fpeps_status fpeps_create(fpeps_ctx* out, int32_t device, void* stream);
fpeps_status fpeps_destroy(fpeps_ctx ctx);
fpeps_status fpeps_set_stream(fpeps_ctx ctx, void* stream);
const char* fpeps_last_error(fpeps_ctx ctx);
const char* fpeps_version(void);

/* Device memory of the context's workspace (chain intermediates, sketch and
 * range matrices, plans) from the caller's allocator, for instance a
 * framework's caching allocator: alloc(bytes, user) returns device memory of
 * the context's device or NULL (the call needing it then fails with
 * FPEPS_ERR_NOMEM); free_(ptr, user) takes back a pointer alloc returned.
 * The library frees a buffer only after the work using it on every stream
 * of the context has finished. Both NULL restores hipMalloc / hipFree.
 * Workspace held from the previous allocator is freed to it first (the call
 * waits for the device). Not to be called while another call on the same
 * context runs. */
fpeps_status fpeps_set_allocator(fpeps_ctx ctx, void* (*alloc)(size_t bytes, void* user),
                                 void (*free_)(void* ptr, void* user), void* user);

/* Absorb one row of L sites into the top environment env_in[0..L-1].
 * ket[x] (5 legs) and pepo[x] (6 legs) are the row tensors; the bra is the
 * ket. env_out[x] receives the new environment sites (5 legs, layout above):
 * sites 0..L-2 are isometries over (a, k, w, b') and site L-1 has unit norm.
 * *log_norm (host, in/out) is increased by the logarithm of the norms that
 * were divided out. Left and right boundary legs must have dimension 1.
 * Synchronises the stream once per site (the kept sector sizes decide the
 * next site's shapes). */
fpeps_status fpeps_env_absorb(fpeps_ctx ctx, int32_t L, const fpeps_tensor* env_in,
                              const fpeps_tensor* ket, const fpeps_tensor* pepo,
                              const fpeps_opts* opts, fpeps_tensor* env_out,
                              double* log_norm, fpeps_report* report);

/* fpeps_env_absorb with its slice budget and GEMM tiles chosen by
 * measurement on this row (the autotuner). When opts->slice_budget is 0 the
 * row is first absorbed once per budget candidate (32 GiB and 64 GiB when
 * below the default of fpeps_opts.slice_budget, and that default) on the
 * library's streams and the fastest is kept. Then, at that budget, it is
 * absorbed tile_candidates times (1 to 4) on one stream with every GEMM
 * launch timed: run r gives every grouped GEMM step the r-th tile of the
 * planner's padding-efficiency ranking, and each step signature (a hash of
 * the step and its output block sizes and contracted extents) keeps the
 * tile with the smallest mean launch time. The table is stored in the
 * context: later fpeps_env_absorb and fpeps_site_apply calls use the tuned
 * tile of every step whose signature it holds (other steps keep the model's
 * tile), and the tuned budget when their opts->slice_budget is 0. Finally the
 * row is absorbed with the tuned choices into env_out, *log_norm and the
 * report, as fpeps_env_absorb does (the tuning runs' results are discarded).
 * Results differ from the untuned call only by rounding (tiles change the
 * split of long contractions). On failure the context keeps its previous
 * table. Synchronises many times; costs 4 + tile_candidates absorptions
 * (1 + tile_candidates when opts->slice_budget is set). */
fpeps_status fpeps_autotune_absorb(fpeps_ctx ctx, int32_t L, const fpeps_tensor* env_in,
                                   const fpeps_tensor* ket, const fpeps_tensor* pepo,
                                   const fpeps_opts* opts, int32_t tile_candidates,
                                   fpeps_tensor* env_out, double* log_norm,
                                   fpeps_report* report);
/* The context's tuned table as a text file (on-disk autotune cache), and
 * back. Format: lines starting with '#' are comments; "fpeps-tune 1";
 * "slice_budget <bytes>"; then one "<signature, 16 hex digits> <mt> <nt>"
 * line per tuned step. fpeps_tune_save fails with FPEPS_ERR_ARG when the
 * context has no table or the file cannot be written; fpeps_tune_load
 * replaces the context's table and fails, keeping it, on a file that is not
 * a table of this format (or names a tile the kernel does not have).
 * fpeps_tune_clear drops the table (the planner's model again).
 * fpeps_tune_info: number of tuned signatures (-1 without a table) and the
 * tuned slice budget in bytes (0: none). */
fpeps_status fpeps_tune_save(fpeps_ctx ctx, const char* path);
fpeps_status fpeps_tune_load(fpeps_ctx ctx, const char* path);
fpeps_status fpeps_tune_clear(fpeps_ctx ctx);
fpeps_status fpeps_tune_info(fpeps_ctx ctx, int32_t* entries, int64_t* slice_budget);

/* Per-site diagnostics of the last fpeps_env_absorb on this context:
 * the singular values of every sector (sectors in label order, each
 * descending), the sector of each value and the kept count per sector. */
fpeps_status fpeps_absorb_diag(fpeps_ctx ctx, int32_t site, int32_t capacity, double* sigma,
                               int32_t* sector, int32_t* count, int32_t* nsectors,
                               int32_t* kept /* [capacity] per sector */);

/* Sector structure of the site operator M_x with remainder R (legs
 * [c, a, lk, lw, lb]), environment site T, ket A and PEPO W.
 * nsect (out): number of sketch sectors J (label order). For each J:
 * labels [nsect * nlab], m[J] (rows), n[J] (columns). Arrays have
 * ``capacity`` entries. */
fpeps_status fpeps_site_shape(fpeps_ctx ctx, const fpeps_tensor* R, const fpeps_tensor* T,
                              const fpeps_tensor* A, const fpeps_tensor* W,
                              const fpeps_opts* opts, int32_t capacity, int32_t* nsect,
                              int32_t* labels, int64_t* m, int64_t* n);

/* Apply M_x (transpose = 0) or M_x^T (transpose = 1) to per-sector blocks
 * of k[J] vectors. x_in holds, for each sector J in order, the n[J] x k[J]
 * (M) or m[J] x k[J] (M^T) row-major matrix; y_out receives m[J] x k[J]
 * (or n[J] x k[J]). Rows follow the canonical order: sector tuples of the
 * row legs (c, dk, dw, db) or column legs (b, rk, rw, rb) in lexicographic
 * order of sector indices, row-major inside a tuple. Device pointers. */
fpeps_status fpeps_site_apply(fpeps_ctx ctx, const fpeps_tensor* R, const fpeps_tensor* T,
                              const fpeps_tensor* A, const fpeps_tensor* W,
                              const fpeps_opts* opts, int32_t transpose, const int32_t* k,
                              const double* x_in, double* y_out, fpeps_report* report);

/* Randomized SVD of nmat explicit row-major matrices A_i (m_i x n_i, device),
 * one truncation to opts->chi over the batch. Sketch of matrix i: Philox
 * counter (element/2, i, opts->tag, 0). Outputs (device): U_i (m_i x kept_i,
 * row-major, capacity m_i * min(m_i, n_i)), R_i = S V^T (kept_i x n_i,
 * capacity min(m_i, n_i) * n_i). Host outputs: kept[nmat]; sigma (kept values
 * of matrix 0, then 1, ...; capacity sum min(m_i, n_i)). */
fpeps_status fpeps_rsvd_truncate(fpeps_ctx ctx, int32_t nmat, const int64_t* m,
                                 const int64_t* n, const double* const* A,
                                 const fpeps_opts* opts, double* const* U_out,
                                 double* const* R_out, int32_t* kept, double* sigma,
                                 fpeps_report* report);

/* The same for several independent truncation problems in one call (for
 * instance the per-site truncations of a row, Sec. 4; the batching of all of
 * a row's truncations into grouped launches): matrix i belongs to problem
 * group[i] (host array, values 0 .. nmat-1). Each group has its own sketch
 * widths and its own cut to opts->chi; its sketch counters are
 * (element/2, ordinal of the matrix inside its group, opts->tag + group[i], 0).
 * A grouped call therefore returns what one fpeps_rsvd_truncate call per
 * group (matrices in the same order, tag + g) returns, up to rounding order.
 * The report gives the smallest relative gap and the largest discarded
 * weight over the groups. */
fpeps_status fpeps_rsvd_truncate_grouped(fpeps_ctx ctx, int32_t nmat, const int64_t* m,
                                         const int64_t* n, const double* const* A,
                                         const int32_t* group, const fpeps_opts* opts,
                                         double* const* U_out, double* const* R_out,
                                         int32_t* kept, double* sigma, fpeps_report* report);

/* Controlled bond expansion of explicit matrices: for each A_i (m_i x n_i)
 * with kept left space U_i (m_i x r_i, orthonormal columns) and kept right
 * space V_i (r_i x n_i, orthonormal rows), the opts->cbe_extra most weighty
 * directions (over the batch) of (1 - U U^T) A (1 - V^T V). Sketch of matrix
 * i: Philox counter (element/2, i, opts->tag, 1 << 16). Output Q_i (device,
 * m_i x e_i row-major, orthogonal to U_i; capacity m_i * min(m_i, n_i)),
 * e_i in kept[i] (host), the matching singular values in sigma (host). */
fpeps_status fpeps_cbe_expand(fpeps_ctx ctx, int32_t nmat, const int64_t* m, const int64_t* n,
                              const double* const* A, const int32_t* r,
                              const double* const* U, const double* const* V,
                              const fpeps_opts* opts, double* const* Q_out, int32_t* kept,
                              double* sigma, fpeps_report* report);

/* Bond expansion of several independent problems in one call: group[i] as in
 * fpeps_rsvd_truncate_grouped; opts->cbe_extra directions per group, sketch
 * counters (element/2, ordinal inside the group, opts->tag + group[i],
 * 1 << 16). */
fpeps_status fpeps_cbe_expand_grouped(fpeps_ctx ctx, int32_t nmat, const int64_t* m,
                                      const int64_t* n, const double* const* A,
                                      const int32_t* group, const int32_t* r,
                                      const double* const* U, const double* const* V,
                                      const fpeps_opts* opts, double* const* Q_out,
                                      int32_t* kept, double* sigma, fpeps_report* report);

/* Network value Z of a top environment (L sites) and a bottom environment
 * whose bundle legs (k, w, b') match the top's (Sec. 2, Fig. 1 once both
 * environments exist): the contraction of all sites, left and right bonds
 * of dimension 1 at the ends, times exp(log_norm_top + log_norm_bottom)
 * (the logarithms of the norms the absorptions divided out). Returned as
 * *sign (host: +1, -1, or 0 for an exact zero) and *log_abs = log |Z| (host;
 * -inf for zero): the partial contraction is normalised after every site
 * and its logarithm accumulated, so |Z| may lie far outside the range of a
 * double. Non-finite data gives FPEPS_ERR_NUMERIC. Synchronises. */
fpeps_status fpeps_expect(fpeps_ctx ctx, int32_t L, const fpeps_tensor* top,
                          const fpeps_tensor* bottom, double log_norm_top,
                          double log_norm_bottom, int32_t* sign, double* log_abs);

/* The effective single-site operator of the Davidson step applied to a PEPS
 * tensor (Sec. 3, contraction pattern of Fig. 2(b)):
 *   y[q, lb, rb, tb, db] = sum T[a, tk, tw, tb, b] L[a, lk, lw, lb, c]
 *                              B[c, dk, dw, db, d] R[b, rk, rw, rb, d]
 *                              W[q, p, lw, rw, tw, dw] A[p, lk, rk, tk, dk]
 * with T the top boundary site, L and R the left and right environments, B
 * the bottom boundary site (each leg k, w, b' facing the ket, PEPO and bra
 * legs of the site), W the site's PEPO and A the ket (the Davidson vector).
 * Evaluated as ((T L) C) (B R), the sandwich C = (A, W) applied layer by
 * layer; every step is one grouped block-pair GEMM, and for FPEPS_SYM_SU2
 * each block pair carries the synthetic scalar of its step (11 .. 15) and
 * blocks, so this association is part of the definition. Inputs are device
 * tensors in the block layout above; y_out (bra-side legs q, lb, rb, tb, db)
 * is filled like an absorption output (FPEPS_ERR_CAPACITY and the required
 * sizes in the report when a capacity is short). FP64 only. The report
 * gives the algorithmic flops (2 m n k over the block pairs) and the device
 * time. Synchronises. */
fpeps_status fpeps_heff_apply(fpeps_ctx ctx, const fpeps_tensor* T, const fpeps_tensor* L,
                              const fpeps_tensor* B, const fpeps_tensor* R, const fpeps_tensor* W,
                              const fpeps_tensor* A, const fpeps_opts* opts, fpeps_tensor* y_out,
                              fpeps_report* report);

/* The same operator prepared for repeated products with one environment
 * (the Davidson iterations of a site, Sec. 3): T L and B R do not depend on
 * the vector and are contracted once here; the three vector-dependent
 * products are captured as a HIP graph and replayed by
 * fpeps_heff_apply_prepared. Arguments as fpeps_heff_apply; A gives the
 * structure of the vectors (and its data the first product, written to
 * y_out with the output structure). T, L, B, R, W and A may be freed after
 * the call: the handle keeps what it needs on the device, in buffers of its
 * own. With FPEPS_FLAG_NO_GRAPH in opts->flags nothing is captured and each
 * product launches the kernels directly. Synchronises. The handle belongs
 * to ctx, must be released before fpeps_destroy, and is invalidated by
 * fpeps_set_allocator (later products fail with FPEPS_ERR_ARG). */
typedef struct fpeps_heff_s* fpeps_heff;
fpeps_status fpeps_heff_prepare(fpeps_ctx ctx, const fpeps_tensor* T, const fpeps_tensor* L,
                                const fpeps_tensor* B, const fpeps_tensor* R,
                                const fpeps_tensor* W, const fpeps_tensor* A,
                                const fpeps_opts* opts, fpeps_tensor* y_out, fpeps_heff* op,
                                fpeps_report* report);
/* y = H_eff a for a vector a in the prepared structure: a (device, a_elems
 * doubles, equal to the prepared A's nelem) in A's block layout, y (device,
 * y_elems >= the output's nelem) in the output layout written by the
 * prepare call. Runs on the context's stream (copy in, graph replay, copy
 * out) and synchronises; the report gives the three products' flops and the
 * device time. Calls on one handle must not overlap. */
fpeps_status fpeps_heff_apply_prepared(fpeps_heff op, const double* a, int64_t a_elems,
                                       double* y, int64_t y_elems, fpeps_report* report);
fpeps_status fpeps_heff_release(fpeps_heff op);

/* fpeps_expect for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same value, computed by the same kernels in the same order, with every
 * workspace buffer (partial contractions, intermediates, reductions, GEMM
 * plans) taken from one library-owned device array of 64 MiB per GPU,
 * reserved for the life of the process. The call makes no hipMalloc,
 * hipFree or other device allocation. A problem whose workspace exceeds the
 * array (roughly environment bonds above 150 at D w D = 144) fails with
 * FPEPS_ERR_CAPACITY and a message giving the bytes it needs. All calls on
 * one GPU share its array: calls that overlap in time on one GPU (several
 * contexts or host threads) race and must be serialised by the caller. The
 * array keeps the last call's contents; every buffer a call reads is
 * written by that call first. Host-side planning still uses the host heap.
 * Synchronises. */
fpeps_status fpeps_expect_noalloc(fpeps_ctx ctx, int32_t L, const fpeps_tensor* top,
                                  const fpeps_tensor* bottom, double log_norm_top,
                                  double log_norm_bottom, int32_t* sign, double* log_abs);

#ifdef __cplusplus
}
#endif
#endif /* FPEPS_H */
