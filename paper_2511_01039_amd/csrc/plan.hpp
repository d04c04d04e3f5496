// Host planner of the block-sparse contraction chain.
//
// Every contraction of the chain (Sec. 3: the environment T, L, B contracted
// with the ket, PEPO and bra layers) is planned as a list of small dense
// products, one per pair of blocks that agree on the contracted legs. The
// planner turns them into GEMM work for the device: for each output block a
// list of (A block, B block, alpha) pairs and, for every operand, tables of
// element offsets along the M, N and K index of the product. Output blocks
// are disjoint, so each output tile is owned by one workgroup and needs no
// atomics (the slices of Sec. 3 "do not overlap").
#pragma once

#include <array>
#include <cstdint>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

namespace fp {

enum SymKind { SYM_NONE = 0, SYM_U1U1 = 1, SYM_SU2 = 2 };

// Leg names of the chain (identifiers only; data layouts are per tensor).
enum LegName : int {
  N_a = 0, N_tk, N_tw, N_tb, N_b, N_rk, N_rw, N_rb, N_j, N_p, N_q, N_lk, N_lw, N_lb,
  N_dk, N_dw, N_db, N_c, N_d, N_COUNT
};

constexpr int MAXL = 10;

struct Leg {
  int nlab = 1;
  int dir = 1;
  std::vector<int32_t> lab;  // nsect * nlab
  std::vector<int32_t> dim;  // nsect
  int nsect() const { return (int)dim.size(); }
  const int32_t* label(int s) const { return lab.data() + (size_t)s * nlab; }
  int64_t total() const {
    int64_t t = 0;
    for (int d : dim) t += d;
    return t;
  }
  bool same_sectors(const Leg& o) const { return nlab == o.nlab && lab == o.lab && dim == o.dim; }
};
using LegP = std::shared_ptr<const Leg>;

struct Block {
  std::array<uint16_t, MAXL> sect{};   // sector index per storage position
  int64_t base = 0;                    // element offset of element (0,...,0)
  std::array<int64_t, MAXL> stride{};  // element stride per storage position
};

// Structure of a block-sparse tensor: leg names and catalogues in storage
// order, and its blocks. ``size`` is the number of elements of the buffer
// holding it (for bounds checks).
struct BT {
  std::vector<int> names;
  std::vector<LegP> cat;
  std::vector<Block> blocks;
  int64_t size = 0;
  int pos(int name) const {
    for (size_t i = 0; i < names.size(); ++i)
      if (names[i] == name) return (int)i;
    return -1;
  }
  int nlegs() const { return (int)names.size(); }
  int dim(const Block& b, int p) const { return cat[p]->dim[b.sect[p]]; }
  int64_t block_elems(const Block& b) const {
    int64_t n = 1;
    for (int p = 0; p < nlegs(); ++p) n *= dim(b, p);
    return n;
  }
};

// Row-major contiguous strides for a block of ``bt`` given its sectors.
void set_rowmajor(const BT& bt, Block& b);

// Measured tile choices (the autotuner's table): GEMM step signature ->
// tile (M, N), and the slice budget that was fastest for the tuned row.
struct TuneTable {
  std::unordered_map<uint64_t, std::array<int16_t, 2>> tiles;
  int64_t slice_budget = 0;   // bytes; 0: not tuned
};

struct SymInfo {
  int kind = SYM_NONE;
  bool fermionic = false;
  uint64_t coef_seed = 0;
  // GEMM tile selection: a tuned tile for the step's signature when the
  // table has one; else, with tile_rank >= 0, that candidate of the padding
  // model's ranking (autotuning runs); else the model's first choice
  const TuneTable* tune = nullptr;
  int tile_rank = -1;
};

// One block-pair product inside a GEMM job. Offsets are element offsets
// relative to the A / B buffers; t* are offsets into the table pool.
struct GemmPair {
  int64_t a_off;
  int64_t b_off;
  int32_t K;
  int32_t tam, tak, tbk, tbn;
  int32_t flags;   // bit0: A rows contiguous along K; bit1: B contiguous along N
  // > 0: that table is i * stride (a row-major run of its legs), so the
  // kernel computes the offset instead of reading it; 0: read the table
  int32_t sam, sak, sbk, sbn;
  double alpha;
};

struct GemmJob {
  int64_t c_off;
  int32_t M, N;
  int32_t m0, n0;
  int32_t tcm, tcn;
  int32_t p0, p1;   // pair range
  int32_t k0, k1;   // K range inside each pair (split-K), k1 = INT32_MAX for all
};

struct TablePool {
  std::vector<int32_t> data;
  std::unordered_map<std::string, int32_t> index;
  int32_t add(const std::vector<int32_t>& dims, const std::vector<int64_t>& strides, bool* ok);
  // a table given by its values
  int32_t add_raw(const std::vector<int32_t>& v, bool* ok);
};

// Sum of the split parts of one output block into C (table addressed).
struct ReduceTab {
  int64_t c_off, p_off;
  int32_t tcm, tcn;
  int32_t M, N, nsplit, pad;
};

struct GemmPlan {
  std::vector<GemmJob> jobs;
  std::vector<GemmPair> pairs;
  double flops = 0;        // 2 m n k over all pairs (algorithmic)
  int64_t a_extent = 0;    // largest element index + 1 read from A
  int64_t b_extent = 0;
  int64_t c_extent = 0;
  int mt = 64, nt = 64;    // tile used for the jobs
  // signature of the step's shape (step, operand roles, output block sizes
  // and contracted extents): the key of tuned tiles
  uint64_t sig = 0;
  double bytes = 0;        // algorithmic: distinct A, B blocks read once, C written once
  // split-K: when partial_size > 0 every job writes a row-major part of its
  // output block into a partial buffer of that many elements, and
  // ``reduces`` sums the parts into C (fixed order, deterministic)
  int64_t partial_size = 0;
  int64_t max_red_mn = 0;
  std::vector<ReduceTab> reduces;
};

// Tile shape choice for a list of output blocks: (M, N) sizes and the
// contracted extent summed over each block's pairs.
void choose_tile(const std::vector<std::pair<int64_t, int64_t>>& mn,
                 const std::vector<int64_t>& ktot, int* mt, int* nt);
// The tiles the autotuner tries, best first by the padding model: its first
// choice, then the other tiles within 30% of the best padding efficiency in
// order of efficiency (at most ``max_n``).
std::vector<std::array<int, 2>> tile_candidates(const std::vector<std::pair<int64_t, int64_t>>& mn,
                                                const std::vector<int64_t>& ktot, int max_n);
// Whether (mt, nt) is one of the GEMM kernel's tile shapes.
bool valid_tile(int mt, int nt);

// Per-pair scalar of a chain step: synthetic recoupling coefficient (SU(2))
// times the parity sign. ``xlabs`` are the labels of the sketch-side
// intermediate block in its canonical leg order, ``tlabs`` those of the step
// tensor block; ``xshared``/``tshared`` flag the contracted legs.
// ``nx`` and ``nt`` count the entries of the label and flag arrays.
double pair_alpha(const SymInfo& sym, int step, const int32_t* const* xlabs, int nx,
                  const int32_t* const* tlabs, int nt, const char* xshared, const char* tshared,
                  int nlab);

uint64_t splitmix64_mix(uint64_t z);

// One contraction step. X and S are contracted over their shared leg names.
// The output is created with leg storage order ``out_names`` (blocks sorted
// by sector tuple, contiguous row-major, starting at offset 0) unless
// ``fixed_out`` is given, in which case exactly those blocks are produced
// (blocks of fixed_out without contributions are written as zeros).
// ``m_is_x`` selects the operand whose free legs form the M index.
// ``key_side`` (0: X, 1: output) names the tensor whose block labels, in
// the canonical order ``key_order``, key the per-pair scalar.
struct StepSpec {
  int step = 0;                 // 1..5
  bool m_is_x = true;
  int key_side = 0;
  std::vector<int> out_names;
  std::vector<int> key_order;   // canonical leg order of the sketch-side intermediate
  bool symbolic = false;        // only produce the output block structure
  // with a fixed output layout: drop pairs whose output block lies outside it
  // (restriction of the product to the layout's blocks) instead of failing
  bool restrict_to_fixed = false;
};

struct StepResult {
  BT out;
  GemmPlan plan;
};

bool plan_step(const BT& X, const BT& S, const StepSpec& spec, const SymInfo& sym,
               TablePool& pool, const BT* fixed_out, StepResult& res, std::string& err);

// Row-thread form of a layer step (ket, PEPO or bra contracted into the
// sketch-side intermediate; contracted and free legs of the layer tensor are
// a few virtual/physical indices, the free legs of X span the environment
// and sketch indices). Rows of the product are grouped by the sectors of X's
// free legs; inside a group a row is addressed by its indices along up to
// RT_MAXLEV "levels" (runs of legs contiguous in both X and the output), so
// a row offset is a short dot product and no per-row tables exist. Each
// output block is cut into column chunks of nc <= RT_NC columns; the layer
// tensor's sub-block of every pair, scaled by the pair's scalar, is packed
// row-major [Kb][nc] once per plan. A workgroup takes ``rows`` consecutive
// rows of one group; when the group's distinct X blocks fit, their values for
// those rows are staged once in LDS (each X element leaves HBM once) and the
// four waves split the output chunks.
constexpr int RT_MAXLEV = 4;
constexpr int RT_NC = 16;
// Groups whose output needs four or more chunks (the four waves share the
// chunks of the tile) and whose 128 staged rows fit RT_PAIR_LDS take 128-row
// tiles with two rows per lane and chunks of at most RT_NC2 columns: each
// packed layer value loaded by a wave then feeds two products.
constexpr int RT_NC2 = 8;
constexpr int RT_PAIR_LDS = 32 * 1024;
constexpr int RT_THREADS = 256;
constexpr int RT_LDS_BYTES = 64 * 1024;   // staging budget per workgroup
constexpr int RT_NCLASS = 4;              // LDS classes: 0 (unstaged), <=16K, <=32K, <=64K

struct RtGroup {
  uint64_t mg[RT_MAXLEV];      // floor((2^64 - 1) / md) + 1: n / md = umulhi64(n, mg) for
                               // n < 2^31 (md = 1 levels are skipped)
  int32_t tile0;               // first workgroup of the group
  int32_t M;                   // rows
  int32_t md[RT_MAXLEV];       // level dims, innermost last (unused levels 1)
  int32_t o0, o1;              // output chunk range
  int32_t k0, k1;              // X block range (RtKblk)
  int32_t rows;                // rows per workgroup: 64, 128 or 256
  int32_t staged;              // 1: X rows staged in LDS (rows * ktot doubles); 2: also two
                               // rows per lane (rows = 128, chunks of <= RT_NC2 columns)
  int32_t ktot;                // sum of Kb over the group's X blocks
  int32_t c0;                  // first staged column (RtCol), ktot of them
};
// One staged column of a group: X element of row (level indices i) at
// xbase + sum_l i_l xs[l] (the X block base plus the column's contracted
// offset, and the block's level strides).
struct RtCol {
  int64_t xbase;
  int32_t xs[RT_MAXLEV];
};
struct RtOut {
  int64_t base;                // output block element offset
  int32_t ms[RT_MAXLEV];       // level strides in the output block
  int32_t nc;                  // columns of this chunk
  int32_t ntab;                // table of the nc column offsets
  int32_t p0, p1;              // pair range
};
// One X block of a group (contracted sector combination).
struct RtKblk {
  int64_t xbase;               // X block element offset
  int32_t xs[RT_MAXLEV];       // level strides in the X block
  int32_t Kb;
  int32_t xktab;               // table of the Kb contracted offsets in the X block
  int32_t koff;                // first staged column of this block in LDS
  int32_t pad;
};
struct RtPair {
  int64_t pk;                  // packed [Kb][nc] layer sub-block
  int32_t kblk;                // X block (RtKblk index)
  int32_t koff;                // its staged column offset
  int32_t Kb;
  int32_t pad;
};
struct RtPack {
  int64_t dst;                 // = RtPair::pk
  int64_t sbase;               // layer block element offset
  int32_t Kb, nc;
  int32_t sktab, sntab;        // layer block offsets along K (Kb) and N (chunk, nc)
  double alpha;
};
struct RtPlan {
  std::vector<RtGroup> groups;
  std::vector<RtOut> outs;
  std::vector<RtKblk> kblks;
  std::vector<RtCol> cols;
  std::vector<RtPair> pairs;
  std::vector<RtPack> packs;
  int64_t pack_size = 0;       // doubles
  int32_t ntiles = 0;
  int32_t lds_bytes = 0;       // largest staged group
  // groups are ordered by LDS class so that each class is one launch with
  // its own dynamic LDS size (a launch reserves its largest group's LDS for
  // every workgroup, which would cap the occupancy of small groups)
  int32_t nlaunch = 0;
  int32_t l_tile0[RT_NCLASS] = {0}, l_ntiles[RT_NCLASS] = {0}, l_lds[RT_NCLASS] = {0};
  double l_flops[RT_NCLASS] = {0}, l_bytes[RT_NCLASS] = {0};   // per launch
  double flops = 0;
  int64_t x_extent = 0, c_extent = 0, s_extent = 0;
  // algorithmic HBM bytes: every input element read once, every output
  // element written once; x_loads counts the element loads the rows issue
  double bytes = 0, x_loads = 0;
};

bool plan_step_rt(const BT& X, const BT& S, const StepSpec& spec, const SymInfo& sym,
                  TablePool& pool, StepResult& res, RtPlan& rt, std::string& err);

// Build the GEMM jobs of a plain dense product C = alpha op(A) op(B) where all
// three are strided matrices (used by the factorisation steps).
struct DenseOp {
  int64_t a_off, b_off, c_off;
  int32_t M, N, K;
  int64_t a_rs, a_cs;   // A(m, k) at a_off + m*a_rs + k*a_cs
  int64_t b_rs, b_cs;   // B(k, n) at b_off + k*b_rs + n*b_cs
  int64_t c_rs, c_cs;   // C(m, n) at c_off + m*c_rs + n*c_cs
  double alpha;
  int32_t ksplit = 0;   // > 1: this op's own K split (overrides the plan's)
};
// ``ksplit`` > 1 splits K into that many chunks written to consecutive
// partial matrices (c_off + chunk * M * N, row-major M x N) for a later sum.
bool plan_dense(const std::vector<DenseOp>& ops, TablePool& pool, int mt, int nt, int ksplit,
                GemmPlan& plan, std::string& err);

}  // namespace fp
