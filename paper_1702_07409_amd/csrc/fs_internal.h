// Internal declarations shared by the host runtime and the HIP kernels of libfs.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "fs_api.h"

// The opaque graph: host CSR/CSC plus one device allocation holding the same
// four arrays (int32).  Immutable after build.
struct fs_graph {
  uint32_t k = 0, n = 0;
  uint64_t nnz = 0;
  uint32_t max_deg = 0, max_cdeg = 0;
  fs_graph_params params{};
  std::vector<double> finite_w;  // owned copy of the finite table
  std::vector<int32_t> row_ptr, col, col_ptr, rowidx;
  // Encode segments: rows cut into runs of at most kSegMax edges, so that a
  // row of huge degree (the Robust Soliton tail) is spread over many
  // workgroups, ordered longest first.  seg_col[seg_ptr[s]..seg_ptr[s+1]) are
  // the edges of segment s, part of row seg_row[s]; seg_atomic[s] = 1 when
  // the row has several segments (combined by atomic XOR into a zeroed row);
  // heavy lists those rows once.
  std::vector<int32_t> seg_ptr, seg_row, seg_col, heavy;
  std::vector<uint8_t> seg_atomic;
  uint32_t nseg = 0;          // encode segments
  bool host_arrays = true;    // false: built on the device (the host vectors
                              // above are empty, except heavy)
  int device = -1;
  void *d_base = nullptr;
  bool pooled = false;        // d_base came from the graph memory pool
  const int32_t *d_row_ptr = nullptr, *d_col = nullptr, *d_col_ptr = nullptr,
                *d_rowidx = nullptr;
  const int32_t *d_seg_ptr = nullptr, *d_seg_row = nullptr, *d_seg_col = nullptr, *d_heavy = nullptr;
  const uint8_t *d_seg_atomic = nullptr;
};

// An array-LDPC precode (check #1, Algorithm 2) on the host and the device.
struct fs_precode {
  uint32_t b = 0, k = 0, p = 0, kp = 0, jp = 0, m = 0;   // m = k - b checks
  std::vector<int32_t> enc_ptr, enc_col;   // row r of L(1): the blocks whose XOR is parity b + r
  std::vector<int32_t> chk_ptr, chk_col;   // members of check r: its row and b + r
  std::vector<int32_t> sym_ptr, sym_chk;   // the checks of every block
  int device = -1;
  void *d_base = nullptr;
  const int32_t *d_enc_ptr = nullptr, *d_enc_col = nullptr, *d_chk_ptr = nullptr, *d_chk_col = nullptr,
                *d_sym_ptr = nullptr, *d_sym_chk = nullptr;
};

// Check #2 / check #3 equations of a graph (Algorithm 4) on the host and the
// device.
struct fs_checks {
  uint32_t k = 0, n = 0, sweeps = 0, zero_columns = 0, max_group = 0;
  std::vector<int32_t> grp_ptr, grp_col;          // check #3 groups, smallest first
  std::vector<int32_t> c2_input, c2_ptr, c2_col;  // check #2: input and its coded blocks
  std::vector<int32_t> sym_ptr, sym_grp;          // the groups of every coded block, in group order
  int device = -1;
  void *d_base = nullptr;
  const int32_t *d_grp_ptr = nullptr, *d_grp_col = nullptr, *d_sym_ptr = nullptr, *d_sym_grp = nullptr;
};

namespace fs {

constexpr uint32_t kSegMax = 64;

// thread-local error text; returns s for chaining
fs_status fail(fs_status s, const std::string &msg);
void clear_error();

// host graph construction (graph_host.cpp)
fs_status degree_weights(const fs_graph_params &p, std::vector<double> &w);
fs_status degree_thresholds(const std::vector<double> &w, std::vector<uint64_t> &T);
fs_status build_host_graph(const fs_graph_params &p, fs_graph &g);
// the same graph built by kernels on the current device (api.cpp, graph_dev.hip)
fs_status build_device_graph(const fs_graph_params &p, hipStream_t stream, fs_graph &g);

// device facts cached per device
struct DeviceInfo {
  int cu_count = 256;
  int max_lds_per_block = 65536;
};
const DeviceInfo &device_info(int dev);

// the process-wide tuning (fs_set_tune)
fs_tune tune_snapshot();

// shape of the last single-stripe gather and replay of this thread (fs_last_launch)
fs_launch_info &launch_record();

// workspace carving: aligned sub-buffers of one caller workspace
struct Carver {
  uint8_t *base;
  size_t off = 0;
  explicit Carver(void *b) : base(static_cast<uint8_t *>(b)) {}
  template <class T>
  T *take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  size_t size() const { return (off + 255) & ~size_t(255); }
};

// ---- kernel launchers (kernels.hip) ----

struct GatherJob {
  const uint8_t *src;      // source block b at src + b * src_stride
  uint64_t src_stride;
  uint8_t *dst;            // output block o at dst + o * dst_stride
  uint64_t dst_stride;
  const int32_t *ptr;      // sources of CSR row j: idx[ptr[j] .. ptr[j+1])
  const int32_t *idx;
  const uint32_t *csr_map; // CSR row of output item r (null: r)
  const int32_t *out_map;  // output block of item r (null: csr row)
  const uint8_t *row_ok;   // item r is zero-filled when row_ok[r] == 0 (null: all ok)
  const int32_t *nrows_dev;  // device item count (null: nrows)
  const int32_t *skip_flag;  // non-zero: the launch writes nothing
  const uint8_t *seg_atomic; // item r XORs atomically into its (zeroed) output when set
  uint32_t nrows;          // item count, or its upper bound with nrows_dev
  uint32_t csr_rows;       // CSR rows; items mapping beyond are skipped
  uint64_t t;              // bytes per block (multiple of 16)
  int accumulate;          // XOR into the existing output
  uint32_t slab_k;         // encode jobs: source blocks (k), for the LDS-slab
                           // kernel; 0 for every other job
};

fs_status launch_gather(const GatherJob &job, const fs_tune &tune, hipStream_t s);
// zero the listed blocks (dst + rows[i] * t)
fs_status launch_zero_rows(uint8_t *dst, const int32_t *rows, uint32_t nrows, uint64_t t, hipStream_t s);

struct PeelJob {
  uint32_t k, n;
  const int32_t *row_ptr, *col, *col_ptr, *rowidx;
  const uint8_t *erased;     // device uint8[n]
  uint32_t maxit;
  uint8_t *recovered;        // uint8[k]
  int32_t *status;           // int32[3]
  int32_t *level_ptr;        // int32[k+1]
  int32_t *dp_f, *dp_g;      // int32[k]
  // global-state workspace (used when the state does not fit in LDS)
  unsigned long long *acc, *best;
  int32_t *front_a, *front_b, *dlist;
  uint32_t *mask, *decmask;
  const int32_t *skip_flag;  // non-zero: write status only
  uint64_t nnz;              // edges (0: unknown; the compact all-LDS variant needs it)
  int32_t *status_out;       // int32[3] or null: a second copy of status (the caller's)
  uint32_t acc_ready;        // 1: acc holds the initial row states (count << 40 | id sum,
                             // erased rows flagged), made by the many-workgroup init kernels
};

size_t peel_ws_bytes(uint32_t k, uint32_t n);
void peel_carve(Carver &cv, PeelJob &j);
size_t peel_lds_bytes(uint32_t k, uint32_t n);
// max_deg selects the LDS variant (row degrees kept as 16-bit in LDS)
fs_status launch_peel(const PeelJob &job, hipStream_t s, uint32_t max_deg);

struct ReplayJob {
  uint32_t k, n;
  const int32_t *row_ptr, *col;
  const uint8_t *c;
  uint8_t *x;
  uint64_t t;
  const int32_t *status, *level_ptr, *dp_f, *dp_g;
  const int32_t *skip_flag;  // non-zero: the launch writes nothing
};
// Replay program built from a schedule (workspace arrays).
struct ProgJob {
  uint32_t k, n;
  const int32_t *row_ptr, *col;
  const int32_t *status, *level_ptr, *dp_f, *dp_g;
  int32_t *gsrc;       // int32[k]
  int32_t *finv;       // int32[n]: input decoded by row g, or -1
  int32_t *gl, *fl;    // int32[k]: decoding rows ascending, and their inputs
  int32_t *poff;       // int32[k+1]
  int32_t *pidx;       // int32[pidx_cap]
  int32_t *meta;       // int32[4]
  uint32_t *psums;     // block sums of the many-workgroup build (scans over k pairs and n rows)
  uint32_t pidx_cap;
  const int32_t *skip_flag;
  // dependency-slab form of the program (graphs with k, n <= 65535): per
  // input 2 + its slab slot when some pair reads it (la_slot); per pair a
  // prefix count (la_pre) and a record {f, g, entries offset, 1 + slot of f}
  // (la_pair); la_idx holds the slots of each pair's other inputs; la_meta =
  // {usable, slots, largest level}
  int32_t *la_slot, *la_pre, *la_idx, *la_meta;
  int32_t *la_pair;    // int32[4 k]
};
void prog_carve(Carver &cv, ProgJob &p, uint64_t nnz);
// whether launch_prog also builds the lookahead form for this graph
bool prog_has_lookahead(const ProgJob &p);
fs_status launch_prog_lookahead(const ProgJob &prog, hipStream_t s);

// prog: workspace for the replay program (null: global-memory replay only).
// launch_replay builds the program then replays; launch_prog and
// launch_replay_prog are the two halves.
fs_status launch_replay(const ReplayJob &job, const ProgJob *prog, hipStream_t s);
fs_status launch_prog(const ProgJob &prog, hipStream_t s);
fs_status launch_replay_prog(const ReplayJob &job, const ProgJob *prog, hipStream_t s);
// the peel and the replay program in one launch (one workgroup): a decode plan
fs_status launch_plan(const PeelJob &job, const ProgJob &prog, hipStream_t s, uint32_t max_deg);

// lost-row validation / masks for repair
struct RepairPrepJob {
  uint32_t n, k;
  const uint32_t *lost;
  uint32_t n_lost;
  const uint8_t *erased;   // may be null
  uint8_t *erased2;        // may be null (mode A): erased | lost
  uint32_t *seen;          // uint32[ceil(n/32)] scratch
  int32_t *flag;           // out: 0 ok, FS_ERR_INVALID bad ids
  uint8_t *repaired;       // out: default value
  int32_t *status;         // out
  // Repair from inputs: the lost rows' edges copied into one compact CSR of
  // pieces of at most 64 edges for the gather (sptr null: not made).  Rows
  // of several pieces are zeroed here; their pieces XOR into them
  // atomically.
  const int32_t *row_ptr, *col;
  int32_t *sptr;           // [seg_cap + 1]: first edge of each piece in sidx
  int32_t *sidx;           // [nnz]: the lost rows' edges, row after row
  int32_t *roff;           // [n]: first edge of each lost row in sidx
  int32_t *sout;           // [seg_cap]: row of each piece
  uint8_t *satomic;        // [seg_cap]: 1 when the row has several pieces
  int32_t *nseg;           // out: pieces
  uint32_t seg_cap;
  uint8_t *c;              // coded blocks (rows of several pieces zeroed)
  uint64_t t;
};
fs_status launch_repair_prep(const RepairPrepJob &job, hipStream_t s);
struct RepairBufs;
struct GatherJob;
// A repair from inputs: the prep job's piece fields, and the gather over the
// pieces (rows of more than 64 edges no longer hold one workgroup per slice
// for their whole length).
void repair_pieces_prep(RepairPrepJob &pj, const struct fs_graph *g, const RepairBufs &b, void *c, uint64_t t);
GatherJob repair_pieces_job(const struct fs_graph *g, const RepairBufs &b, uint32_t n_lost, const void *x, void *c,
                            uint64_t t);

// Lost-row list and erasure vector of a code extension: ids[i] = n_old + i
// for i < n - n_old; erased_full (if non-null) = erased on [0, n_old), 0 above.
struct ExtendPrepJob {
  uint32_t n, n_old;
  const uint8_t *erased;   // may be null: nothing erased
  uint32_t *ids;           // uint32[n - n_old]
  uint8_t *erased_full;    // uint8[n], may be null
};
fs_status launch_extend_prep(const ExtendPrepJob &job, hipStream_t s);

// Disk-failure sweep (simdisk.hip).  Per-combination state lives in LDS
// (byte counts + 16-bit index XORs, or one word a row) when it fits, else in
// kSimDiskSlots per-workgroup slots of the workspace.
enum { kSimDiskByte = 0, kSimDiskXor16 = 1, kSimDiskGlobal = 2 };
constexpr uint32_t kSimDiskSlots = 256;
struct SimDiskLayout {
  int mode;
  size_t image_bytes;                 // per-row state image (rowinfo and the copy in LDS / a slot)
  size_t off_w, off_dec, off_fresh, off_chk;   // byte offsets in LDS or in one slot
  size_t bytes;                       // LDS bytes, or bytes of one slot
};
SimDiskLayout simdisk_layout(uint32_t k, uint32_t n, uint32_t max_deg, uint32_t checks, size_t max_lds);
struct SimDiskJob {
  uint32_t k, n, s, f, maxit;
  uint64_t first, count;
  const int32_t *row_ptr, *col, *col_ptr, *rowidx;
  uint64_t *binom;      // uint64[65 * 65], C(a, b) at a * 65 + b (written by the setup)
  uint32_t *rowinfo;    // the initial per-row state image (written by the setup)
  uint8_t *slots;       // global mode: kSimDiskSlots slots of slot_bytes
  size_t slot_bytes, off_w, off_dec, off_fresh, off_chk;
  uint32_t pc_b, pc_m;  // precode: data blocks and checks (pc_m = 0: none)
  const int32_t *chk_ptr, *chk_col, *sym_ptr, *sym_chk;   // precode check sets
  int32_t *result;      // int32[count][3], or [count][4] with a precode
};
fs_status launch_simdisk(const SimDiskJob &job, const SimDiskLayout &layout, hipStream_t s);

// Precode (precode.hip): host construction of the checks and the second BP
// pass of the two-stage decode.
uint32_t largest_prime_factor(uint32_t k);
fs_status build_precode_host(uint32_t b, uint32_t k, fs_precode &pc);
size_t precode_peel_lds(uint32_t k, uint32_t m);
struct PrecodePeelJob {
  uint32_t b, k, m;
  const int32_t *chk_ptr, *chk_col, *sym_ptr, *sym_chk;
  uint8_t *recovered;        // uint8[k]: in, the LDGM pass; out, both passes
  const int32_t *status1;    // int32[3] of the LDGM pass
  int32_t *status;           // int32[4] out
  int32_t *pair_sym, *pair_chk;   // int32[k]: (block, check) in level order
  int32_t *level_ptr;        // int32[k + 1]
  int32_t *meta;             // int32[2]: levels, pairs
};
fs_status launch_precode_peel(const PrecodePeelJob &job, hipStream_t s);
struct PrecodeReplayJob {
  uint8_t *x;
  uint64_t t;
  const int32_t *chk_ptr, *chk_col, *pair_sym, *pair_chk, *level_ptr, *meta;
};
fs_status launch_precode_replay(const PrecodeReplayJob &job, hipStream_t s);
// after a two-stage decode: mark the parity blocks known when every data
// block came back, else set skip[0] (also when bad[0] is set)
fs_status launch_parity_known(const int32_t *status, uint8_t *recovered, uint32_t b, uint32_t k, const int32_t *bad,
                              int32_t *skip, hipStream_t s);

// Check generation and local repair (checks.hip).
struct CgaJob {
  uint32_t k, n, kw, nw;     // 32-bit words per B column (k bits) and per L column (n bits)
  uint32_t max_sweeps;       // 0: until converged or unchanged
  uint32_t max_w;            // largest column weight of B (its largest row degree)
  const int32_t *row_ptr, *col, *col_ptr, *rowidx;
  uint32_t *bcol;            // [n][kw]
  uint32_t *lcol;            // [n][nw]
  uint32_t *rrow;            // [k][nw] rows of B: the columns holding each input
  uint32_t *w;               // [n] column weights of B
  int32_t *meta;             // [2] sweeps, zero columns
};
fs_status run_cga(const CgaJob &job, hipStream_t s);
struct LocalPlanJob {
  uint32_t n, n_lost;
  const uint32_t *lost;
  const uint8_t *erased;     // may be null
  const int32_t *grp_ptr, *grp_col, *sym_ptr, *sym_grp;
  int32_t *chosen;           // ws: [n_lost] group per lost block, -1 none
  int32_t *level;            // ws: [n_lost] BP level that rebuilds it, -1 none
  int32_t *pos;              // ws: [n_lost] its place in level order
  // ws: items in level order (unrebuilt blocks last, with no sources): the
  // blocks item p is the XOR of, item_col[item_ptr[p] .. item_ptr[p+1]),
  // its destination item_dst[p]; items of level l at [lvl_ptr[l], lvl_ptr[l+1])
  int32_t *item_ptr, *item_col, *item_dst, *lvl_ptr;
  int32_t *meta;             // ws: [4] {levels}
  int32_t *flag;             // ws: non-zero = bad ids, nothing written
  uint8_t *repaired;         // out [n_lost]
  int32_t *status;           // out [3]
  // group peel state: per group (unknown members << 40 | sum of their ids),
  // per block its lost index (-1) and smallest usable group, two frontiers of
  // (group, unknown block) pairs
  uint32_t n_groups;
  unsigned long long *gacc;  // ws: [2n]
  int32_t *rof, *best;       // ws: [n] each
  int32_t *fa, *fb;          // ws: [2 * 2n] each
  uint32_t *unk;             // ws: [ceil(n / 32)] unknown blocks (bitset)
};
fs_status launch_local_plan(const LocalPlanJob &job, hipStream_t s);
// the rebuild of the lost blocks in c, level by level, from a local plan
fs_status launch_local_apply(const LocalPlanJob &plan, uint8_t *c, uint64_t t, hipStream_t s);
// the largest n local repair plans for (its unknown-block bitset sits in LDS)
constexpr uint32_t kLocalMaxN = 524288;

struct RepairCheckJob {
  const int32_t *row_ptr, *col;
  uint32_t n;
  const uint32_t *lost;
  uint32_t n_lost;
  const uint8_t *recovered;   // from the conventional decode
  const int32_t *flag;
  uint8_t *repaired;
  int32_t *status;
};
fs_status launch_repair_check(const RepairCheckJob &job, hipStream_t s);

struct UpdatePlanJob {
  uint32_t k, n;
  const int32_t *col_ptr, *rowidx;
  const uint32_t *ids;
  uint32_t n_ids;
  uint32_t *seen;      // uint32[ceil(k/32)]
  int32_t *cnt;        // int32[n]
  int32_t *arow;       // int32[n]
  int32_t *aptr;       // int32[n+1]
  int32_t *asrc;       // int32[max pairs]
  int32_t *n_aff;      // int32[1]
  int32_t *flag;       // int32[1]
  int32_t *status;     // int32[3]
};
fs_status launch_update_plan(const UpdatePlanJob &job, hipStream_t s);

struct UpdateDeltaJob {
  uint8_t *x;
  const uint8_t *new_blocks;
  uint8_t *delta;
  const uint32_t *ids;
  uint32_t n_ids;
  uint64_t t;
  const int32_t *flag;
};
fs_status launch_update_delta(const UpdateDeltaJob &job, hipStream_t s);

// ---- batched launches (one launch for many stripes) ----
// the batched gather's per-XCD work counters lie kCounterStride words apart
constexpr uint32_t kCounterStride = 32;

struct ZeroEntry {
  uint8_t *base;
  uint64_t t;
  int64_t row;
};
// device arrays of job descriptors; see kernels.hip for the item spaces
// d_counter: a device word the launch resets and then uses to hand out items
fs_status launch_gather_batch(const GatherJob *d_jobs, unsigned long long *d_prefix, uint32_t njobs,
                              unsigned long long *d_counter, const fs_tune &tune, uint32_t grid,
                              uint64_t total_items, hipStream_t s);
// mode: where the peel keeps its state (peel_mode); lds_bytes: dynamic LDS
fs_status launch_peel_batch(const PeelJob *d_jobs, uint32_t njobs, int mode, size_t lds_bytes, hipStream_t s);
// 2: all of the peel's state fits LDS, 1: its per-row counters do, 0: none
int peel_mode(uint32_t k, uint32_t n, uint32_t max_deg);
fs_status launch_prog_batch(const ProgJob *d_jobs, uint32_t njobs, hipStream_t s);
// prog_lds: dynamic LDS of each workgroup, enough for the 16-bit program of
// the largest item (replay_prog_lds_bound); items whose program does not fit
// read it from global memory
fs_status launch_replay_batch(const ReplayJob *d_rj, const ProgJob *d_pj, const uint32_t *d_wg_prefix,
                              uint32_t nitems, uint32_t total_wg, size_t prog_lds, hipStream_t s);
// largest LDS size of the 16-bit replay program of a graph with k inputs and
// pidx_cap program entries
size_t replay_prog_lds_bound(uint32_t k, uint32_t pidx_cap);
fs_status launch_repair_prep_batch(const RepairPrepJob *d_jobs, uint32_t njobs, hipStream_t s);
fs_status launch_update_plan_batch(const UpdatePlanJob *d_jobs, uint32_t njobs, hipStream_t s);
fs_status launch_update_delta_batch(const UpdateDeltaJob *d_jobs, const uint32_t *d_prefix, uint32_t njobs,
                                    uint32_t total_wg, hipStream_t s);
fs_status launch_zero_batch(const ZeroEntry *d_rows, uint32_t nrows, uint64_t max_t, hipStream_t s);
// set the LDS limits of the batched kernels (before a graph capture)
void prepare_batch_kernels();
// batch replay geometry: 16-byte lanes per symbol (W = 16 LPS) and slices per workgroup
constexpr uint32_t kBatchReplayLanes = 16;
constexpr uint32_t kBatchReplaySlicesPerWg = 8;
constexpr uint32_t kDeltaBytesPerWg = 4096;

// ---- workspace layouts and argument checks shared by the entry points ----

// Schedule arrays kept in a decode workspace.
struct SchedBufs {
  int32_t *status, *level_ptr, *dp_f, *dp_g;
  uint8_t *recovered;
};
// Decode workspace: schedule arrays, peel state, replay program.
struct DecodeBufs {
  SchedBufs sched;
  PeelJob peel;
  ProgJob prog;
};
struct RepairBufs {
  uint32_t *seen;
  int32_t *flag;
  // repair from inputs: the pieces of the lost rows (RepairPrepJob)
  int32_t *sptr, *sidx, *roff, *sout, *nseg;
  uint8_t *satomic;
  uint32_t seg_cap;
  uint8_t *erased2;
  SchedBufs sched;
  PeelJob peel;
  ProgJob prog;
  uint8_t *x;
};
struct UpdateBufs {
  uint32_t *seen;
  int32_t *cnt, *arow, *aptr, *asrc, *n_aff, *flag;
  uint8_t *delta;
  uint32_t max_rows;
};

// Device copy of a graph: its nine arrays, 256-byte aligned, in one buffer.
struct GraphImage {
  struct Part {
    const void *src;
    size_t bytes;
    size_t off;
  } parts[9];
  size_t total;
};
void graph_image(const fs_graph &g, GraphImage &img);
// the same layout from the array sizes alone (no host sources)
void graph_image_sized(uint32_t k, uint32_t n, uint64_t nnz, uint32_t nseg, uint32_t nheavy, GraphImage &img);

// ---- device graph construction (graph_dev.hip) ----
enum {
  kScalarMaxDeg = 0,
  kScalarSegs = 1,
  kScalarHeavy = 2,
  kScalarMaxCdeg = 3,
  kScalarMidCols = 4,    // columns of 65 .. 1024 rows
  kScalarLongCols = 5,   // longer columns
  kScalarCount = 6,
  kScalarWords = 8       // the scalars, then the 64-bit edge count
};
struct DevGraphJob {
  uint32_t k, n, D;
  uint32_t nnz;            // known once the degrees are
  uint64_t seed, stripe_key;
  // scratch
  const uint64_t *T;       // degree thresholds (D)
  int32_t *deg;            // degree of each row (n)
  uint32_t *blk_hist;      // per block of rows: segment bucket counts, then offsets
  uint32_t *blk_max, *blk_sum;   // per block of rows: largest degree, degree sum
  int32_t *bucket;         // per segment bucket: first segment, then first edge
  int32_t *scalars;        // kScalar*, the edge count, then the heavy rows
  unsigned long long *edges;   // sum of the degrees (nnz) in 64 bits
  uint32_t *sums;          // scan block sums
  int32_t *ccnt, *cfill;   // column counts and fill cursors (k)
  int32_t *seg_len, *seg_beg;   // per segment: edges and first edge (nseg)
  int32_t *unsorted;       // each column's rows before its sort (nnz)
  int32_t *col_list;       // columns of more than 64 rows (k)
  const int32_t *row_src;  // row_ptr as the degree pass left it (n + 1)
  // the graph image
  int32_t *row_ptr, *col, *col_ptr, *rowidx, *seg_ptr, *seg_row, *heavy, *seg_col;
  uint8_t *seg_atomic;
};
// scratch before the sizes are known: deg, a row_ptr copy, block
// histograms and totals, bucket starts, scalars (with room for n heavy rows)
// and scan sums for n and k elements (T is set apart)
void dev_graph_carve(Carver &cv, DevGraphJob &J, uint32_t k, uint32_t n);
// scratch once the sizes are known: seg_len, seg_beg, the unsorted columns,
// the long-column list and scan sums for max(n, k) elements
void dev_graph_carve_rows(Carver &cv, DevGraphJob &J, uint32_t k, uint32_t n, uint32_t nseg, uint64_t nnz);
// degrees, row_ptr, segment and heavy-row counts (scalars)
fs_status launch_dev_graph_degrees(const DevGraphJob &J, hipStream_t s);
// neighbours, segments, heavy rows and the transpose (scalars: max_cdeg)
fs_status launch_dev_graph_rows(const DevGraphJob &J, uint32_t nseg, uint32_t nheavy, hipStream_t s);
void bind_image(fs_graph &g, const GraphImage &img, void *base);

fs_tune current_tune();
// the tuning with its gather tiling filled in for graph g when left open
fs_tune tile_for(const fs_tune &t, const fs_graph *g);
fs_status check_graph(const fs_graph *g);
fs_status check_payload(const void *p, uint64_t t, const char *name);
void carve_sched(Carver &cv, uint32_t k, SchedBufs &s, bool with_recovered);
void carve_repair(Carver &cv, const fs_graph *g, uint64_t t, bool conventional, RepairBufs &b);
void carve_update(Carver &cv, const fs_graph *g, uint64_t t, uint32_t n_ids, UpdateBufs &b);
void carve_decode(Carver &cv, const fs_graph *g, DecodeBufs &b);
PeelJob peel_job(const fs_graph *g, const uint8_t *erased, uint32_t maxit, uint8_t *recovered, int32_t *status,
                 int32_t *level_ptr, int32_t *dp_f, int32_t *dp_g);
ProgJob prog_job(const fs_graph *g, Carver &cv, const int32_t *status, const int32_t *level_ptr,
                 const int32_t *dp_f, const int32_t *dp_g);
ReplayJob replay_job(const fs_graph *g, const void *c, void *x, uint64_t t, const int32_t *status,
                     const int32_t *level_ptr, const int32_t *dp_f, const int32_t *dp_g);
// the graph's encode as one gather job (segments of long rows combine atomically)
GatherJob encode_job(const fs_graph *g, const void *x, void *c, uint64_t t);

}  // namespace fs
