/*
 * fs_api.h - C ABI of libfs: the data-parallel XOR path of an LDGM fountain
 * erasure code (Founsure 1.0, Arslan, SoftwareX) on one AMD MI355X (gfx950).
 *
 * The code: k input blocks x_0..x_{k-1} and n coded blocks c_0..c_{n-1}, all
 * of t bytes.  Coded block g is the region XOR of the d_g input blocks in its
 * neighbour set N(g) (paper §2.2); d_g is drawn from a degree distribution
 * (Robust Soliton, or any finite max-degree table such as the Raptor Omega of
 * §2.2) and N(g) is drawn uniformly without replacement.  Everything follows
 * from (k, n, distribution, seed, stripe key), so a graph is regenerable
 * (§2.2, per-object seed).  The generator matrix B in F_2^{k x n} of
 * Algorithms 1 and 5 has column g = indicator of N(g).
 *
 * Conventions shared by every call
 *  - Payload, mask, id, flag, schedule and workspace pointers are DEVICE
 *    pointers owned by the caller; the library never allocates on a payload
 *    call.  Payloads are block-major: block b of a stripe starts at
 *    base + b * t.  t must be a positive multiple of 16 and every payload base
 *    16-byte aligned, else FS_ERR_ALIGN.
 *  - Calls are asynchronous on the given HIP stream (0 = the null stream);
 *    results land in device memory.  Argument errors found on the host are
 *    returned before anything is enqueued; out-parameters are then untouched.
 *  - Data-dependent outcomes (decode failure, a row that cannot be repaired,
 *    a bad id inside a device array) are RESULTS written to device status
 *    arrays, never host error codes.
 *  - Graphs are immutable after fs_graph_build and may be used concurrently
 *    from several streams.  Calls that share a workspace must not overlap.
 *  - Arithmetic is bytewise XOR (GF(2)): results are exact and deterministic.
 */
#ifndef FS_API_H
#define FS_API_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FS_API __attribute__((visibility("default")))

typedef enum fs_status {
  FS_OK = 0,
  FS_ERR_INVALID = 1,     /* a parameter is out of range or inconsistent    */
  FS_ERR_ALIGN = 2,       /* t % 16 != 0 or a payload base not 16-B aligned */
  FS_ERR_NOMEM = 3,       /* host or device allocation failed (build/plan)  */
  FS_ERR_HIP = 4,         /* a HIP runtime call failed; see fs_last_error   */
  FS_ERR_UNSUPPORTED = 5, /* valid request the library does not handle       */
  FS_ERR_WORKSPACE = 6    /* workspace pointer null or smaller than needed  */
} fs_status;

/* Degree distributions (paper §1 and §2.2). */
enum {
  FS_DIST_RSD = 0,     /* Robust Soliton (Luby): R = c ln(k/delta) sqrt(k),
                          spike at M = clamp(floor(k/R), 1, k); needs c > 0,
                          0 < delta < 1 and R/delta > 1                         */
  FS_DIST_FINITE = 1,  /* finite table: weights w_1..w_dmax >= 0, normalised;
                          degrees above k are dropped                          */
  FS_DIST_RAPTOR = 2   /* the Raptor Omega printed in §2.2 (finite, max 65)    */
};

/* Default object seed quoted in the paper (§2.2, footnote on the seed). */
#define FS_DEFAULT_SEED 1389488782ULL

/* fs_graph_params.flags */
enum {
  FS_GRAPH_HOST_ONLY = 1,  /* build the host arrays only (no device copy, no
                              HIP call): for fs_graph_export on any machine  */
  FS_GRAPH_ON_DEVICE = 2   /* build the graph with kernels on the current
                              device (the same arrays, element for element);
                              the host keeps no copy of the CSR/CSC          */
};

typedef struct fs_graph_params {
  uint32_t k;              /* input blocks, >= 1                               */
  uint32_t n;              /* coded blocks, >= 1                               */
  uint32_t dist;           /* FS_DIST_*                                        */
  uint32_t finite_dmax;    /* FS_DIST_FINITE: length of finite_w (>= 1)        */
  double rsd_c;            /* FS_DIST_RSD: c                                   */
  double rsd_delta;        /* FS_DIST_RSD: delta                               */
  const double *finite_w;  /* FS_DIST_FINITE: host array w_1..w_dmax           */
  uint64_t seed;           /* object seed                                      */
  uint64_t stripe_key;     /* per-stripe key (0: one graph shared per object)  */
  uint32_t flags;          /* FS_GRAPH_*                                       */
  uint32_t reserved;       /* must be 0                                        */
} fs_graph_params;

typedef struct fs_graph fs_graph;   /* opaque; owns host + device CSR and CSC */
typedef struct fs_precode fs_precode;   /* opaque; owns host + device check sets */
typedef struct fs_checks fs_checks;     /* opaque; check #2 / #3 equations of a graph */

/*
 * Degree table: the integer inverse-CDF thresholds used
 * to draw a coded row's degree.  Weights are summed in float64 in order
 * d = 1..D into W, p_d = w_d / W, C_d is the running sum and
 * T_d = min(2^53, floor(C_d 2^53)) for d < D, T_D = 2^53.  A 64-bit draw u
 * gives d = min{d : (u >> 11) < T_d}.  Host-only; writes D to *D_out and, if
 * T_out is non-null and cap >= D, T_1..T_D to T_out[0..D-1].
 * Errors: FS_ERR_INVALID for bad parameters or cap < D with T_out non-null.
 */
FS_API fs_status fs_degree_table(const fs_graph_params *params, uint64_t *T_out, uint32_t cap,
                          uint32_t *D_out);

/*
 * Build the seeded graph (§2.2 encoding step 2, "pseudo-randomly
 * selected" neighbours).  Row j uses the stream
 *   key = mix(mix(mix(mix(seed + G) ^ 1) ^ stripe_key) ^ j)
 *   draw i = mix(key + (i + 1) G)  (mix: SplitMix64's output function,
 *   G = 0x9E3779B97F4A7C15),
 * draw 0 picks d_j by the degree table, draws 1..d_j drive Floyd's sampler
 * (value r = k - d_j + s, v = ((draw >> 32) (r + 1)) >> 32; r if v is taken),
 * and the row is sorted ascending.  Rows do not depend on n.
 * Unless FS_GRAPH_HOST_ONLY, the CSR/CSC are copied to the current device on
 * `stream` and the call returns after the copy has completed.
 * With FS_GRAPH_ON_DEVICE the rows are drawn by kernels on `stream` instead
 * (16 lanes per row of at most 16 neighbours, a wave per row of up to 64, a
 * workgroup per longer row), the transpose and the encode segments likewise;
 * the call synchronises the stream twice (for the sizes, then the heavy-row
 * list) and returns with the graph complete.  The degree thresholds of the
 * last distribution built on a thread stay on the device for its next build.
 * Its scratch memory is kept per calling thread and device
 * (grown, never freed, so that builds beside other work do not wait for the
 * device); builds on different threads and streams run concurrently.  The
 * graph's device memory comes from a memory pool per device that keeps
 * freed memory for later builds (hipMalloc when no pool can be made).
 * fs_graph_export then copies from the device, and fs_graph_image_size /
 * fs_graph_upload do not apply.
 * *out receives the graph (freed with fs_graph_free).
 * Errors: FS_ERR_INVALID (parameters, unknown or conflicting flags,
 * nnz >= 2^31), FS_ERR_NOMEM, FS_ERR_HIP.
 */
FS_API fs_status fs_graph_build(const fs_graph_params *params, hipStream_t stream, fs_graph **out);

/* Sizes of a built graph (any out pointer may be null). */
FS_API fs_status fs_graph_info(const fs_graph *g, uint32_t *k, uint32_t *n, uint64_t *nnz,
                        uint32_t *max_degree, uint32_t *max_column_degree);

/*
 * Copy the graph to caller HOST arrays (any may be null): row_ptr[n+1] and
 * col[nnz] (CSR by coded row, ascending within a row), col_ptr[k+1] and
 * rowidx[nnz] (CSC by input, rows ascending within a column).
 */
FS_API fs_status fs_graph_export(const fs_graph *g, int32_t *row_ptr, int32_t *col,
                          int32_t *col_ptr, int32_t *rowidx);

/* Release a graph and its device memory.  Like hipFree, it waits for all
 * work on the graph's device first. */
FS_API void fs_graph_free(fs_graph *g);

/*
 * Device copy of a graph in caller memory, for request loops that keep
 * graphs in memory they manage.  fs_graph_image_size gives the bytes of the
 * copy (CSR, CSC and the encode segments, each 256-byte aligned).
 * fs_graph_upload copies a graph built with FS_GRAPH_HOST_ONLY into dev_mem
 * (device memory, 256-byte aligned, at least the image size, owned by the
 * caller and kept while the graph is used) on `stream`, and makes the graph
 * usable on the current device.  host_stage is null (the call returns after
 * the copy has completed) or pinned host memory of at least the image size
 * that the caller leaves untouched until the stream has passed the copy (the
 * call then returns at once; work on other streams that uses the graph must
 * be ordered after the copy).  fs_graph_free never frees dev_mem.
 * Errors: FS_ERR_INVALID (null, or the graph already has a device copy),
 * FS_ERR_ALIGN, FS_ERR_WORKSPACE (dev_mem too small), FS_ERR_HIP.
 */
FS_API fs_status fs_graph_image_size(const fs_graph *g, size_t *bytes);
FS_API fs_status fs_graph_upload(fs_graph *g, void *dev_mem, size_t bytes, void *host_stage, hipStream_t stream);

/*
 * Encode (§2.2 encoding step 2): c_g = XOR_{i in N(g)} x_i for every
 * g in [0, n).  x: device uint8[k][t]; c: device uint8[n][t] (written, not
 * read).  x and c must not overlap.
 */
FS_API fs_status fs_encode(const fs_graph *g, const void *x, void *c, uint64_t t, hipStream_t stream);

/* Operations for fs_workspace_size. */
enum { FS_OP_ENCODE = 0, FS_OP_PEEL = 1, FS_OP_DECODE = 2, FS_OP_REPAIR = 3,
       FS_OP_REPAIR_CONVENTIONAL = 4, FS_OP_UPDATE = 5, FS_OP_REPLAY = 6, FS_OP_EXTEND = 7,
       FS_OP_EXTEND_CONVENTIONAL = 8, FS_OP_SIM_DISKS = 9, FS_OP_DECODE_PRECODED = 10,
       FS_OP_REPAIR_LOCAL = 11, FS_OP_REPAIR_PRECODED = 12, FS_OP_EXTEND_LOCAL = 13 };

/*
 * Workspace bytes the operation needs for this graph and block size
 * (n_items: lost rows for repair, updated ids for update; ignored otherwise).
 */
FS_API fs_status fs_workspace_size(const fs_graph *g, int op, uint64_t t, uint32_t n_items,
                            size_t *bytes);

/*
 * Peeling schedule Algorithm 5 (DPG) with the level-synchronous
 * ("delayed") BP of §3.1.  With F the undecoded inputs (initially all k) and
 * S the coded rows with erased[g] == 0, each level:
 *   - every g in S with exactly one neighbour f(g) in F names f(g);
 *   - each named f is decoded by its namer of least (d_g, g), d_g the
 *     ORIGINAL degree, ties to the lower row index;
 *   - the decoded inputs leave F.
 * It stops when F is empty, no row names anything, or maxit levels ran
 * (maxit == 0: no limit).
 * Inputs : erased  device uint8[n] (non-zero = erased).
 * Outputs: recovered device uint8[k]  (1 = decoded);
 *          status    device int32[3]  {ok (F empty), |F|, levels L};
 *          level_ptr device int32[k+1] (entries 0..L valid, level_ptr[0] = 0);
 *          dp_f      device int32[k]: pairs of level l at [level_ptr[l],
 *                    level_ptr[l+1]) by ascending f, then F ascending;
 *          dp_g      device int32[k]: the decoding row of each pair, -1 for F.
 * ws: FS_OP_PEEL bytes of device workspace.
 */
FS_API fs_status fs_peel(const fs_graph *g, const uint8_t *erased, uint32_t maxit, uint8_t *recovered,
                  int32_t *status, int32_t *level_ptr, int32_t *dp_f, int32_t *dp_g, void *ws,
                  size_t ws_bytes, hipStream_t stream);

/*
 * Replay a schedule (§3.1): level by level,
 *   x_f = c_g XOR (XOR of x_i for i in N(g), i != f),
 * then x_f = 0 for every f left in F.  Reads c (device uint8[n][t]), writes
 * every block of x (device uint8[k][t]).  status/level_ptr/dp_f/dp_g are the
 * device outputs of fs_peel for the same graph.  ws: FS_OP_REPLAY bytes (the
 * schedule is flattened there into a replay program).  A schedule that does
 * not come from fs_peel never makes the call touch memory outside x, c and ws,
 * but the bytes it leaves in x are then unspecified.
 */
FS_API fs_status fs_replay(const fs_graph *g, const void *c, const int32_t *status,
                    const int32_t *level_ptr, const int32_t *dp_f, const int32_t *dp_g, void *x,
                    uint64_t t, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Decode (Algorithms 1/5, "founsureDec"): fs_peel into the
 * workspace then fs_replay.  A failed decode is a result: status[0] = 0,
 * recovered[] tells which blocks of x are valid, the others are zero.
 */
FS_API fs_status fs_decode(const fs_graph *g, const void *c, const uint8_t *erased, uint32_t maxit,
                    void *x, uint8_t *recovered, int32_t *status, uint64_t t, void *ws,
                    size_t ws_bytes, hipStream_t stream);

/*
 * fs_decode without a workspace argument, for callers that cannot allocate
 * memory (code under stream capture, tight request loops, harnesses that
 * forbid allocation calls): the workspace is a fixed 16 MiB device array
 * inside the library, one per GPU, held until the process ends.  The call
 * allocates nothing; arguments, outputs and results are those of fs_decode on
 * the current device (the graph must live there).  Every call on a GPU shares
 * that GPU's array: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller.
 * Errors: as fs_decode; FS_ERR_WORKSPACE when the graph's decode needs more
 * than 16 MiB of workspace (fs_workspace_size(FS_OP_DECODE); every graph with
 * k, n <= 65535 and Robust Soliton degrees fits), FS_ERR_INVALID when the
 * graph was built for another device.
 */
FS_API fs_status fs_decode_noalloc(const fs_graph *g, const void *c, const uint8_t *erased, uint32_t maxit,
                                   void *x, uint8_t *recovered, int32_t *status, uint64_t t,
                                   hipStream_t stream);

/*
 * Repair (the repair engine of §2.1 / §4).  lost: device uint32[n_lost]
 * coded rows to rebuild in place in c.
 *   x != NULL  re-encode from resident inputs: c_j = XOR_{i in N(j)} x_i.
 *   x == NULL  conventional repair (§4): peel + replay over the rows that are
 *              neither erased nor lost (into the workspace), then rebuild each
 *              lost row whose neighbours were all recovered; other lost rows
 *              are zero-filled.  erased: device uint8[n] (may be NULL = none).
 * repaired: device uint8[n_lost], 1 where c_j was rebuilt.
 * status: device int32[3] {all rebuilt, rows not rebuilt, 0 or an FS_ERR_*
 *         code for a bad lost id (>= n or repeated: nothing is written)}.
 */
FS_API fs_status fs_repair(const fs_graph *g, const void *x, void *c, const uint8_t *erased,
                    const uint32_t *lost, uint32_t n_lost, uint8_t *repaired, int32_t *status,
                    uint64_t t, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Update replace inputs ids[u] by new_blocks[u] and bring every
 * adjacent coded block up to date by adding the delta x_old ^ x_new (the
 * region XOR is linear, §2.2), i.e. the result equals re-encoding from
 * scratch.  ids: device uint32[n_ids], distinct, < k; new_blocks: device
 * uint8[n_ids][t].  x and c are updated in place.
 * status: device int32[3] {affected coded rows, pairs (row, id), 0 or
 *         FS_ERR_INVALID if an id is out of range or repeated, in which case
 *         nothing is written}.
 */
FS_API fs_status fs_update(const fs_graph *g, void *x, void *c, const uint32_t *ids, uint32_t n_ids,
                    const void *new_blocks, int32_t *status, uint64_t t, void *ws,
                    size_t ws_bytes, hipStream_t stream);

/*
 * Code extension, the paper's update (§2.9): the code is made
 * stronger by new coded blocks while no existing block changes.  g is the
 * graph of the longer code (n rows); since a row depends only on its own
 * index and the seeds, its first n_old rows are those of the original code.
 * c: device uint8[n][t]; rows [0, n_old) hold the existing blocks, rows
 * [n_old, n) are written and nothing else is.
 *   x != NULL  the new rows are encoded from the resident inputs.
 *   x == NULL  they are made the way the repair engine makes missing blocks:
 *              peel + replay over the existing rows that are not erased,
 *              then each new row whose neighbours were all recovered is
 *              encoded; other new rows are zero-filled.  erased: device
 *              uint8[n_old] (may be NULL = none).
 * made: device uint8[n - n_old], 1 where the new block was made.
 * status: device int32[3] {all made, rows not made, 0}.
 * ws: FS_OP_EXTEND (x given) or FS_OP_EXTEND_CONVENTIONAL bytes; neither
 * depends on n_old.  Making the code weaker (dropping coded rows) needs no
 * call: the shorter code is the prefix of rows it keeps.
 */
FS_API fs_status fs_extend(const fs_graph *g, uint32_t n_old, const void *x, void *c,
                    const uint8_t *erased, uint8_t *made, int32_t *status, uint64_t t,
                    void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Code extension through local groups, as §2.9 describes the update: the new
 * coded rows n_old..n-1 of the longer graph g are made from existing coded
 * blocks only, each as the XOR of the other members of a check #3 group of
 * the longer code, smallest groups first (fs_repair_local with the new rows
 * as the lost ones).  ch: the check #2/#3 equations of g (fs_checks_generate
 * on the longer graph, or its check data loaded).  erased: device uint8[n_old]
 * (the old rows that are unavailable) or NULL.  made: device
 * uint8[n - n_old]; status: device int32[3] as fs_repair_local's.  Rows no
 * local group reaches are left zero-filled (made 0) for fs_extend.
 * ws: FS_OP_EXTEND_LOCAL bytes with n_items = n - n_old.
 */
FS_API fs_status fs_extend_local(const fs_graph *g, const fs_checks *ch, uint32_t n_old, void *c,
                                 const uint8_t *erased, uint8_t *made, int32_t *status, uint64_t t,
                                 void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Disk-failure sweep, the simDisk utility (§2.1, §2.2): which combinations
 * of f failed disks out of s the code tolerates.  The n coded rows are
 * striped over the s disks equally and in order: disk d holds rows
 * [floor(d n / s), floor((d+1) n / s)).  The f-subsets of the disks are
 * ranked in lexicographic order of their sorted disk lists (rank 0 = disks
 * 0..f-1); for each rank r in [first, first + count) the rows of the failed
 * disks are erased and the peeling decode runs (maxit levels, 0 = no limit).
 * result: device int32[count][3]; entry r - first is the status triple that
 *   fs_peel gives for that erasure pattern: {ok (every input decoded),
 *   undecoded inputs, levels}.  No payload is read.
 * Requires 1 <= s <= min(64, n), f <= s and first + count <= C(s, f)
 * (FS_ERR_INVALID otherwise, nothing launched).
 * ws: FS_OP_SIM_DISKS bytes with n_items = 0 (a binomial table, the rows'
 *   initial state, and per-workgroup state when it does not fit in LDS); t
 *   is ignored for it.
 */
FS_API fs_status fs_sim_disks(const fs_graph *g, uint32_t s, uint32_t f, uint64_t first,
                       uint64_t count, uint32_t maxit, int32_t *result, void *ws,
                       size_t ws_bytes, hipStream_t stream);

/*
 * Array-LDPC precode, check #1 (§2.4, Algorithm 2).  A (b, k, n) code first
 * extends b data blocks to k with k - b parity blocks, then encodes the k
 * blocks with an LDGM graph of k inputs (§2.2).  With p the largest prime
 * factor of k, k' = k / p and j' = k' - b / p, b must be a multiple of p and
 * 1 <= j' < k' (FS_ERR_INVALID otherwise).  Row r of L(1) lists the k' - j'
 * blocks whose XOR is parity block b + r; they lie in the data or in earlier
 * block rows of p checks.  Check r is that row together with block b + r
 * (its members XOR to zero).
 * host_only != 0 builds the host tables only (for export; no device use).
 * Errors: FS_ERR_INVALID, FS_ERR_NOMEM, FS_ERR_HIP.
 */
FS_API fs_status fs_precode_build(uint32_t b, uint32_t k, int host_only, hipStream_t stream,
                           fs_precode **out);
FS_API fs_status fs_precode_info(const fs_precode *pc, uint32_t *b, uint32_t *k, uint32_t *p,
                          uint32_t *kp, uint32_t *jp);
/* L(1) on the host: row_ptr int32[k - b + 1], col int32[(k - b)(k' - j')],
 * each row ascending. */
FS_API fs_status fs_precode_export(const fs_precode *pc, int32_t *row_ptr, int32_t *col);
FS_API void fs_precode_free(fs_precode *pc);

/*
 * Precode encode: x device uint8[k][t] with the b data blocks in rows
 * 0..b-1; rows b..k-1 are written with the parity blocks, block row by block
 * row (j' launches).  Then fs_encode with the LDGM graph of k inputs makes
 * the coded blocks.
 */
FS_API fs_status fs_precode_encode(const fs_precode *pc, void *x, uint64_t t, hipStream_t stream);

/*
 * Two-stage decode (§2.2: BP at most twice, on the LDGM graph and then on
 * the precode).  The first pass is fs_decode into x (device uint8[k][t]) and
 * recovered (device uint8[k]).  If data blocks (rows < b) are still missing,
 * the second pass runs BP over the checks: at each level every check with
 * exactly one unknown member names it, and each named block becomes the XOR
 * of the other members of one of its naming checks; it ends when no check
 * names anything.  The second pass does not feed back into the first.
 * Blocks left unknown are zero, recovered[] marks the others.
 * status: device int32[4] {all b data blocks recovered, data blocks not
 *   recovered, levels of the first pass, levels of the second}.
 * g->k must equal the precode's k.  ws: FS_OP_DECODE_PRECODED bytes.
 * FS_ERR_UNSUPPORTED when the second pass's state (8 bytes per check plus a
 * bit per block) exceeds one workgroup's LDS.
 */
FS_API fs_status fs_decode_precoded(const fs_graph *g, const fs_precode *pc, const void *c,
                             const uint8_t *erased, uint32_t maxit, void *x, uint8_t *recovered,
                             int32_t *status, uint64_t t, void *ws, size_t ws_bytes,
                             hipStream_t stream);

/*
 * Conventional repair of a precoded code (§4: decode the entire data, then
 * re-run the encoding of the lost chunks): the two-stage decode of
 * fs_decode_precoded from the rows neither erased nor lost; if every data
 * block comes back, the parity blocks are encoded again from it, so every
 * input is known.  A lost row is rebuilt in c when all its inputs are known,
 * else zero-filled.  lost, repaired, status and the id checks are as in
 * fs_repair.  ws: FS_OP_REPAIR_PRECODED bytes.  g->k must equal pc's k.
 */
FS_API fs_status fs_repair_precoded(const fs_graph *g, const fs_precode *pc, void *c, const uint8_t *erased,
                                    const uint32_t *lost, uint32_t n_lost, uint8_t *repaired,
                                    int32_t *status, uint64_t t, void *ws, size_t ws_bytes,
                                    hipStream_t stream);

/*
 * Disk-failure sweep of a precoded code: as fs_sim_disks, with a
 * combination tolerable when the two-stage decode of fs_decode_precoded
 * recovers all b data blocks (maxit limits the first pass).  result: device
 * int32[count][4], each {ok, data blocks missing, levels of the first pass,
 * levels of the second}.  g->k must equal the precode's k.  ws:
 * FS_OP_SIM_DISKS bytes with n_items = k - b (the precode's checks).
 */
FS_API fs_status fs_sim_disks_precoded(const fs_graph *g, const fs_precode *pc, uint32_t s,
                                uint32_t f, uint64_t first, uint64_t count, uint32_t maxit,
                                int32_t *result, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Check #2 and check #3 generation (§2.6, Algorithm 4 "CGA"), on the device.
 * Columns of the generator matrix B (column j = the inputs of coded block j)
 * are XORed into each other while that lowers their weight: for j = 0..n-1
 * and i = 0..n-1 (i != j), if 2 w(b_j) > w(b_i) and w(b_j ^ b_i) < w(b_j)
 * then b_j ^= b_i and l_j ^= l_i, with L the n x n identity at the start.
 * Sweeps repeat until B has n - k zero columns, a sweep changes nothing, or
 * max_sweeps sweeps ran (0 = no limit).  Then a column of weight one is a
 * check #2 equation (its input = XOR of the coded blocks of l_j; the first
 * such column per input is kept) and a column of weight zero a check #3
 * group (its coded blocks XOR to zero), groups ordered by size, smallest
 * first, ties by column.  Runs on the stream, waits for it, and keeps the
 * groups on the host and the device.  Errors: FS_ERR_NOMEM, FS_ERR_HIP.
 */
FS_API fs_status fs_checks_generate(const fs_graph *g, uint32_t max_sweeps, hipStream_t stream,
                             fs_checks **out);
FS_API fs_status fs_checks_info(const fs_checks *ch, uint32_t *n_check2, uint32_t *n_check3,
                         uint32_t *sweeps, uint32_t *zero_columns, uint64_t *check2_entries,
                         uint64_t *check3_entries);
/* Host copies: check #3 groups c3_ptr int32[n_check3 + 1], c3_col
 * int32[check3_entries]; check #2 equations by ascending input, c2_input
 * int32[n_check2], c2_ptr int32[n_check2 + 1], c2_col int32[check2_entries].
 * Members ascending. */
FS_API fs_status fs_checks_export(const fs_checks *ch, int32_t *c3_ptr, int32_t *c3_col,
                           int32_t *c2_input, int32_t *c2_ptr, int32_t *c2_col);
FS_API void fs_checks_free(fs_checks *ch);

/*
 * The check data file (§2.7; read back as §2.8 describes): one integer array.  A check #2 equation is the
 * record 1, input, L, then the L coded blocks whose XOR is that input; a
 * check #3 group is the record 0, L, then its L coded blocks.
 *
 * fs_checks_serialize writes the check #2 records by ascending input, then
 * the check #3 groups in their stored order (smallest first), into out
 * (host int32[cap]); *len is the number of integers (with out == NULL only
 * *len is set).  FS_ERR_INVALID, nothing written, when cap is too small.
 *
 * fs_checks_load reads such an array (host int32[len]) for graph g: the
 * first check #2 record of each input is kept, the check #3 groups are
 * ordered by cardinality with ties in file order, as the repair engine sorts
 * them, and members become ascending sets.  The groups are uploaded on
 * stream (the call waits for the copy).  FS_ERR_INVALID for an unknown
 * flag, a record running past the end or an index out of range (input >= k,
 * coded block >= n).  The result serves fs_repair_local like a generated one.
 */
/*
 * More check #3 groups (§2.5), added to ch for graph g:
 *   (1) for each coded block j of degree one whose input i has a check #2
 *       set S_i, the group S_i xor {j} (c_j = x_i);
 *   (2) with pc non-null (the precode of g's inputs, pc's k = g's k), for each
 *       check #1 set D whose members all have check #2 sets, the symmetric
 *       difference of those sets (Eqs. (1)-(4)).
 * Empty groups and groups equal to one already held are skipped; all groups
 * are then ordered by cardinality, held ones first on ties.  added (may be
 * NULL): the number of groups added.  The device copies are replaced (the
 * call waits for the upload); on an error ch is left as it was.
 */
FS_API fs_status fs_checks_add_groups(fs_checks *ch, const fs_graph *g, const fs_precode *pc,
                                      hipStream_t stream, uint32_t *added);
FS_API fs_status fs_checks_serialize(const fs_checks *ch, int32_t *out, uint64_t cap, uint64_t *len);
FS_API fs_status fs_checks_load(const fs_graph *g, const int32_t *data, uint64_t len, hipStream_t stream,
                                fs_checks **out);

/*
 * Local-group repair, the repair engine's fast path (§2.3, §2.8, §4): BP
 * over the check #3 groups.  At each level every lost coded row s still
 * unknown is rebuilt in place in c as the XOR of the other members of the
 * first (smallest) group holding s whose other members are all known:
 * neither erased nor lost, or rebuilt at an earlier level.  The loop ends at
 * a level that rebuilds nothing; rows left unknown are zero-filled for
 * fs_repair.  lost: device uint32[n_lost]; erased: device uint8[n] or NULL.
 * repaired: device uint8[n_lost].  status: device int32[3] {all rebuilt,
 * rows not rebuilt, levels run}, or {0, n_lost, -FS_ERR_INVALID} for a bad
 * lost id (>= n or repeated; then nothing is written).  ws:
 * FS_OP_REPAIR_LOCAL bytes with n_items = n_lost.  FS_ERR_UNSUPPORTED for
 * codes of more than 524288 rows or checks with more than 2n groups.
 */
FS_API fs_status fs_repair_local(const fs_graph *g, const fs_checks *ch, void *c,
                          const uint8_t *erased, const uint32_t *lost, uint32_t n_lost,
                          uint8_t *repaired, int32_t *status, uint64_t t, void *ws,
                          size_t ws_bytes, hipStream_t stream);

/*
 * Decode in two halves.  fs_decode_plan runs the peeling schedule of fs_peel
 * for the erasure pattern and flattens it into a replay program, all inside
 * the workspace (FS_OP_DECODE bytes); it reads no payload.  recovered
 * (device uint8[k]) and status (device int32[3], may be NULL) are as in
 * fs_peel.  fs_decode_apply replays that plan on c into x (as fs_replay).  A
 * plan may be computed on one stream while the coded blocks are still being
 * written on another, and applied once both are done; a plan can be applied
 * to any number of stripes that share the graph and the erasure pattern.
 */
FS_API fs_status fs_decode_plan(const fs_graph *g, const uint8_t *erased, uint32_t maxit,
                                uint8_t *recovered, int32_t *status, void *ws, size_t ws_bytes,
                                hipStream_t stream);
FS_API fs_status fs_decode_apply(const fs_graph *g, const void *c, void *x, uint64_t t,
                                 const void *ws, size_t ws_bytes, hipStream_t stream);

/* Tuning of the gather-XOR kernel family (encode, repair, update). */
typedef struct fs_tune {
  uint32_t lanes_per_row;  /* 8, 16, 32, 64, 128 or 256 lanes share one coded
                              row (128 and 256: one or two rows per
                              workgroup, for jobs of few rows)               */
  uint32_t chunks;         /* 16-byte chunks per lane per slice: 1, 2 or 4
                              (1 or 2 with 128 and 256 lanes; both 0: chosen
                              per graph, see fs_set_tune)                    */
  uint32_t xcd_remap;      /* 1: keep each XCD on a contiguous slice range   */
  uint32_t nt_store;       /* 1: non-temporal stores for outputs             */
  uint32_t replay_prog_global; /* 1: keep decode replay programs in global
                                  memory instead of LDS (slower; for checks)  */
  uint32_t encode_slab;    /* 1: encode stripes with k <= 8192 whose block is
                              wide enough to fill the device from an LDS copy
                              of each byte slice of every input (below)       */
  uint32_t replay_lookahead; /* 1: decode replays of large k (k, n <= 65535)
                              keep every input a later pair reads in an LDS
                              slab and load the coded blocks eight levels
                              ahead; slices narrow to what the slab allows
                              (16-128 bytes).  Off by default: on the
                              k = 4096 x 64 KiB stripe it takes 0.38 ms
                              against 0.21 ms for the wide-slice replay    */
  uint32_t claim_chunk;    /* items a workgroup of the batched gather claims
                              from its XCD's counter at a time, 1..1024
                              (0: by the plan's item count and grid)        */
} fs_tune;

/*
 * Override (or with NULL restore) the gather tuning used by this process.
 * The default is {0, 0, 1, 1, 0, 1, 0, 0}: the gather slice is chosen per graph
 * (4 KiB for graphs of mean degree <= 6, which read each neighbour block in
 * long runs; for denser graphs 2 MiB / k within [512 B, 4 KiB], so that one
 * slice of every input stays in an XCD's L2), the LDS-slab encode where it
 * applies, and the wide-slice decode replay.
 */
FS_API fs_status fs_set_tune(const fs_tune *tune);
FS_API fs_status fs_get_tune(fs_tune *tune);

/*
 * Shape of the last single-stripe gather (fs_encode, fs_repair, fs_update,
 * fs_extend, the precode encode) and the last decode replay that the calling
 * thread launched, as chosen by the tuning and the per-graph rules above.
 * For tests and tuning tools; plans report their own choices through
 * fs_plan_get_info.  Fields are 0 until the first launch of that kind.
 */
typedef struct fs_launch_info {
  uint32_t gather_kind;          /* 1 gather kernel, 2 LDS-slab encode           */
  uint32_t gather_lanes_per_row; /* lanes per coded row (slab: lanes per slice) */
  uint32_t gather_chunks;        /* 16-byte chunks per lane (slab: 1)           */
  uint32_t gather_slice_bytes;   /* bytes of each block one item covers         */
  uint32_t replay_kind;          /* 1 LDS slab, 2 wide slices, 3 lookahead,
                                    4 no program (global-memory replay)          */
  uint32_t replay_slice_bytes;   /* bytes of each block one workgroup covers    */
  uint32_t replay_workgroups;    /* grid of the replay launch                   */
  uint32_t reserved;
} fs_launch_info;
FS_API fs_status fs_last_launch(fs_launch_info *info);

/* ---------------------------------------------------------------------------
 * Batches: many stripes of uneven k and block size in one captured launch.
 *
 * A plan binds a list of work items (encode, decode, repair from resident
 * inputs, update) to their buffers.  At creation it lays out one device
 * workspace for all items, writes the job descriptors to device memory and
 * captures the launch sequence in a hipGraph:
 *   branch A: peeling schedules of every decode (one workgroup per stripe),
 *             their replay programs, then the replays;
 *   branch B: zeroing of split rows, repair id checks, update plans and
 *             deltas, then ONE persistent gather-XOR kernel over the tiles
 *             of every encode, repair and update job.
 * fs_plan_launch replays the graph.  Items of one plan must be independent:
 * no item may write a buffer another item of the plan reads or writes.
 * Results are those of the single-stripe calls (bit for bit).
 *
 * Batching has no counterpart in the paper: it changes only how independent
 * single-stripe operations are scheduled, never their arithmetic.  The
 * nearest passages are the paper's processing of a file as independent
 * partitions, each coded on its own (§2.2), and its dynamic thread
 * scheduling over unevenly sized work in the decoder (§3.1).
 * ------------------------------------------------------------------------- */
enum { FS_WORK_ENCODE = 0, FS_WORK_DECODE = 1, FS_WORK_REPAIR = 2, FS_WORK_UPDATE = 3 };

typedef struct fs_work {
  uint32_t op;              /* FS_WORK_*                                              */
  uint32_t n_ids;           /* repair: lost rows; update: updated inputs              */
  const fs_graph *graph;    /* built on the current device                            */
  uint64_t t;               /* block bytes, multiple of 16                            */
  void *x;                  /* encode: in; decode: out; repair: in; update: in/out    */
  void *c;                  /* encode: out; decode: in; repair, update: in/out        */
  const uint8_t *erased;    /* decode: device uint8[n]                                */
  uint32_t maxit;           /* decode (0 = no limit)                                  */
  uint32_t reserved;        /* must be 0                                              */
  uint8_t *recovered;       /* decode: device uint8[k] (out)                          */
  int32_t *status;          /* device int32[3] (out) as the single call; decode: may
                               be NULL                                                 */
  const uint32_t *ids;      /* repair: device lost rows; update: device input ids     */
  const void *new_blocks;   /* update: device uint8[n_ids][t]                         */
  uint8_t *repaired;        /* repair: device uint8[n_ids] (out)                      */
} fs_work;

typedef struct fs_plan fs_plan;

/* fs_plan_create flags */
enum {
  FS_PLAN_AUTOTUNE = 1,  /* time candidate gather tilings on the bound buffers and
                            keep the fastest (encode and repair outputs are
                            written during the timing; updates are not run)     */
  FS_PLAN_NO_GRAPH = 2   /* launch the kernels one by one instead of a hipGraph */
};

typedef struct fs_plan_info {
  uint32_t items, gather_jobs, decode_items, update_items, repair_items, encode_items;
  uint64_t gather_tiles;     /* items of the persistent gather                   */
  uint32_t replay_workgroups;
  uint32_t tune_source;      /* 0 default, 1 timed now, 2 read from the cache    */
  fs_tune tune;              /* gather tiling used by the plan                   */
  uint64_t workspace_bytes;  /* device memory owned by the plan                  */
  double tuned_ms;           /* timed gather of the chosen tiling (0 if none)    */
} fs_plan_info;

/*
 * Create a plan for count items.  tune_cache: optional path of a text file
 * of tilings keyed by the plan's shape (read, and appended after timing).
 * The stream is used for uploads and timing; the call synchronises it.
 * Errors: FS_ERR_INVALID / FS_ERR_ALIGN for a bad item (fs_last_error names
 * it), FS_ERR_UNSUPPORTED for a repair without resident inputs (x == NULL),
 * FS_ERR_NOMEM, FS_ERR_HIP.
 */
FS_API fs_status fs_plan_create(const fs_work *items, uint32_t count, const char *tune_cache, uint32_t flags,
                                hipStream_t stream, fs_plan **out);
/*
 * Memory a plan of these items needs for fs_plan_create_in: device_bytes of
 * device memory (workspace and descriptors) and stage_bytes (may be null) of
 * host staging for the descriptors.
 */
FS_API fs_status fs_plan_memory_size(const fs_work *items, uint32_t count, size_t *device_bytes,
                                     size_t *stage_bytes);
/*
 * As fs_plan_create, but the plan lives in caller device memory mem (256-byte
 * aligned, at least device_bytes, owned by the caller and kept until
 * fs_plan_free) and is launched without a graph, all on the launch stream: no
 * device allocation, stream or graph is created.  For request loops that
 * build a plan per tick (FS_PLAN_AUTOTUNE is ignored; the process tuning of
 * fs_set_tune applies).  The workspace is cleared and the descriptors copied
 * on `stream`: from host_stage (pinned host memory of at least stage_bytes,
 * left untouched by the caller until the stream has passed the copy) the
 * call returns at once; with host_stage null it returns after the copy.
 * Errors: as fs_plan_create, and FS_ERR_ALIGN (mem), FS_ERR_WORKSPACE (mem or
 * host_stage too small).
 */
FS_API fs_status fs_plan_create_in(const fs_work *items, uint32_t count, void *mem, size_t mem_bytes,
                                   void *host_stage, size_t stage_bytes, hipStream_t stream, fs_plan **out);
/* Run the plan on a stream (asynchronous). */
FS_API fs_status fs_plan_launch(fs_plan *plan, hipStream_t stream);
/*
 * Point the plan at new buffers: same count and, item by item, the same op,
 * graph, t and n_ids (else FS_ERR_INVALID).  The descriptors are rewritten
 * in device memory on the stream.  The captured graph is reused when every
 * job of the plan runs inside the shared persistent kernels; a plan that
 * also holds stripes large enough for launches of their own (their
 * arguments are captured by value) is captured again, which costs a graph
 * capture and instantiation on the host.  A launch already enqueued on
 * another stream must have completed.
 */
FS_API fs_status fs_plan_rebind(fs_plan *plan, const fs_work *items, uint32_t count, hipStream_t stream);
FS_API fs_status fs_plan_get_info(const fs_plan *plan, fs_plan_info *info);
FS_API void fs_plan_free(fs_plan *plan);

FS_API const char *fs_status_string(fs_status s);
/* Message of the last error on the calling thread ("" if none). */
FS_API const char *fs_last_error(void);
/* Library version string. */
FS_API const char *fs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FS_API_H */
