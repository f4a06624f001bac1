// Batches of stripes: descriptors in device memory, one workspace, a captured
// hipGraph, and an autotuner for the gather tiling.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "fs_internal.h"

using namespace fs;

struct fs_plan {
  int device = -1;
  uint32_t flags = 0;
  std::vector<fs_work> items;
  fs_tune tune{};
  uint32_t tune_source = 0;
  double tuned_ms = 0.0;

  // host copies of the descriptor arrays
  std::vector<GatherJob> gjobs;          // encode, repair and update-accumulate jobs
  std::vector<uint8_t> gjob_accumulate;  // 1 for update jobs (not run while tuning)
  std::vector<unsigned long long> gprefix;
  std::vector<PeelJob> peels;
  std::vector<ProgJob> progs;
  std::vector<ReplayJob> replays;
  std::vector<uint32_t> rprefix;
  std::vector<RepairPrepJob> rpreps;
  std::vector<UpdatePlanJob> uplans;
  std::vector<UpdateDeltaJob> udeltas;
  std::vector<uint32_t> uprefix;
  std::vector<ZeroEntry> zeros;
  uint64_t zero_max_t = 0;
  // large jobs run as launches of their own: gathers (1 = accumulating) and
  // the replays of large decodes (program index into progs)
  std::vector<GatherJob> solo;
  std::vector<uint8_t> solo_accumulate;
  std::vector<const fs_graph *> solo_graph;   // graph of each solo job (its tiling)
  std::vector<const fs_graph *> gjob_graph;   // graph of each gather job while building
  std::vector<ReplayJob> solo_replays;
  std::vector<uint32_t> solo_replay_prog;
  std::vector<ProgJob> replay_progs;   // programs of the batched replays, in their order
  std::vector<PeelJob> peels_rows;     // schedules whose row counters alone fit LDS
  size_t peel_rows_bytes = 0;
  size_t peel_rows32_bytes = 0;
  std::vector<PeelJob> peels_rows32;   // schedules whose row counters fit LDS packed in 32 bits
  std::vector<PeelJob> peels_global;   // schedules too large for LDS
  bool peel_lds = true;
  size_t peel_lds_bytes = 0;
  size_t replay_lds = 256;   // dynamic LDS of the batched replay
  uint32_t gather_grid = 0;

  // device memory
  void *d_ws = nullptr;
  size_t ws_bytes = 0;
  void *d_desc = nullptr;
  size_t desc_bytes = 0;
  std::vector<uint8_t> himage;   // host image of the descriptor buffer
  GatherJob *d_gjobs = nullptr;
  unsigned long long *d_gprefix = nullptr;
  PeelJob *d_peels = nullptr;
  PeelJob *d_peels_rows = nullptr;
  PeelJob *d_peels_rows32 = nullptr;
  PeelJob *d_peels_global = nullptr;
  ProgJob *d_progs = nullptr;
  ReplayJob *d_replays = nullptr;
  ProgJob *d_replay_progs = nullptr;
  uint32_t *d_rprefix = nullptr;
  RepairPrepJob *d_rpreps = nullptr;
  UpdatePlanJob *d_uplans = nullptr;
  UpdateDeltaJob *d_udeltas = nullptr;
  uint32_t *d_uprefix = nullptr;
  ZeroEntry *d_zeros = nullptr;
  // tuning runs: the gather jobs without the accumulating ones
  GatherJob *d_tjobs = nullptr;
  unsigned long long *d_tprefix = nullptr;
  uint32_t n_tjobs = 0;
  unsigned long long *d_counter = nullptr;   // 8 work counters (one per XCD, 256 bytes apart) of the persistent gather

  bool external = false;   // workspace and descriptors in caller memory
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

namespace {

#define PL_TRY(expr)              \
  do {                            \
    fs_status _s = (expr);        \
    if (_s != FS_OK) return _s;   \
  } while (0)

fs_status hip_ok(hipError_t e, const char *what) {
  if (e == hipSuccess) return FS_OK;
  return fail(FS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

fs_status check_item(const fs_work &w, uint32_t i) {
  const std::string at = "item " + std::to_string(i) + ": ";
  fs_status st = check_graph(w.graph);
  if (st != FS_OK) return fail(st, at + fs_last_error());
  if (w.reserved != 0) return fail(FS_ERR_INVALID, at + "reserved field must be 0");
  if (w.t == 0 || (w.t & 15)) return fail(FS_ERR_ALIGN, at + "t must be a positive multiple of 16");
  auto al = [&](const void *p, const char *name, bool need) -> fs_status {
    if (!p) return need ? fail(FS_ERR_INVALID, at + name + " is null") : FS_OK;
    if (reinterpret_cast<uintptr_t>(p) & 15) return fail(FS_ERR_ALIGN, at + name + " is not 16-byte aligned");
    return FS_OK;
  };
  switch (w.op) {
    case FS_WORK_ENCODE:
      PL_TRY(al(w.x, "x", true));
      PL_TRY(al(w.c, "c", true));
      return FS_OK;
    case FS_WORK_DECODE:
      PL_TRY(al(w.x, "x", true));
      PL_TRY(al(w.c, "c", true));
      if (!w.erased || !w.recovered) return fail(FS_ERR_INVALID, at + "erased and recovered must be non-null");
      return FS_OK;
    case FS_WORK_REPAIR:
      if (!w.x) return fail(FS_ERR_UNSUPPORTED, at + "batched repair needs the resident inputs (x)");
      PL_TRY(al(w.x, "x", true));
      PL_TRY(al(w.c, "c", true));
      if (!w.status || (w.n_ids && (!w.ids || !w.repaired)))
        return fail(FS_ERR_INVALID, at + "ids, repaired and status must be non-null");
      return FS_OK;
    case FS_WORK_UPDATE:
      PL_TRY(al(w.x, "x", true));
      PL_TRY(al(w.c, "c", true));
      if (w.n_ids) PL_TRY(al(w.new_blocks, "new_blocks", true));
      if (!w.status || (w.n_ids && !w.ids)) return fail(FS_ERR_INVALID, at + "ids and status must be non-null");
      return FS_OK;
  }
  return fail(FS_ERR_INVALID, at + "unknown op");
}

// Per item workspace carving (also used for sizing with base == nullptr).
struct ItemWs {
  DecodeBufs dec;
  RepairBufs rep;
  UpdateBufs upd;
};

void carve_item(Carver &cv, const fs_work &w, ItemWs &b) {
  switch (w.op) {
    case FS_WORK_DECODE: carve_decode(cv, w.graph, b.dec); break;
    case FS_WORK_REPAIR: carve_repair(cv, w.graph, w.t, false, b.rep); break;
    case FS_WORK_UPDATE: carve_update(cv, w.graph, w.t, w.n_ids, b.upd); break;
    default: break;
  }
}

uint64_t gather_items_of(const GatherJob &j, const fs_tune &tune) {
  const uint32_t rpb = 256 / tune.lanes_per_row;
  const uint64_t w = 16ull * tune.lanes_per_row * tune.chunks;
  const uint64_t nslices = (j.t + w - 1) / w;
  const uint64_t ntiles = (j.nrows + rpb - 1) / rpb;
  return nslices * ntiles;
}

// A gather job of at least this many (slice, tile) items at the default
// tiling fills the device by itself: it runs as its own launch, where the
// hardware dispatcher balances it with no claim traffic.  Smaller jobs share
// the persistent kernel.
constexpr uint64_t kSoloItems = 8192;
// A decode whose k t reaches this size replays with the one-stripe kernels
// (which pick the slice width and LDS layout for its shape).
constexpr uint64_t kSoloReplayBytes = 32ull << 20;

// The persistent kernel's tiling: the plan's (tuned or set) tiling, or,
// left open, by its jobs' blocks: 64 lanes x 4 chunks (4 KiB slices) when
// every block is at least 64 KiB, else 16 lanes x 2 chunks.  Four chunks
// per lane keep more loads in flight: the update of 128 resident stripes of
// 256 KiB blocks took 1.89 ms so against 2.48 ms at 16 x 2.
fs_tune batch_tune(const fs_tune &t, uint64_t min_t) {
  if (t.lanes_per_row != 0) return t;
  fs_tune r = t;
  const bool long_blocks = min_t >= (64u << 10);
  r.lanes_per_row = long_blocks ? 64 : 16;
  r.chunks = long_blocks ? 4 : 2;
  return r;
}

uint64_t min_block(const std::vector<GatherJob> &jobs) {
  uint64_t m = ~0ull;
  for (const GatherJob &j : jobs) m = std::min<uint64_t>(m, j.t);
  return jobs.empty() ? 0 : m;
}

bool solo_gather(const GatherJob &j) {
  // jobs sized on the device (update deltas) only know a bound: they stay
  // in the persistent kernel, which skips their dead tiles cheaply
  if (j.nrows_dev) return false;
  const fs_tune dflt{16, 2, 1, 1, 0, 0};
  return gather_items_of(j, dflt) >= kSoloItems;
}

// Build every descriptor of the plan from its items (device pointers into the
// items' buffers and into the plan workspace).
void build_descriptors(fs_plan &P) {
  P.gjobs.clear();
  P.gjob_accumulate.clear();
  P.peels.clear();
  P.progs.clear();
  P.replays.clear();
  P.rprefix.assign(1, 0);
  P.rpreps.clear();
  P.uplans.clear();
  P.udeltas.clear();
  P.uprefix.assign(1, 0);
  P.zeros.clear();
  P.zero_max_t = 0;
  P.solo.clear();
  P.solo_accumulate.clear();
  P.solo_graph.clear();
  P.gjob_graph.clear();
  P.solo_replays.clear();
  P.solo_replay_prog.clear();
  P.replay_progs.clear();
  P.peels_global.clear();
  P.peels_rows.clear();
  P.peels_rows32.clear();
  P.peel_rows_bytes = 0;
  P.peel_rows32_bytes = 0;
  P.peel_lds = true;
  P.peel_lds_bytes = 0;
  P.replay_lds = 256;
  Carver cv(P.d_ws);
  for (const fs_work &w : P.items) {
    const fs_graph *g = w.graph;
    ItemWs b{};
    carve_item(cv, w, b);
    switch (w.op) {
      case FS_WORK_ENCODE: {
        for (int32_t row : g->heavy) P.zeros.push_back(ZeroEntry{static_cast<uint8_t *>(w.c), w.t, row});
        if (!g->heavy.empty()) P.zero_max_t = std::max(P.zero_max_t, w.t);
        P.gjobs.push_back(encode_job(g, w.x, w.c, w.t));
        P.gjob_accumulate.push_back(0);
        P.gjob_graph.push_back(g);
        break;
      }
      case FS_WORK_DECODE: {
        int32_t *status = w.status ? w.status : b.dec.sched.status;
        PeelJob pj = peel_job(g, w.erased, w.maxit, w.recovered, status, b.dec.sched.level_ptr, b.dec.sched.dp_f,
                              b.dec.sched.dp_g);
        pj.acc = b.dec.peel.acc;
        pj.best = b.dec.peel.best;
        pj.front_a = b.dec.peel.front_a;
        pj.front_b = b.dec.peel.front_b;
        pj.dlist = b.dec.peel.dlist;
        pj.mask = b.dec.peel.mask;
        pj.decmask = b.dec.peel.decmask;
        const int mode = peel_mode(g->k, g->n, g->max_deg);
        if (mode == 2) {
          P.peel_lds_bytes = std::max(P.peel_lds_bytes, peel_lds_bytes(g->k, g->n));
          P.peels.push_back(pj);
        } else if (mode == 1) {
          P.peel_rows_bytes = std::max<size_t>(P.peel_rows_bytes, 8ull * g->n);
          P.peels_rows.push_back(pj);
        } else if (mode == 3 || mode == 5) {
          // (the batched peel keeps only the packed counters in LDS)
          P.peel_rows32_bytes = std::max<size_t>(P.peel_rows32_bytes, 4ull * g->n);
          P.peels_rows32.push_back(pj);
        } else {
          P.peels_global.push_back(pj);
        }
        ProgJob prog = b.dec.prog;
        prog.status = status;
        P.progs.push_back(prog);
        const ReplayJob rj = replay_job(g, w.c, w.x, w.t, status, b.dec.sched.level_ptr, b.dec.sched.dp_f,
                                        b.dec.sched.dp_g);
        if ((uint64_t)g->k * w.t >= kSoloReplayBytes) {
          P.solo_replays.push_back(rj);
          P.solo_replay_prog.push_back((uint32_t)(P.progs.size() - 1));
          break;
        }
        P.replay_lds = std::max(P.replay_lds, replay_prog_lds_bound(g->k, prog.pidx_cap));
        P.replays.push_back(rj);
        P.replay_progs.push_back(prog);
        const uint64_t wsl = 16ull * kBatchReplayLanes;
        const uint64_t nslices = (w.t + wsl - 1) / wsl;
        const uint32_t nwg = (uint32_t)((nslices + kBatchReplaySlicesPerWg - 1) / kBatchReplaySlicesPerWg);
        P.rprefix.push_back(P.rprefix.back() + nwg);
        break;
      }
      case FS_WORK_REPAIR: {
        RepairPrepJob rp{};
        rp.n = g->n;
        rp.k = g->k;
        rp.lost = w.ids;
        rp.n_lost = w.n_ids;
        rp.seen = b.rep.seen;
        rp.flag = b.rep.flag;
        rp.repaired = w.repaired;
        rp.status = w.status;
        if (b.rep.sptr) repair_pieces_prep(rp, g, b.rep, w.c, w.t);
        P.rpreps.push_back(rp);
        if (w.n_ids && b.rep.sptr) {
          // rows of more than 64 edges: the lost rows in pieces
          P.gjobs.push_back(repair_pieces_job(g, b.rep, w.n_ids, w.x, w.c, w.t));
          P.gjob_accumulate.push_back(0);
          P.gjob_graph.push_back(g);
        } else if (w.n_ids) {
          GatherJob gj{};
          gj.src = static_cast<const uint8_t *>(w.x);
          gj.src_stride = w.t;
          gj.dst = static_cast<uint8_t *>(w.c);
          gj.dst_stride = w.t;
          gj.ptr = g->d_row_ptr;
          gj.idx = g->d_col;
          gj.csr_map = w.ids;
          gj.out_map = reinterpret_cast<const int32_t *>(w.ids);
          gj.skip_flag = b.rep.flag;
          gj.nrows = w.n_ids;
          gj.csr_rows = g->n;
          gj.t = w.t;
          P.gjobs.push_back(gj);
          P.gjob_accumulate.push_back(0);
          P.gjob_graph.push_back(g);
        }
        break;
      }
      case FS_WORK_UPDATE: {
        UpdatePlanJob up{};
        up.k = g->k;
        up.n = g->n;
        up.col_ptr = g->d_col_ptr;
        up.rowidx = g->d_rowidx;
        up.ids = w.ids;
        up.n_ids = w.n_ids;
        up.seen = b.upd.seen;
        up.cnt = b.upd.cnt;
        up.arow = b.upd.arow;
        up.aptr = b.upd.aptr;
        up.asrc = b.upd.asrc;
        up.n_aff = b.upd.n_aff;
        up.flag = b.upd.flag;
        up.status = w.status;
        P.uplans.push_back(up);
        UpdateDeltaJob dj{};
        dj.x = static_cast<uint8_t *>(w.x);
        dj.new_blocks = static_cast<const uint8_t *>(w.new_blocks);
        dj.delta = b.upd.delta;
        dj.ids = w.ids;
        dj.n_ids = w.n_ids;
        dj.t = w.t;
        dj.flag = b.upd.flag;
        P.udeltas.push_back(dj);
        const uint32_t per = (uint32_t)((w.t + kDeltaBytesPerWg - 1) / kDeltaBytesPerWg);
        P.uprefix.push_back(P.uprefix.back() + per * w.n_ids);
        if (w.n_ids && b.upd.max_rows) {
          GatherJob gj{};
          gj.src = b.upd.delta;
          gj.src_stride = w.t;
          gj.dst = static_cast<uint8_t *>(w.c);
          gj.dst_stride = w.t;
          gj.ptr = b.upd.aptr;
          gj.idx = b.upd.asrc;
          gj.out_map = b.upd.arow;
          gj.nrows_dev = b.upd.n_aff;
          gj.skip_flag = b.upd.flag;
          gj.nrows = b.upd.max_rows;
          gj.csr_rows = b.upd.max_rows;
          gj.t = w.t;
          gj.accumulate = 1;
          P.gjobs.push_back(gj);
          P.gjob_accumulate.push_back(1);
          P.gjob_graph.push_back(g);
        }
        break;
      }
      default: break;
    }
  }
  // move the large gather jobs out of the persistent kernel
  std::vector<GatherJob> shared;
  std::vector<uint8_t> shared_acc;
  for (size_t i = 0; i < P.gjobs.size(); ++i) {
    if (solo_gather(P.gjobs[i])) {
      P.solo.push_back(P.gjobs[i]);
      P.solo_accumulate.push_back(P.gjob_accumulate[i]);
      P.solo_graph.push_back(P.gjob_graph[i]);
    } else {
      shared.push_back(P.gjobs[i]);
      shared_acc.push_back(P.gjob_accumulate[i]);
    }
  }
  P.gjobs.swap(shared);
  P.gjob_accumulate.swap(shared_acc);
}

void gather_prefix(const std::vector<GatherJob> &jobs, const fs_tune &tune, std::vector<unsigned long long> &pre) {
  pre.assign(1, 0);
  for (const GatherJob &j : jobs) pre.push_back(pre.back() + gather_items_of(j, tune));
}

template <class T>
T *place(uint8_t *base, size_t &off, size_t count) {
  off = (off + 255) & ~size_t(255);
  T *p = reinterpret_cast<T *>(base + off);
  off += std::max<size_t>(count, 1) * sizeof(T);
  return p;
}

// Lay out every descriptor array in one device buffer (sizes are fixed for
// the life of the plan), pack the same layout into a host image and copy it
// with one transfer.  With `stage` (pinned host memory of >= desc_bytes that
// the caller keeps until the stream passes the copy) the copy is
// asynchronous; otherwise it is made from the plan's own host image and the
// call waits for it.
fs_status upload_descriptors(fs_plan &P, hipStream_t s, bool allocate, void *stage = nullptr) {
  std::vector<GatherJob> tjobs;
  for (size_t i = 0; i < P.gjobs.size(); ++i)
    if (!P.gjob_accumulate[i]) tjobs.push_back(P.gjobs[i]);
  std::vector<unsigned long long> tprefix;
  gather_prefix(tjobs, batch_tune(P.tune, min_block(P.gjobs)), tprefix);
  gather_prefix(P.gjobs, batch_tune(P.tune, min_block(P.gjobs)), P.gprefix);
  size_t off = 0;
  uint8_t *base = static_cast<uint8_t *>(P.d_desc);
  P.d_gjobs = place<GatherJob>(base, off, P.gjobs.size());
  P.d_gprefix = place<unsigned long long>(base, off, P.gprefix.size());
  P.d_peels = place<PeelJob>(base, off, P.peels.size());
  P.d_peels_rows = place<PeelJob>(base, off, P.peels_rows.size());
  P.d_peels_rows32 = place<PeelJob>(base, off, P.peels_rows32.size());
  P.d_peels_global = place<PeelJob>(base, off, P.peels_global.size());
  P.d_progs = place<ProgJob>(base, off, P.progs.size());
  P.d_replays = place<ReplayJob>(base, off, P.replays.size());
  P.d_replay_progs = place<ProgJob>(base, off, P.replay_progs.size());
  P.d_rprefix = place<uint32_t>(base, off, P.rprefix.size());
  P.d_rpreps = place<RepairPrepJob>(base, off, P.rpreps.size());
  P.d_uplans = place<UpdatePlanJob>(base, off, P.uplans.size());
  P.d_udeltas = place<UpdateDeltaJob>(base, off, P.udeltas.size());
  P.d_uprefix = place<uint32_t>(base, off, P.uprefix.size());
  P.d_zeros = place<ZeroEntry>(base, off, P.zeros.size());
  P.d_tjobs = place<GatherJob>(base, off, tjobs.size());
  P.d_tprefix = place<unsigned long long>(base, off, tprefix.size());
  P.d_counter = place<unsigned long long>(base, off, 8 * kCounterStride);
  P.n_tjobs = (uint32_t)tjobs.size();
  off = (off + 255) & ~size_t(255);
  if (allocate) {
    P.desc_bytes = off;
    return FS_OK;   // caller allocates desc_bytes and calls again
  }
  if (off > P.desc_bytes) return fail(FS_ERR_INVALID, "descriptor layout changed");
  uint8_t *img = static_cast<uint8_t *>(stage);
  if (!img) {
    P.himage.assign(P.desc_bytes, 0);
    img = P.himage.data();
  } else {
    std::memset(img, 0, P.desc_bytes);
  }
  auto put = [&](const void *dst, const void *src, size_t bytes) {
    if (bytes) std::memcpy(img + (static_cast<const uint8_t *>(dst) - base), src, bytes);
  };
  put(P.d_gjobs, P.gjobs.data(), P.gjobs.size() * sizeof(GatherJob));
  put(P.d_gprefix, P.gprefix.data(), P.gprefix.size() * sizeof(unsigned long long));
  put(P.d_peels, P.peels.data(), P.peels.size() * sizeof(PeelJob));
  put(P.d_peels_rows, P.peels_rows.data(), P.peels_rows.size() * sizeof(PeelJob));
  put(P.d_peels_rows32, P.peels_rows32.data(), P.peels_rows32.size() * sizeof(PeelJob));
  put(P.d_peels_global, P.peels_global.data(), P.peels_global.size() * sizeof(PeelJob));
  put(P.d_progs, P.progs.data(), P.progs.size() * sizeof(ProgJob));
  put(P.d_replays, P.replays.data(), P.replays.size() * sizeof(ReplayJob));
  put(P.d_replay_progs, P.replay_progs.data(), P.replay_progs.size() * sizeof(ProgJob));
  put(P.d_rprefix, P.rprefix.data(), P.rprefix.size() * sizeof(uint32_t));
  put(P.d_rpreps, P.rpreps.data(), P.rpreps.size() * sizeof(RepairPrepJob));
  put(P.d_uplans, P.uplans.data(), P.uplans.size() * sizeof(UpdatePlanJob));
  put(P.d_udeltas, P.udeltas.data(), P.udeltas.size() * sizeof(UpdateDeltaJob));
  put(P.d_uprefix, P.uprefix.data(), P.uprefix.size() * sizeof(uint32_t));
  put(P.d_zeros, P.zeros.data(), P.zeros.size() * sizeof(ZeroEntry));
  put(P.d_tjobs, tjobs.data(), tjobs.size() * sizeof(GatherJob));
  put(P.d_tprefix, tprefix.data(), tprefix.size() * sizeof(unsigned long long));
  PL_TRY(hip_ok(hipMemcpyAsync(P.d_desc, img, P.desc_bytes, hipMemcpyHostToDevice, s), "descriptor upload"));
  if (!stage) PL_TRY(hip_ok(hipStreamSynchronize(s), "descriptor upload"));
  return FS_OK;
}

uint32_t gather_grid_for(uint64_t items) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  const uint64_t cap = (uint64_t)device_info(dev).cu_count * 8;   // persistent: ~8 workgroups per CU
  return (uint32_t)std::min<uint64_t>(items, cap);
}

// The whole plan as launches on s (branch A on P.side when it exists).
fs_status enqueue(fs_plan &P, hipStream_t s) {
  const bool fork = P.side != nullptr && !(P.peels.empty() && P.peels_rows.empty() && P.peels_rows32.empty() && P.peels_global.empty());
  hipStream_t a = fork ? P.side : s;
  if (fork) {
    PL_TRY(hip_ok(hipEventRecord(P.fork, s), "fork"));
    PL_TRY(hip_ok(hipStreamWaitEvent(P.side, P.fork, 0), "fork wait"));
  }
  // branch A: decodes (schedule, program, replay)
  PL_TRY(launch_peel_batch(P.d_peels, (uint32_t)P.peels.size(), 2, P.peel_lds_bytes, a));
  PL_TRY(launch_peel_batch(P.d_peels_rows, (uint32_t)P.peels_rows.size(), 1, P.peel_rows_bytes, a));
  PL_TRY(launch_peel_batch(P.d_peels_rows32, (uint32_t)P.peels_rows32.size(), 3, P.peel_rows32_bytes, a));
  PL_TRY(launch_peel_batch(P.d_peels_global, (uint32_t)P.peels_global.size(), 0, 0, a));
  PL_TRY(launch_prog_batch(P.d_progs, (uint32_t)P.progs.size(), a));
  // replays[i] runs the program replay_progs[i] (built above for every decode)
  PL_TRY(launch_replay_batch(P.d_replays, P.d_replay_progs, P.d_rprefix, (uint32_t)P.replays.size(),
                             P.rprefix.back(), P.replay_lds, a));
  for (size_t i = 0; i < P.solo_replays.size(); ++i) {
    PL_TRY(launch_prog_lookahead(P.progs[P.solo_replay_prog[i]], a));
    PL_TRY(launch_replay_prog(P.solo_replays[i], &P.progs[P.solo_replay_prog[i]], a));
  }
  // branch B: zeroing, checks, update planning, then the persistent gather
  PL_TRY(launch_zero_batch(P.d_zeros, (uint32_t)P.zeros.size(), P.zero_max_t, s));
  PL_TRY(launch_repair_prep_batch(P.d_rpreps, (uint32_t)P.rpreps.size(), s));
  PL_TRY(launch_update_plan_batch(P.d_uplans, (uint32_t)P.uplans.size(), s));
  PL_TRY(launch_update_delta_batch(P.d_udeltas, P.d_uprefix, (uint32_t)P.udeltas.size(), P.uprefix.back(), s));
  PL_TRY(launch_gather_batch(P.d_gjobs, P.d_gprefix, (uint32_t)P.gjobs.size(), P.d_counter, batch_tune(P.tune, min_block(P.gjobs)),
                             P.gather_grid, P.gprefix.back(), s));
  for (size_t i = 0; i < P.solo.size(); ++i) PL_TRY(launch_gather(P.solo[i], tile_for(P.tune, P.solo_graph[i]), s));
  if (fork) {
    PL_TRY(hip_ok(hipEventRecord(P.join, P.side), "join"));
    PL_TRY(hip_ok(hipStreamWaitEvent(s, P.join, 0), "join wait"));
  }
  return FS_OK;
}

// Capture the plan's launches into a graph and instantiate it (replacing
// any earlier one: a rebind changes the arguments of the large jobs' own
// launches, which a graph holds by value).
fs_status capture(fs_plan &P) {
  if (P.exec) (void)hipGraphExecDestroy(P.exec);
  if (P.graph) (void)hipGraphDestroy(P.graph);
  P.exec = nullptr;
  P.graph = nullptr;
  hipStream_t cap = nullptr;
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
    return fail(FS_ERR_HIP, "capture stream creation failed");
  fs_status st = FS_OK;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    st = enqueue(P, cap);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (st == FS_OK && e2 != hipSuccess) st = fail(FS_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e2));
    P.graph = g;
  } else {
    st = fail(FS_ERR_HIP, std::string("begin capture: ") + hipGetErrorString(e));
  }
  (void)hipStreamDestroy(cap);
  if (st != FS_OK) return st;
  if (hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0) != hipSuccess)
    return fail(FS_ERR_HIP, "graph instantiation failed");
  return FS_OK;
}

std::string shape_key(const fs_plan &P) {
  // the plan's shape: per item op, k, n, nnz, t (arch first)
  std::ostringstream os;
  os << "gfx950.v3";   // v3: tuned with live row counts (entries carry the claim chunk)
  uint64_t h = 1469598103934665603ull;
  for (const fs_work &w : P.items) {
    const uint64_t v[5] = {w.op, w.graph->k, w.graph->n, w.graph->nnz, w.t};
    for (uint64_t x : v) {
      h ^= x;
      h *= 1099511628211ull;
    }
  }
  os << ":" << P.items.size() << ":" << std::hex << h;
  return os.str();
}

bool cache_lookup(const char *path, const std::string &key, fs_tune &t) {
  if (!path) return false;
  std::ifstream f(path);
  std::string k;
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    uint32_t lpr, ch, rm, nt, cc;
    if (!(is >> k >> lpr >> ch >> rm >> nt >> cc) || k != key) continue;
    t.lanes_per_row = lpr;
    t.chunks = ch;
    t.xcd_remap = rm;
    t.nt_store = nt;
    t.claim_chunk = cc;
    found = true;   // the last entry wins
  }
  return found;
}

void cache_store(const char *path, const std::string &key, const fs_tune &t) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << t.lanes_per_row << " " << t.chunks << " " << t.xcd_remap << " " << t.nt_store << " "
    << t.claim_chunk << "\n";
}

// Time the plan's gathers (the persistent kernel and the large jobs' own
// launches, without the accumulating update jobs) under candidate tunings
// and keep the fastest:
//   1. every tiling (lanes per row x chunks), and the per-graph rule (the
//      persistent kernel by its jobs' blocks, each large job at its graph's
//      tiling), with XCD remap and non-temporal stores on: one warm run,
//      median of three timed;
//   2. the three fastest again, median of five timed runs each;
//   3. the winner with XCD remap off, then with plain stores, then with
//      claim chunks of 1, 4 and 32 items: each kept when its median of five
//      is faster.
fs_status autotune(fs_plan &P, hipStream_t s) {
  size_t solo_tuned = 0;
  for (uint8_t a : P.solo_accumulate) solo_tuned += a == 0;
  if (P.n_tjobs == 0 && solo_tuned == 0) return FS_OK;
  static const uint32_t cand[][2] = {{0, 0},  {16, 1}, {16, 2}, {16, 4}, {32, 1},  {32, 2},  {32, 4},
                                     {64, 1}, {64, 2}, {64, 4}, {128, 2}, {256, 1}, {256, 2}};
  hipEvent_t e0, e1;
  PL_TRY(hip_ok(hipEventCreate(&e0), "event"));
  PL_TRY(hip_ok(hipEventCreate(&e1), "event"));
  std::vector<GatherJob> tjobs;
  for (size_t i = 0; i < P.gjobs.size(); ++i)
    if (!P.gjob_accumulate[i]) tjobs.push_back(P.gjobs[i]);
  // the repairs' pieces are counted by their prep kernel: without it the
  // timed gathers would find no live rows (it writes only the plan's
  // workspace, the items' status outputs and lost rows of c)
  PL_TRY(launch_repair_prep_batch(P.d_rpreps, (uint32_t)P.rpreps.size(), s));
  // median time of `reps` timed runs (after one warm run) of the gathers under tuning t
  auto measure = [&](const fs_tune &t, int reps, float &median) -> fs_status {
    const fs_tune bt = batch_tune(t, min_block(P.gjobs));
    std::vector<unsigned long long> pre;
    gather_prefix(tjobs, bt, pre);
    PL_TRY(hip_ok(hipMemcpyAsync(P.d_tprefix, pre.data(), pre.size() * sizeof(unsigned long long),
                                 hipMemcpyHostToDevice, s), "tune prefix"));
    const uint32_t grid = gather_grid_for(pre.back());
    auto run = [&]() -> fs_status {
      PL_TRY(launch_gather_batch(P.d_tjobs, P.d_tprefix, P.n_tjobs, P.d_counter, bt, grid, pre.back(), s));
      for (size_t i = 0; i < P.solo.size(); ++i)
        if (!P.solo_accumulate[i]) PL_TRY(launch_gather(P.solo[i], tile_for(t, P.solo_graph[i]), s));
      return FS_OK;
    };
    PL_TRY(run());
    std::vector<float> ms;
    for (int r = 0; r < reps; ++r) {
      PL_TRY(hip_ok(hipEventRecord(e0, s), "tune event"));
      PL_TRY(run());
      PL_TRY(hip_ok(hipEventRecord(e1, s), "tune event"));
      PL_TRY(hip_ok(hipEventSynchronize(e1), "tune sync"));
      float m = 0.0f;
      (void)hipEventElapsedTime(&m, e0, e1);
      ms.push_back(m);
    }
    std::sort(ms.begin(), ms.end());
    median = ms[ms.size() / 2];
    return FS_OK;
  };
  fs_status st = FS_OK;
  std::vector<std::pair<float, fs_tune>> first;
  for (const auto &c : cand) {
    fs_tune t = P.tune;
    t.lanes_per_row = c[0];
    t.chunks = c[1];
    t.xcd_remap = 1;
    t.nt_store = 1;
    float m = 0.0f;
    st = measure(t, 3, m);
    if (st != FS_OK) break;
    first.emplace_back(m, t);
  }
  float best = 1e30f;
  fs_tune best_t = P.tune;
  if (st == FS_OK) {
    std::stable_sort(first.begin(), first.end(),
                     [](const std::pair<float, fs_tune> &a, const std::pair<float, fs_tune> &b) {
                       return a.first < b.first;
                     });
    for (size_t i = 0; i < first.size() && i < 3 && st == FS_OK; ++i) {
      float m = 0.0f;
      st = measure(first[i].second, 5, m);
      if (st == FS_OK && m < best) {
        best = m;
        best_t = first[i].second;
      }
    }
  }
  for (int flip = 0; flip < 5 && st == FS_OK; ++flip) {
    if (flip >= 2 && P.n_tjobs == 0) break;   // claim chunks apply to the persistent kernel only
    fs_tune t = best_t;
    if (flip == 0) t.xcd_remap = 0;
    else if (flip == 1) t.nt_store = 0;
    else t.claim_chunk = flip == 2 ? 1u : flip == 3 ? 4u : 32u;
    float m = 0.0f;
    st = measure(t, 5, m);
    if (st == FS_OK && m < best) {
      best = m;
      best_t = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != FS_OK) return st;
  P.tune = best_t;
  P.tuned_ms = best;
  P.tune_source = 1;
  return FS_OK;
}

void release(fs_plan *P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->fork) (void)hipEventDestroy(P->fork);
  if (P->join) (void)hipEventDestroy(P->join);
  if (P->side) (void)hipStreamDestroy(P->side);
  if (!P->external) {
    if (P->d_desc) (void)hipFree(P->d_desc);
    if (P->d_ws) (void)hipFree(P->d_ws);
  }
  delete P;
}

}  // namespace

extern "C" {

fs_status fs_plan_create(const fs_work *items, uint32_t count, const char *tune_cache, uint32_t flags,
                         hipStream_t stream, fs_plan **out) {
  clear_error();
  if (!out || (count && !items)) return fail(FS_ERR_INVALID, "items and out must be non-null");
  if (flags & ~3u) return fail(FS_ERR_INVALID, "unknown plan flags");
  for (uint32_t i = 0; i < count; ++i) PL_TRY(check_item(items[i], i));
  fs_plan *P = new (std::nothrow) fs_plan();
  if (!P) return fail(FS_ERR_NOMEM, "host allocation failed");
  P->flags = flags;
  P->items.assign(items, items + count);
  P->tune = current_tune();
  (void)hipGetDevice(&P->device);
  auto bail = [&](fs_status s) {
    const std::string msg = fs_last_error();
    release(P);
    return fail(s, msg);
  };
  // workspace
  {
    Carver cv(nullptr);
    for (const fs_work &w : P->items) {
      ItemWs b{};
      carve_item(cv, w, b);
    }
    P->ws_bytes = cv.size();
    if (P->ws_bytes && hipMalloc(&P->d_ws, P->ws_bytes) != hipSuccess)
      return bail(fail(FS_ERR_NOMEM, "plan workspace allocation failed"));
    // flags start cleared (tuning runs read them before any check kernel ran)
    if (P->ws_bytes && hipMemsetAsync(P->d_ws, 0, P->ws_bytes, stream) != hipSuccess)
      return bail(fail(FS_ERR_HIP, "plan workspace clear failed"));
  }
  build_descriptors(*P);
  fs_status st = upload_descriptors(*P, stream, true);   // sizes only
  if (st != FS_OK) return bail(st);
  if (hipMalloc(&P->d_desc, P->desc_bytes) != hipSuccess)
    return bail(fail(FS_ERR_NOMEM, "plan descriptor allocation failed"));
  const std::string key = shape_key(*P);
  if (cache_lookup(tune_cache, key, P->tune)) P->tune_source = 2;
  st = upload_descriptors(*P, stream, false);
  if (st != FS_OK) return bail(st);
  if ((flags & FS_PLAN_AUTOTUNE) && P->tune_source != 2) {
    st = autotune(*P, stream);
    if (st != FS_OK) return bail(st);
    cache_store(tune_cache, key, P->tune);
    st = upload_descriptors(*P, stream, false);   // prefix of the chosen tiling
    if (st != FS_OK) return bail(st);
  }
  P->gather_grid = gather_grid_for(P->gprefix.back());
  if (hipStreamSynchronize(stream) != hipSuccess) return bail(fail(FS_ERR_HIP, "plan upload failed"));
  if (!P->peels.empty() || !P->peels_rows.empty() || !P->peels_rows32.empty() || !P->peels_global.empty()) {
    if (hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&P->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&P->join, hipEventDisableTiming) != hipSuccess)
      return bail(fail(FS_ERR_HIP, "plan stream/event creation failed"));
  }
  prepare_batch_kernels();
  if (!(flags & FS_PLAN_NO_GRAPH)) {
    st = capture(*P);
    if (st != FS_OK) return bail(st);
  }
  *out = P;
  return FS_OK;
}

fs_status fs_plan_launch(fs_plan *plan, hipStream_t stream) {
  clear_error();
  if (!plan) return fail(FS_ERR_INVALID, "plan is null");
  int dev = -1;
  (void)hipGetDevice(&dev);
  if (dev != plan->device) return fail(FS_ERR_INVALID, "plan lives on another device");
  if (plan->exec) return hip_ok(hipGraphLaunch(plan->exec, stream), "graph launch");
  return enqueue(*plan, stream);
}

fs_status fs_plan_rebind(fs_plan *plan, const fs_work *items, uint32_t count, hipStream_t stream) {
  clear_error();
  if (!plan || (count && !items)) return fail(FS_ERR_INVALID, "plan and items must be non-null");
  if (count != plan->items.size()) return fail(FS_ERR_INVALID, "rebind needs the same number of items");
  for (uint32_t i = 0; i < count; ++i) {
    const fs_work &a = plan->items[i], &b = items[i];
    if (a.op != b.op || a.graph != b.graph || a.t != b.t || a.n_ids != b.n_ids)
      return fail(FS_ERR_INVALID, "item " + std::to_string(i) + ": rebind must keep op, graph, t and n_ids");
    PL_TRY(check_item(b, i));
    // the decode status slot moves between caller memory and the workspace
    if (a.op == FS_WORK_DECODE && ((a.status == nullptr) != (b.status == nullptr)))
      return fail(FS_ERR_INVALID, "item " + std::to_string(i) + ": rebind must keep status null or not");
  }
  plan->items.assign(items, items + count);
  build_descriptors(*plan);
  PL_TRY(upload_descriptors(*plan, stream, false));
  if (plan->exec && !plan->solo.size() && !plan->solo_replays.size()) return FS_OK;
  return plan->exec ? capture(*plan) : FS_OK;
}

fs_status fs_plan_get_info(const fs_plan *plan, fs_plan_info *info) {
  clear_error();
  if (!plan || !info) return fail(FS_ERR_INVALID, "plan and info must be non-null");
  std::memset(info, 0, sizeof(*info));
  info->items = (uint32_t)plan->items.size();
  for (const fs_work &w : plan->items) {
    info->decode_items += w.op == FS_WORK_DECODE;
    info->update_items += w.op == FS_WORK_UPDATE;
    info->repair_items += w.op == FS_WORK_REPAIR;
    info->encode_items += w.op == FS_WORK_ENCODE;
  }
  info->gather_jobs = (uint32_t)(plan->gjobs.size() + plan->solo.size());
  info->gather_tiles = plan->gprefix.empty() ? 0 : plan->gprefix.back();
  info->replay_workgroups = plan->rprefix.back();
  info->tune_source = plan->tune_source;
  info->tune = plan->tune;
  info->workspace_bytes = plan->ws_bytes + plan->desc_bytes;
  info->tuned_ms = plan->tuned_ms;
  return FS_OK;
}

void fs_plan_free(fs_plan *plan) { release(plan); }

fs_status fs_plan_memory_size(const fs_work *items, uint32_t count, size_t *device_bytes, size_t *stage_bytes) {
  clear_error();
  if (!device_bytes || (count && !items)) return fail(FS_ERR_INVALID, "items and device_bytes must be non-null");
  for (uint32_t i = 0; i < count; ++i) PL_TRY(check_item(items[i], i));
  fs_plan P;
  P.items.assign(items, items + count);
  P.tune = current_tune();
  Carver cv(nullptr);
  for (const fs_work &w : P.items) {
    ItemWs b{};
    carve_item(cv, w, b);
  }
  P.ws_bytes = cv.size();
  build_descriptors(P);
  PL_TRY(upload_descriptors(P, nullptr, true));
  *device_bytes = P.ws_bytes + P.desc_bytes + 512;
  if (stage_bytes) *stage_bytes = P.desc_bytes;
  return FS_OK;
}

fs_status fs_plan_create_in(const fs_work *items, uint32_t count, void *mem, size_t mem_bytes, void *host_stage,
                            size_t stage_bytes, hipStream_t stream, fs_plan **out) {
  clear_error();
  if (!out || (count && !items)) return fail(FS_ERR_INVALID, "items and out must be non-null");
  if (!mem || (reinterpret_cast<uintptr_t>(mem) & 255)) return fail(FS_ERR_ALIGN, "mem must be 256-byte aligned");
  for (uint32_t i = 0; i < count; ++i) PL_TRY(check_item(items[i], i));
  fs_plan *P = new (std::nothrow) fs_plan();
  if (!P) return fail(FS_ERR_NOMEM, "host allocation failed");
  P->external = true;
  P->flags = FS_PLAN_NO_GRAPH;
  P->items.assign(items, items + count);
  P->tune = current_tune();
  (void)hipGetDevice(&P->device);
  Carver cv(nullptr);
  for (const fs_work &w : P->items) {
    ItemWs b{};
    carve_item(cv, w, b);
  }
  P->ws_bytes = cv.size();
  P->d_ws = mem;
  build_descriptors(*P);   // carves the workspace at d_ws
  fs_status st = upload_descriptors(*P, stream, true);
  if (st == FS_OK && P->ws_bytes + P->desc_bytes > mem_bytes)
    st = fail(FS_ERR_WORKSPACE, "plan memory too small: need " + std::to_string(P->ws_bytes + P->desc_bytes));
  if (st == FS_OK && host_stage && stage_bytes < P->desc_bytes)
    st = fail(FS_ERR_WORKSPACE, "host stage too small: need " + std::to_string(P->desc_bytes));
  if (st == FS_OK) {
    P->d_desc = static_cast<uint8_t *>(mem) + P->ws_bytes;
    // flags of the workspace start cleared; descriptors follow
    if (P->ws_bytes) st = hip_ok(hipMemsetAsync(P->d_ws, 0, P->ws_bytes, stream), "plan workspace clear");
  }
  if (st == FS_OK) st = upload_descriptors(*P, stream, false, host_stage);
  if (st != FS_OK) {
    const std::string msg = fs_last_error();
    release(P);
    return fail(st, msg);
  }
  P->gather_grid = gather_grid_for(P->gprefix.back());
  prepare_batch_kernels();
  *out = P;
  return FS_OK;
}

}  // extern "C"
