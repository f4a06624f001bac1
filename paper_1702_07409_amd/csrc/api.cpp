// C ABI entry points of libfs: argument checks, workspace layout, launches.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <set>

#include "fs_internal.h"

namespace fs {

static thread_local std::string g_last_error;

fs_status fail(fs_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}
void clear_error() { g_last_error.clear(); }

const DeviceInfo &device_info(int dev) {
  static std::mutex mu;
  static DeviceInfo info[64];
  static bool have[64] = {false};
  std::lock_guard<std::mutex> lock(mu);
  if (dev < 0 || dev >= 64) return info[0];
  if (!have[dev]) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      info[dev].cu_count = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
      info[dev].max_lds_per_block = v;
    have[dev] = true;
  }
  return info[dev];
}

namespace {
std::mutex g_tune_mu;
fs_tune g_tune = {0, 0, 1, 1, 0, 1, 0, 0};

}  // namespace

fs_tune current_tune() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  return g_tune;
}

// Gather tiling for a graph when the tuning leaves it open (lanes_per_row
// 0).  Sparse graphs (mean degree <= 6) with k <= 8192 read each neighbour
// block in 4 KiB runs; denser ones (the Robust Soliton graphs), and sparse
// ones of more inputs, re-read every input about d times from slices too
// large to stay on chip, so the slice narrows as k grows: W = 4 MiB / k
// (one slice of every input block, k x W bytes, about one XCD's L2),
// within [512 B, 4 KiB].  Measured with the inputs out of the caches, on
// Robust Soliton stripes of 1024 x 256 KiB, 2048 x 128 KiB, 4096 x 64 KiB
// and 8192 x 32 KiB: this width within 0-4 % of the best of 512 B - 4 KiB,
// where 2 MiB / k was up to 16 % slower; on the k = 4096 finite-degree stripe
// 4 KiB slices 14 % faster than 512-byte ones; on the k = 10246 Raptor code
// (mean degree 5.7, 7 KiB blocks) 512-byte slices 0.082 ms against 0.25 ms.
fs_tune tile_for(const fs_tune &t, const fs_graph *g) {
  if (t.lanes_per_row != 0) return t;
  fs_tune r = t;
  const double dbar = g->n ? (double)g->nnz / (double)g->n : 1.0;
  uint64_t w = 4096;
  if (dbar > 6.0 || g->k > 8192) {
    w = (4ull << 20) / std::max<uint32_t>(g->k, 1);
    w = std::min<uint64_t>(4096, std::max<uint64_t>(512, w));
  }
  if (w >= 4096) {
    r.lanes_per_row = 64; r.chunks = 4;
  } else if (w >= 2048) {
    r.lanes_per_row = 64; r.chunks = 2;
  } else if (w >= 1024) {
    r.lanes_per_row = 32; r.chunks = 2;
  } else {
    r.lanes_per_row = 16; r.chunks = 2;
  }
  return r;
}

static bool tune_ok(const fs_tune &t) {
  const bool auto_tile = t.lanes_per_row == 0 && t.chunks == 0;
  const bool lpr = auto_tile || t.lanes_per_row == 8 || t.lanes_per_row == 16 || t.lanes_per_row == 32 ||
                   t.lanes_per_row == 64 ||
                   t.lanes_per_row == 128 || t.lanes_per_row == 256;
  // row-wide tilings (one or two rows per workgroup) take 1 or 2 chunks
  const bool ch = auto_tile || t.chunks == 1 || t.chunks == 2 || (t.chunks == 4 && t.lanes_per_row <= 64);
  return lpr && ch && t.xcd_remap <= 1 && t.nt_store <= 1 && t.replay_prog_global <= 1 && t.encode_slab <= 1 &&
         t.replay_lookahead <= 1 && t.claim_chunk <= 1024;
}

// The device copy of a graph: nine arrays, each 256-byte aligned, in one buffer.
void graph_image_sized(uint32_t k, uint32_t n, uint64_t nnz, uint32_t nseg, uint32_t nheavy, GraphImage &img) {
  const size_t bytes[9] = {((size_t)n + 1) * 4, nnz * 4,  ((size_t)k + 1) * 4,      nnz * 4, ((size_t)nseg + 1) * 4,
                           (size_t)nseg * 4,    (size_t)nheavy * 4, (size_t)nseg, nnz * 4};
  size_t total = 0;
  for (int i = 0; i < 9; ++i) {
    img.parts[i] = {nullptr, bytes[i], total};
    total += (bytes[i] + 255) & ~size_t(255);
  }
  img.total = total + 256;
}

void graph_image(const fs_graph &g, GraphImage &img) {
  graph_image_sized(g.k, g.n, g.nnz, g.nseg, (uint32_t)g.heavy.size(), img);
  img.parts[0].src = g.row_ptr.data();
  img.parts[1].src = g.col.data();
  img.parts[2].src = g.col_ptr.data();
  img.parts[3].src = g.rowidx.data();
  img.parts[4].src = g.seg_ptr.data();
  img.parts[5].src = g.seg_row.data();
  img.parts[6].src = g.heavy.data();
  img.parts[7].src = g.seg_atomic.data();
  img.parts[8].src = g.seg_col.data();
}

void bind_image(fs_graph &g, const GraphImage &img, void *base) {
  uint8_t *p = static_cast<uint8_t *>(base);
  g.d_row_ptr = reinterpret_cast<const int32_t *>(p + img.parts[0].off);
  g.d_col = reinterpret_cast<const int32_t *>(p + img.parts[1].off);
  g.d_col_ptr = reinterpret_cast<const int32_t *>(p + img.parts[2].off);
  g.d_rowidx = reinterpret_cast<const int32_t *>(p + img.parts[3].off);
  g.d_seg_ptr = reinterpret_cast<const int32_t *>(p + img.parts[4].off);
  g.d_seg_row = reinterpret_cast<const int32_t *>(p + img.parts[5].off);
  g.d_heavy = reinterpret_cast<const int32_t *>(p + img.parts[6].off);
  g.d_seg_atomic = reinterpret_cast<const uint8_t *>(p + img.parts[7].off);
  g.d_seg_col = reinterpret_cast<const int32_t *>(p + img.parts[8].off);
}

fs_status check_graph(const fs_graph *g) {
  if (!g) return fail(FS_ERR_INVALID, "graph is null");
  if (!g->d_row_ptr) return fail(FS_ERR_INVALID, "graph has no device copy (host-only and not uploaded)");
  int dev = -1;
  if (const hipError_t e = hipGetDevice(&dev); e != hipSuccess)
    return fail(FS_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev != g->device) return fail(FS_ERR_INVALID, "graph lives on another device");
  return FS_OK;
}

fs_status check_payload(const void *p, uint64_t t, const char *name) {
  if (t == 0 || (t & 15)) return fail(FS_ERR_ALIGN, "t must be a positive multiple of 16");
  if (!p) return fail(FS_ERR_INVALID, std::string(name) + " is null");
  if (reinterpret_cast<uintptr_t>(p) & 15) return fail(FS_ERR_ALIGN, std::string(name) + " is not 16-byte aligned");
  return FS_OK;
}

#define FS_TRY(expr)                  \
  do {                                \
    fs_status _s = (expr);            \
    if (_s != FS_OK) return _s;       \
  } while (0)


void carve_sched(Carver &cv, uint32_t k, SchedBufs &s, bool with_recovered) {
  s.status = cv.take<int32_t>(4);
  s.level_ptr = cv.take<int32_t>((size_t)k + 1);
  s.dp_f = cv.take<int32_t>(k);
  s.dp_g = cv.take<int32_t>(k);
  s.recovered = with_recovered ? cv.take<uint8_t>(k) : nullptr;
}


void carve_repair(Carver &cv, const fs_graph *g, uint64_t t, bool conventional, RepairBufs &b) {
  b.seen = cv.take<uint32_t>((g->n + 31) / 32);
  b.flag = cv.take<int32_t>(4);
  b.sptr = b.sidx = b.roff = b.sout = b.nseg = nullptr;
  b.satomic = nullptr;
  b.seg_cap = 0;
  if (!conventional && g->max_deg > kSegMax) {
    // every row of the graph in pieces of at most 64 edges: its encode segments
    b.seg_cap = std::max<uint32_t>(g->nseg, 1);
    b.sptr = cv.take<int32_t>((size_t)b.seg_cap + 1);
    b.sidx = cv.take<int32_t>(std::max<uint64_t>(g->nnz, 1));
    b.roff = cv.take<int32_t>(g->n);
    b.sout = cv.take<int32_t>(b.seg_cap);
    b.satomic = cv.take<uint8_t>(b.seg_cap);
    b.nseg = cv.take<int32_t>(1);
  }
  b.erased2 = nullptr;
  b.x = nullptr;
  b.sched = SchedBufs{};
  b.peel = PeelJob{};
  b.prog = ProgJob{};
  if (conventional) {
    b.erased2 = cv.take<uint8_t>(g->n);
    carve_sched(cv, g->k, b.sched, true);
    b.peel.k = g->k;
    b.peel.n = g->n;
    peel_carve(cv, b.peel);
    b.prog.k = g->k;
    b.prog.n = g->n;
    prog_carve(cv, b.prog, g->nnz);
    b.x = cv.take<uint8_t>((size_t)g->k * t);
  }
}


void carve_update(Carver &cv, const fs_graph *g, uint64_t t, uint32_t n_ids, UpdateBufs &b) {
  const uint64_t max_pairs = (uint64_t)n_ids * g->max_cdeg;
  b.max_rows = (uint32_t)std::min<uint64_t>(g->n, max_pairs);
  b.seen = cv.take<uint32_t>((g->k + 31) / 32);
  b.cnt = cv.take<int32_t>(g->n);
  b.arow = cv.take<int32_t>(g->n);
  b.aptr = cv.take<int32_t>((size_t)g->n + 1);
  b.asrc = cv.take<int32_t>(std::max<uint64_t>(max_pairs, 1));
  b.n_aff = cv.take<int32_t>(1);
  b.flag = cv.take<int32_t>(1);
  b.delta = cv.take<uint8_t>((size_t)n_ids * t);
}

struct LocalBufs {
  int32_t *chosen, *level, *pos, *item_ptr, *item_col, *item_dst, *lvl_ptr, *meta, *flag;
  unsigned long long *gacc;
  int32_t *rof, *best, *fa, *fb;
  uint32_t *unk;
};

// the XOR lists are bounded by n blocks per lost row
void carve_local(Carver &cv, const fs_graph *g, uint32_t n_lost, LocalBufs &b) {
  const size_t m = std::max<uint32_t>(n_lost, 1);
  b.chosen = cv.take<int32_t>(m);
  b.level = cv.take<int32_t>(m);
  b.pos = cv.take<int32_t>(m);
  b.item_ptr = cv.take<int32_t>((size_t)n_lost + 1);
  b.item_col = cv.take<int32_t>(std::max<uint64_t>((uint64_t)n_lost * g->n, 1));
  b.item_dst = cv.take<int32_t>(m);
  b.lvl_ptr = cv.take<int32_t>((size_t)n_lost + 2);
  b.meta = cv.take<int32_t>(4);
  b.flag = cv.take<int32_t>(4);
  // group peel: at most 2n groups (n - k from the generation, at most n + k added)
  b.gacc = cv.take<unsigned long long>(2ull * g->n + 1);
  b.rof = cv.take<int32_t>((size_t)g->n + 1);
  b.best = cv.take<int32_t>((size_t)g->n + 1);
  b.fa = cv.take<int32_t>(4ull * g->n + 2);
  b.fb = cv.take<int32_t>(4ull * g->n + 2);
  b.unk = cv.take<uint32_t>(((size_t)g->n + 31) / 32);
}

struct PrecodeBufs {
  int32_t *status1, *pair_sym, *pair_chk, *level_ptr, *meta;
};

void carve_precode(Carver &cv, uint32_t k, PrecodeBufs &b) {
  b.status1 = cv.take<int32_t>(4);
  b.pair_sym = cv.take<int32_t>(k);
  b.pair_chk = cv.take<int32_t>(k);
  b.level_ptr = cv.take<int32_t>((size_t)k + 1);
  b.meta = cv.take<int32_t>(4);
}

size_t workspace_bytes(const fs_graph *g, int op, uint64_t t, uint32_t n_items);

SimDiskLayout simdisk_layout_for(const fs_graph *g, uint32_t checks) {
  const int dev = g->device < 0 ? 0 : g->device;
  return simdisk_layout(g->k, g->n, g->max_deg, checks, (size_t)device_info(dev).max_lds_per_block);
}

void carve_simdisk(Carver &cv, const fs_graph *g, uint32_t checks, SimDiskJob &j) {
  const SimDiskLayout L = simdisk_layout_for(g, checks);
  const bool global = (L.mode == kSimDiskGlobal);
  j.binom = cv.take<uint64_t>(65 * 65);
  j.rowinfo = cv.take<uint32_t>(L.image_bytes / 4);
  j.slots = global ? cv.take<uint8_t>((size_t)kSimDiskSlots * L.bytes) : nullptr;
}

size_t workspace_bytes(const fs_graph *g, int op, uint64_t t, uint32_t n_items) {
  Carver cv(nullptr);
  switch (op) {
    case FS_OP_ENCODE: return 0;
    case FS_OP_PEEL: {
      PeelJob j{};
      j.k = g->k;
      j.n = g->n;
      peel_carve(cv, j);
      return cv.size();
    }
    case FS_OP_DECODE: {
      SchedBufs s;
      carve_sched(cv, g->k, s, false);
      PeelJob j{};
      j.k = g->k;
      j.n = g->n;
      peel_carve(cv, j);
      ProgJob pj{};
      pj.k = g->k;
      pj.n = g->n;
      prog_carve(cv, pj, g->nnz);
      return cv.size();
    }
    case FS_OP_REPLAY: {
      ProgJob pj{};
      pj.k = g->k;
      pj.n = g->n;
      prog_carve(cv, pj, g->nnz);
      return cv.size();
    }
    case FS_OP_REPAIR:
    case FS_OP_REPAIR_CONVENTIONAL: {
      RepairBufs b;
      carve_repair(cv, g, t, op == FS_OP_REPAIR_CONVENTIONAL, b);
      return cv.size();
    }
    case FS_OP_UPDATE: {
      UpdateBufs b;
      carve_update(cv, g, t, n_items, b);
      return cv.size();
    }
    case FS_OP_SIM_DISKS: {
      SimDiskJob j{};
      carve_simdisk(cv, g, n_items, j);
      return cv.size();
    }
    case FS_OP_REPAIR_LOCAL: {
      LocalBufs b;
      carve_local(cv, g, n_items, b);
      return cv.size();
    }
    case FS_OP_EXTEND_LOCAL: {
      cv.take<uint32_t>(g->n);
      cv.take<uint8_t>(g->n);
      LocalBufs b;
      carve_local(cv, g, n_items, b);
      return cv.size();
    }
    case FS_OP_DECODE_PRECODED: {
      cv.take<uint8_t>(workspace_bytes(g, FS_OP_DECODE, t, 0));
      PrecodeBufs b;
      carve_precode(cv, g->k, b);
      return cv.size();
    }
    case FS_OP_REPAIR_PRECODED: {
      RepairBufs b;
      carve_repair(cv, g, t, true, b);
      cv.take<uint8_t>(workspace_bytes(g, FS_OP_DECODE_PRECODED, t, 0));
      cv.take<int32_t>(4);
      return cv.size();
    }
    case FS_OP_EXTEND:
    case FS_OP_EXTEND_CONVENTIONAL: {
      const bool conventional = (op == FS_OP_EXTEND_CONVENTIONAL);
      cv.take<uint32_t>(g->n);
      if (conventional) cv.take<uint8_t>(g->n);
      RepairBufs b;
      carve_repair(cv, g, t, conventional, b);
      return cv.size();
    }
  }
  return 0;
}

fs_status check_ws(const fs_graph *g, int op, uint64_t t, uint32_t n_items, void *ws, size_t ws_bytes) {
  const size_t need = workspace_bytes(g, op, t, n_items);
  if (need == 0) return FS_OK;
  if (!ws) return fail(FS_ERR_WORKSPACE, "workspace is null");
  if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(FS_ERR_ALIGN, "workspace must be 256-byte aligned");
  if (ws_bytes < need)
    return fail(FS_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  return FS_OK;
}

PeelJob peel_job(const fs_graph *g, const uint8_t *erased, uint32_t maxit, uint8_t *recovered,
                 int32_t *status, int32_t *level_ptr, int32_t *dp_f, int32_t *dp_g) {
  PeelJob j{};
  j.k = g->k;
  j.n = g->n;
  j.row_ptr = g->d_row_ptr;
  j.col = g->d_col;
  j.col_ptr = g->d_col_ptr;
  j.rowidx = g->d_rowidx;
  j.erased = erased;
  j.maxit = maxit;
  j.recovered = recovered;
  j.status = status;
  j.level_ptr = level_ptr;
  j.dp_f = dp_f;
  j.dp_g = dp_g;
  j.nnz = g->nnz;
  return j;
}

ProgJob prog_job(const fs_graph *g, Carver &cv, const int32_t *status, const int32_t *level_ptr,
                 const int32_t *dp_f, const int32_t *dp_g) {
  ProgJob p{};
  p.k = g->k;
  p.n = g->n;
  p.row_ptr = g->d_row_ptr;
  p.col = g->d_col;
  p.status = status;
  p.level_ptr = level_ptr;
  p.dp_f = dp_f;
  p.dp_g = dp_g;
  prog_carve(cv, p, g->nnz);
  return p;
}

ReplayJob replay_job(const fs_graph *g, const void *c, void *x, uint64_t t, const int32_t *status,
                     const int32_t *level_ptr, const int32_t *dp_f, const int32_t *dp_g) {
  ReplayJob r{};
  r.k = g->k;
  r.n = g->n;
  r.row_ptr = g->d_row_ptr;
  r.col = g->d_col;
  r.c = static_cast<const uint8_t *>(c);
  r.x = static_cast<uint8_t *>(x);
  r.t = t;
  r.status = status;
  r.level_ptr = level_ptr;
  r.dp_f = dp_f;
  r.dp_g = dp_g;
  return r;
}

fs_tune tune_snapshot() { return current_tune(); }

namespace {
// Scratch of the device graph builds, kept per thread and device and grown
// when a build needs more: a hipFree waits for the whole device, so builds
// made while other work runs (a request loop) must not free memory, and
// builds on different threads (each on its own stream) run side by side.
// The buffers live until the process ends.
struct BuildScratch {
  void *buf[64][3] = {};     // slots: before the sizes, after them, thresholds
  size_t bytes[64][3] = {};
};

fs_status build_scratch(int dev, int slot, size_t need, void **out) {
  static thread_local BuildScratch sc;
  if (dev < 0 || dev >= 64) return fail(FS_ERR_INVALID, "device index out of range");
  if (sc.bytes[dev][slot] < need) {
    if (sc.buf[dev][slot]) (void)hipFree(sc.buf[dev][slot]);
    sc.buf[dev][slot] = nullptr;
    sc.bytes[dev][slot] = 0;
    const size_t grow = std::max(need, (size_t)4 << 20);
    if (hipMalloc(&sc.buf[dev][slot], grow) != hipSuccess) return fail(FS_ERR_NOMEM, "graph scratch allocation failed");
    sc.bytes[dev][slot] = grow;
  }
  *out = sc.buf[dev][slot];
  return FS_OK;
}

// Images of device-built graphs come from one memory pool per device that
// keeps freed memory for reuse, so that a build does not wait on the mapping
// of new memory (a request loop builds graphs while other work runs).  Null
// when the pool cannot be made; builds then use hipMalloc.
hipMemPool_t graph_pool(int dev) {
  static std::mutex mu;
  static hipMemPool_t pools[64] = {};
  static bool tried[64] = {};
  if (dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!tried[dev]) {
    tried[dev] = true;
    hipMemPoolProps props = {};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) == hipSuccess) {
      uint64_t keep = UINT64_MAX;
      if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) == hipSuccess) pools[dev] = pool;
      else (void)hipMemPoolDestroy(pool);
    }
    (void)hipGetLastError();
  }
  return pools[dev];
}

// The degree thresholds of the last distribution a thread built with, on
// the host and in its threshold scratch: a request loop builds many graphs
// of one distribution, and RSD has k thresholds.
struct ThresholdCache {
  bool valid = false;
  uint32_t dist = 0, k = 0;
  double c = 0.0, delta = 0.0;
  std::vector<double> finite;
  std::vector<uint64_t> T;
  void *dev = nullptr;
};

fs_status device_thresholds(const fs_graph_params &p, int dev, hipStream_t stream, const uint64_t **T_dev,
                            uint32_t *D) {
  static thread_local ThresholdCache cache[64];
  ThresholdCache &tc = cache[dev];
  bool same = tc.valid && tc.dist == p.dist && tc.k == p.k;
  if (same && p.dist == FS_DIST_RSD) same = tc.c == p.rsd_c && tc.delta == p.rsd_delta;
  if (same && p.dist == FS_DIST_FINITE)
    same = tc.finite.size() == p.finite_dmax && p.finite_w &&
           std::equal(tc.finite.begin(), tc.finite.end(), p.finite_w);
  if (!same) {
    tc.valid = false;
    std::vector<double> w;
    FS_TRY(degree_weights(p, w));
    degree_thresholds(w, tc.T);
    tc.dist = p.dist;
    tc.k = p.k;
    tc.c = p.rsd_c;
    tc.delta = p.rsd_delta;
    if (p.dist == FS_DIST_FINITE) tc.finite.assign(p.finite_w, p.finite_w + p.finite_dmax);
    else tc.finite.clear();
  }
  void *buf = nullptr;
  FS_TRY(build_scratch(dev, 2, tc.T.size() * sizeof(uint64_t), &buf));
  if (!same || buf != tc.dev) {
    // tc.T stays unchanged until the build that uses it has synchronised
    const hipError_t e = hipMemcpyAsync(buf, tc.T.data(), tc.T.size() * sizeof(uint64_t), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return fail(FS_ERR_HIP, std::string("graph thresholds: ") + hipGetErrorString(e));
    tc.dev = buf;
  }
  tc.valid = true;
  *T_dev = static_cast<const uint64_t *>(buf);
  *D = (uint32_t)tc.T.size();
  return FS_OK;
}

void free_graph_memory(fs_graph &g) {
  if (!g.d_base) return;
  if (g.pooled) {
    // work on any stream may still read the image: wait for the device, as
    // hipFree does, then hand the memory back to the pool
    (void)hipDeviceSynchronize();
    (void)hipFreeAsync(g.d_base, nullptr);
    (void)hipStreamSynchronize(nullptr);
  } else {
    (void)hipFree(g.d_base);
  }
  g.d_base = nullptr;
}
}  // namespace

// Device construction (graph_dev.hip): thresholds on the host (kept for the
// next build of the same distribution), then the
// degree pass, one copy of the sizes back (nnz, segments, heavy rows), the
// image allocated to fit, the rows, segments and transpose, and the heavy-row
// list and largest column copied back.
fs_status build_device_graph(const fs_graph_params &p, hipStream_t stream, fs_graph &g) {
  if (p.k < 1 || p.n < 1) return fail(FS_ERR_INVALID, "k and n must be >= 1");
  if (p.k > (1u << 20)) return fail(FS_ERR_INVALID, "k above 2^20 is not supported");
  if (p.reserved != 0) return fail(FS_ERR_INVALID, "reserved field must be 0");
  g.k = p.k;
  g.n = p.n;
  g.params = p;
  g.params.flags = p.flags;
  if (p.dist == FS_DIST_FINITE) {
    g.finite_w.assign(p.finite_w, p.finite_w + p.finite_dmax);
    g.params.finite_w = g.finite_w.data();
  } else {
    g.params.finite_w = nullptr;
  }
  g.host_arrays = false;
  if (const hipError_t e = hipGetDevice(&g.device); e != hipSuccess)
    return fail(FS_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  DevGraphJob J{};
  J.k = p.k;
  J.n = p.n;
  FS_TRY(device_thresholds(p, g.device, stream, &J.T, &J.D));
  J.seed = p.seed;
  J.stripe_key = p.stripe_key;
  Carver sz(nullptr);
  dev_graph_carve(sz, J, J.k, J.n);
  void *scratch = nullptr, *scratch2 = nullptr;
  FS_TRY(build_scratch(g.device, 0, sz.size(), &scratch));
  auto done = [&](fs_status st) { return st; };
  Carver cv(scratch);
  dev_graph_carve(cv, J, J.k, J.n);
  int32_t *row_ptr_tmp = J.row_ptr;
  // the degree pass clears the scalars and the edge count itself
  fs_status st = launch_dev_graph_degrees(J, stream);
  if (st != FS_OK) return done(st);
  int32_t sizes[kScalarWords] = {};
  hipError_t e = hipMemcpyAsync(sizes, J.scalars, sizeof(sizes), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  unsigned long long edges = 0;
  std::memcpy(&edges, sizes + kScalarCount, sizeof(edges));
  if (e != hipSuccess) return done(fail(FS_ERR_HIP, std::string("graph sizes: ") + hipGetErrorString(e)));
  // row_ptr is int32 (its scan wraps past 2^31 edges)
  if (edges >= (unsigned long long)INT32_MAX) return done(fail(FS_ERR_INVALID, "graph has 2^31 or more edges"));
  g.nnz = edges;
  J.nnz = (uint32_t)edges;
  g.max_deg = (uint32_t)sizes[kScalarMaxDeg];
  g.nseg = (uint32_t)sizes[kScalarSegs];
  const uint32_t nheavy = (uint32_t)sizes[kScalarHeavy];
  GraphImage img;
  graph_image_sized(g.k, g.n, g.nnz, g.nseg, nheavy, img);
  if (hipMemPool_t pool = graph_pool(g.device)) {
    g.pooled = hipMallocFromPoolAsync(&g.d_base, img.total, pool, stream) == hipSuccess;
    if (!g.pooled) {
      g.d_base = nullptr;
      (void)hipGetLastError();
    }
  }
  if (!g.d_base && hipMalloc(&g.d_base, img.total) != hipSuccess) {
    g.d_base = nullptr;
    return done(fail(FS_ERR_NOMEM, "device allocation for the graph failed"));
  }
  bind_image(g, img, g.d_base);
  uint8_t *base = static_cast<uint8_t *>(g.d_base);
  J.row_ptr = reinterpret_cast<int32_t *>(base + img.parts[0].off);
  J.col = reinterpret_cast<int32_t *>(base + img.parts[1].off);
  J.col_ptr = reinterpret_cast<int32_t *>(base + img.parts[2].off);
  J.rowidx = reinterpret_cast<int32_t *>(base + img.parts[3].off);
  J.seg_ptr = reinterpret_cast<int32_t *>(base + img.parts[4].off);
  J.seg_row = reinterpret_cast<int32_t *>(base + img.parts[5].off);
  J.heavy = reinterpret_cast<int32_t *>(base + img.parts[6].off);
  J.seg_atomic = base + img.parts[7].off;
  J.seg_col = reinterpret_cast<int32_t *>(base + img.parts[8].off);
  Carver sz2(nullptr);
  dev_graph_carve_rows(sz2, J, J.k, J.n, g.nseg, g.nnz);
  FS_TRY(build_scratch(g.device, 1, sz2.size(), &scratch2));
  Carver cv2(scratch2);
  dev_graph_carve_rows(cv2, J, J.k, J.n, g.nseg, g.nnz);
  J.row_src = row_ptr_tmp;   // copied into the image by the first kernel
  st = launch_dev_graph_rows(J, g.nseg, nheavy, stream);
  if (st != FS_OK) return done(st);
  // the scalars and, after them, the heavy-row list in one copy
  std::vector<int32_t> tail((size_t)kScalarWords + nheavy);
  e = hipMemcpyAsync(tail.data(), J.scalars, tail.size() * sizeof(int32_t), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return done(fail(FS_ERR_HIP, std::string("graph build: ") + hipGetErrorString(e)));
  g.heavy.assign(tail.begin() + kScalarWords, tail.end());
  g.max_cdeg = (uint32_t)tail[kScalarMaxCdeg];
  return done(FS_OK);
}

void repair_pieces_prep(RepairPrepJob &pj, const fs_graph *g, const RepairBufs &b, void *c, uint64_t t) {
  pj.row_ptr = g->d_row_ptr;
  pj.col = g->d_col;
  pj.sptr = b.sptr;
  pj.sidx = b.sidx;
  pj.roff = b.roff;
  pj.sout = b.sout;
  pj.satomic = b.satomic;
  pj.nseg = b.nseg;
  pj.seg_cap = b.seg_cap;
  pj.c = static_cast<uint8_t *>(c);
  pj.t = t;
}

GatherJob repair_pieces_job(const fs_graph *g, const RepairBufs &b, uint32_t n_lost, const void *x, void *c,
                            uint64_t t) {
  GatherJob gj{};
  gj.src = static_cast<const uint8_t *>(x);
  gj.src_stride = t;
  gj.dst = static_cast<uint8_t *>(c);
  gj.dst_stride = t;
  gj.ptr = b.sptr;
  gj.idx = b.sidx;
  gj.out_map = b.sout;
  gj.seg_atomic = b.satomic;
  gj.skip_flag = b.flag;
  // the pieces are counted on the device; at most n_lost rows of the
  // largest degree
  const uint64_t per = ((uint64_t)std::max<uint32_t>(g->max_deg, 1) + kSegMax - 1) / kSegMax;
  gj.nrows = (uint32_t)std::min<uint64_t>(b.seg_cap, (uint64_t)n_lost * per);
  gj.nrows_dev = b.nseg;
  gj.csr_rows = b.seg_cap;
  gj.t = t;
  return gj;
}

fs_launch_info &launch_record() {
  static thread_local fs_launch_info rec = {};
  return rec;
}

}  // namespace fs

using namespace fs;

extern "C" {

const char *fs_version(void) { return "libfs 0.1 (gfx950)"; }

const char *fs_status_string(fs_status s) {
  switch (s) {
    case FS_OK: return "ok";
    case FS_ERR_INVALID: return "invalid argument";
    case FS_ERR_ALIGN: return "misaligned size or pointer";
    case FS_ERR_NOMEM: return "out of memory";
    case FS_ERR_HIP: return "HIP runtime error";
    case FS_ERR_UNSUPPORTED: return "unsupported";
    case FS_ERR_WORKSPACE: return "workspace missing or too small";
  }
  return "unknown status";
}

const char *fs_last_error(void) { return g_last_error.c_str(); }

fs_status fs_last_launch(fs_launch_info *info) {
  clear_error();
  if (!info) return fail(FS_ERR_INVALID, "info must be non-null");
  *info = launch_record();
  return FS_OK;
}

fs_status fs_set_tune(const fs_tune *tune) {
  clear_error();
  std::lock_guard<std::mutex> lock(g_tune_mu);
  if (!tune) {
    g_tune = fs_tune{0, 0, 1, 1, 0, 1, 0, 0};
    return FS_OK;
  }
  if (!tune_ok(*tune)) return fail(FS_ERR_INVALID, "tuning out of range");
  g_tune = *tune;
  return FS_OK;
}

fs_status fs_get_tune(fs_tune *tune) {
  if (!tune) return fail(FS_ERR_INVALID, "tune is null");
  *tune = current_tune();
  return FS_OK;
}

fs_status fs_degree_table(const fs_graph_params *params, uint64_t *T_out, uint32_t cap, uint32_t *D_out) {
  clear_error();
  if (!params) return fail(FS_ERR_INVALID, "params is null");
  std::vector<double> w;
  FS_TRY(degree_weights(*params, w));
  std::vector<uint64_t> T;
  degree_thresholds(w, T);
  if (T_out && cap < T.size()) return fail(FS_ERR_INVALID, "threshold buffer too small");
  if (D_out) *D_out = (uint32_t)T.size();
  if (T_out) std::memcpy(T_out, T.data(), T.size() * sizeof(uint64_t));
  return FS_OK;
}

fs_status fs_graph_build(const fs_graph_params *params, hipStream_t stream, fs_graph **out) {
  clear_error();
  if (!params || !out) return fail(FS_ERR_INVALID, "params and out must be non-null");
  if ((params->flags & FS_GRAPH_HOST_ONLY) && (params->flags & FS_GRAPH_ON_DEVICE))
    return fail(FS_ERR_INVALID, "FS_GRAPH_HOST_ONLY and FS_GRAPH_ON_DEVICE exclude each other");
  if (params->flags & ~3u) return fail(FS_ERR_INVALID, "unknown graph flags");
  fs_graph *g = new (std::nothrow) fs_graph();
  if (!g) return fail(FS_ERR_NOMEM, "host allocation failed");
  if (params->flags & FS_GRAPH_ON_DEVICE) {
    const fs_status st = build_device_graph(*params, stream, *g);
    if (st != FS_OK) {
      free_graph_memory(*g);
      delete g;
      return st;
    }
    *out = g;
    return FS_OK;
  }
  fs_status st = build_host_graph(*params, *g);
  if (st != FS_OK) {
    delete g;
    return st;
  }
  if (!(params->flags & FS_GRAPH_HOST_ONLY)) {
    if (const hipError_t e = hipGetDevice(&g->device); e != hipSuccess) {
      delete g;
      return fail(FS_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    GraphImage img;
    graph_image(*g, img);
    void *base = nullptr;
    if (hipMalloc(&base, img.total) != hipSuccess) {
      delete g;
      return fail(FS_ERR_NOMEM, "device allocation for the graph failed");
    }
    hipError_t e = hipSuccess;
    for (const GraphImage::Part &pt : img.parts)
      if (e == hipSuccess && pt.bytes)
        e = hipMemcpyAsync(static_cast<uint8_t *>(base) + pt.off, pt.src, pt.bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      (void)hipFree(base);
      delete g;
      return fail(FS_ERR_HIP, std::string("graph upload: ") + hipGetErrorString(e));
    }
    g->d_base = base;
    bind_image(*g, img, base);
  }
  *out = g;
  return FS_OK;
}

fs_status fs_graph_image_size(const fs_graph *g, size_t *bytes) {
  clear_error();
  if (!g || !bytes) return fail(FS_ERR_INVALID, "graph and bytes must be non-null");
  if (!g->host_arrays) return fail(FS_ERR_INVALID, "graph was built on the device and has no host image");
  GraphImage img;
  graph_image(*g, img);
  *bytes = img.total;
  return FS_OK;
}

fs_status fs_graph_upload(fs_graph *g, void *dev_mem, size_t bytes, void *host_stage, hipStream_t stream) {
  clear_error();
  if (!g || !dev_mem) return fail(FS_ERR_INVALID, "graph and dev_mem must be non-null");
  if (g->d_row_ptr) return fail(FS_ERR_INVALID, "graph is already on a device");
  if (reinterpret_cast<uintptr_t>(dev_mem) & 255) return fail(FS_ERR_ALIGN, "dev_mem must be 256-byte aligned");
  GraphImage img;
  graph_image(*g, img);
  if (bytes < img.total) return fail(FS_ERR_WORKSPACE, "graph image needs " + std::to_string(img.total) + " bytes");
  int dev = 0;
  if (const hipError_t e = hipGetDevice(&dev); e != hipSuccess)
    return fail(FS_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  uint8_t *dst = static_cast<uint8_t *>(dev_mem);
  hipError_t e = hipSuccess;
  if (host_stage) {
    uint8_t *st = static_cast<uint8_t *>(host_stage);
    for (const GraphImage::Part &pt : img.parts)
      if (pt.bytes) std::memcpy(st + pt.off, pt.src, pt.bytes);
    e = hipMemcpyAsync(dst, st, img.total, hipMemcpyHostToDevice, stream);
  } else {
    for (const GraphImage::Part &pt : img.parts)
      if (e == hipSuccess && pt.bytes) e = hipMemcpyAsync(dst + pt.off, pt.src, pt.bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
  }
  if (e != hipSuccess) return fail(FS_ERR_HIP, std::string("graph upload: ") + hipGetErrorString(e));
  g->device = dev;
  bind_image(*g, img, dev_mem);
  return FS_OK;
}

fs_status fs_graph_info(const fs_graph *g, uint32_t *k, uint32_t *n, uint64_t *nnz, uint32_t *max_degree,
                        uint32_t *max_column_degree) {
  clear_error();
  if (!g) return fail(FS_ERR_INVALID, "graph is null");
  if (k) *k = g->k;
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  if (max_degree) *max_degree = g->max_deg;
  if (max_column_degree) *max_column_degree = g->max_cdeg;
  return FS_OK;
}

fs_status fs_graph_export(const fs_graph *g, int32_t *row_ptr, int32_t *col, int32_t *col_ptr, int32_t *rowidx) {
  clear_error();
  if (!g) return fail(FS_ERR_INVALID, "graph is null");
  if (!g->host_arrays) {
    // built on the device: copy from the device image (synchronous)
    const struct {
      int32_t *dst;
      const int32_t *src;
      size_t count;
    } parts[4] = {{row_ptr, g->d_row_ptr, (size_t)g->n + 1},
                  {col, g->d_col, (size_t)g->nnz},
                  {col_ptr, g->d_col_ptr, (size_t)g->k + 1},
                  {rowidx, g->d_rowidx, (size_t)g->nnz}};
    for (const auto &pt : parts)
      if (pt.dst && pt.count)
        if (const hipError_t e = hipMemcpy(pt.dst, pt.src, pt.count * 4, hipMemcpyDeviceToHost); e != hipSuccess)
          return fail(FS_ERR_HIP, std::string("graph export: ") + hipGetErrorString(e));
    return FS_OK;
  }
  if (row_ptr) std::memcpy(row_ptr, g->row_ptr.data(), g->row_ptr.size() * 4);
  if (col) std::memcpy(col, g->col.data(), g->col.size() * 4);
  if (col_ptr) std::memcpy(col_ptr, g->col_ptr.data(), g->col_ptr.size() * 4);
  if (rowidx) std::memcpy(rowidx, g->rowidx.data(), g->rowidx.size() * 4);
  return FS_OK;
}

void fs_graph_free(fs_graph *g) {
  if (!g) return;
  free_graph_memory(*g);
  delete g;
}

fs_status fs_workspace_size(const fs_graph *g, int op, uint64_t t, uint32_t n_items, size_t *bytes) {
  clear_error();
  if (!g || !bytes) return fail(FS_ERR_INVALID, "graph and bytes must be non-null");
  if (op < FS_OP_ENCODE || op > FS_OP_EXTEND_LOCAL) return fail(FS_ERR_INVALID, "unknown operation");
  if ((op == FS_OP_REPAIR_CONVENTIONAL || op == FS_OP_EXTEND_CONVENTIONAL || op == FS_OP_UPDATE ||
       op == FS_OP_REPAIR_PRECODED) &&
      (t == 0 || (t & 15)))
    return fail(FS_ERR_ALIGN, "t must be a positive multiple of 16");
  *bytes = workspace_bytes(g, op, t, n_items);
  return FS_OK;
}

fs_status fs_encode(const fs_graph *g, const void *x, void *c, uint64_t t, hipStream_t stream) {
  clear_error();
  FS_TRY(check_graph(g));
  FS_TRY(check_payload(x, t, "x"));
  FS_TRY(check_payload(c, t, "c"));
  // rows split into several segments are zeroed, then combined atomically
  if (!g->heavy.empty())
    FS_TRY(launch_zero_rows(static_cast<uint8_t *>(c), g->d_heavy, (uint32_t)g->heavy.size(), t, stream));
  return launch_gather(encode_job(g, x, c, t), tile_for(current_tune(), g), stream);
}

fs_status fs_peel(const fs_graph *g, const uint8_t *erased, uint32_t maxit, uint8_t *recovered, int32_t *status,
                  int32_t *level_ptr, int32_t *dp_f, int32_t *dp_g, void *ws, size_t ws_bytes,
                  hipStream_t stream) {
  clear_error();
  FS_TRY(check_graph(g));
  if (!erased || !recovered || !status || !level_ptr || !dp_f || !dp_g)
    return fail(FS_ERR_INVALID, "peel arrays must be non-null");
  FS_TRY(check_ws(g, FS_OP_PEEL, 0, 0, ws, ws_bytes));
  PeelJob j = peel_job(g, erased, maxit, recovered, status, level_ptr, dp_f, dp_g);
  Carver cv(ws);
  peel_carve(cv, j);
  return launch_peel(j, stream, g->max_deg);
}

fs_status fs_replay(const fs_graph *g, const void *c, const int32_t *status, const int32_t *level_ptr,
                    const int32_t *dp_f, const int32_t *dp_g, void *x, uint64_t t, void *ws, size_t ws_bytes,
                    hipStream_t stream) {
  clear_error();
  FS_TRY(check_graph(g));
  FS_TRY(check_payload(c, t, "c"));
  FS_TRY(check_payload(x, t, "x"));
  if (!status || !level_ptr || !dp_f || !dp_g) return fail(FS_ERR_INVALID, "schedule arrays must be non-null");
  FS_TRY(check_ws(g, FS_OP_REPLAY, t, 0, ws, ws_bytes));
  Carver cv(ws);
  ProgJob p = prog_job(g, cv, status, level_ptr, dp_f, dp_g);
  return launch_replay(replay_job(g, c, x, t, status, level_ptr, dp_f, dp_g), &p, stream);
}

}  // extern "C"

namespace fs {
GatherJob encode_job(const fs_graph *g, const void *x, void *c, uint64_t t) {
  GatherJob j{};
  j.src = static_cast<const uint8_t *>(x);
  j.src_stride = t;
  j.dst = static_cast<uint8_t *>(c);
  j.dst_stride = t;
  j.ptr = g->d_seg_ptr;
  j.idx = g->d_seg_col;
  j.out_map = g->d_seg_row;
  j.seg_atomic = g->heavy.empty() ? nullptr : g->d_seg_atomic;
  j.nrows = g->nseg;
  j.csr_rows = j.nrows;
  j.t = t;
  j.slab_k = g->k;
  return j;
}

void carve_decode(Carver &cv, const fs_graph *g, DecodeBufs &b) {
  carve_sched(cv, g->k, b.sched, false);
  b.peel = PeelJob{};
  b.peel.k = g->k;
  b.peel.n = g->n;
  peel_carve(cv, b.peel);
  b.prog = prog_job(g, cv, b.sched.status, b.sched.level_ptr, b.sched.dp_f, b.sched.dp_g);
}
}  // namespace fs

using namespace fs;


namespace fs {

// The groups of every coded block (the transpose of the check #3 groups)
// and the largest group, on the host.
void checks_transpose(fs_checks *ch) {
  const uint32_t n = ch->n;
  ch->max_group = 0;
  for (size_t q = 0; q + 1 < ch->grp_ptr.size(); ++q)
    ch->max_group = std::max<uint32_t>(ch->max_group, (uint32_t)(ch->grp_ptr[q + 1] - ch->grp_ptr[q]));
  ch->sym_ptr.assign(n + 1, 0);
  for (int32_t v : ch->grp_col) ++ch->sym_ptr[v + 1];
  for (uint32_t u = 0; u < n; ++u) ch->sym_ptr[u + 1] += ch->sym_ptr[u];
  ch->sym_grp.assign(ch->grp_col.size(), 0);
  {
    std::vector<int32_t> fill(ch->sym_ptr.begin(), ch->sym_ptr.end() - 1);
    for (size_t q = 0; q + 1 < ch->grp_ptr.size(); ++q)
      for (int32_t m = ch->grp_ptr[q]; m < ch->grp_ptr[q + 1]; ++m) ch->sym_grp[fill[ch->grp_col[m]]++] = (int32_t)q;
  }
}

// The transpose, then the device copies the local repair reads; the device
// pointers change only on success.
fs_status finish_checks(fs_checks *ch, hipStream_t stream) {
  checks_transpose(ch);
  const std::vector<int32_t> *parts[4] = {&ch->grp_ptr, &ch->grp_col, &ch->sym_ptr, &ch->sym_grp};
  size_t off[4], dtotal = 0;
  for (int q = 0; q < 4; ++q) {
    off[q] = dtotal;
    dtotal += (std::max<size_t>(parts[q]->size(), 1) * sizeof(int32_t) + 255) & ~size_t(255);
  }
  (void)hipGetDevice(&ch->device);
  void *dbase = nullptr;
  if (hipMalloc(&dbase, dtotal) != hipSuccess) return fail(FS_ERR_NOMEM, "device allocation for the checks failed");
  hipError_t e = hipSuccess;
  for (int q = 0; q < 4; ++q)
    if (e == hipSuccess && !parts[q]->empty())
      e = hipMemcpyAsync(static_cast<uint8_t *>(dbase) + off[q], parts[q]->data(), parts[q]->size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    (void)hipFree(dbase);
    return fail(FS_ERR_HIP, std::string("checks upload: ") + hipGetErrorString(e));
  }
  ch->d_base = dbase;
  const int32_t **dst[4] = {&ch->d_grp_ptr, &ch->d_grp_col, &ch->d_sym_ptr, &ch->d_sym_grp};
  for (int q = 0; q < 4; ++q) *dst[q] = reinterpret_cast<const int32_t *>(static_cast<uint8_t *>(dbase) + off[q]);
  return FS_OK;
}

}  // namespace fs

extern "C" {

fs_status fs_decode_plan(const fs_graph *g, const uint8_t *erased, uint32_t maxit, uint8_t *recovered,
                         int32_t *status, void *ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  FS_TRY(check_graph(g));
  if (!erased || !recovered) return fail(FS_ERR_INVALID, "erased and recovered must be non-null");
  FS_TRY(check_ws(g, FS_OP_DECODE, 16, 0, ws, ws_bytes));
  Carver cv(ws);
  DecodeBufs b;
  carve_decode(cv, g, b);
  PeelJob j = peel_job(g, erased, maxit, recovered, b.sched.status, b.sched.level_ptr, b.sched.dp_f,
                       b.sched.dp_g);
  j.acc = b.peel.acc;
  j.best = b.peel.best;
  j.front_a = b.peel.front_a;
  j.front_b = b.peel.front_b;
  j.dlist = b.peel.dlist;
  j.mask = b.peel.mask;
  j.decmask = b.peel.decmask;
  j.status_out = status;   // the peel writes the caller's copy too: no extra dispatch
  return launch_plan(j, b.prog, stream, g->max_deg);
}

fs_status fs_decode_apply(const fs_graph *g, const void *c, void *x, uint64_t t, const void *ws, size_t ws_bytes,
                          hipStream_t stream) {
  clear_error();
  FS_TRY(check_graph(g));
  FS_TRY(check_payload(c, t, "c"));
  FS_TRY(check_payload(x, t, "x"));
  FS_TRY(check_ws(g, FS_OP_DECODE, t, 0, const_cast<void *>(ws), ws_bytes));
  Carver cv(const_cast<void *>(ws));
  DecodeBufs b;
  carve_decode(cv, g, b);
  return launch_replay_prog(replay_job(g, c, x, t, b.sched.status, b.sched.level_ptr, b.sched.dp_f, b.sched.dp_g),
                            &b.prog, stream);
}

fs_status fs_decode(const fs_graph *g, const void *c, const uint8_t *erased, uint32_t maxit, void *x,
                    uint8_t *recovered, int32_t *status, uint64_t t, void *ws, size_t ws_bytes,
                    hipStream_t stream) {
  clear_error();
  FS_TRY(check_graph(g));
  FS_TRY(check_payload(c, t, "c"));
  FS_TRY(check_payload(x, t, "x"));
  if (!erased || !recovered || !status) return fail(FS_ERR_INVALID, "erased, recovered and status must be non-null");
  FS_TRY(fs_decode_plan(g, erased, maxit, recovered, status, ws, ws_bytes, stream));
  return fs_decode_apply(g, c, x, t, ws, ws_bytes, stream);
}

// Repair of the rows lost[0..n_lost) with the workspace already checked; cv
// points at the part of it that carve_repair lays out.
static fs_status precode_encode_impl(const fs_precode *pc, void *x, uint64_t t, const int32_t *skip_flag,
                                     hipStream_t stream);

// The end of a conventional repair: a lost row is rebuilt when all its
// inputs were recovered into b.x, else zero-filled.
static fs_status repair_finish(const fs_graph *g, const uint32_t *lost, uint32_t n_lost, uint8_t *repaired,
                               int32_t *status, RepairBufs &b, GatherJob &gj, hipStream_t stream) {
  RepairCheckJob cj{};
  cj.row_ptr = g->d_row_ptr;
  cj.col = g->d_col;
  cj.n = g->n;
  cj.lost = lost;
  cj.n_lost = n_lost;
  cj.recovered = b.sched.recovered;
  cj.flag = b.flag;
  cj.repaired = repaired;
  cj.status = status;
  FS_TRY(launch_repair_check(cj, stream));
  gj.src = b.x;
  gj.row_ok = repaired;
  return launch_gather(gj, tile_for(current_tune(), g), stream);
}

static fs_status repair_impl(const fs_graph *g, const void *x, void *c, const uint8_t *erased,
                             const uint32_t *lost, uint32_t n_lost, uint8_t *repaired, int32_t *status,
                             uint64_t t, Carver &cv, hipStream_t stream, const fs_precode *pc = nullptr) {
  const bool conventional = (x == nullptr);
  RepairBufs b;
  carve_repair(cv, g, t, conventional, b);
  uint8_t *pws = nullptr;
  int32_t *skip = nullptr;
  const size_t pws_bytes = pc ? workspace_bytes(g, FS_OP_DECODE_PRECODED, t, 0) : 0;
  if (pc) {
    pws = cv.take<uint8_t>(pws_bytes);
    skip = cv.take<int32_t>(4);
  }

  RepairPrepJob pj{};
  pj.n = g->n;
  pj.k = g->k;
  pj.lost = lost;
  pj.n_lost = n_lost;
  pj.erased = erased;
  pj.erased2 = b.erased2;
  pj.seen = b.seen;
  pj.flag = b.flag;
  pj.repaired = repaired;
  pj.status = status;
  // graphs with rows of more than 64 edges repair through pieces
  const bool pieces = !conventional && b.sptr;
  if (pieces) repair_pieces_prep(pj, g, b, c, t);
  FS_TRY(launch_repair_prep(pj, stream));
  if (n_lost == 0) return FS_OK;
  if (pieces) return launch_gather(repair_pieces_job(g, b, n_lost, x, c, t), tile_for(current_tune(), g), stream);

  GatherJob gj{};
  gj.src_stride = t;
  gj.dst = static_cast<uint8_t *>(c);
  gj.dst_stride = t;
  gj.ptr = g->d_row_ptr;
  gj.idx = g->d_col;
  gj.csr_map = lost;
  gj.out_map = reinterpret_cast<const int32_t *>(lost);
  gj.skip_flag = b.flag;
  gj.nrows = n_lost;
  gj.csr_rows = g->n;
  gj.t = t;
  if (!conventional) {
    gj.src = static_cast<const uint8_t *>(x);
    return launch_gather(gj, tile_for(current_tune(), g), stream);
  }
  if (pc) {
    // two-stage decode of everything, then the parity again when the data is complete
    FS_TRY(fs_decode_precoded(g, pc, c, b.erased2, 0, b.x, b.sched.recovered, b.sched.status, t, pws, pws_bytes,
                              stream));
    FS_TRY(launch_parity_known(b.sched.status, b.sched.recovered, pc->b, pc->k, b.flag, skip, stream));
    FS_TRY(precode_encode_impl(pc, b.x, t, skip, stream));
    return repair_finish(g, lost, n_lost, repaired, status, b, gj, stream);
  }
  PeelJob j = peel_job(g, b.erased2, 0, b.sched.recovered, b.sched.status, b.sched.level_ptr, b.sched.dp_f,
                       b.sched.dp_g);
  j.acc = b.peel.acc;
  j.best = b.peel.best;
  j.front_a = b.peel.front_a;
  j.front_b = b.peel.front_b;
  j.dlist = b.peel.dlist;
  j.mask = b.peel.mask;
  j.decmask = b.peel.decmask;
  j.skip_flag = b.flag;
  FS_TRY(launch_peel(j, stream, g->max_deg));
  ReplayJob r = replay_job(g, c, b.x, t, b.sched.status, b.sched.level_ptr, b.sched.dp_f, b.sched.dp_g);
  r.skip_flag = b.flag;
  ProgJob p = b.prog;
  p.n = g->n;
  p.row_ptr = g->d_row_ptr;
  p.col = g->d_col;
  p.status = b.sched.status;
  p.level_ptr = b.sched.level_ptr;
  p.dp_f = b.sched.dp_f;
  p.dp_g = b.sched.dp_g;
  p.skip_flag = b.flag;
  FS_TRY(launch_replay(r, &p, stream));
  return repair_finish(g, lost, n_lost, repaired, status, b, gj, stream);
}

fs_status fs_repair(const fs_graph *g, const void *x, void *c, const uint8_t *erased, const uint32_t *lost,
                    uint32_t n_lost, uint8_t *repaired, int32_t *status, uint64_t t, void *ws, size_t ws_bytes,
                    hipStream_t stream) {
  clear_error();
  FS_TRY(check_graph(g));
  FS_TRY(check_payload(c, t, "c"));
  if (x) FS_TRY(check_payload(x, t, "x"));
  if ((n_lost && (!lost || !repaired)) || !status)
    return fail(FS_ERR_INVALID, "lost, repaired and status must be non-null");
  const int op = x ? FS_OP_REPAIR : FS_OP_REPAIR_CONVENTIONAL;
  FS_TRY(check_ws(g, op, t, n_lost, ws, ws_bytes));
  Carver cv(ws);
  return repair_impl(g, x, c, erased, lost, n_lost, repaired, status, t, cv, stream);
}

fs_status fs_extend(const fs_graph *g, uint32_t n_old, const void *x, void *c, const uint8_t *erased,
                    uint8_t *made, int32_t *status, uint64_t t, void *ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  FS_TRY(check_graph(g));
  FS_TRY(check_payload(c, t, "c"));
  if (x) FS_TRY(check_payload(x, t, "x"));
  if (n_old > g->n) return fail(FS_ERR_INVALID, "n_old exceeds the rows of the graph");
  const uint32_t n_new = g->n - n_old;
  if ((n_new && !made) || !status) return fail(FS_ERR_INVALID, "made and status must be non-null");
  const int op = x ? FS_OP_EXTEND : FS_OP_EXTEND_CONVENTIONAL;
  FS_TRY(check_ws(g, op, t, 0, ws, ws_bytes));
  Carver cv(ws);
  ExtendPrepJob ej{};
  ej.n = g->n;
  ej.n_old = n_old;
  ej.erased = erased;
  ej.ids = cv.take<uint32_t>(g->n);
  ej.erased_full = x ? nullptr : cv.take<uint8_t>(g->n);
  FS_TRY(launch_extend_prep(ej, stream));
  return repair_impl(g, x, c, ej.erased_full, ej.ids, n_new, made, status, t, cv, stream);
}

fs_status fs_update(const fs_graph *g, void *x, void *c, const uint32_t *ids, uint32_t n_ids,
                    const void *new_blocks, int32_t *status, uint64_t t, void *ws, size_t ws_bytes,
                    hipStream_t stream) {
  clear_error();
  FS_TRY(check_graph(g));
  FS_TRY(check_payload(x, t, "x"));
  FS_TRY(check_payload(c, t, "c"));
  if (n_ids) {
    FS_TRY(check_payload(new_blocks, t, "new_blocks"));
    if (!ids) return fail(FS_ERR_INVALID, "ids is null");
  }
  if (!status) return fail(FS_ERR_INVALID, "status is null");
  FS_TRY(check_ws(g, FS_OP_UPDATE, t, n_ids, ws, ws_bytes));
  Carver cv(ws);
  UpdateBufs b;
  carve_update(cv, g, t, n_ids, b);
  UpdatePlanJob pj{};
  pj.k = g->k;
  pj.n = g->n;
  pj.col_ptr = g->d_col_ptr;
  pj.rowidx = g->d_rowidx;
  pj.ids = ids;
  pj.n_ids = n_ids;
  pj.seen = b.seen;
  pj.cnt = b.cnt;
  pj.arow = b.arow;
  pj.aptr = b.aptr;
  pj.asrc = b.asrc;
  pj.n_aff = b.n_aff;
  pj.flag = b.flag;
  pj.status = status;
  FS_TRY(launch_update_plan(pj, stream));
  if (n_ids == 0) return FS_OK;
  UpdateDeltaJob dj{};
  dj.x = static_cast<uint8_t *>(x);
  dj.new_blocks = static_cast<const uint8_t *>(new_blocks);
  dj.delta = b.delta;
  dj.ids = ids;
  dj.n_ids = n_ids;
  dj.t = t;
  dj.flag = b.flag;
  FS_TRY(launch_update_delta(dj, stream));
  GatherJob gj{};
  gj.src = b.delta;
  gj.src_stride = t;
  gj.dst = static_cast<uint8_t *>(c);
  gj.dst_stride = t;
  gj.ptr = b.aptr;
  gj.idx = b.asrc;
  gj.out_map = b.arow;
  gj.nrows_dev = b.n_aff;
  gj.skip_flag = b.flag;
  gj.nrows = b.max_rows;
  gj.csr_rows = b.max_rows;
  gj.t = t;
  gj.accumulate = 1;
  return launch_gather(gj, tile_for(current_tune(), g), stream);
}

static fs_status sim_disks_impl(const fs_graph *g, const fs_precode *pc, uint32_t s, uint32_t f, uint64_t first,
                                uint64_t count, uint32_t maxit, int32_t *result, void *ws, size_t ws_bytes,
                                hipStream_t stream) {
  clear_error();
  FS_TRY(check_graph(g));
  if (pc) {
    if (!pc->d_base) return fail(FS_ERR_INVALID, "precode was built host-only");
    if (pc->k != g->k) return fail(FS_ERR_INVALID, "the graph's k differs from the precode's");
  }
  if (s < 1 || s > 64 || s > g->n) return fail(FS_ERR_INVALID, "s must be in [1, min(64, n)]");
  if (f > s) return fail(FS_ERR_INVALID, "f exceeds s");
  // C(s, f) by the multiplicative formula, exact for s <= 64 in 128-bit
  unsigned __int128 total = 1;
  for (uint32_t i = 1; i <= f; ++i) total = total * (s - f + i) / i;
  if (first > (uint64_t)total || count > (uint64_t)total - first)
    return fail(FS_ERR_INVALID, "combination ranks beyond C(s, f) = " + std::to_string((uint64_t)total));
  if (count && !result) return fail(FS_ERR_INVALID, "result is null");
  const uint32_t checks = pc ? pc->m : 0;
  FS_TRY(check_ws(g, FS_OP_SIM_DISKS, 0, checks, ws, ws_bytes));
  Carver cv(ws);
  SimDiskJob j{};
  carve_simdisk(cv, g, checks, j);
  j.k = g->k;
  j.n = g->n;
  j.s = s;
  j.f = f;
  j.maxit = maxit;
  j.first = first;
  j.count = count;
  j.row_ptr = g->d_row_ptr;
  j.col = g->d_col;
  j.col_ptr = g->d_col_ptr;
  j.rowidx = g->d_rowidx;
  j.result = result;
  if (pc) {
    j.pc_b = pc->b;
    j.pc_m = pc->m;
    j.chk_ptr = pc->d_chk_ptr;
    j.chk_col = pc->d_chk_col;
    j.sym_ptr = pc->d_sym_ptr;
    j.sym_chk = pc->d_sym_chk;
  }
  return launch_simdisk(j, simdisk_layout_for(g, checks), stream);
}

fs_status fs_sim_disks(const fs_graph *g, uint32_t s, uint32_t f, uint64_t first, uint64_t count,
                       uint32_t maxit, int32_t *result, void *ws, size_t ws_bytes, hipStream_t stream) {
  return sim_disks_impl(g, nullptr, s, f, first, count, maxit, result, ws, ws_bytes, stream);
}

fs_status fs_sim_disks_precoded(const fs_graph *g, const fs_precode *pc, uint32_t s, uint32_t f, uint64_t first,
                                uint64_t count, uint32_t maxit, int32_t *result, void *ws, size_t ws_bytes,
                                hipStream_t stream) {
  if (!pc) {
    clear_error();
    return fail(FS_ERR_INVALID, "precode is null");
  }
  return sim_disks_impl(g, pc, s, f, first, count, maxit, result, ws, ws_bytes, stream);
}

fs_status fs_precode_build(uint32_t b, uint32_t k, int host_only, hipStream_t stream, fs_precode **out) {
  clear_error();
  if (!out) return fail(FS_ERR_INVALID, "out is null");
  *out = nullptr;
  fs_precode *pc = new (std::nothrow) fs_precode();
  if (!pc) return fail(FS_ERR_NOMEM, "host allocation failed");
  fs_status st = build_precode_host(b, k, *pc);
  if (st != FS_OK) {
    delete pc;
    return st;
  }
  if (!host_only) {
    if (const hipError_t e = hipGetDevice(&pc->device); e != hipSuccess) {
      delete pc;
      return fail(FS_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    const std::vector<int32_t> *parts[6] = {&pc->enc_ptr, &pc->enc_col, &pc->chk_ptr,
                                            &pc->chk_col, &pc->sym_ptr, &pc->sym_chk};
    size_t off[6], total = 0;
    for (int i = 0; i < 6; ++i) {
      off[i] = total;
      total += (parts[i]->size() * sizeof(int32_t) + 255) & ~size_t(255);
    }
    void *base = nullptr;
    if (hipMalloc(&base, total) != hipSuccess) {
      delete pc;
      return fail(FS_ERR_NOMEM, "device allocation for the precode failed");
    }
    hipError_t e = hipSuccess;
    for (int i = 0; i < 6; ++i)
      if (e == hipSuccess && !parts[i]->empty())
        e = hipMemcpyAsync(static_cast<uint8_t *>(base) + off[i], parts[i]->data(), parts[i]->size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      (void)hipFree(base);
      delete pc;
      return fail(FS_ERR_HIP, std::string("precode upload: ") + hipGetErrorString(e));
    }
    pc->d_base = base;
    const int32_t **dst[6] = {&pc->d_enc_ptr, &pc->d_enc_col, &pc->d_chk_ptr,
                              &pc->d_chk_col, &pc->d_sym_ptr, &pc->d_sym_chk};
    for (int i = 0; i < 6; ++i) *dst[i] = reinterpret_cast<const int32_t *>(static_cast<uint8_t *>(base) + off[i]);
  }
  *out = pc;
  return FS_OK;
}

fs_status fs_precode_info(const fs_precode *pc, uint32_t *b, uint32_t *k, uint32_t *p, uint32_t *kp, uint32_t *jp) {
  clear_error();
  if (!pc) return fail(FS_ERR_INVALID, "precode is null");
  if (b) *b = pc->b;
  if (k) *k = pc->k;
  if (p) *p = pc->p;
  if (kp) *kp = pc->kp;
  if (jp) *jp = pc->jp;
  return FS_OK;
}

fs_status fs_precode_export(const fs_precode *pc, int32_t *row_ptr, int32_t *col) {
  clear_error();
  if (!pc || !row_ptr || !col) return fail(FS_ERR_INVALID, "precode, row_ptr and col must be non-null");
  std::copy(pc->enc_ptr.begin(), pc->enc_ptr.end(), row_ptr);
  std::copy(pc->enc_col.begin(), pc->enc_col.end(), col);
  return FS_OK;
}

void fs_precode_free(fs_precode *pc) {
  if (!pc) return;
  if (pc->d_base) (void)hipFree(pc->d_base);
  delete pc;
}

static fs_status check_precode(const fs_precode *pc) {
  if (!pc) return fail(FS_ERR_INVALID, "precode is null");
  if (!pc->d_base) return fail(FS_ERR_INVALID, "precode was built host-only");
  return FS_OK;
}

fs_status fs_precode_encode(const fs_precode *pc, void *x, uint64_t t, hipStream_t stream) {
  clear_error();
  FS_TRY(check_precode(pc));
  FS_TRY(check_payload(x, t, "x"));
  return precode_encode_impl(pc, x, t, nullptr, stream);
}

// The parity block rows of the precode as gathers (skip_flag: as GatherJob's).
// A launch has only p rows, so 1 KiB slices by default give it more items:
// on the k = 10246 code (p = 109, 7 KiB blocks) the three launches took
// 0.057 ms against 0.086 ms with 4 KiB slices.
static fs_status precode_encode_impl(const fs_precode *pc, void *x, uint64_t t, const int32_t *skip_flag,
                                     hipStream_t stream) {
  fs_tune tune = current_tune();
  if (tune.lanes_per_row == 0) {
    tune.lanes_per_row = 64;
    tune.chunks = 1;
  }
  for (uint32_t j = 0; j < pc->jp; ++j) {
    GatherJob gj{};
    gj.src = static_cast<const uint8_t *>(x);
    gj.src_stride = t;
    gj.dst = static_cast<uint8_t *>(x) + (uint64_t)(pc->b + j * pc->p) * t;
    gj.dst_stride = t;
    gj.ptr = pc->d_enc_ptr + (size_t)j * pc->p;
    gj.idx = pc->d_enc_col;
    gj.nrows = pc->p;
    gj.csr_rows = pc->p;
    gj.t = t;
    gj.skip_flag = skip_flag;
    FS_TRY(launch_gather(gj, tune, stream));
  }
  return FS_OK;
}

fs_status fs_repair_precoded(const fs_graph *g, const fs_precode *pc, void *c, const uint8_t *erased,
                             const uint32_t *lost, uint32_t n_lost, uint8_t *repaired, int32_t *status, uint64_t t,
                             void *ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  FS_TRY(check_graph(g));
  FS_TRY(check_precode(pc));
  if (pc->k != g->k) return fail(FS_ERR_INVALID, "the graph's k differs from the precode's");
  FS_TRY(check_payload(c, t, "c"));
  if ((n_lost && (!lost || !repaired)) || !status)
    return fail(FS_ERR_INVALID, "lost, repaired and status must be non-null");
  FS_TRY(check_ws(g, FS_OP_REPAIR_PRECODED, t, n_lost, ws, ws_bytes));
  Carver cv(ws);
  return repair_impl(g, nullptr, c, erased, lost, n_lost, repaired, status, t, cv, stream, pc);
}

fs_status fs_decode_precoded(const fs_graph *g, const fs_precode *pc, const void *c, const uint8_t *erased,
                             uint32_t maxit, void *x, uint8_t *recovered, int32_t *status, uint64_t t, void *ws,
                             size_t ws_bytes, hipStream_t stream) {
  clear_error();
  FS_TRY(check_graph(g));
  FS_TRY(check_precode(pc));
  if (pc->k != g->k) return fail(FS_ERR_INVALID, "the graph's k differs from the precode's");
  if (!erased || !recovered || !status) return fail(FS_ERR_INVALID, "erased, recovered and status must be non-null");
  FS_TRY(check_payload(c, t, "c"));
  FS_TRY(check_payload(x, t, "x"));
  const int dev = g->device < 0 ? 0 : g->device;
  if (precode_peel_lds(pc->k, pc->m) > (size_t)device_info(dev).max_lds_per_block)
    return fail(FS_ERR_UNSUPPORTED, "the precode's check state exceeds one workgroup's LDS");
  FS_TRY(check_ws(g, FS_OP_DECODE_PRECODED, t, 0, ws, ws_bytes));
  const size_t dec = workspace_bytes(g, FS_OP_DECODE, t, 0);
  Carver cv(ws);
  uint8_t *dws = cv.take<uint8_t>(dec);
  PrecodeBufs b;
  carve_precode(cv, g->k, b);
  FS_TRY(fs_decode(g, c, erased, maxit, x, recovered, b.status1, t, dws, dec, stream));
  PrecodePeelJob pj{};
  pj.b = pc->b;
  pj.k = pc->k;
  pj.m = pc->m;
  pj.chk_ptr = pc->d_chk_ptr;
  pj.chk_col = pc->d_chk_col;
  pj.sym_ptr = pc->d_sym_ptr;
  pj.sym_chk = pc->d_sym_chk;
  pj.recovered = recovered;
  pj.status1 = b.status1;
  pj.status = status;
  pj.pair_sym = b.pair_sym;
  pj.pair_chk = b.pair_chk;
  pj.level_ptr = b.level_ptr;
  pj.meta = b.meta;
  FS_TRY(launch_precode_peel(pj, stream));
  PrecodeReplayJob rj{};
  rj.x = static_cast<uint8_t *>(x);
  rj.t = t;
  rj.chk_ptr = pc->d_chk_ptr;
  rj.chk_col = pc->d_chk_col;
  rj.pair_sym = b.pair_sym;
  rj.pair_chk = b.pair_chk;
  rj.level_ptr = b.level_ptr;
  rj.meta = b.meta;
  return launch_precode_replay(rj, stream);
}

fs_status fs_checks_generate(const fs_graph *g, uint32_t max_sweeps, hipStream_t stream, fs_checks **out) {
  clear_error();
  FS_TRY(check_graph(g));
  if (!out) return fail(FS_ERR_INVALID, "out is null");
  *out = nullptr;
  const uint32_t k = g->k, n = g->n, kw = (k + 31) / 32, nw = (n + 31) / 32;
  const size_t b_bytes = 4ull * n * kw, l_bytes = 4ull * n * nw, w_bytes = 4ull * n, r_bytes = 4ull * k * nw;
  const size_t o_l = (b_bytes + 255) & ~size_t(255), o_w = o_l + ((l_bytes + 255) & ~size_t(255)),
               o_r = o_w + ((w_bytes + 255) & ~size_t(255)), o_m = o_r + ((r_bytes + 255) & ~size_t(255)),
               total = o_m + 256;
  if (4ull * (kw + nw + g->max_deg) + 64 > 160ull * 1024)
    return fail(FS_ERR_UNSUPPORTED, "check generation keeps a column of B and of L in LDS: k + n too large");
  void *scratch = nullptr;
  if (hipMalloc(&scratch, total) != hipSuccess) return fail(FS_ERR_NOMEM, "device allocation for the checks failed");
  uint8_t *base = static_cast<uint8_t *>(scratch);
  CgaJob j{};
  j.k = k;
  j.n = n;
  j.kw = kw;
  j.nw = nw;
  j.max_sweeps = max_sweeps;
  j.max_w = g->max_deg;
  j.row_ptr = g->d_row_ptr;
  j.col = g->d_col;
  j.col_ptr = g->d_col_ptr;
  j.rowidx = g->d_rowidx;
  j.bcol = reinterpret_cast<uint32_t *>(base);
  j.lcol = reinterpret_cast<uint32_t *>(base + o_l);
  j.w = reinterpret_cast<uint32_t *>(base + o_w);
  j.rrow = reinterpret_cast<uint32_t *>(base + o_r);
  j.meta = reinterpret_cast<int32_t *>(base + o_m);
  std::vector<uint32_t> hb((size_t)n * kw), hl((size_t)n * nw), hw(n);
  int32_t meta[2] = {0, 0};
  fs_status st = run_cga(j, stream);
  hipError_t e = hipSuccess;
  if (st == FS_OK) {
    e = hipMemcpyAsync(hb.data(), j.bcol, b_bytes, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hl.data(), j.lcol, l_bytes, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hw.data(), j.w, w_bytes, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(meta, j.meta, sizeof(meta), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
  }
  (void)hipFree(scratch);
  if (st != FS_OK) return st;
  if (e != hipSuccess) return fail(FS_ERR_HIP, std::string("check generation: ") + hipGetErrorString(e));
  fs_checks *ch = new (std::nothrow) fs_checks();
  if (!ch) return fail(FS_ERR_NOMEM, "host allocation failed");
  ch->k = k;
  ch->n = n;
  ch->sweeps = (uint32_t)meta[0];
  ch->zero_columns = (uint32_t)meta[1];
  // check #3 groups (weight zero), smallest first, ties by column; check #2
  // equations (weight one), the first column per input
  struct Grp {
    uint32_t size, col;
  };
  std::vector<Grp> groups;
  std::vector<int32_t> c2_of(k, -1);
  auto members = [&](uint32_t col, std::vector<int32_t> &dst) {
    const uint32_t *l = hl.data() + (size_t)col * nw;
    for (uint32_t q = 0; q < nw; ++q)
      for (uint32_t x = l[q]; x; x &= x - 1) dst.push_back((int32_t)(32 * q + (uint32_t)__builtin_ctz(x)));
  };
  for (uint32_t c = 0; c < n; ++c) {
    if (hw[c] == 0) {
      uint32_t size = 0;
      for (uint32_t q = 0; q < nw; ++q) size += (uint32_t)__builtin_popcount(hl[(size_t)c * nw + q]);
      groups.push_back({size, c});
    } else if (hw[c] == 1) {
      const uint32_t *b = hb.data() + (size_t)c * kw;
      for (uint32_t q = 0; q < kw; ++q)
        if (b[q]) {
          const uint32_t i = 32 * q + (uint32_t)__builtin_ctz(b[q]);
          if (i < k && c2_of[i] < 0) c2_of[i] = (int32_t)c;
          break;
        }
    }
  }
  std::stable_sort(groups.begin(), groups.end(), [](const Grp &a, const Grp &b) { return a.size < b.size; });
  ch->grp_ptr.assign(1, 0);
  for (const Grp &gr : groups) {
    members(gr.col, ch->grp_col);
    ch->grp_ptr.push_back((int32_t)ch->grp_col.size());
    ch->max_group = std::max(ch->max_group, gr.size);
  }
  ch->c2_ptr.assign(1, 0);
  for (uint32_t i = 0; i < k; ++i)
    if (c2_of[i] >= 0) {
      ch->c2_input.push_back((int32_t)i);
      members((uint32_t)c2_of[i], ch->c2_col);
      ch->c2_ptr.push_back((int32_t)ch->c2_col.size());
    }
  const fs_status fin = finish_checks(ch, stream);
  if (fin != FS_OK) {
    delete ch;
    return fin;
  }
  *out = ch;
  return FS_OK;
}

fs_status fs_checks_info(const fs_checks *ch, uint32_t *n_check2, uint32_t *n_check3, uint32_t *sweeps,
                         uint32_t *zero_columns, uint64_t *check2_entries, uint64_t *check3_entries) {
  clear_error();
  if (!ch) return fail(FS_ERR_INVALID, "checks is null");
  if (n_check2) *n_check2 = (uint32_t)ch->c2_input.size();
  if (n_check3) *n_check3 = (uint32_t)(ch->grp_ptr.size() - 1);
  if (sweeps) *sweeps = ch->sweeps;
  if (zero_columns) *zero_columns = ch->zero_columns;
  if (check2_entries) *check2_entries = ch->c2_col.size();
  if (check3_entries) *check3_entries = ch->grp_col.size();
  return FS_OK;
}

fs_status fs_checks_export(const fs_checks *ch, int32_t *c3_ptr, int32_t *c3_col, int32_t *c2_input, int32_t *c2_ptr,
                           int32_t *c2_col) {
  clear_error();
  if (!ch || !c3_ptr || !c3_col || !c2_input || !c2_ptr || !c2_col)
    return fail(FS_ERR_INVALID, "checks and every array must be non-null");
  std::copy(ch->grp_ptr.begin(), ch->grp_ptr.end(), c3_ptr);
  std::copy(ch->grp_col.begin(), ch->grp_col.end(), c3_col);
  std::copy(ch->c2_input.begin(), ch->c2_input.end(), c2_input);
  std::copy(ch->c2_ptr.begin(), ch->c2_ptr.end(), c2_ptr);
  std::copy(ch->c2_col.begin(), ch->c2_col.end(), c2_col);
  return FS_OK;
}

fs_status fs_checks_serialize(const fs_checks *ch, int32_t *out, uint64_t cap, uint64_t *len) {
  clear_error();
  if (!ch || !len) return fail(FS_ERR_INVALID, "checks and len must be non-null");
  const uint64_t ngroups = ch->grp_ptr.empty() ? 0 : ch->grp_ptr.size() - 1;
  const uint64_t need = 3ull * ch->c2_input.size() + ch->c2_col.size() + 2ull * ngroups + ch->grp_col.size();
  if (out) {
    if (cap < need) return fail(FS_ERR_INVALID, "the output holds fewer integers than the check data");
    uint64_t p = 0;
    for (size_t q = 0; q < ch->c2_input.size(); ++q) {
      out[p++] = 1;
      out[p++] = ch->c2_input[q];
      out[p++] = ch->c2_ptr[q + 1] - ch->c2_ptr[q];
      for (int32_t m = ch->c2_ptr[q]; m < ch->c2_ptr[q + 1]; ++m) out[p++] = ch->c2_col[m];
    }
    for (uint64_t q = 0; q < ngroups; ++q) {
      out[p++] = 0;
      out[p++] = ch->grp_ptr[q + 1] - ch->grp_ptr[q];
      for (int32_t m = ch->grp_ptr[q]; m < ch->grp_ptr[q + 1]; ++m) out[p++] = ch->grp_col[m];
    }
  }
  *len = need;
  return FS_OK;
}

fs_status fs_checks_load(const fs_graph *g, const int32_t *data, uint64_t len, hipStream_t stream,
                         fs_checks **out) {
  clear_error();
  FS_TRY(check_graph(g));
  if (!out || (len && !data)) return fail(FS_ERR_INVALID, "out and data must be non-null");
  *out = nullptr;
  const uint32_t k = g->k, n = g->n;
  struct Grp {
    std::vector<int32_t> m;
  };
  std::vector<Grp> groups;
  std::vector<std::vector<int32_t>> c2(k);
  std::vector<uint8_t> c2_seen(k, 0);
  uint64_t p = 0;
  auto members = [&](uint64_t at, int64_t L, std::vector<int32_t> &dst) -> bool {
    if (L < 0 || at + (uint64_t)L > len) return false;
    for (int64_t q = 0; q < L; ++q) {
      const int32_t v = data[at + q];
      if (v < 0 || (uint32_t)v >= n) return false;
      dst.push_back(v);
    }
    std::sort(dst.begin(), dst.end());
    return true;
  };
  while (p < len) {
    const int32_t flag = data[p];
    if (flag == 1) {
      if (p + 3 > len) return fail(FS_ERR_INVALID, "check data: a check #2 record runs past the end");
      const int32_t i = data[p + 1], L = data[p + 2];
      if (i < 0 || (uint32_t)i >= k) return fail(FS_ERR_INVALID, "check data: input index out of range");
      std::vector<int32_t> m;
      if (!members(p + 3, L, m)) return fail(FS_ERR_INVALID, "check data: a check #2 record is past the end or out of range");
      if (!c2_seen[i]) {
        c2_seen[i] = 1;
        c2[i] = std::move(m);
      }
      p += 3 + (uint64_t)L;
    } else if (flag == 0) {
      if (p + 2 > len) return fail(FS_ERR_INVALID, "check data: a check #3 record runs past the end");
      const int32_t L = data[p + 1];
      Grp gr;
      if (!members(p + 2, L, gr.m)) return fail(FS_ERR_INVALID, "check data: a check #3 record is past the end or out of range");
      groups.push_back(std::move(gr));
      p += 2 + (uint64_t)L;
    } else {
      return fail(FS_ERR_INVALID, "check data: unknown record flag");
    }
  }
  // the repair engine takes the smallest groups first (ties in file order)
  std::stable_sort(groups.begin(), groups.end(), [](const Grp &a, const Grp &b) { return a.m.size() < b.m.size(); });
  fs_checks *ch = new (std::nothrow) fs_checks();
  if (!ch) return fail(FS_ERR_NOMEM, "host allocation failed");
  ch->k = k;
  ch->n = n;
  ch->sweeps = 0;
  ch->zero_columns = (uint32_t)groups.size();
  ch->grp_ptr.assign(1, 0);
  for (const Grp &gr : groups) {
    ch->grp_col.insert(ch->grp_col.end(), gr.m.begin(), gr.m.end());
    ch->grp_ptr.push_back((int32_t)ch->grp_col.size());
  }
  ch->c2_ptr.assign(1, 0);
  for (uint32_t i = 0; i < k; ++i)
    if (c2_seen[i]) {
      ch->c2_input.push_back((int32_t)i);
      ch->c2_col.insert(ch->c2_col.end(), c2[i].begin(), c2[i].end());
      ch->c2_ptr.push_back((int32_t)ch->c2_col.size());
    }
  const fs_status fin = finish_checks(ch, stream);
  if (fin != FS_OK) {
    delete ch;
    return fin;
  }
  *out = ch;
  return FS_OK;
}

fs_status fs_checks_add_groups(fs_checks *ch, const fs_graph *g, const fs_precode *pc, hipStream_t stream,
                               uint32_t *added) {
  clear_error();
  FS_TRY(check_graph(g));
  if (!ch) return fail(FS_ERR_INVALID, "checks is null");
  if (ch->n != g->n || ch->k != g->k) return fail(FS_ERR_INVALID, "the checks belong to another graph shape");
  if (pc) {
    FS_TRY(check_precode(pc));
    if (pc->k != g->k) return fail(FS_ERR_INVALID, "the precode's k differs from the graph's");
  }
  // check #2 set of every input (-1: none)
  std::vector<int32_t> c2_of(g->k, -1);
  for (size_t q = 0; q < ch->c2_input.size(); ++q) c2_of[ch->c2_input[q]] = (int32_t)q;
  auto set_of = [&](int32_t i, std::vector<int32_t> &dst) {
    const int32_t q = c2_of[i];
    dst.assign(ch->c2_col.begin() + ch->c2_ptr[q], ch->c2_col.begin() + ch->c2_ptr[q + 1]);
  };
  // symmetric difference of two ascending sets
  auto sym_xor = [](const std::vector<int32_t> &a, const std::vector<int32_t> &b, std::vector<int32_t> &out) {
    out.clear();
    size_t i = 0, j = 0;
    while (i < a.size() || j < b.size()) {
      if (j == b.size() || (i < a.size() && a[i] < b[j])) out.push_back(a[i++]);
      else if (i == a.size() || b[j] < a[i]) out.push_back(b[j++]);
      else { ++i; ++j; }
    }
  };
  std::vector<std::vector<int32_t>> groups;
  const size_t held = ch->grp_ptr.empty() ? 0 : ch->grp_ptr.size() - 1;
  for (size_t q = 0; q < held; ++q) groups.emplace_back(ch->grp_col.begin() + ch->grp_ptr[q], ch->grp_col.begin() + ch->grp_ptr[q + 1]);
  std::set<std::vector<int32_t>> seen(groups.begin(), groups.end());
  uint32_t count = 0;
  auto offer = [&](std::vector<int32_t> &&grp) {
    if (grp.empty() || seen.count(grp)) return;
    seen.insert(grp);
    groups.push_back(std::move(grp));
    ++count;
  };
  std::vector<int32_t> acc, tmp, set;
  // (1) coded blocks of degree one: c_j = x_i, so S_i xor {j} XORs to zero
  for (uint32_t j = 0; j < g->n; ++j) {
    if (g->row_ptr[j + 1] - g->row_ptr[j] != 1) continue;
    const int32_t i = g->col[g->row_ptr[j]];
    if (c2_of[i] < 0) continue;
    set_of(i, set);
    sym_xor(set, std::vector<int32_t>{(int32_t)j}, acc);
    offer(std::move(acc));
    acc = {};
  }
  // (2) check #1 sets whose members all have check #2 sets (Eqs. (1)-(4))
  if (pc) {
    for (uint32_t r = 0; r < pc->m; ++r) {
      bool all = true;
      for (int32_t e = pc->chk_ptr[r]; e < pc->chk_ptr[r + 1] && all; ++e) all = c2_of[pc->chk_col[e]] >= 0;
      if (!all) continue;
      acc.clear();
      for (int32_t e = pc->chk_ptr[r]; e < pc->chk_ptr[r + 1]; ++e) {
        set_of(pc->chk_col[e], set);
        sym_xor(acc, set, tmp);
        acc.swap(tmp);
      }
      offer(std::move(acc));
      acc = {};
    }
  }
  // smallest first, the held groups before new ones of the same size
  std::stable_sort(groups.begin(), groups.end(),
                   [](const std::vector<int32_t> &a, const std::vector<int32_t> &b) { return a.size() < b.size(); });
  std::vector<int32_t> ptr(1, 0), col;
  for (const auto &gr : groups) {
    col.insert(col.end(), gr.begin(), gr.end());
    ptr.push_back((int32_t)col.size());
  }
  void *old = ch->d_base;
  const int old_dev = ch->device;
  ch->grp_ptr.swap(ptr);
  ch->grp_col.swap(col);
  ch->d_base = nullptr;
  const fs_status fin = finish_checks(ch, stream);
  if (fin != FS_OK) {
    // keep the object as it was
    ch->grp_ptr.swap(ptr);
    ch->grp_col.swap(col);
    ch->d_base = old;
    ch->device = old_dev;
    checks_transpose(ch);
    return fin;
  }
  if (old) (void)hipFree(old);
  if (added) *added = count;
  return FS_OK;
}

void fs_checks_free(fs_checks *ch) {
  if (!ch) return;
  if (ch->d_base) (void)hipFree(ch->d_base);
  delete ch;
}

static fs_status local_repair_impl(const fs_graph *g, const fs_checks *ch, void *c, const uint8_t *erased,
                                   const uint32_t *lost, uint32_t n_lost, uint8_t *repaired, int32_t *status,
                                   uint64_t t, Carver &cv, hipStream_t stream);

static fs_status check_local(const fs_graph *g, const fs_checks *ch, void *c, uint64_t t) {
  FS_TRY(check_graph(g));
  if (!ch || !ch->d_base) return fail(FS_ERR_INVALID, "checks is null");
  if (ch->n != g->n || ch->k != g->k) return fail(FS_ERR_INVALID, "the checks belong to another graph shape");
  if (g->n > kLocalMaxN) return fail(FS_ERR_UNSUPPORTED, "local repair plans codes of at most 524288 blocks");
  return check_payload(c, t, "c");
}

fs_status fs_repair_local(const fs_graph *g, const fs_checks *ch, void *c, const uint8_t *erased, const uint32_t *lost,
                          uint32_t n_lost, uint8_t *repaired, int32_t *status, uint64_t t, void *ws, size_t ws_bytes,
                          hipStream_t stream) {
  clear_error();
  FS_TRY(check_local(g, ch, c, t));
  if ((n_lost && (!lost || !repaired)) || !status)
    return fail(FS_ERR_INVALID, "lost, repaired and status must be non-null");
  FS_TRY(check_ws(g, FS_OP_REPAIR_LOCAL, t, n_lost, ws, ws_bytes));
  Carver cv(ws);
  return local_repair_impl(g, ch, c, erased, lost, n_lost, repaired, status, t, cv, stream);
}

fs_status fs_extend_local(const fs_graph *g, const fs_checks *ch, uint32_t n_old, void *c, const uint8_t *erased,
                          uint8_t *made, int32_t *status, uint64_t t, void *ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  FS_TRY(check_local(g, ch, c, t));
  if (n_old > g->n) return fail(FS_ERR_INVALID, "n_old exceeds the rows of the graph");
  const uint32_t n_new = g->n - n_old;
  if ((n_new && !made) || !status) return fail(FS_ERR_INVALID, "made and status must be non-null");
  FS_TRY(check_ws(g, FS_OP_EXTEND_LOCAL, t, n_new, ws, ws_bytes));
  Carver cv(ws);
  ExtendPrepJob ej{};
  ej.n = g->n;
  ej.n_old = n_old;
  ej.erased = erased;
  ej.ids = cv.take<uint32_t>(g->n);
  ej.erased_full = cv.take<uint8_t>(g->n);
  FS_TRY(launch_extend_prep(ej, stream));
  return local_repair_impl(g, ch, c, ej.erased_full, ej.ids, n_new, made, status, t, cv, stream);
}

}  // extern "C"

static fs_status local_repair_impl(const fs_graph *g, const fs_checks *ch, void *c, const uint8_t *erased,
                                   const uint32_t *lost, uint32_t n_lost, uint8_t *repaired, int32_t *status,
                                   uint64_t t, Carver &cv, hipStream_t stream) {
  LocalBufs b;
  carve_local(cv, g, n_lost, b);
  LocalPlanJob pj{};
  pj.n = g->n;
  pj.n_lost = n_lost;
  pj.lost = lost;
  pj.erased = erased;
  pj.grp_ptr = ch->d_grp_ptr;
  pj.grp_col = ch->d_grp_col;
  pj.sym_ptr = ch->d_sym_ptr;
  pj.sym_grp = ch->d_sym_grp;
  pj.chosen = b.chosen;
  pj.level = b.level;
  pj.pos = b.pos;
  pj.item_ptr = b.item_ptr;
  pj.item_col = b.item_col;
  pj.item_dst = b.item_dst;
  pj.lvl_ptr = b.lvl_ptr;
  pj.meta = b.meta;
  pj.flag = b.flag;
  pj.repaired = repaired;
  pj.status = status;
  pj.n_groups = (uint32_t)(ch->grp_ptr.size() - 1);
  pj.gacc = b.gacc;
  pj.rof = b.rof;
  pj.best = b.best;
  pj.fa = b.fa;
  pj.fb = b.fb;
  pj.unk = b.unk;
  if ((uint64_t)pj.n_groups > 2ull * g->n) return fail(FS_ERR_UNSUPPORTED, "more than 2n check #3 groups");
  FS_TRY(launch_local_plan(pj, stream));
  if (n_lost == 0) return FS_OK;
  return launch_local_apply(pj, static_cast<uint8_t *>(c), t, stream);
}
