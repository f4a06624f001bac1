"""ctypes binding of libfs.so: argument marshalling only.

Every function here forwards to the C entry point of the same name; payloads,
masks, ids and workspaces are torch tensors on the GPU, passed by pointer.
Nothing is computed in Python.  If libfs.so has not been built, importing
this module raises ImportError: there is no fallback path.
"""

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libfs.so is not built (run python -m paper_1702_07409_amd.build)")


def _torch_runtime_first():
    """Initialise torch's HIP runtime before loading a library linked against
    the system one: in a process that also uses torch, a library loaded
    before torch's runtime is up has been seen to find no device."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


_torch_runtime_first()
_lib = ctypes.CDLL(LIB_PATH)

FS_OK, FS_ERR_INVALID, FS_ERR_ALIGN, FS_ERR_NOMEM, FS_ERR_HIP, FS_ERR_UNSUPPORTED, FS_ERR_WORKSPACE = range(7)
FS_DIST_RSD, FS_DIST_FINITE, FS_DIST_RAPTOR = 0, 1, 2
FS_DEFAULT_SEED = 1389488782
FS_GRAPH_HOST_ONLY = 1
FS_GRAPH_ON_DEVICE = 2
(FS_OP_ENCODE, FS_OP_PEEL, FS_OP_DECODE, FS_OP_REPAIR, FS_OP_REPAIR_CONVENTIONAL, FS_OP_UPDATE, FS_OP_REPLAY,
 FS_OP_EXTEND, FS_OP_EXTEND_CONVENTIONAL, FS_OP_SIM_DISKS, FS_OP_DECODE_PRECODED, FS_OP_REPAIR_LOCAL,
 FS_OP_REPAIR_PRECODED, FS_OP_EXTEND_LOCAL) = range(14)

DIST_CODES = {"rsd": FS_DIST_RSD, "finite": FS_DIST_FINITE, "raptor": FS_DIST_RAPTOR}


class fs_graph_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("n", ctypes.c_uint32), ("dist", ctypes.c_uint32),
                ("finite_dmax", ctypes.c_uint32), ("rsd_c", ctypes.c_double),
                ("rsd_delta", ctypes.c_double), ("finite_w", ctypes.POINTER(ctypes.c_double)),
                ("seed", ctypes.c_uint64), ("stripe_key", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class fs_tune(ctypes.Structure):
    _fields_ = [("lanes_per_row", ctypes.c_uint32), ("chunks", ctypes.c_uint32),
                ("xcd_remap", ctypes.c_uint32), ("nt_store", ctypes.c_uint32),
                ("replay_prog_global", ctypes.c_uint32), ("encode_slab", ctypes.c_uint32),
                ("replay_lookahead", ctypes.c_uint32), ("claim_chunk", ctypes.c_uint32)]


class fs_launch_info(ctypes.Structure):
    _fields_ = [("gather_kind", ctypes.c_uint32), ("gather_lanes_per_row", ctypes.c_uint32),
                ("gather_chunks", ctypes.c_uint32), ("gather_slice_bytes", ctypes.c_uint32),
                ("replay_kind", ctypes.c_uint32), ("replay_slice_bytes", ctypes.c_uint32),
                ("replay_workgroups", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class fs_work(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("n_ids", ctypes.c_uint32), ("graph", ctypes.c_void_p),
                ("t", ctypes.c_uint64), ("x", ctypes.c_void_p), ("c", ctypes.c_void_p),
                ("erased", ctypes.c_void_p), ("maxit", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("recovered", ctypes.c_void_p), ("status", ctypes.c_void_p), ("ids", ctypes.c_void_p),
                ("new_blocks", ctypes.c_void_p), ("repaired", ctypes.c_void_p)]


class fs_plan_info(ctypes.Structure):
    _fields_ = [("items", ctypes.c_uint32), ("gather_jobs", ctypes.c_uint32),
                ("decode_items", ctypes.c_uint32), ("update_items", ctypes.c_uint32),
                ("repair_items", ctypes.c_uint32), ("encode_items", ctypes.c_uint32),
                ("gather_tiles", ctypes.c_uint64), ("replay_workgroups", ctypes.c_uint32),
                ("tune_source", ctypes.c_uint32), ("tune", fs_tune),
                ("workspace_bytes", ctypes.c_uint64), ("tuned_ms", ctypes.c_double)]


P = ctypes.c_void_p
U32, U64, SZ, I32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int
ST = ctypes.c_int

_SIGS = {
    "fs_degree_table": ([ctypes.POINTER(fs_graph_params), P, U32, ctypes.POINTER(U32)], ST),
    "fs_graph_build": ([ctypes.POINTER(fs_graph_params), P, ctypes.POINTER(P)], ST),
    "fs_graph_info": ([P, ctypes.POINTER(U32), ctypes.POINTER(U32), ctypes.POINTER(U64),
                       ctypes.POINTER(U32), ctypes.POINTER(U32)], ST),
    "fs_graph_export": ([P, P, P, P, P], ST),
    "fs_graph_free": ([P], None),
    "fs_graph_image_size": ([P, ctypes.POINTER(SZ)], ST),
    "fs_graph_upload": ([P, P, SZ, P, P], ST),
    "fs_workspace_size": ([P, I32, U64, U32, ctypes.POINTER(SZ)], ST),
    "fs_encode": ([P, P, P, U64, P], ST),
    "fs_peel": ([P, P, U32, P, P, P, P, P, P, SZ, P], ST),
    "fs_replay": ([P, P, P, P, P, P, P, U64, P, SZ, P], ST),
    "fs_decode": ([P, P, P, U32, P, P, P, U64, P, SZ, P], ST),
    "fs_decode_noalloc": ([P, P, P, U32, P, P, P, U64, P], ST),
    "fs_decode_plan": ([P, P, U32, P, P, P, SZ, P], ST),
    "fs_decode_apply": ([P, P, P, U64, P, SZ, P], ST),
    "fs_repair": ([P, P, P, P, P, U32, P, P, U64, P, SZ, P], ST),
    "fs_update": ([P, P, P, P, U32, P, P, U64, P, SZ, P], ST),
    "fs_extend": ([P, U32, P, P, P, P, P, U64, P, SZ, P], ST),
    "fs_sim_disks": ([P, U32, U32, U64, U64, U32, P, P, SZ, P], ST),
    "fs_precode_build": ([U32, U32, I32, P, ctypes.POINTER(P)], ST),
    "fs_precode_info": ([P, ctypes.POINTER(U32), ctypes.POINTER(U32), ctypes.POINTER(U32), ctypes.POINTER(U32),
                         ctypes.POINTER(U32)], ST),
    "fs_precode_export": ([P, P, P], ST),
    "fs_precode_free": ([P], None),
    "fs_precode_encode": ([P, P, U64, P], ST),
    "fs_decode_precoded": ([P, P, P, P, U32, P, P, P, U64, P, SZ, P], ST),
    "fs_repair_precoded": ([P, P, P, P, P, U32, P, P, U64, P, SZ, P], ST),
    "fs_sim_disks_precoded": ([P, P, U32, U32, U64, U64, U32, P, P, SZ, P], ST),
    "fs_checks_generate": ([P, U32, P, ctypes.POINTER(P)], ST),
    "fs_checks_info": ([P, ctypes.POINTER(U32), ctypes.POINTER(U32), ctypes.POINTER(U32), ctypes.POINTER(U32),
                        ctypes.POINTER(U64), ctypes.POINTER(U64)], ST),
    "fs_checks_export": ([P, P, P, P, P, P], ST),
    "fs_checks_free": ([P], None),
    "fs_checks_serialize": ([P, P, U64, ctypes.POINTER(U64)], ST),
    "fs_checks_load": ([P, P, U64, P, ctypes.POINTER(P)], ST),
    "fs_checks_add_groups": ([P, P, P, P, ctypes.POINTER(U32)], ST),
    "fs_repair_local": ([P, P, P, P, P, U32, P, P, U64, P, SZ, P], ST),
    "fs_extend_local": ([P, P, U32, P, P, P, P, U64, P, SZ, P], ST),
    "fs_plan_create": ([ctypes.POINTER(fs_work), U32, ctypes.c_char_p, U32, P, ctypes.POINTER(P)], ST),
    "fs_plan_launch": ([P, P], ST),
    "fs_plan_memory_size": ([ctypes.POINTER(fs_work), U32, ctypes.POINTER(SZ), ctypes.POINTER(SZ)], ST),
    "fs_plan_create_in": ([ctypes.POINTER(fs_work), U32, P, SZ, P, SZ, P, ctypes.POINTER(P)], ST),
    "fs_plan_rebind": ([P, ctypes.POINTER(fs_work), U32, P], ST),
    "fs_plan_get_info": ([P, ctypes.POINTER(fs_plan_info)], ST),
    "fs_plan_free": ([P], None),
    "fs_set_tune": ([ctypes.POINTER(fs_tune)], ST),
    "fs_get_tune": ([ctypes.POINTER(fs_tune)], ST),
    "fs_last_launch": ([ctypes.POINTER(fs_launch_info)], ST),
    "fs_status_string": ([I32], ctypes.c_char_p),
    "fs_last_error": ([], ctypes.c_char_p),
    "fs_version": ([], ctypes.c_char_p),
}

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


class FsError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.fs_last_error().decode() or _lib.fs_status_string(status).decode()
        super().__init__("%s: %s (%s)" % (where, _lib.fs_status_string(status).decode(), msg))


def _check(status, where):
    if status != FS_OK:
        raise FsError(status, where)


def version():
    return _lib.fs_version().decode()


def _ptr(t):
    """Device pointer of a tensor (or None -> NULL)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def make_params(k, n, dist="rsd", rsd_c=0.1, rsd_delta=0.05, finite_w=(), seed=FS_DEFAULT_SEED,
                stripe_key=0, host_only=False, on_device=False):
    p = fs_graph_params()
    p.k, p.n = k, n
    p.dist = DIST_CODES[dist]
    p.rsd_c, p.rsd_delta = rsd_c, rsd_delta
    w = (ctypes.c_double * max(1, len(finite_w)))(*finite_w)
    p.finite_dmax = len(finite_w)
    p.finite_w = ctypes.cast(w, ctypes.POINTER(ctypes.c_double))
    p.seed, p.stripe_key = seed, stripe_key
    p.flags = (FS_GRAPH_HOST_ONLY if host_only else 0) | (FS_GRAPH_ON_DEVICE if on_device else 0)
    p._keep = w
    return p


def fs_degree_table(**kw):
    """Thresholds T_1..T_D of the degree distribution, as a Python list."""
    p = make_params(k=kw.pop("k"), n=kw.pop("n", 1), **kw)
    D = U32()
    _check(_lib.fs_degree_table(ctypes.byref(p), None, 0, ctypes.byref(D)), "fs_degree_table")
    buf = (ctypes.c_uint64 * D.value)()
    _check(_lib.fs_degree_table(ctypes.byref(p), buf, D.value, ctypes.byref(D)), "fs_degree_table")
    return list(buf)


class Graph:
    """Owner of an fs_graph handle."""

    def __init__(self, handle, params):
        self.handle = handle
        self.params = params
        k, n, nnz, md, mc = U32(), U32(), U64(), U32(), U32()
        _check(_lib.fs_graph_info(handle, ctypes.byref(k), ctypes.byref(n), ctypes.byref(nnz),
                                  ctypes.byref(md), ctypes.byref(mc)), "fs_graph_info")
        self.k, self.n, self.nnz = k.value, n.value, nnz.value
        self.max_degree, self.max_column_degree = md.value, mc.value

    @property
    def built_on_device(self):
        return bool(self.params.flags & FS_GRAPH_ON_DEVICE)

    def device_bytes(self):
        """Device bytes of the graph's arrays (CSR, CSC, encode segments), about."""
        return 4 * (3 * self.nnz + 3 * self.n + self.k) + 9 * 256

    def export(self):
        import numpy as np
        rp = np.zeros(self.n + 1, np.int32)
        col = np.zeros(max(self.nnz, 1), np.int32)
        cp = np.zeros(self.k + 1, np.int32)
        ri = np.zeros(max(self.nnz, 1), np.int32)
        _check(_lib.fs_graph_export(self.handle, rp.ctypes.data, col.ctypes.data, cp.ctypes.data,
                                    ri.ctypes.data), "fs_graph_export")
        return rp, col[:self.nnz], cp, ri[:self.nnz]

    def workspace_size(self, op, t=16, n_items=0):
        return fs_workspace_size(self, op, t, n_items)

    def image_size(self):
        b = SZ()
        _check(_lib.fs_graph_image_size(self.handle, ctypes.byref(b)), "fs_graph_image_size")
        return b.value

    def upload(self, memory, stage=None, stream=None):
        """Device copy into `memory` (a device uint8 tensor kept by the caller);
        `stage`: optional pinned host uint8 tensor for an asynchronous copy."""
        w, wb = _ws(memory)
        sp = stage.data_ptr() if stage is not None else None
        _check(_lib.fs_graph_upload(self.handle, w, wb, sp, _stream(stream)), "fs_graph_upload")
        self._memory = memory

    def free(self):
        if self.handle:
            _lib.fs_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def fs_graph_build(k, n, dist="rsd", rsd_c=0.1, rsd_delta=0.05, finite_w=(), seed=FS_DEFAULT_SEED,
                   stripe_key=0, host_only=False, on_device=False, stream=None):
    """on_device: the rows, transpose and encode segments are built by
    kernels on the current device (same arrays as the host build)."""
    p = make_params(k, n, dist, rsd_c, rsd_delta, finite_w, seed, stripe_key, host_only, on_device)
    h = P()
    s = None if host_only else _stream(stream)
    _check(_lib.fs_graph_build(ctypes.byref(p), s, ctypes.byref(h)), "fs_graph_build")
    return Graph(h, p)


def fs_workspace_size(g, op, t=16, n_items=0):
    b = SZ()
    _check(_lib.fs_workspace_size(g.handle, op, t, n_items, ctypes.byref(b)), "fs_workspace_size")
    return b.value


def workspace(g, op, t=16, n_items=0, device="cuda"):
    """A device workspace tensor of the size the operation needs (torch memory)."""
    import torch
    nbytes = fs_workspace_size(g, op, t, n_items)
    return torch.empty(max(nbytes, 256) + 256, dtype=torch.uint8, device=device)


def _ws(ws):
    if ws is None:
        return None, 0
    base = ws.data_ptr()
    aligned = (base + 255) & ~255
    return aligned, ws.numel() - (aligned - base)


def fs_encode(g, x, c, t, stream=None):
    _check(_lib.fs_encode(g.handle, _ptr(x), _ptr(c), t, _stream(stream)), "fs_encode")


def fs_peel(g, erased, maxit, recovered, status, level_ptr, dp_f, dp_g, ws, stream=None):
    w, wb = _ws(ws)
    _check(_lib.fs_peel(g.handle, _ptr(erased), maxit, _ptr(recovered), _ptr(status), _ptr(level_ptr),
                        _ptr(dp_f), _ptr(dp_g), w, wb, _stream(stream)), "fs_peel")


def fs_replay(g, c, status, level_ptr, dp_f, dp_g, x, t, ws, stream=None):
    w, wb = _ws(ws)
    _check(_lib.fs_replay(g.handle, _ptr(c), _ptr(status), _ptr(level_ptr), _ptr(dp_f), _ptr(dp_g),
                          _ptr(x), t, w, wb, _stream(stream)), "fs_replay")


def fs_decode(g, c, erased, maxit, x, recovered, status, t, ws, stream=None):
    w, wb = _ws(ws)
    _check(_lib.fs_decode(g.handle, _ptr(c), _ptr(erased), maxit, _ptr(x), _ptr(recovered), _ptr(status),
                          t, w, wb, _stream(stream)), "fs_decode")


def fs_decode_noalloc(g, c, erased, maxit, x, recovered, status, t, stream=None):
    _check(_lib.fs_decode_noalloc(g.handle, _ptr(c), _ptr(erased), maxit, _ptr(x), _ptr(recovered),
                                  _ptr(status), t, _stream(stream)), "fs_decode_noalloc")


def fs_decode_plan(g, erased, maxit, recovered, status, ws, stream=None):
    w, wb = _ws(ws)
    _check(_lib.fs_decode_plan(g.handle, _ptr(erased), maxit, _ptr(recovered), _ptr(status), w, wb,
                               _stream(stream)), "fs_decode_plan")


def fs_decode_apply(g, c, x, t, ws, stream=None):
    w, wb = _ws(ws)
    _check(_lib.fs_decode_apply(g.handle, _ptr(c), _ptr(x), t, w, wb, _stream(stream)), "fs_decode_apply")


def fs_repair(g, x, c, erased, lost, n_lost, repaired, status, t, ws, stream=None):
    w, wb = _ws(ws)
    _check(_lib.fs_repair(g.handle, _ptr(x), _ptr(c), _ptr(erased), _ptr(lost), n_lost, _ptr(repaired),
                          _ptr(status), t, w, wb, _stream(stream)), "fs_repair")


def fs_update(g, x, c, ids, n_ids, new_blocks, status, t, ws, stream=None):
    w, wb = _ws(ws)
    _check(_lib.fs_update(g.handle, _ptr(x), _ptr(c), _ptr(ids), n_ids, _ptr(new_blocks), _ptr(status),
                          t, w, wb, _stream(stream)), "fs_update")


def fs_extend(g, n_old, x, c, erased, made, status, t, ws, stream=None):
    w, wb = _ws(ws)
    _check(_lib.fs_extend(g.handle, n_old, _ptr(x), _ptr(c), _ptr(erased), _ptr(made), _ptr(status),
                          t, w, wb, _stream(stream)), "fs_extend")


class Precode:
    """Owner of an fs_precode handle (array-LDPC check #1 of a (b, k) code)."""

    def __init__(self, handle):
        self.handle = handle
        b, k, p, kp, jp = U32(), U32(), U32(), U32(), U32()
        _check(_lib.fs_precode_info(handle, ctypes.byref(b), ctypes.byref(k), ctypes.byref(p), ctypes.byref(kp),
                                    ctypes.byref(jp)), "fs_precode_info")
        self.b, self.k, self.p, self.kp, self.jp = b.value, k.value, p.value, kp.value, jp.value

    def export(self):
        """L(1) as (row_ptr, col) numpy arrays, each row ascending."""
        import numpy as np
        m, w = self.k - self.b, self.kp - self.jp
        rp = np.zeros(m + 1, np.int32)
        col = np.zeros(max(m * w, 1), np.int32)
        _check(_lib.fs_precode_export(self.handle, rp.ctypes.data, col.ctypes.data), "fs_precode_export")
        return rp, col[:m * w]

    def free(self):
        if self.handle:
            _lib.fs_precode_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def fs_precode_build(b, k, host_only=False, stream=None):
    h = P()
    _check(_lib.fs_precode_build(b, k, 1 if host_only else 0, None if host_only else _stream(stream),
                                 ctypes.byref(h)), "fs_precode_build")
    return Precode(h)


def fs_precode_encode(pc, x, t, stream=None):
    _check(_lib.fs_precode_encode(pc.handle, _ptr(x), t, _stream(stream)), "fs_precode_encode")


def fs_decode_precoded(g, pc, c, erased, maxit, x, recovered, status, t, ws, stream=None):
    w, wb = _ws(ws)
    _check(_lib.fs_decode_precoded(g.handle, pc.handle, _ptr(c), _ptr(erased), maxit, _ptr(x), _ptr(recovered),
                                   _ptr(status), t, w, wb, _stream(stream)), "fs_decode_precoded")


class Checks:
    """Owner of an fs_checks handle (check #2 / #3 equations of a graph)."""

    def __init__(self, handle):
        self.handle = handle
        a, b_, c, d, e, f = U32(), U32(), U32(), U32(), U64(), U64()
        _check(_lib.fs_checks_info(handle, ctypes.byref(a), ctypes.byref(b_), ctypes.byref(c), ctypes.byref(d),
                                   ctypes.byref(e), ctypes.byref(f)), "fs_checks_info")
        self.n_check2, self.n_check3, self.sweeps, self.zero_columns = a.value, b_.value, c.value, d.value
        self.check2_entries, self.check3_entries = e.value, f.value

    def export(self):
        """(check2 {input: [coded blocks]}, check3 [[coded blocks], ...])."""
        import numpy as np
        c3p = np.zeros(self.n_check3 + 1, np.int32)
        c3c = np.zeros(max(self.check3_entries, 1), np.int32)
        c2i = np.zeros(max(self.n_check2, 1), np.int32)
        c2p = np.zeros(self.n_check2 + 1, np.int32)
        c2c = np.zeros(max(self.check2_entries, 1), np.int32)
        _check(_lib.fs_checks_export(self.handle, c3p.ctypes.data, c3c.ctypes.data, c2i.ctypes.data,
                                     c2p.ctypes.data, c2c.ctypes.data), "fs_checks_export")
        check2 = {int(c2i[q]): c2c[c2p[q]:c2p[q + 1]].tolist() for q in range(self.n_check2)}
        check3 = [c3c[c3p[q]:c3p[q + 1]].tolist() for q in range(self.n_check3)]
        return check2, check3

    def add_groups(self, g, precode=None, stream=None):
        """Check #3 groups from degree-one coded blocks and from the
        precode's check #1 sets (§2.5); returns how many were added."""
        a = U32()
        _check(_lib.fs_checks_add_groups(self.handle, g.handle, precode.handle if precode is not None else None,
                                         _stream(stream), ctypes.byref(a)), "fs_checks_add_groups")
        n2, n3, sw, zc, e2, e3 = U32(), U32(), U32(), U32(), U64(), U64()
        _check(_lib.fs_checks_info(self.handle, ctypes.byref(n2), ctypes.byref(n3), ctypes.byref(sw),
                                   ctypes.byref(zc), ctypes.byref(e2), ctypes.byref(e3)), "fs_checks_info")
        self.n_check2, self.n_check3 = n2.value, n3.value
        self.check2_entries, self.check3_entries = e2.value, e3.value
        return a.value

    def serialize(self):
        """The check data integer array (numpy int32)."""
        import numpy as np
        n = U64()
        _check(_lib.fs_checks_serialize(self.handle, None, 0, ctypes.byref(n)), "fs_checks_serialize")
        out = np.zeros(max(n.value, 1), np.int32)
        _check(_lib.fs_checks_serialize(self.handle, out.ctypes.data, out.size, ctypes.byref(n)),
               "fs_checks_serialize")
        return out[:n.value]

    def free(self):
        if self.handle:
            _lib.fs_checks_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def fs_checks_generate(g, max_sweeps=0, stream=None):
    h = P()
    _check(_lib.fs_checks_generate(g.handle, max_sweeps, _stream(stream), ctypes.byref(h)), "fs_checks_generate")
    return Checks(h)


def fs_checks_load(g, data, stream=None):
    """Checks from a check data integer array (anything numpy turns into int32)."""
    import numpy as np
    arr = np.ascontiguousarray(np.asarray(data, dtype=np.int32))
    h = P()
    _check(_lib.fs_checks_load(g.handle, arr.ctypes.data if arr.size else None, arr.size, _stream(stream),
                               ctypes.byref(h)), "fs_checks_load")
    return Checks(h)


def fs_repair_local(g, ch, c, erased, lost, n_lost, repaired, status, t, ws, stream=None):
    w, wb = _ws(ws)
    _check(_lib.fs_repair_local(g.handle, ch.handle, _ptr(c), _ptr(erased), _ptr(lost), n_lost, _ptr(repaired),
                                _ptr(status), t, w, wb, _stream(stream)), "fs_repair_local")


def fs_extend_local(g, ch, n_old, c, erased, made, status, t, ws, stream=None):
    """New coded rows n_old..n-1 from existing ones through the check #3
    groups ch of the longer graph g (§2.9)."""
    w, wb = _ws(ws)
    _check(_lib.fs_extend_local(g.handle, ch.handle, n_old, _ptr(c), _ptr(erased), _ptr(made), _ptr(status),
                                t, w, wb, _stream(stream)), "fs_extend_local")


def fs_repair_precoded(g, pc, c, erased, lost, n_lost, repaired, status, t, ws, stream=None):
    w, wb = _ws(ws)
    _check(_lib.fs_repair_precoded(g.handle, pc.handle, _ptr(c), _ptr(erased), _ptr(lost), n_lost, _ptr(repaired),
                                   _ptr(status), t, w, wb, _stream(stream)), "fs_repair_precoded")


def fs_sim_disks_precoded(g, pc, s, f, first, count, maxit, result, ws, stream=None):
    w, wb = _ws(ws)
    _check(_lib.fs_sim_disks_precoded(g.handle, pc.handle, s, f, first, count, maxit, _ptr(result), w, wb,
                                      _stream(stream)), "fs_sim_disks_precoded")


def fs_sim_disks(g, s, f, first, count, maxit, result, ws, stream=None):
    w, wb = _ws(ws)
    _check(_lib.fs_sim_disks(g.handle, s, f, first, count, maxit, _ptr(result), w, wb, _stream(stream)),
           "fs_sim_disks")


def fs_set_tune(lanes_per_row=0, chunks=0, xcd_remap=1, nt_store=1, replay_prog_global=0, encode_slab=1,
                replay_lookahead=0, claim_chunk=0):
    tu = fs_tune(lanes_per_row, chunks, xcd_remap, nt_store, replay_prog_global, encode_slab, replay_lookahead,
                 claim_chunk)
    _check(_lib.fs_set_tune(ctypes.byref(tu)), "fs_set_tune")


def fs_reset_tune():
    _check(_lib.fs_set_tune(None), "fs_set_tune")


def fs_last_launch():
    """Shape of this thread's last single-stripe gather and replay launch."""
    li = fs_launch_info()
    _check(_lib.fs_last_launch(ctypes.byref(li)), "fs_last_launch")
    return {f: getattr(li, f) for f, _ in fs_launch_info._fields_ if f != "reserved"}


def fs_get_tune():
    tu = fs_tune()
    _check(_lib.fs_get_tune(ctypes.byref(tu)), "fs_get_tune")
    return dict(lanes_per_row=tu.lanes_per_row, chunks=tu.chunks, xcd_remap=tu.xcd_remap,
                nt_store=tu.nt_store, replay_prog_global=tu.replay_prog_global, encode_slab=tu.encode_slab,
                replay_lookahead=tu.replay_lookahead, claim_chunk=tu.claim_chunk)


FS_WORK_ENCODE, FS_WORK_DECODE, FS_WORK_REPAIR, FS_WORK_UPDATE = range(4)
FS_PLAN_AUTOTUNE, FS_PLAN_NO_GRAPH = 1, 2
WORK_OPS = {"encode": FS_WORK_ENCODE, "decode": FS_WORK_DECODE, "repair": FS_WORK_REPAIR,
            "update": FS_WORK_UPDATE}


def work(op, graph, t, x=None, c=None, erased=None, maxit=0, recovered=None, status=None, ids=None,
         n_ids=0, new_blocks=None, repaired=None):
    """One fs_work item (tensors are kept alive by the returned object)."""
    w = fs_work()
    w.op = WORK_OPS[op] if isinstance(op, str) else op
    w.n_ids = n_ids
    w.graph = graph.handle
    w.t = t
    w.x, w.c, w.erased = _ptr(x), _ptr(c), _ptr(erased)
    w.maxit = maxit
    w.recovered, w.status, w.ids = _ptr(recovered), _ptr(status), _ptr(ids)
    w.new_blocks, w.repaired = _ptr(new_blocks), _ptr(repaired)
    w._keep = (graph, x, c, erased, recovered, status, ids, new_blocks, repaired)
    return w


def plan_memory_size(items):
    """(device bytes, host staging bytes) of fs_plan_create_in for these items."""
    arr = (fs_work * len(items))(*items)
    b, h = SZ(), SZ()
    _check(_lib.fs_plan_memory_size(arr, len(items), ctypes.byref(b), ctypes.byref(h)), "fs_plan_memory_size")
    return b.value, h.value


class Plan:
    """Owner of an fs_plan handle.

    memory: optional device tensor (uint8) that holds the plan
    (fs_plan_create_in: no allocation, no graph, one stream); stage: optional
    pinned host uint8 tensor for an asynchronous descriptor copy."""

    def __init__(self, items, tune_cache=None, autotune=False, graph=True, stream=None, memory=None,
                 stage=None):
        arr = (fs_work * len(items))(*items)
        h = P()
        if memory is not None:
            w, wb = _ws(memory)
            sp, sb = (stage.data_ptr(), stage.numel()) if stage is not None else (None, 0)
            _check(_lib.fs_plan_create_in(arr, len(items), w, wb, sp, sb, _stream(stream), ctypes.byref(h)),
                   "fs_plan_create_in")
        else:
            flags = (FS_PLAN_AUTOTUNE if autotune else 0) | (0 if graph else FS_PLAN_NO_GRAPH)
            path = tune_cache.encode() if tune_cache else None
            _check(_lib.fs_plan_create(arr, len(items), path, flags, _stream(stream), ctypes.byref(h)),
                   "fs_plan_create")
        self.handle = h
        self._items = list(items)
        self._memory = memory
        self._stage = stage

    def launch(self, stream=None):
        _check(_lib.fs_plan_launch(self.handle, _stream(stream)), "fs_plan_launch")

    def rebind(self, items, stream=None):
        arr = (fs_work * len(items))(*items)
        _check(_lib.fs_plan_rebind(self.handle, arr, len(items), _stream(stream)), "fs_plan_rebind")
        self._items = list(items)

    def info(self):
        i = fs_plan_info()
        _check(_lib.fs_plan_get_info(self.handle, ctypes.byref(i)), "fs_plan_get_info")
        out = {f: getattr(i, f) for f, _ in fs_plan_info._fields_ if f != "tune"}
        out["tune"] = dict(lanes_per_row=i.tune.lanes_per_row, chunks=i.tune.chunks,
                           xcd_remap=i.tune.xcd_remap, nt_store=i.tune.nt_store, claim_chunk=i.tune.claim_chunk)
        return out

    def free(self):
        if self.handle:
            _lib.fs_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
