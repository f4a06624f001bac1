"""MI355X (gfx950) implementation of the LDGM fountain-code XOR path of
Founsure 1.0: seeded graph build, encode, level-synchronous peeling decode,
repair, delta update, code extension, the disk-failure sweep and the
array-LDPC precode with its two-stage decode, check #2/#3 generation and
local-group repair, as HIP kernels behind the C ABI of libfs.so
(include/fs_api.h).  This package is the thin ctypes binding; PyTorch only
supplies device memory and streams.

The binding (and libfs.so) is loaded on first use of one of its names, so
that the build module can run before the library exists; a missing library
then raises ImportError.
"""

_BINDING = (
    "EXPORTED", "FS_DEFAULT_SEED", "FS_OP_DECODE", "FS_OP_ENCODE", "FS_OP_PEEL", "FS_OP_REPAIR",
    "FS_OP_REPAIR_CONVENTIONAL", "FS_OP_REPLAY", "FS_OP_UPDATE", "FS_OP_EXTEND",
    "FS_OP_EXTEND_CONVENTIONAL", "FS_OP_SIM_DISKS", "FS_OP_DECODE_PRECODED", "FS_OP_REPAIR_LOCAL", "FS_OP_REPAIR_PRECODED", "FS_OP_EXTEND_LOCAL", "fs_extend_local", "FsError",
    "Graph", "Checks", "fs_checks_generate", "fs_checks_load", "fs_repair_local", "fs_repair_precoded", "fs_decode", "fs_decode_noalloc", "fs_decode_apply", "fs_decode_plan", "fs_degree_table", "fs_encode", "fs_get_tune", "fs_last_launch",
    "fs_graph_build", "fs_peel", "fs_repair", "fs_replay", "fs_reset_tune", "fs_set_tune",
    "fs_update", "fs_extend", "fs_sim_disks", "fs_sim_disks_precoded", "fs_precode_build",
    "fs_precode_encode",
    "fs_decode_precoded", "Precode", "fs_workspace_size", "version", "workspace", "Plan",
    "work", "plan_memory_size",
    "FS_WORK_ENCODE", "FS_WORK_DECODE", "FS_WORK_REPAIR", "FS_WORK_UPDATE",
)


def __getattr__(name):
    if name in _BINDING:
        from . import _lib
        return getattr(_lib, name)
    raise AttributeError("module %r has no attribute %r" % (__name__, name))


def __dir__():
    return sorted(list(globals()) + list(_BINDING))
