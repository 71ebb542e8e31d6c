"""ctypes binding of libpic's C ABI (include/pic.h): structures and the
``pic_*`` functions under the same names.  Argument marshalling only -- every
step of the PIC cycle runs in the HIP kernels of libpic.so.  There is no CPU
fallback: if the library is missing this module raises on first use."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libpic.so")

MAX_SPECIES = 4

PIC_OK = 0
PIC_EINVAL = -1
PIC_ECFL = -2
PIC_ETILE = -3
PIC_EHIP = -4
PIC_EORDER = -5
PIC_ERANGE = -6
PIC_ESORT = -7
PIC_ECOUNT = -8
PIC_EOVERFLOW = -9
PIC_ENOCONV = -10
PIC_ESCRATCH = -11
PIC_GAUSS_NOALLOC_MAX_CELLS = 1 << 20

PIC_FLAG_J_FLOAT = 1
PIC_FLAG_ESIRKEPOV = 2
PIC_FLAG_MOVING_WINDOW = 4
PIC_FLAG_MOTION_SORT = 8
PIC_FLAG_QUADRATIC = 16

PIC_DIAG_ENERGY = 1
PIC_DIAG_RHO_SNAPSHOT = 2
PIC_DIAG_CONTINUITY = 4
PIC_DIAG_COUNTS = 8
PIC_DIAG_GAUSS = 16

KERNELS = ["push", "j_reduce", "sort_scan", "sort_plan", "sort_scatter", "field", "filter"]
PIC_MAX_FILTER = 16

# every symbol the header declares
EXPORTS = [
    "pic_query", "pic_init", "pic_push_deposit", "pic_sort", "pic_sync", "pic_field_advance", "pic_move_window",
    "pic_get_window_origin", "pic_get_counts", "pic_solve_gauss", "pic_solve_gauss_noalloc", "pic_step",
    "pic_check", "pic_diag", "pic_get_state", "pic_set_state", "pic_get_tile_offsets",
    "pic_set_timing", "pic_set_timing_mask", "pic_get_timing",
    "pic_batch_query", "pic_batch_init", "pic_batch_step", "pic_batch_capture", "pic_batch_sim",
    "pic_batch_check", "pic_batch_sync", "pic_batch_destroy",
    "pic_probe_stream", "pic_strerror", "pic_destroy",
]


class pic_species(ctypes.Structure):
    _fields_ = [("qm", ctypes.c_double), ("q", ctypes.c_double), ("n", ctypes.c_int64), ("cap", ctypes.c_int64)]


class pic_config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dt", ctypes.c_double),
                ("tile", ctypes.c_int32), ("j_replicas", ctypes.c_int32),
                ("n_species", ctypes.c_int32), ("flags", ctypes.c_uint32), ("j_filter", ctypes.c_int32),
                ("sort_every", ctypes.c_int32), ("ppl", ctypes.c_int32),
                ("species", pic_species * MAX_SPECIES)]


class pic_particles(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("cell", "x", "y", "ux", "uy", "uz")]


class pic_buffers(ctypes.Structure):
    _fields_ = [("fields", ctypes.c_void_p), ("work", ctypes.c_void_p),
                ("work_bytes", ctypes.c_size_t), ("sp", pic_particles * MAX_SPECIES)]


class pic_sizes(ctypes.Structure):
    _fields_ = [("n_tiles", ctypes.c_int32), ("field_bytes", ctypes.c_size_t),
                ("work_bytes", ctypes.c_size_t)]


class pic_diag_out(ctypes.Structure):
    _fields_ = [("u_e", ctypes.c_double), ("u_b", ctypes.c_double),
                ("u_k", ctypes.c_double * MAX_SPECIES),
                ("continuity_max", ctypes.c_double), ("rho_max", ctypes.c_double),
                ("leavers", ctypes.c_int64 * MAX_SPECIES), ("movers", ctypes.c_int64 * MAX_SPECIES),
                ("gauss_max", ctypes.c_double), ("divb_max", ctypes.c_double)]


class pic_host_state(ctypes.Structure):
    _fields_ = [("fields", ctypes.c_void_p), ("sp", pic_particles * MAX_SPECIES),
                ("n", ctypes.c_int64 * MAX_SPECIES), ("window_origin", ctypes.c_int32)]


class pic_gauss_out(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32 * 2), ("residual", ctypes.c_double * 2)]


class pic_timing_out(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double * 7), ("launches", ctypes.c_int64 * 7)]


class PicError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_L = None


def load(path: str = SO_PATH):
    """Load libpic.so (raises if it has not been built)."""
    global _L
    if _L is not None:
        return _L
    if not os.path.exists(path):
        raise ImportError(f"libpic.so not built at {path}; run __graft_entry__.build()")
    try:
        # torch ships its own HIP runtime; load it first so libpic binds to the
        # same libamdhip64 instance instead of a second copy from /opt/rocm
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.pic_query.argtypes = [P(pic_config), P(pic_sizes)]
    L.pic_init.argtypes = [P(pic_config), P(pic_buffers), vp, P(vp)]
    for name in ("pic_push_deposit", "pic_sort", "pic_sync", "pic_field_advance", "pic_step", "pic_check"):
        getattr(L, name).argtypes = [vp, vp]
    L.pic_diag.argtypes = [vp, ctypes.c_uint, P(pic_diag_out), vp]
    L.pic_get_tile_offsets.argtypes = [vp, ctypes.c_int, vp, vp]
    L.pic_get_state.argtypes = [vp, P(pic_host_state), vp]
    L.pic_move_window.argtypes = [vp, P(pic_particles), P(ctypes.c_int64), vp]
    L.pic_get_counts.argtypes = [vp, P(ctypes.c_int64)]
    L.pic_get_window_origin.argtypes = [vp, P(ctypes.c_int32)]
    L.pic_solve_gauss.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_double, ctypes.c_int, P(pic_gauss_out), vp]
    L.pic_solve_gauss_noalloc.argtypes = [vp, ctypes.c_double, ctypes.c_int, P(pic_gauss_out), vp]
    L.pic_probe_stream.argtypes = [vp, ctypes.c_int64, ctypes.c_int, vp]
    L.pic_set_state.argtypes = [vp, P(pic_host_state), vp]
    L.pic_set_timing.argtypes = [vp, ctypes.c_int]
    L.pic_set_timing_mask.argtypes = [vp, ctypes.c_uint]
    L.pic_get_timing.argtypes = [vp, P(pic_timing_out)]
    L.pic_strerror.argtypes = [ctypes.c_int]
    L.pic_strerror.restype = ctypes.c_char_p
    L.pic_destroy.argtypes = [vp]
    L.pic_destroy.restype = None
    L.pic_batch_query.argtypes = [ctypes.c_int, P(pic_config), P(ctypes.c_size_t)]
    L.pic_batch_init.argtypes = [ctypes.c_int, P(pic_config), P(pic_buffers), vp, ctypes.c_size_t, vp, P(vp)]
    L.pic_batch_step.argtypes = [vp, ctypes.c_int, vp]
    L.pic_batch_capture.argtypes = [vp, vp]
    L.pic_batch_sim.argtypes = [vp, ctypes.c_int]
    L.pic_batch_sim.restype = vp
    L.pic_batch_check.argtypes = [vp, vp]
    L.pic_batch_sync.argtypes = [vp, vp]
    L.pic_batch_destroy.argtypes = [vp]
    L.pic_batch_destroy.restype = None
    for name in EXPORTS:
        if name not in ("pic_strerror", "pic_destroy", "pic_batch_sim", "pic_batch_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _L = L
    return L


def strerror(code: int) -> str:
    return load().pic_strerror(int(code)).decode()


def _chk(rc: int, where: str) -> int:
    if rc != PIC_OK:
        raise PicError(rc, where)
    return rc


# ---- the C functions, same names, raising PicError on a negative code ----

def pic_query(cfg: pic_config) -> pic_sizes:
    out = pic_sizes()
    _chk(load().pic_query(ctypes.byref(cfg), ctypes.byref(out)), "pic_query")
    return out


def pic_init(cfg: pic_config, bufs: pic_buffers, stream: int) -> int:
    h = ctypes.c_void_p()
    _chk(load().pic_init(ctypes.byref(cfg), ctypes.byref(bufs), ctypes.c_void_p(stream), ctypes.byref(h)),
         "pic_init")
    return h.value


def pic_push_deposit(sim: int, stream: int):
    _chk(load().pic_push_deposit(ctypes.c_void_p(sim), ctypes.c_void_p(stream)), "pic_push_deposit")


def pic_sort(sim: int, stream: int):
    _chk(load().pic_sort(ctypes.c_void_p(sim), ctypes.c_void_p(stream)), "pic_sort")


def pic_sync(sim: int, stream: int):
    _chk(load().pic_sync(ctypes.c_void_p(sim), ctypes.c_void_p(stream)), "pic_sync")


def pic_field_advance(sim: int, stream: int):
    _chk(load().pic_field_advance(ctypes.c_void_p(sim), ctypes.c_void_p(stream)), "pic_field_advance")


def pic_step(sim: int, stream: int):
    _chk(load().pic_step(ctypes.c_void_p(sim), ctypes.c_void_p(stream)), "pic_step")


def pic_check(sim: int, stream: int) -> int:
    """Returns the code (does not raise) so callers can test error paths."""
    return load().pic_check(ctypes.c_void_p(sim), ctypes.c_void_p(stream))


def pic_diag(sim: int, what: int, stream: int) -> pic_diag_out:
    out = pic_diag_out()
    _chk(load().pic_diag(ctypes.c_void_p(sim), ctypes.c_uint(what), ctypes.byref(out), ctypes.c_void_p(stream)),
         "pic_diag")
    return out


def pic_move_window(sim: int, inject, n_inject, stream: int):
    """inject: sequence of pic_particles (device pointers), n_inject: counts."""
    arr = (pic_particles * MAX_SPECIES)(*inject)
    cnt = (ctypes.c_int64 * MAX_SPECIES)(*n_inject)
    _chk(load().pic_move_window(ctypes.c_void_p(sim), arr, cnt, ctypes.c_void_p(stream)), "pic_move_window")


def pic_get_window_origin(sim: int) -> int:
    out = ctypes.c_int32()
    _chk(load().pic_get_window_origin(ctypes.c_void_p(sim), ctypes.byref(out)), "pic_get_window_origin")
    return int(out.value)


def gauss_scratch_bytes(nx: int, ny: int) -> int:
    """PIC_GAUSS_SCRATCH_BYTES(nx, ny)."""
    return 32 * nx * ny + 16384


def pic_solve_gauss(sim: int, scratch: int, scratch_bytes: int, tol: float, max_iter: int, stream: int):
    """Returns the pic_gauss_out record; raises PicError (PIC_ENOCONV included)."""
    out = pic_gauss_out()
    _chk(load().pic_solve_gauss(ctypes.c_void_p(sim), ctypes.c_void_p(scratch), scratch_bytes, float(tol),
                                int(max_iter), ctypes.byref(out), ctypes.c_void_p(stream)), "pic_solve_gauss")
    return out


def pic_solve_gauss_noalloc(sim: int, tol: float, max_iter: int, stream: int):
    """pic_solve_gauss in the library's static scratch (no device allocation);
    returns the pic_gauss_out record; raises PicError."""
    out = pic_gauss_out()
    _chk(load().pic_solve_gauss_noalloc(ctypes.c_void_p(sim), float(tol), int(max_iter), ctypes.byref(out),
                                        ctypes.c_void_p(stream)), "pic_solve_gauss_noalloc")
    return out


def pic_probe_stream(arrays, n: int, nontemporal: bool, stream: int):
    """arrays: six device pointers of n float32 each, read and written back."""
    ptrs = (ctypes.c_void_p * 6)(*arrays)
    _chk(load().pic_probe_stream(ptrs, int(n), int(bool(nontemporal)), ctypes.c_void_p(stream)), "pic_probe_stream")


def pic_get_counts(sim: int, n_species: int):
    out = (ctypes.c_int64 * MAX_SPECIES)()
    _chk(load().pic_get_counts(ctypes.c_void_p(sim), out), "pic_get_counts")
    return [int(out[k]) for k in range(n_species)]


def pic_get_state(sim: int, state: pic_host_state, stream: int):
    _chk(load().pic_get_state(ctypes.c_void_p(sim), ctypes.byref(state), ctypes.c_void_p(stream)),
         "pic_get_state")


def pic_set_state(sim: int, state: pic_host_state, stream: int):
    _chk(load().pic_set_state(ctypes.c_void_p(sim), ctypes.byref(state), ctypes.c_void_p(stream)),
         "pic_set_state")


def pic_get_tile_offsets(sim: int, species: int, n_tiles: int, stream: int):
    buf = (ctypes.c_int32 * (n_tiles + 1))()
    _chk(load().pic_get_tile_offsets(ctypes.c_void_p(sim), species, ctypes.cast(buf, ctypes.c_void_p),
                                     ctypes.c_void_p(stream)), "pic_get_tile_offsets")
    return list(buf)


def pic_set_timing(sim: int, enable: bool):
    _chk(load().pic_set_timing(ctypes.c_void_p(sim), 1 if enable else 0), "pic_set_timing")


def pic_set_timing_mask(sim: int, kernels):
    """Time only the named kernels (names from KERNELS); an empty list stops."""
    mask = 0
    for name in kernels:
        mask |= 1 << KERNELS.index(name)
    _chk(load().pic_set_timing_mask(ctypes.c_void_p(sim), mask), "pic_set_timing_mask")


def pic_get_timing(sim: int) -> pic_timing_out:
    out = pic_timing_out()
    _chk(load().pic_get_timing(ctypes.c_void_p(sim), ctypes.byref(out)), "pic_get_timing")
    return out


def pic_destroy(sim: int):
    load().pic_destroy(ctypes.c_void_p(sim))


def pic_batch_query(cfgs) -> int:
    arr = (pic_config * len(cfgs))(*cfgs)
    out = ctypes.c_size_t()
    _chk(load().pic_batch_query(len(cfgs), arr, ctypes.byref(out)), "pic_batch_query")
    return out.value


def pic_batch_init(cfgs, bufs, work: int, work_bytes: int, stream: int) -> int:
    ca = (pic_config * len(cfgs))(*cfgs)
    ba = (pic_buffers * len(bufs))(*bufs)
    h = ctypes.c_void_p()
    _chk(load().pic_batch_init(len(cfgs), ca, ba, ctypes.c_void_p(work), work_bytes, ctypes.c_void_p(stream),
                               ctypes.byref(h)), "pic_batch_init")
    return h.value


def pic_batch_step(batch: int, nsteps: int, stream: int):
    _chk(load().pic_batch_step(ctypes.c_void_p(batch), nsteps, ctypes.c_void_p(stream)), "pic_batch_step")


def pic_batch_capture(batch: int, stream: int):
    _chk(load().pic_batch_capture(ctypes.c_void_p(batch), ctypes.c_void_p(stream)), "pic_batch_capture")


def pic_batch_sim(batch: int, i: int) -> int:
    h = load().pic_batch_sim(ctypes.c_void_p(batch), i)
    if not h:
        raise PicError(PIC_EINVAL, "pic_batch_sim")
    return h


def pic_batch_check(batch: int, stream: int) -> int:
    return load().pic_batch_check(ctypes.c_void_p(batch), ctypes.c_void_p(stream))


def pic_batch_sync(batch: int, stream: int):
    _chk(load().pic_batch_sync(ctypes.c_void_p(batch), ctypes.c_void_p(stream)), "pic_batch_sync")


def pic_batch_destroy(batch: int):
    load().pic_batch_destroy(ctypes.c_void_p(batch))
