"""Periodic 2D PIC simulations on one MI355X, driven through libpic's C ABI.

PyTorch provides the device memory (caller-owned buffers of the C ABI) and the
streams; every step of the cycle runs in libpic's HIP kernels.  These classes
only allocate, upload, pack cell indices (ix | iy << 16) and download."""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _lib

PARTICLE_FIELDS = ("cell", "x", "y", "ux", "uy", "uz")


def pack_cells(ix: np.ndarray, iy: np.ndarray) -> np.ndarray:
    return (np.asarray(ix, np.int32) | (np.asarray(iy, np.int32) << 16)).astype(np.int32)


def unpack_cells(cell: np.ndarray):
    cell = np.asarray(cell, np.int32)
    return (cell & 0xFFFF).astype(np.int32), (cell >> 16).astype(np.int32)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libpic needs a GPU (torch.cuda.is_available() is False)")
    _lib.load()
    return torch


class _Buffers:
    """The caller-owned device buffers of one simulation (torch tensors) and
    the pic_config / pic_buffers structures that describe them."""

    def __init__(self, nx, ny, dx, dy, dt, tile, species, E=None, B=None, j_replicas=0, j_float=False,
                 device="cuda:0", j_filter=0, esirkepov=False, moving_window=False, capacity=None,
                 sort_every=1, motion_sort=False, ppl=0, quadratic=False):
        torch = _torch()
        if not 1 <= len(species) <= _lib.MAX_SPECIES:
            raise ValueError("1..4 species")
        self.nx, self.ny, self.tile = int(nx), int(ny), int(tile)
        cfg = _lib.pic_config()
        cfg.nx, cfg.ny, cfg.dx, cfg.dy, cfg.dt = self.nx, self.ny, float(dx), float(dy), float(dt)
        cfg.tile = self.tile
        cfg.j_replicas = int(j_replicas)
        cfg.n_species = len(species)
        cfg.flags = ((_lib.PIC_FLAG_J_FLOAT if j_float else 0) | (_lib.PIC_FLAG_ESIRKEPOV if esirkepov else 0) |
                     (_lib.PIC_FLAG_MOVING_WINDOW if moving_window else 0) | (_lib.PIC_FLAG_MOTION_SORT if motion_sort else 0) |
                     (_lib.PIC_FLAG_QUADRATIC if quadratic else 0))
        cfg.j_filter = int(j_filter)
        cfg.sort_every = int(sort_every)
        cfg.ppl = int(ppl)
        for k, (qm, q, st) in enumerate(species):
            cfg.species[k].qm = float(qm)
            cfg.species[k].q = float(q)
            cfg.species[k].n = int(np.asarray(st["ix"]).size)
            cfg.species[k].cap = int(capacity[k]) if capacity is not None else 0
        self.cfg = cfg
        sizes = _lib.pic_query(cfg)
        self.n_tiles = sizes.n_tiles
        dev = torch.device(device)
        self.fields = torch.zeros((9, self.ny, self.nx), dtype=torch.float32, device=dev)
        if E is not None:
            self.fields[0:3] = torch.from_numpy(np.ascontiguousarray(E, np.float32)).to(dev)
        if B is not None:
            self.fields[3:6] = torch.from_numpy(np.ascontiguousarray(B, np.float32)).to(dev)
        self.work = torch.empty(sizes.work_bytes + 256, dtype=torch.uint8, device=dev)
        bufs = _lib.pic_buffers()
        bufs.fields = self.fields.data_ptr()
        bufs.work = (self.work.data_ptr() + 255) & ~255
        bufs.work_bytes = sizes.work_bytes
        self.particles: List[Dict[str, "torch.Tensor"]] = []
        for k, (qm, q, st) in enumerate(species):
            n = int(cfg.species[k].n)
            cap = max(n, int(cfg.species[k].cap))
            p = {}
            for name in PARTICLE_FIELDS:
                a = pack_cells(st["ix"], st["iy"]) if name == "cell" else np.ascontiguousarray(st[name], np.float32)
                t = torch.zeros(cap, dtype=torch.int32 if name == "cell" else torch.float32, device=dev)
                if n:
                    t[:n] = torch.from_numpy(a).to(dev)
                p[name] = t
            self.particles.append(p)
            for name in PARTICLE_FIELDS:
                setattr(bufs.sp[k], name, p[name].data_ptr() if p[name].numel() else None)
        self.bufs = bufs


class _SimView:
    """The pic_* calls and host copies of one simulation (a pic_sim handle)."""

    handle: int
    stream: object
    buf: _Buffers

    @property
    def s(self) -> int:
        return self.stream.cuda_stream

    @property
    def nx(self):
        return self.buf.nx

    @property
    def ny(self):
        return self.buf.ny

    @property
    def n_tiles(self):
        return self.buf.n_tiles

    @property
    def fields(self):
        return self.buf.fields

    @property
    def particles(self):
        return self.buf.particles

    def push_deposit(self):
        _lib.pic_push_deposit(self.handle, self.s)

    def sort(self):
        _lib.pic_sort(self.handle, self.s)

    def field_advance(self):
        _lib.pic_field_advance(self.handle, self.s)

    def sync(self):
        """Bring the particle tensors up to date (pic_sync): complete what
        step()'s sort left to the next push (the hole fill, or the
        motion-class sort's copy back) and write every particle's cell into
        the cell tensor (the kernels keep 16-bit tile-relative cells in the
        workspace)."""
        _lib.pic_sync(self.handle, self.s)

    def step(self):
        _lib.pic_step(self.handle, self.s)

    def check(self) -> int:
        return _lib.pic_check(self.handle, self.s)

    def diag(self, what: int):
        return _lib.pic_diag(self.handle, what, self.s)

    def tile_offsets(self, species: int = 0) -> np.ndarray:
        return np.array(_lib.pic_get_tile_offsets(self.handle, species, self.n_tiles, self.s), dtype=np.int64)

    def set_timing(self, enable=True):
        """True / False: time every kernel or none; a list of kernel names
        (_lib.KERNELS): time only those."""
        if isinstance(enable, (list, tuple)):
            _lib.pic_set_timing_mask(self.handle, enable)
        else:
            _lib.pic_set_timing(self.handle, enable)

    def timing(self) -> Dict[str, tuple]:
        t = _lib.pic_get_timing(self.handle)
        return {name: (t.ms_total[k], t.launches[k]) for k, name in enumerate(_lib.KERNELS)}

    def counts(self):
        """Current particle count of every species (the moving window changes them)."""
        return _lib.pic_get_counts(self.handle, self.buf.cfg.n_species)

    def upload_particles(self, st: Dict[str, np.ndarray]) -> Dict[str, object]:
        """Device copies (cell, x, y, ux, uy, uz) of host particle arrays
        (ix, iy, x, y, ux, uy, uz), e.g. to keep new particles resident for
        move_window."""
        torch = _torch()
        dev = self.fields.device
        out = {}
        for name in PARTICLE_FIELDS:
            a = pack_cells(st["ix"], st["iy"]) if name == "cell" else np.ascontiguousarray(st[name], np.float32)
            out[name] = torch.from_numpy(a).to(dev)
        return out

    def move_window(self, inject: Sequence[Dict[str, object]]):
        """One moving-window step (pic_move_window); inject[k]: the new
        particles of species k, all in column nx - 1 and grouped by tile --
        host arrays (ix, iy, x, y, ux, uy, uz) or device tensors from
        upload_particles (cell, x, y, ux, uy, uz)."""
        torch = _torch()
        keep, arr, cnt = [], [], []
        for k in range(self.buf.cfg.n_species):
            st = inject[k]
            if "cell" not in st:
                st = self.upload_particles(st)
            keep.append(st)
            pp = _lib.pic_particles()
            n = int(st["cell"].numel())
            if n:
                for name in PARTICLE_FIELDS:
                    t = st[name]
                    want = torch.int32 if name == "cell" else torch.float32
                    if t.device != self.fields.device or t.dtype != want or not t.is_contiguous() or t.numel() != n:
                        raise ValueError(f"inject[{k}][{name!r}]: expected {n} contiguous {want} values on "
                                         f"{self.fields.device}")
                    setattr(pp, name, t.data_ptr())
            arr.append(pp)
            cnt.append(n)
        torch.cuda.synchronize(self.fields.device)
        _lib.pic_move_window(self.handle, arr, cnt, self.s)

    def state(self, species: int = 0) -> Dict[str, np.ndarray]:
        self.sync()
        self.stream.synchronize()
        p = self.particles[species]
        n = self.counts()[species]
        out = {name: p[name][:n].cpu().numpy() for name in PARTICLE_FIELDS}
        out["ix"], out["iy"] = unpack_cells(out["cell"])
        return out

    def get_state(self) -> Dict[str, object]:
        """Host copy of the step-to-step state through pic_get_state:
        {"fields": (9, ny, nx) float32, "species": [{cell, x, y, ux, uy, uz}],
        "window_origin": int}, in array columns."""
        cfg = self.buf.cfg
        hs = _lib.pic_host_state()
        out = {"fields": np.empty((9, self.ny, self.nx), np.float32), "species": []}
        hs.fields = out["fields"].ctypes.data
        counts = self.counts()
        for k in range(cfg.n_species):
            n = counts[k]
            arrs = {name: np.empty(n, np.int32 if name == "cell" else np.float32) for name in PARTICLE_FIELDS}
            for name in PARTICLE_FIELDS:
                setattr(hs.sp[k], name, arrs[name].ctypes.data if n else None)
            out["species"].append(arrs)
        _lib.pic_get_state(self.handle, hs, self.s)
        out["window_origin"] = int(hs.window_origin)
        return out

    def set_state(self, state: Dict[str, object]):
        """Load a state of the form get_state() returns (pic_set_state); the
        counts are the arrays' lengths."""
        cfg = self.buf.cfg
        hs = _lib.pic_host_state()
        keep = [np.ascontiguousarray(state["fields"], np.float32)]
        if keep[0].shape != (9, self.ny, self.nx):
            raise ValueError("fields must be (9, ny, nx)")
        hs.fields = keep[0].ctypes.data
        for k in range(cfg.n_species):
            sp = state["species"][k]
            n = int(np.asarray(sp["cell"]).size)
            hs.n[k] = n
            for name in PARTICLE_FIELDS:
                a = np.ascontiguousarray(sp[name], np.int32 if name == "cell" else np.float32)
                if a.size != n:
                    raise ValueError(f"species {k}: {name} has {a.size} entries, cell {n}")
                keep.append(a)
                setattr(hs.sp[k], name, a.ctypes.data if a.size else None)
        hs.window_origin = int(state.get("window_origin", 0))
        self.stream.synchronize()
        _lib.pic_set_state(self.handle, hs, self.s)

    def solve_gauss(self, tol: float = 0.0, max_iter: int = 0):
        """Make E and B valid initial fields for the current particles
        (pic_solve_gauss: E satisfies Gauss's law, div B = 0, curls kept).
        Returns the pic_gauss_out record (iterations, final residuals)."""
        torch = _torch()
        nbytes = _lib.gauss_scratch_bytes(self.nx, self.ny)
        scratch = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.fields.device)
        self.stream.synchronize()
        return _lib.pic_solve_gauss(self.handle, (scratch.data_ptr() + 255) & ~255, nbytes, tol, max_iter, self.s)

    def window_origin(self) -> int:
        """Array column of window column 0 (pic_get_window_origin)."""
        return _lib.pic_get_window_origin(self.handle)

    def window_fields(self) -> Dict[str, np.ndarray]:
        """field_arrays() in window columns: window column i is array column
        (i + origin) mod nx."""
        o = self.window_origin()
        return {k: np.roll(v, -o, axis=-1) for k, v in self.field_arrays().items()}

    def window_state(self, species: int = 0) -> Dict[str, np.ndarray]:
        """state() with ix in window columns (array order kept)."""
        o = self.window_origin()
        st = self.state(species)
        st["ix"] = ((st["ix"] - o) % self.nx).astype(np.int32)
        st["cell"] = pack_cells(st["ix"], st["iy"])
        return st

    def field_arrays(self) -> Dict[str, np.ndarray]:
        self.stream.synchronize()
        f = self.fields.cpu().numpy()
        return {"E": f[0:3].copy(), "B": f[3:6].copy(), "J": f[6:9].copy()}


class Sim(_SimView):
    """One simulation that owns its device buffers.

    species: list of (qm, q, state) where state is a dict of numpy arrays
    ix, iy (int32), x, y, ux, uy, uz (float32), in any order (pic_init groups
    them by tile).  The options map to pic_config: j_replicas, j_float
    (PIC_FLAG_J_FLOAT), j_filter, esirkepov (PIC_FLAG_ESIRKEPOV), quadratic
    (PIC_FLAG_QUADRATIC, the quadratic particle shape), moving_window and
    capacity, sort_every, motion_sort (PIC_FLAG_MOTION_SORT), ppl."""

    def __init__(self, nx: int, ny: int, dx: float, dy: float, dt: float, tile: int,
                 species: Sequence, E: Optional[np.ndarray] = None, B: Optional[np.ndarray] = None,
                 j_replicas: int = 0, j_float: bool = False, device: str = "cuda:0", stream=None,
                 j_filter: int = 0, esirkepov: bool = False, moving_window: bool = False, capacity=None,
                 sort_every: int = 1, motion_sort: bool = False, ppl: int = 0, quadratic: bool = False):
        torch = _torch()
        self.handle = None
        self.stream = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
        self.buf = _Buffers(nx, ny, dx, dy, dt, tile, species, E, B, j_replicas, j_float, device, j_filter,
                            esirkepov, moving_window, capacity, sort_every, motion_sort, ppl, quadratic)
        self.cfg = self.buf.cfg
        torch.cuda.synchronize(torch.device(device))
        self.handle = _lib.pic_init(self.cfg, self.buf.bufs, self.s)

    def close(self):
        if getattr(self, "handle", None):
            _lib.pic_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchMember(_SimView):
    """A member of a Batch (its pic_sim is owned by the batch)."""

    def __init__(self, batch, i, buf):
        self.batch = batch
        self.buf = buf
        self.stream = batch.stream
        self.handle = _lib.pic_batch_sim(batch.handle, i)


class Batch:
    """Many independent simulations advanced together: one launch per phase
    for all of them, optionally replayed from a captured HIP graph.

    members: list of dicts with keys nx, ny, dx, dy, dt, species (as for Sim)
    and optionally E, B.  All share tile, j_replicas, j_float, j_filter, the
    deposit scheme and particle shape, and the sort cadence."""

    def __init__(self, members: Sequence[dict], tile: int, j_replicas: int = 0, j_float: bool = False,
                 device: str = "cuda:0", stream=None, j_filter: int = 0, esirkepov: bool = False,
                 sort_every: int = 1, ppl: int = 0, motion_sort: bool = False, quadratic: bool = False):
        torch = _torch()
        self.handle = None
        self.stream = stream if stream is not None else torch.cuda.Stream(torch.device(device))
        self.bufs = [_Buffers(m["nx"], m["ny"], m["dx"], m["dy"], m["dt"], tile, m["species"], m.get("E"),
                              m.get("B"), j_replicas, j_float, device, j_filter, esirkepov,
                              sort_every=sort_every, ppl=ppl, motion_sort=motion_sort, quadratic=quadratic)
                     for m in members]
        cfgs = [b.cfg for b in self.bufs]
        nbytes = _lib.pic_batch_query(cfgs)
        self.work = torch.empty(nbytes + 256, dtype=torch.uint8, device=torch.device(device))
        torch.cuda.synchronize(torch.device(device))
        self.handle = _lib.pic_batch_init(cfgs, [b.bufs for b in self.bufs], (self.work.data_ptr() + 255) & ~255,
                                          nbytes, self.stream.cuda_stream)
        self.members = [BatchMember(self, i, b) for i, b in enumerate(self.bufs)]
        self.captured = False
        self.sort_every = max(1, int(sort_every))

    def __len__(self):
        return len(self.members)

    def __getitem__(self, i) -> BatchMember:
        return self.members[i]

    def step(self, nsteps: int = 1):
        _lib.pic_batch_step(self.handle, nsteps, self.stream.cuda_stream)

    def capture(self):
        _lib.pic_batch_capture(self.handle, self.stream.cuda_stream)
        self.captured = True

    def check(self) -> int:
        return _lib.pic_batch_check(self.handle, self.stream.cuda_stream)

    def sync(self):
        """pic_sync for every member at once (pic_batch_sync)."""
        _lib.pic_batch_sync(self.handle, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            _lib.pic_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
