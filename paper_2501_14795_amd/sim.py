"""A periodic 2D PIC simulation on one MI355X, driven through libpic's C ABI.

PyTorch provides the device memory (caller-owned buffers of the C ABI) and the
stream; every step of the cycle runs in libpic's HIP kernels.  This class only
allocates, uploads, packs cell indices (ix | iy << 16) and downloads."""
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


class Sim:
    """Owns the device buffers of one simulation.

    species: list of (qm, q, state) where state is a dict of numpy arrays
    ix, iy (int32), x, y, ux, uy, uz (float32), grouped by tile."""

    def __init__(self, nx: int, ny: int, dx: float, dy: float, dt: float, tile: int,
                 species: Sequence, E: Optional[np.ndarray] = None, B: Optional[np.ndarray] = None,
                 j_replicas: int = 0, j_float: bool = False, device: str = "cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libpic needs a GPU (torch.cuda.is_available() is False)")
        _lib.load()
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.nx, self.ny, self.tile = int(nx), int(ny), int(tile)
        cfg = _lib.pic_config()
        cfg.nx, cfg.ny, cfg.dx, cfg.dy, cfg.dt = self.nx, self.ny, float(dx), float(dy), float(dt)
        cfg.tile = self.tile
        cfg.j_replicas = int(j_replicas)
        cfg.n_species = len(species)
        cfg.flags = _lib.PIC_FLAG_J_FLOAT if j_float else 0
        if not 1 <= len(species) <= _lib.MAX_SPECIES:
            raise ValueError("1..4 species")
        for k, (qm, q, st) in enumerate(species):
            cfg.species[k].qm = float(qm)
            cfg.species[k].q = float(q)
            cfg.species[k].n = int(np.asarray(st["ix"]).size)
        self.cfg = cfg
        sizes = _lib.pic_query(cfg)
        self.n_tiles = sizes.n_tiles
        dev = self.device
        self.fields = torch.zeros((9, self.ny, self.nx), dtype=torch.float32, device=dev)
        if E is not None:
            self.fields[0:3] = torch.from_numpy(np.ascontiguousarray(E, np.float32)).to(dev)
        if B is not None:
            self.fields[3:6] = torch.from_numpy(np.ascontiguousarray(B, np.float32)).to(dev)
        self.work = torch.empty(sizes.work_bytes + 256, dtype=torch.uint8, device=dev)
        work_ptr = (self.work.data_ptr() + 255) & ~255
        self.particles: List[Dict[str, "torch.Tensor"]] = []
        bufs = _lib.pic_buffers()
        bufs.fields = self.fields.data_ptr()
        bufs.work = work_ptr
        bufs.work_bytes = sizes.work_bytes
        for k, (qm, q, st) in enumerate(species):
            cell = pack_cells(st["ix"], st["iy"])
            p = {"cell": torch.from_numpy(cell).to(dev)}
            for name in PARTICLE_FIELDS[1:]:
                p[name] = torch.from_numpy(np.ascontiguousarray(st[name], np.float32)).to(dev)
            self.particles.append(p)
            for name in PARTICLE_FIELDS:
                setattr(bufs.sp[k], name, p[name].data_ptr() if p[name].numel() else None)
        self.bufs = bufs
        torch.cuda.synchronize(dev)
        self.handle = _lib.pic_init(cfg, bufs, self.stream.cuda_stream)

    # ---- the C functions
    @property
    def s(self) -> int:
        return self.stream.cuda_stream

    def push_deposit(self):
        _lib.pic_push_deposit(self.handle, self.s)

    def sort(self):
        _lib.pic_sort(self.handle, self.s)

    def field_advance(self):
        _lib.pic_field_advance(self.handle, self.s)

    def step(self):
        _lib.pic_step(self.handle, self.s)

    def check(self) -> int:
        return _lib.pic_check(self.handle, self.s)

    def diag(self, what: int):
        return _lib.pic_diag(self.handle, what, self.s)

    def tile_offsets(self, species: int = 0) -> np.ndarray:
        return np.array(_lib.pic_get_tile_offsets(self.handle, species, self.n_tiles, self.s), dtype=np.int64)

    def set_timing(self, enable: bool = True):
        _lib.pic_set_timing(self.handle, enable)

    def timing(self) -> Dict[str, tuple]:
        t = _lib.pic_get_timing(self.handle)
        return {name: (t.ms_total[k], t.launches[k]) for k, name in enumerate(_lib.KERNELS)}

    # ---- host copies
    def state(self, species: int = 0) -> Dict[str, np.ndarray]:
        self.stream.synchronize()
        p = self.particles[species]
        out = {name: p[name].cpu().numpy() for name in PARTICLE_FIELDS}
        out["ix"], out["iy"] = unpack_cells(out["cell"])
        return out

    def field_arrays(self) -> Dict[str, np.ndarray]:
        self.stream.synchronize()
        f = self.fields.cpu().numpy()
        return {"E": f[0:3].copy(), "B": f[3:6].copy(), "J": f[6:9].copy()}

    def close(self):
        if getattr(self, "handle", None):
            _lib.pic_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
