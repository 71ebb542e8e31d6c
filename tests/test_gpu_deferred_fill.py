"""pic_step's sort leaves its last part -- the copy of the staged movers into
their holes -- to the next push, which streams those slots anyway.

* Until then the caller's x, y, ux, uy, uz arrays hold stale values in
  exactly those slots (at most one per mover of the step), and pic_sync()
  makes them equal, bit for bit, to a twin that sorted eagerly
  (pic_push_deposit, pic_sort, pic_field_advance); the next pic_step needs no
  sync in between.  The cell array (the kernels keep tile-relative cells in
  the workspace) is written by pic_sync() only.
* With a sort cadence of 2 the fill is consumed by the first push after the
  sort and not done again by the unsorted push that follows.
* pic_batch_sync() completes the fill of every member in one launch: the
  members' raw arrays then equal their own pic_sync-ed state.
"""
import numpy as np
import pytest

import pic_workloads as pw
from _parity import flush, species_states

pytestmark = pytest.mark.gpu

DX = DY = 0.1
DT = 0.07
FIELDS = ("cell", "x", "y", "ux", "uy", "uz")
STREAMED = FIELDS[1:]   # what the kernels write in the caller's arrays


def _raw(sim, k=0):
    """The particle tensors as they are on the device, without any sync."""
    import torch
    torch.cuda.synchronize()
    n = sim.counts()[k]
    return {f: sim.particles[k][f][:n].cpu().numpy() for f in FIELDS}


@pytest.mark.parametrize("tile,every", [(16, 1), (32, 1), (8, 2)])
def test_sync_completes_the_deferred_fill(tile, every):
    from paper_2501_14795_amd import Sim, _lib
    nx = ny = 64
    spec = pw.SpeciesSpec(-1.0, (3, 3), (0.25, 0.25, 0.2), (0.3, -0.2, 0.1))
    state = species_states(nx, ny, tile, [spec], 31)[0]
    E, B = pw.random_fields(nx, ny, 0.05, 31)
    lazy = Sim(nx, ny, DX, DY, DT, tile, [(spec.qm, spec.q, state)], E=E, B=B, sort_every=every)
    eager = Sim(nx, ny, DX, DY, DT, tile, [(spec.qm, spec.q, state)], E=E, B=B, sort_every=every)
    for k in range(6):
        lazy.step()   # never synced before the last step: every fill is the next push's
        eager.push_deposit()
        sorted_now = (k + 1) % every == 0
        if sorted_now:
            eager.sort()
        eager.field_advance()
        got, want = _raw(lazy), _raw(eager)
        stale = np.zeros(want["x"].size, bool)
        for f in STREAMED:
            stale |= got[f] != want[f]
        # the movers of this step (pic_diag's counts read the count records
        # and mover counts only; it completes the fill too, so use a twin)
        movers = eager.diag(_lib.PIC_DIAG_COUNTS).movers[0] if sorted_now else 0
        assert stale.sum() <= movers, (k, stale.sum(), movers)
        if not sorted_now:
            assert stale.sum() == 0, k   # the push placed the last sort's movers, once
        assert np.array_equal(lazy.tile_offsets(0), eager.tile_offsets(0))
        flush(f"T{tile} every {every} step {k}: {stale.sum()} stale slots ({movers} movers)")
    lazy.sync()
    eager.sync()   # no fill pending: writes its cells
    got, want = _raw(lazy), _raw(eager)
    for f in FIELDS:
        assert np.array_equal(got[f], want[f]), f
    fa, fb = lazy.field_arrays(), eager.field_arrays()
    for c in fa:
        assert np.array_equal(fa[c], fb[c]), c
    flush(f"T{tile} every {every}: after pic_sync equal to the eager twin bit for bit")
    assert lazy.check() == 0 and eager.check() == 0
    lazy.close()
    eager.close()


def test_batch_sync_fills_every_member():
    from paper_2501_14795_amd import Batch
    specs = pw.batched_members(6, 9, sizes=(32, 48, 64), ppcs=(8, 16))
    members = []
    for m in specs:
        st = pw.species_state(m["nx"], m["ny"], 16, m["spec"], m["seed"])
        members.append({"nx": m["nx"], "ny": m["ny"], "dx": m["dx"], "dy": m["dy"], "dt": m["dt"],
                        "species": [(m["spec"].qm, m["spec"].q, st)]})
    b = Batch(members, tile=16)
    b.step(3)
    b.sync()
    for i in range(len(members)):
        raw = _raw(b[i])
        st = b[i].state(0)
        for f in FIELDS:
            assert np.array_equal(raw[f], st[f]), (i, f)
    assert b.check() == 0
    flush(f"{len(members)} members: raw arrays after pic_batch_sync equal their synced state")
    b.close()


@pytest.mark.parametrize("tile", [8, 32])
def test_cells_right_after_a_sort(tile):
    """A particle that crossed into a tile and already sits inside that
    tile's new section is not moved by the canonical sort, so its 16-bit cell
    is still relative to the tile it left; right after a sort the cells are
    read modulo the tile edge (the publish, the next push).  The case occurs
    here (counted from the oracle's permutation), every sorted state read back
    is the oracle's canonical sort, bit for bit, and every push from such a
    state agrees with the oracle's push of it (positions, as ix + x, and
    momenta within 1e-5)."""
    import oracle
    from _parity import oracle_from_gpu, particle_errors, sort_replay
    from paper_2501_14795_amd import Sim
    nx = ny = 64
    spec = pw.SpeciesSpec(-1.0, (4, 4), (0.3, 0.3, 0.2), (0.35, -0.25, 0.1))
    state = species_states(nx, ny, tile, [spec], 47)[0]
    E, B = pw.random_fields(nx, ny, 0.05, 47)
    sim = Sim(nx, ny, DX, DY, DT, tile, [(spec.qm, spec.q, state)], E=E, B=B)
    in_place = 0
    for k in range(5):
        ref = oracle_from_gpu(sim, [spec], DX, DY, DT)   # the state right after the sort
        ref.push_deposit()
        sim.push_deposit()   # reads its cells modulo the edge
        pos, du = particle_errors(sim.state(0), ref.species[0], nx, ny)
        assert pos <= 1e-5 and du <= 1e-5, (k, pos, du)
        old_off = sim.tile_offsets(0)
        pre = sort_replay(sim, [spec], tile)[0]   # publish right after the sort: modulo the edge
        _, src = oracle.sort_canonical(nx, ny, tile, pre["ix"], pre["iy"])
        slots = np.arange(src.size)
        held_by = np.searchsorted(old_off, slots, side="right") - 1   # tile of the old section
        now_in = (pre["iy"] // tile) * (nx // tile) + pre["ix"] // tile
        in_place += int(np.count_nonzero((src == slots) & (now_in != held_by)))
        sim.field_advance()
    assert in_place > 0
    assert sim.check() == 0
    flush(f"T{tile}: {in_place} particles entered a tile in place over 5 sorts; every sort bit-exact")
    sim.close()
