"""The alternative sort (PIC_FLAG_MOTION_SORT; the motion-class sort Sec. 4.3
cites, after Germaschewski et al.): after the push every particle is moved,
in one counting pass over the push's per-class counts, to its slot in the
order (new tile, motion class, old slot), out of place, and copied back (in
pic_step, read back by the next push).

Bit-exact against the oracle's motion-class sort of the GPU's post-push state
and tile_offset (every array and the new tile_offset), with one and two
species, at T = 8, 16, 32, with a sort cadence of 2, and on grids of one and
two tiles per axis (where the classes of the two neighbours coincide); free
runs within the usual tolerances of the oracle, and the same physics as the
in-place sort (fields within round-off after 10 steps); batched members equal
to standalone runs bit for bit."""
import numpy as np
import pytest

import oracle
import pic_workloads as pw
from _parity import flush, make_pair, matched_particle_errors, oracle_from_gpu, particle_errors, rel_err, species_states

pytestmark = pytest.mark.gpu

DX = DY = 0.1
DT = 0.07
ARRAYS = ("ix", "iy", "x", "y", "ux", "uy", "uz")


def _specs(nspecies):
    drifts = [(0.6, -0.4, 0.2), (-0.5, 0.3, 0.0)]
    return [pw.SpeciesSpec(-1.0, (3, 3), (0.3, 0.3, 0.3), drifts[k]) for k in range(nspecies)]


@pytest.mark.parametrize("nx,ny,tile,nspecies,every", [(64, 64, 16, 1, 1), (96, 64, 32, 2, 1), (64, 32, 8, 1, 2),
                                                       (32, 16, 16, 1, 1), (16, 32, 8, 2, 1)])
def test_motion_sort_replay(nx, ny, tile, nspecies, every):
    specs = _specs(nspecies)
    states = species_states(nx, ny, tile, specs, 6)
    E, B = pw.random_fields(nx, ny, 0.05, 6)
    sim, _ = make_pair(nx, ny, DX, DY, DT, tile, specs, states, E, B, sort_every=every, motion_sort=True)
    worst = [0.0, 0.0, 0.0]
    moved = 0
    for step in range(3 * every):
        ref = oracle_from_gpu(sim, specs, DX, DY, DT)
        ref.push_deposit()
        sim.push_deposit()
        assert sim.check() == 0
        for k in range(nspecies):
            pos, du = particle_errors(sim.state(k), ref.species[k], nx, ny)
            worst[0], worst[1] = max(worst[0], pos), max(worst[1], du)
        worst[2] = max(worst[2], rel_err(sim.field_arrays()["J"], ref.J))
        if step % every == every - 1:
            pre = [sim.state(k) for k in range(nspecies)]
            off_old = [sim.tile_offsets(k) for k in range(nspecies)]
            sim.sort()
            assert sim.check() == 0
            for k in range(nspecies):
                off, src = oracle.sort_motion_classes(nx, ny, tile, pre[k]["ix"], pre[k]["iy"], off_old[k])
                post = sim.state(k)
                for a in ARRAYS:
                    assert np.array_equal(post[a], pre[k][a][src]), a
                assert np.array_equal(sim.tile_offsets(k), off)
                moved += int((src != np.arange(src.size)).sum())
        sim.field_advance()
    flush(f"motion sort {nx}x{ny} T{tile} x{nspecies} k={every}: pos {worst[0]:.2e} u {worst[1]:.2e} "
          f"J {worst[2]:.2e}; regrouping bit-exact ({moved} particles changed slot)")
    assert worst[0] < 1e-5 and worst[1] < 1e-5 and worst[2] < 1e-5
    assert moved > 0
    sim.close()


def test_motion_sort_free_run_matches_oracle_and_in_place_sort():
    nx = ny = 64
    specs = _specs(1)
    states = species_states(nx, ny, 16, specs, 7)
    motion, ora = make_pair(nx, ny, DX, DY, DT, 16, specs, states, motion_sort=True)
    inplace, _ = make_pair(nx, ny, DX, DY, DT, 16, specs, states)
    for _ in range(10):
        motion.step()
        inplace.step()
        ora.step(T=16)
    assert motion.check() == 0 and inplace.check() == 0
    fm, fi = motion.field_arrays(), inplace.field_arrays()
    e_ora = {c: rel_err(fm[c], getattr(ora, c)) for c in ("E", "B", "J")}
    same = {c: bool(np.array_equal(fm[c], fi[c])) for c in ("E", "B", "J")}
    pos, du, _ = matched_particle_errors(motion.state(0), ora.species[0], nx, ny)
    flush(f"motion sort, 10 steps: vs oracle {e_ora}, bit-identical to the in-place sort {same}; "
          f"particles {pos:.2e} {du:.2e}")
    # the fixed-point current does not depend on particle order: E, B, J equal the in-place sort's
    assert all(same.values())
    assert max(e_ora.values()) <= 1e-5
    assert pos < 1e-5 and du < 1e-5
    motion.close()
    inplace.close()


@pytest.mark.parametrize("tile,every", [(16, 1), (8, 2)])
def test_batched_motion_sort_equals_members_run_alone(tile, every):
    from paper_2501_14795_amd import Batch, Sim
    specs = pw.batched_members(5, 40 + tile, sizes=(32, 48, 64, 96), ppcs=(8, 16))
    members = []
    for m in specs:
        st = pw.species_state(m["nx"], m["ny"], tile, m["spec"], m["seed"])
        members.append({"nx": m["nx"], "ny": m["ny"], "dx": m["dx"], "dy": m["dy"], "dt": m["dt"],
                        "species": [(m["spec"].qm, m["spec"].q, st)]})
    batch = Batch(members, tile=tile, sort_every=every, motion_sort=True)
    alone = [Sim(m["nx"], m["ny"], m["dx"], m["dy"], m["dt"], tile, m["species"], sort_every=every,
                 motion_sort=True) for m in members]
    for step in range(4):
        if step == 2:
            batch.capture()
        batch.step()
        for s in alone:
            s.step()
    assert batch.check() == 0
    for i, s in enumerate(alone):
        assert s.check() == 0
        sa, sb = s.state(0), batch[i].state(0)
        for k in sa:
            assert np.array_equal(sa[k], sb[k]), k
        fa, fb = s.field_arrays(), batch[i].field_arrays()
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), k
        assert np.array_equal(s.tile_offsets(0), batch[i].tile_offsets(0))
        s.close()
    flush(f"batched motion sort T={tile} k={every}: {len(members)} members equal their standalone runs")
    batch.close()


@pytest.mark.parametrize("tile,every", [(16, 1), (32, 1), (8, 2)])
def test_step_leaves_the_copy_back_to_the_next_push(tile, every):
    """pic_step's motion-class sort leaves its last pass (the staging arrays
    copied back) to the next push, which reads the particles from the staging
    arrays; a state read in between completes the copy instead.  Six steps,
    one state read after the third, against a twin that sorts eagerly
    (pic_push_deposit, pic_sort, pic_field_advance): every array, the fields
    and tile_offset equal bit for bit."""
    from paper_2501_14795_amd import Sim
    nx, ny = 64, 64
    spec = _specs(1)[0]
    state = species_states(nx, ny, tile, [spec], 17)[0]
    E, B = pw.random_fields(nx, ny, 0.05, 17)
    lazy = Sim(nx, ny, DX, DY, DT, tile, [(spec.qm, spec.q, state)], E=E, B=B, sort_every=every, motion_sort=True)
    eager = Sim(nx, ny, DX, DY, DT, tile, [(spec.qm, spec.q, state)], E=E, B=B, sort_every=every, motion_sort=True)

    def same():
        a, b = lazy.state(0), eager.state(0)
        for k in a:
            assert np.array_equal(a[k], b[k]), k
        fa, fb = lazy.field_arrays(), eager.field_arrays()
        for c in fa:
            assert np.array_equal(fa[c], fb[c]), c
        assert np.array_equal(lazy.tile_offsets(0), eager.tile_offsets(0))

    for k in range(6):
        lazy.step()
        eager.push_deposit()
        if (k + 1) % every == 0:
            eager.sort()
        eager.field_advance()
        if k == 2:
            same()   # completes the pending copy; the next push reads the particle arrays
    same()
    assert lazy.check() == 0 and eager.check() == 0
    flush(f"T{tile} every {every}: deferred copy back equal to the eager sort bit for bit")
    lazy.close()
    eager.close()


@pytest.mark.parametrize("motion", [True, False])
def test_set_state_while_the_copy_back_is_pending(motion):
    """A state loaded (pic_set_state) while pic_step's copy back (motion-class
    sort) or hole fill (in-place sort) is still pending replaces the
    particles: the next push reads the loaded ones, not the staging arrays or
    records.  The run from there equals a fresh simulation loaded from the
    same state, bit for bit."""
    from paper_2501_14795_amd import Sim
    nx = ny = 64
    tile = 16
    spec = _specs(1)[0]
    a = species_states(nx, ny, tile, [spec], 23)[0]
    b = species_states(nx, ny, tile, [spec], 24)[0]
    E, B = pw.random_fields(nx, ny, 0.05, 23)
    donor = Sim(nx, ny, DX, DY, DT, tile, [(spec.qm, spec.q, b)], E=E, B=B, motion_sort=motion)
    for _ in range(2):
        donor.step()
    ck = donor.get_state()
    busy = Sim(nx, ny, DX, DY, DT, tile, [(spec.qm, spec.q, a)], E=E, B=B, motion_sort=motion)
    busy.step()               # its copy back (or hole fill) is now pending
    busy.set_state(ck)
    fresh = Sim(nx, ny, DX, DY, DT, tile, [(spec.qm, spec.q, a)], E=E, B=B, motion_sort=motion)
    fresh.set_state(ck)
    for _ in range(3):
        busy.step()
        fresh.step()
    sa, sb = busy.state(0), fresh.state(0)
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    fa, fb = busy.field_arrays(), fresh.field_arrays()
    for c in fa:
        assert np.array_equal(fa[c], fb[c]), c
    assert busy.check() == 0 and fresh.check() == 0
    flush(f"motion sort {motion}: set_state during a pending copy back / fill: the loaded state is the one pushed")
    for s in (donor, busy, fresh):
        s.close()
