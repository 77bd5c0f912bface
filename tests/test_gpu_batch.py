"""GPU parity of batched stepping (pss_batch_*): every member of a batch must
end bit for bit where the same lattice stepped alone ends, and a member must
stay on the FP64 oracle."""

import numpy as np
import pytest

from tests.conftest import gpu_available
from tests import inputs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402
from paper_2405_02410_amd import Mono, PssError  # noqa: E402
from oracle import model as om  # noqa: E402
from oracle.spectral import Lattice as OLattice  # noqa: E402


def _model_b(n, seed, D=0.01, dt=0.01, a=-1.0):
    lat = pss.Lattice(n, dt=dt, seed=seed)
    f, _ = pss.model_b(lat, a=a, D=D)
    lat.init_uniform(f, -0.1, 0.1)
    return lat


def _two_field(n, seed):
    lat = pss.Lattice(n, dt=0.005, seed=seed)
    phi = lat.field("phi")
    psi = lat.field("psi")
    lat.term(phi, [Mono(1.0, q2=1), Mono(-1.0, q2=2)], [(phi, 1)], implicit=True)
    lat.term(phi, [Mono(-1.0, q2=1)], [(phi, 3)])
    lat.term(phi, [Mono(-0.15, q2=1)], [(phi, 1), (psi, 2)])
    lat.term(psi, [Mono(0.5), Mono(-1.0, q2=1)], [(psi, 1)], implicit=True)
    lat.term(psi, [Mono(-1.0)], [(psi, 3)])
    lat.term(psi, [Mono(-0.3)], [(phi, 1), (psi, 1)])
    lat.noise(phi, [Mono(0.005, q2=1)])
    lat.noise(psi, [Mono(0.005)])
    lat.init_uniform(phi)
    lat.init_uniform(psi)
    return lat


# members of uneven size and model; the builder of each is called twice
MEMBERS = [
    lambda: _model_b((64, 64), 1),
    lambda: _model_b((64, 64), 2),
    lambda: _model_b((64, 64), 2**40 + 7),
    lambda: _model_b((64, 64), 4, D=0.0),      # noiseless, same class
    lambda: _model_b((128, 128), 10),
    lambda: _model_b((128, 128), 11, a=-0.5),  # other coefficients, same class
    lambda: _model_b((32, 128), 12),
    lambda: _model_b((256, 16), 13),
    lambda: _two_field((64, 64), 14),
]


def _fields(lat):
    return range(len(lat.names))


def test_batch_is_bitwise_the_single_lattice_path():
    mem = [b() for b in MEMBERS]
    twins = [b() for b in MEMBERS]
    batch = pss.Batch(mem)
    nc, of = batch.classes()
    assert nc == 5 and of[:4] == [0, 0, 0, 0] and of[4] == of[5] != of[0]
    # LDS-resident: the 64^2 and 128^2 Model B classes.  Fused: the update of
    # 32x128 and the x pass of 256x16.  On their own: the update of 256x16
    # (lines of 16), the x pass of 32x128 (rows of 32), both of the two-field
    # class
    assert batch.launches() == (6, 1, 2)
    batch.step(7)
    batch.step(60)  # crosses a graph chunk
    batch.sync()
    for lat, tw in zip(mem, twins):
        tw.step(67)
        assert lat.step_index == 67
        for f in _fields(lat):
            assert np.array_equal(lat.spectrum(f), tw.spectrum(f)), (lat.n, f)
    batch.close()


def test_batch_member_on_the_oracle():
    p = inputs.MODEL_B
    mem = [_model_b((64, 64), s) for s in (3, 5, 8)]
    batch = pss.Batch(mem)
    mass0 = mem[1].mass(0)
    batch.step(100)
    m = om.model_b(OLattice(64, 64, 1), p["dt"], a=p["a"], b=p["b"], k=p["k"], D=0.01, seed=5)
    m.init_uniform(0, -0.1, 0.1)
    m.step(100)
    phi = mem[1].download(0)
    assert np.max(np.abs(phi - m.real(0)[0])) <= 1e-4
    assert abs(mem[1].mass(0) - mass0) <= 1e-6 * np.sum(np.abs(phi))
    batch.close()


def test_batch_seeds_and_interleaving_with_own_steps():
    mem = [_model_b((64, 64), 0) for _ in range(3)]  # same initial field, noise keys set by the batch
    twins = [_model_b((64, 64), 0) for _ in range(3)]
    for tw, s in zip(twins, (21, 22, 23)):
        tw.seed(s)
    batch = pss.Batch(mem, seeds=[21, 22, 23])
    mem[0].step(5)          # alone first
    batch.step(10)
    mem[2].set_coef(1, 0, -2.0)   # coefficient change between batch steps
    twins[2].step(10)
    twins[2].set_coef(1, 0, -2.0)
    batch.step(6)
    mem[1].step(3)          # alone after
    twins[0].step(16 + 5)
    twins[1].step(16 + 3)
    twins[2].step(6)
    for i, (lat, tw) in enumerate(zip(mem, twins)):
        assert lat.step_index == tw.step_index, i
        assert np.array_equal(lat.spectrum(0), tw.spectrum(0)), i
    batch.close()


def test_batch_restores_after_state_load():
    a = _model_b((128, 64), 31)
    b = _model_b((128, 64), 32)
    batch = pss.Batch([a, b])
    batch.step(20)
    blob = a.save()
    ref = _model_b((128, 64), 31)
    ref.step(20)
    batch.step(5)
    a.load(blob)             # back to step 20: channels rebuilt before the next batch step
    batch.step(5)
    ref.step(5)
    assert np.array_equal(a.spectrum(0), ref.spectrum(0))
    batch.close()


def test_member_outlives_its_batch():
    a = _model_b((64, 64), 1)
    batch = pss.Batch([a])
    batch.step(2)
    with pytest.raises(PssError) as e:
        a.close()
    assert e.value.name == "PSS_E_STATE"
    batch.close()
    a.step(1)
    a.close()


def test_batch_kernel_timing_and_bytes():
    mem = [_model_b((256, 256), s) for s in range(4)]
    single = _model_b((256, 256), 9)
    batch = pss.Batch(mem)
    blobs = [lat.save() for lat in mem]  # timing launches overwrite the state
    ms, nbytes = batch.time_kernel(0, pss.KERNEL_UPDATE, 20)
    assert ms > 0 and nbytes == 4 * single.kernel_bytes(pss.KERNEL_UPDATE)
    ms, nbytes = batch.time_kernel(0, pss.KERNEL_X, 20)
    assert ms > 0 and nbytes == 4 * single.kernel_bytes(pss.KERNEL_X)
    for which in (pss.KERNEL_UPDATE, pss.KERNEL_X):  # the fused launches
        ms, nbytes = batch.time_kernel(-1, which, 20)
        assert ms > 0 and nbytes == 4 * single.kernel_bytes(which)
    with pytest.raises(PssError):
        batch.time_kernel(-2, pss.KERNEL_UPDATE, 5)  # no LDS-resident class
    # restore the states; the next batch step must rebuild the stale channels
    twins = [_model_b((256, 256), s) for s in range(4)]
    for lat, blob in zip(mem, blobs):
        lat.load(blob)
    batch.step(3)
    for lat, tw in zip(mem, twins):
        tw.step(3)
        assert np.array_equal(lat.spectrum(0), tw.spectrum(0))
    batch.close()
    # the LDS-resident launch: per-step time and HBM bytes (state and channel
    # array in and out once per launch of `reps` steps)
    res = [_model_b((128, 128), s) for s in range(3)]
    rb = pss.Batch(res)
    blobs = [lat.save() for lat in res]
    ms, nbytes = rb.time_kernel(-2, pss.KERNEL_UPDATE, 10)
    assert ms > 0 and nbytes == 16 * 128 * 128 * 3 / 10
    with pytest.raises(PssError):
        rb.time_kernel(-1, pss.KERNEL_UPDATE, 5)  # no fused launch
    for lat, blob in zip(res, blobs):
        lat.load(blob)
    rb.step(4)
    twins = [_model_b((128, 128), s) for s in range(3)]
    for lat, tw in zip(res, twins):
        tw.step(4)
        assert np.array_equal(lat.spectrum(0), tw.spectrum(0))
    rb.close()


def test_full_ensemble_configuration_sampled():
    # the batched ensemble exactly as bench.py runs it (256 x 128^2 + 64 x 256^2
    # + 16 x 512^2, seeds 1000 + i); two members of each size re-run alone
    sizes = [128] * 256 + [256] * 64 + [512] * 16
    mem = [_model_b((s, s), 1000 + i) for i, s in enumerate(sizes)]
    batch = pss.Batch(mem)
    assert batch.classes()[0] == 3
    # 128^2 LDS-resident; 256^2 and 512^2 in one fused launch per phase
    assert batch.launches() == (2, 2, 1)
    batch.step(25)
    for i in (0, 255, 256, 319, 320, 335):
        twin = _model_b((sizes[i], sizes[i]), 1000 + i)
        twin.step(25)
        assert np.array_equal(mem[i].spectrum(0), twin.spectrum(0)), i
    batch.close()


@pytest.mark.parametrize("n", [(64, 64), (128, 128), (64, 128), (128, 64)])
def test_resident_launch_is_bitwise_the_single_path(n, monkeypatch):
    """Every lattice shape of the LDS-resident kernel, with and without noise,
    and a member whose state went non-finite: equal bit for bit to the lattice
    stepped alone and to the batch with the resident launch turned off; steps
    that cross graph chunks, and a chunk of one step."""
    def make():
        return [_model_b(n, 40 + i, D=0.0 if i == 1 else 0.01) for i in range(3)]
    mem, off, twins = make(), None, make()
    batch = pss.Batch(mem)
    assert batch.launches()[2] == 1
    monkeypatch.setenv("PSS_BATCH_RESIDENT", "0")
    off = make()
    batch_off = pss.Batch(off)
    assert batch_off.launches()[2] == 0
    monkeypatch.delenv("PSS_BATCH_RESIDENT")
    for k in (1, 60, 7):
        batch.step(k)
        batch_off.step(k)
    batch.sync()
    batch_off.sync()
    for lat, lo, tw in zip(mem, off, twins):
        tw.step(68)
        assert lat.step_index == 68
        assert np.array_equal(lat.spectrum(0), tw.spectrum(0))
        assert np.array_equal(lo.spectrum(0), tw.spectrum(0))
    # after the batch: the member's own steps continue from the right counter
    mem[0].step(5)
    twins[0].step(5)
    assert np.array_equal(mem[0].spectrum(0), twins[0].spectrum(0))
    batch.close()
    batch_off.close()


def test_resident_member_matches_the_oracle():
    n, steps = (128, 128), 100
    lat = _model_b(n, 77)
    other = _model_b(n, 78)
    batch = pss.Batch([lat, other])
    assert batch.launches()[2] == 1
    batch.step(steps)
    batch.sync()
    m = om.model_b(OLattice(n[0], n[1], 1), 0.01, a=-1.0, b=1.0, k=1.0, D=0.01, seed=77)
    m.init_uniform(0, -0.1, 0.1)
    m.step(steps)
    want = m.real(0)[0]
    assert np.max(np.abs(lat.download(0) - want)) <= 1e-4 * max(1.0, np.max(np.abs(want)))
    batch.close()


def test_resident_nonfinite_flag():
    lat = _model_b((64, 64), 5)
    other = _model_b((64, 64), 6)
    bad = np.zeros((64, 64), dtype=np.float32)
    bad[3, 7] = np.inf
    lat.upload(0, bad)
    batch = pss.Batch([lat, other])
    assert batch.launches()[2] == 1
    batch.step(2)
    with pytest.raises(PssError) as e:
        batch.sync()
    assert e.value.name == "PSS_E_NONFINITE"
    batch.close()


def test_member_stream_is_fixed_while_a_batch_holds_it():
    import torch
    lats = []
    for s in (1, 2):
        lat = pss.Lattice((64, 64), dt=0.01, seed=s)
        f, _ = pss.model_b(lat)
        lat.init_uniform(f)
        lats.append(lat)
    b = pss.Batch(lats)
    st = torch.cuda.Stream()
    with pytest.raises(pss.PssError) as e:
        lats[0].stream(st.cuda_stream)
    assert e.value.name == "PSS_E_STATE"
    b.step(3)
    b.sync()
    b.close()
    lats[0].stream(st.cuda_stream)  # allowed once the batch is gone
    lats[0].step(2)
    lats[0].sync()
    assert lats[0].step_index == 5


def test_batch_of_multi_field_models_is_bitwise_the_single_path():
    # Model H members (three fields, general operators, shared channels) and
    # a two-field member run in per-class launches: each member gets bit for
    # bit what pss_step gives it alone
    def mh(seed):
        lat = pss.Lattice((64, 64), dt=0.01, seed=seed)
        ids, _ = pss.model_h(lat, D=0.01)
        lat.init_uniform(ids[0], -0.4, 0.4)
        return lat, ids

    def two(seed):
        lat = pss.Lattice((128, 64), dt=0.01, seed=seed)
        a = lat.field("a")
        b = lat.field("b")
        lat.term(a, [Mono(-0.5), Mono(-1.0, q2=1)], [(a, 1)], implicit=True)
        lat.term(b, [Mono(-0.2, q2=1)], [(b, 1)], implicit=True)
        lat.term(a, [Mono(-1.0)], [(a, 3)])
        lat.term(b, [Mono(0.3)], [(a, 1), (b, 1)])
        lat.noise(a, [Mono(0.004)])
        for f in (a, b):
            lat.init_uniform(f, -0.3, 0.3)
        return lat, (a, b)

    members = [mh(3), mh(5), two(7), mh(9)]
    alone = [mh(3), mh(5), two(7), mh(9)]
    batch = pss.Batch([m for m, _ in members])
    batch.step(40)
    batch.sync()
    for (m, ids), (r, _) in zip(members, alone):
        r.step(40)
        for f in ids:
            assert np.array_equal(m.spectrum(f), r.spectrum(f))
    batch.close()
