"""pss_field_bind on the GPU: a torch tensor holds a field's Fourier state.

Checks, through the C interface: a bound lattice steps bitwise like an
unbound twin; the tensor is byte for byte the field's block of the saved
state; a state written into the tensor by torch and announced with
pss_state_changed is the one the next steps start from (bitwise against a
lattice that holds that state itself); and the library never frees the
tensor's memory.
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X")]

import paper_2405_02410_amd as pss  # noqa: E402


def _lat(bound, lo=-0.1, hi=0.1, n=(256, 128)):
    import torch
    lat = pss.Lattice(n, dt=0.01, seed=3)
    f, _ = pss.model_b(lat)
    t = None
    if bound:
        t = torch.full((lat.state_bytes(f) // 8,), 7.0, dtype=torch.complex64, device="cuda")
        lat.bind(f, t)
    lat.init_uniform(f, lo, hi)
    return lat, f, t


def test_bound_tensor_holds_the_state():
    import torch
    a, f, t = _lat(True)
    b, g, _ = _lat(False)
    a.step(60)
    b.step(60)
    assert np.array_equal(a.spectrum(f), b.spectrum(g))
    blob = a.save()
    a.sync()
    torch.cuda.synchronize()
    need = a.state_bytes(f)
    assert t.cpu().numpy().tobytes() == bytes(blob[len(blob) - need:])


def test_state_written_through_the_tensor():
    import torch
    a, f, t = _lat(True)
    c, g, _ = _lat(False, -0.3, 0.2)
    a.step(40)
    c.step(40)
    assert not np.array_equal(a.spectrum(f), c.spectrum(g))
    blob = c.save()
    need = c.state_bytes(g)
    src = torch.frombuffer(bytearray(blob[len(blob) - need:]), dtype=torch.complex64).to("cuda")
    a.sync()
    t.copy_(src)
    torch.cuda.synchronize()
    a.state_changed()
    a.step(30)
    c.step(30)
    assert np.array_equal(a.spectrum(f), c.spectrum(g))


def test_the_library_does_not_free_bound_memory():
    import torch
    a, f, t = _lat(True)
    a.step(5)
    a.sync()
    a.close()
    torch.cuda.synchronize()
    assert torch.isfinite(t.view(torch.float32)).all()
    t.add_(1.0)  # still ours
    torch.cuda.synchronize()


def test_bind_after_the_plan_is_built_is_refused():
    import torch
    a, f, _ = _lat(False)
    t = torch.zeros(a.state_bytes(f) // 8, dtype=torch.complex64, device="cuda")
    with pytest.raises(pss.PssError) as e:
        a.bind(f, t)
    assert e.value.name == "PSS_E_STATE"
