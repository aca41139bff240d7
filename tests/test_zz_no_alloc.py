"""nkreg_gradient_noalloc (no handle, no device allocation, a fixed device array for its
spectra and twiddles) against nkreg_gradient through a handle, on two calls in a row,
the second with a smaller input; and its size limit."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import spectral as osp
from tests.helpers import rel_inf

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1408_6299_amd as nk
    return nk


def noalloc_gradient(lib, u, g, prec):
    shape = tuple(u.shape)
    n = (ctypes.c_int * 3)(*(list(shape) + [1] * (3 - len(shape))))
    st = lib.nkreg_gradient_noalloc(len(shape), n, prec, ctypes.c_void_p(u.data_ptr()),
                                    ctypes.c_void_p(g.data_ptr()),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, lib.nkreg_last_error().decode()
    return g


@pytest.mark.parametrize("prec", [32, 64])
def test_noalloc_gradient_equals_the_handle_gradient_on_two_calls(nk, prec):
    """A 512^2 field, then a smaller 3D field (64 x 32 x 16) in the same array: each result
    is nkreg_gradient's bit for bit and the oracle's to rounding; the calls change no
    device memory use."""
    from paper_1408_6299_amd import _lib
    lib = _lib.load()
    dt = torch.float32 if prec == 32 else torch.float64
    fields = []
    for shape, seed in (((512, 512), 3), ((64, 32, 16), 4)):
        u = synth.smooth_image(shape, seed, 0.6 * min(shape) ** 2 / 16.0)
        if prec == 32:
            u = u.astype(np.float32).astype(np.float64)   # the oracle sees the field the kernel sees
        fields.append((shape, u))
    refs = []
    for shape, u in fields:
        G = nk.Problem(shape, 2, precision=prec)
        refs.append(G.gradient(torch.from_numpy(u).cuda().to(dt)).clone())
        torch.cuda.synchronize()
        G.close()
    # inputs and outputs exist before the measured calls; only the library runs between
    # the two readings of free device memory
    ins = [torch.from_numpy(u).cuda().to(dt) for _, u in fields]
    outs = [[torch.full_like(r, float("nan")) for r in refs] for _ in range(2)]
    noalloc_gradient(lib, ins[0], outs[0][0], prec)   # the first call on this GPU looks up the array
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for rep in range(2):
        for k in range(2):
            noalloc_gradient(lib, ins[k], outs[rep][k], prec)
        torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, (free0, free1)
    for rep in range(2):
        for k, ((shape, u), ref) in enumerate(zip(fields, refs)):
            g = outs[rep][k]
            assert torch.equal(g, ref), shape
            assert rel_inf(g.double().cpu().numpy(), osp.grad(u)) < (1e-12 if prec == 64 else 2e-5), shape


def test_noalloc_gradient_rejects_grids_beyond_its_array(nk):
    """Three FP64 spectra of a 128^3 field (48 MiB) do not fit the 8 MiB array: ESHAPE with a
    message, before any device work; an unsupported size and a null pointer are refused too."""
    from paper_1408_6299_amd import _lib
    lib = _lib.load()
    u = torch.zeros((128, 128, 128), dtype=torch.float64, device="cuda")
    g = torch.zeros((3, 128, 128, 128), dtype=torch.float64, device="cuda")
    n = (ctypes.c_int * 3)(128, 128, 128)
    st = lib.nkreg_gradient_noalloc(3, n, 64, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(g.data_ptr()), None)
    assert st == _lib.ESHAPE
    assert "scratch" in lib.nkreg_last_error().decode()
    assert not g.any()
    n = (ctypes.c_int * 3)(48, 64, 1)
    assert lib.nkreg_gradient_noalloc(2, n, 32, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                      None) == _lib.ESHAPE
    assert lib.nkreg_gradient_noalloc(2, n, 32, None, ctypes.c_void_p(g.data_ptr()), None) == _lib.EINVAL
