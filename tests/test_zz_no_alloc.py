"""The imaging entry point that allocates nothing (vista_image_noalloc) against the one that
does (vista_image), through the C ABI: two calls in a row, the second on a smaller grid,
each identical to vista_image's images (the same kernels; the no-alloc form takes the
channels in passes that fit its fixed scratch)."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2609_01897_amd import vista  # noqa: E402


def _grid(nu, nv, nchan):
    return dict(nu=nu, nv=nv, du=1.0, dv=1.0, nchan=nchan, freq_lo=1e11, dfreq=1e7, flags=0)


def _inputs(nu, nv, nchan, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    S = torch.complex(torch.randn((nchan, nv, nu), generator=g, device="cuda"),
                      torch.randn((nchan, nv, nu), generator=g, device="cuda"))
    W = torch.rand((nchan, nv, nu), generator=g, device="cuda")
    W[nchan // 2] = 0.0                           # a channel without weight images to 0
    return S, W


@pytest.mark.parametrize("beam", [True, False])
def test_noalloc_image_equals_vista_image_on_two_calls(beam):
    # 1024 x 512 planes (4 MiB of staging each): 70 channels take five passes of the scratch;
    # then a smaller 256 x 128 grid of 9 channels in one pass
    for (nu, nv, nchan, seed) in ((1024, 512, 70, 1), (256, 128, 9, 2)):
        grid = _grid(nu, nv, nchan)
        S, W = _inputs(nu, nv, nchan, seed)
        ref, ref_beam, _ = vista.image(grid, S, W, beam=beam)
        img = torch.full_like(W, float("nan"))
        bm = torch.full_like(W, float("nan")) if beam else None
        vista.image_noalloc(grid, S, W, img, bm)
        torch.cuda.synchronize()
        assert torch.equal(img, ref), float((img - ref).abs().max())
        if beam:
            assert torch.equal(bm, ref_beam)
        assert not torch.any(img[nchan // 2] != 0)


def test_noalloc_image_refuses_planes_beyond_its_scratch():
    grid = _grid(4096, 4096, 1)
    S = torch.zeros((1, 1, 1), dtype=torch.complex64, device="cuda")
    W = torch.zeros((1, 1, 1), dtype=torch.float32, device="cuda")
    with pytest.raises(vista.VistaError) as e:
        vista.image_noalloc(grid, S, W, W)
    assert e.value.code == vista.VISTA_E_ARG and "scratch" in str(e.value)
