"""Host-side pieces of the differentiable path, on CPU tensors: the centred
FFT pair (checkerboard form against the shift form, and F^dagger F = n I
on the centred grid), and the weighted-residual chi^2 of Eq. ImChisq as one
autograd Function (value and gradients against the plain torch expression,
and gradcheck in FP64)."""

import pytest

torch = pytest.importorskip("torch")

from paper_2508_17187_amd.autograd import (WeightedResidual, centred_fft2,  # noqa: E402
                                           centred_ifft2)


def shifted_fft2(x):
    return torch.fft.fftshift(torch.fft.fft2(torch.fft.ifftshift(x, dim=(-2, -1))), dim=(-2, -1))


def shifted_ifft2(x):
    n = x.shape[-1] * x.shape[-2]
    return torch.fft.fftshift(torch.fft.ifft2(torch.fft.ifftshift(x, dim=(-2, -1))),
                              dim=(-2, -1)) * n


@pytest.mark.parametrize("shape", [(1, 4, 64, 64), (2, 1, 96, 128), (1, 2, 10, 6),
                                   (1, 1, 7, 9), (3, 2, 2)])
def test_centred_fft_pair_equals_the_shift_form(shape):
    g = torch.Generator().manual_seed(5)
    x = torch.complex(torch.randn(shape, generator=g, dtype=torch.float64),
                      torch.randn(shape, generator=g, dtype=torch.float64))
    a, b = centred_fft2(x), shifted_fft2(x)
    assert torch.max(torch.abs(a - b)) <= 1e-13 * torch.max(torch.abs(b))
    a, b = centred_ifft2(x), shifted_ifft2(x)
    assert torch.max(torch.abs(a - b)) <= 1e-13 * torch.max(torch.abs(b))
    # unnormalised pair: F^dagger F = (nx ny) I
    n = shape[-1] * shape[-2]
    assert torch.max(torch.abs(centred_ifft2(centred_fft2(x)) - n * x)) <= 1e-12 * n


def test_centred_fft_of_a_point_at_the_centre_pixel_is_flat():
    # pixel (n/2, n/2) is l = m = 0: its transform is 1 everywhere
    x = torch.zeros((1, 1, 16, 12), dtype=torch.complex128)
    x[..., 8, 6] = 1.0
    assert torch.allclose(centred_fft2(x), torch.ones_like(x), atol=1e-15)


@pytest.mark.parametrize("cdt,rdt,tol", [(torch.complex128, torch.float64, 1e-12),
                                         (torch.complex64, torch.float32, 2e-6)])
def test_weighted_residual_value_and_gradients(cdt, rdt, tol):
    g = torch.Generator().manual_seed(7)
    sh = (50, 3, 4)

    def c():
        return torch.complex(torch.randn(sh, generator=g, dtype=rdt),
                             torch.randn(sh, generator=g, dtype=rdt)).to(cdt)

    v = c().requires_grad_(True)
    o = c().requires_grad_(True)
    w = torch.rand(sh, generator=g, dtype=rdt).requires_grad_(True)
    w.data[0] = 0.0                      # a flagged sample contributes nothing
    loss = WeightedResidual.apply(v, o, w)
    r = o - v
    ref = (w * (r.real ** 2 + r.imag ** 2)).sum()
    assert abs(loss.item() - ref.item()) <= tol * abs(ref.item())
    for a, b in zip(torch.autograd.grad(loss, (v, o, w)), torch.autograd.grad(ref, (v, o, w))):
        assert torch.max(torch.abs(a - b)) <= tol * torch.max(torch.abs(b))


def test_weighted_residual_gradcheck():
    g = torch.Generator().manual_seed(8)
    v = torch.randn((6, 2), generator=g, dtype=torch.complex128).requires_grad_(True)
    o = torch.randn((6, 2), generator=g, dtype=torch.complex128).requires_grad_(True)
    w = torch.rand((6, 2), generator=g, dtype=torch.float64).requires_grad_(True)
    assert torch.autograd.gradcheck(WeightedResidual.apply, (v, o, w))
