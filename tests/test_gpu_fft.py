"""Batched FFT building block (the transform behind the evaluations at roots of
unity, eq. (vandprod), and the products of Alg. 1) against numpy's FFT."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_6945_amd as P
    return P


# single-pass lengths of every radix mix, the LDS limit, and two-pass lengths
LENGTHS = [1, 2, 3, 5, 8, 16, 48, 72, 80, 96, 144, 240, 256, 320, 1152, 2304, 3072, 3840, 4096,
           4608, 9216, 36864]


@pytest.mark.parametrize("L", LENGTHS)
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft_matches_numpy(P, L, sign):
    rng = np.random.default_rng(L * 7 + (sign > 0))
    items = 3
    lines = max(1, min(37, 20000 // L))
    x = rng.standard_normal((items, lines, L)) + 1j * rng.standard_normal((items, lines, L))
    ref = np.fft.fft(x, axis=-1) if sign < 0 else np.fft.ifft(x, axis=-1) * L
    t = torch.tensor(x, device="cuda")
    P.fft_batched(t, sign)
    got = t.cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    # FP64 FFT: error grows like eps * log2(L)
    assert err < 1e-14 * max(1.0, np.log2(L)), (L, sign, err)


def test_fft_invalid(P):
    t = torch.zeros((1, 1, 7), dtype=torch.complex128, device="cuda")
    with pytest.raises(P.TikhError):
        P.fft_batched(t, -1)            # 7 is not 5-smooth
    t = torch.zeros((1, 1, 8), dtype=torch.complex128, device="cuda")
    with pytest.raises(P.TikhError):
        P.fft_batched(t, 2)             # sign must be +-1
