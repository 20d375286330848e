"""GPU parity of the data-preparation kernels against the oracle."""
import numpy as np
import pytest
import torch

from oracle import prep as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_06819_amd as gk
    return gk


def test_ml_from_colour_matches_oracle(gk):
    rng = np.random.default_rng(11)
    n = 300 * 301 + 7                                     # not a multiple of the block
    mb = rng.uniform(15, 22, n).astype(np.float32)
    mg = (mb - rng.uniform(-0.2, 1.6, n)).astype(np.float32)
    eb = rng.uniform(0.01, 0.3, n).astype(np.float32)
    eg = rng.uniform(0.01, 0.3, n).astype(np.float32)
    mb[::97] = np.nan
    eg[5::131] = np.inf
    a, b, s = -0.70, 0.89, 0.07
    ml, err = gk.ml_from_colour(*[torch.tensor(x, device="cuda") for x in (mb, mg, eb, eg)], a, b, s)
    ml, err = ml.cpu().numpy(), err.cpu().numpy()
    rml, rerr = P.ml_from_colour(mb, mg, eb, eg, a, b, s)
    assert np.array_equal(np.isnan(ml), np.isnan(rml))          # identical masks
    ok = ~np.isnan(rml)
    np.testing.assert_allclose(ml[ok], rml[ok], rtol=2e-6)
    np.testing.assert_allclose(err[ok], rerr[ok], rtol=2e-6)
    assert np.all(err[~ok] == 0)
    assert gk.ml_from_colour(*[torch.empty(0, device="cuda")] * 4, a, b, s)[0].numel() == 0
    # inputs one float off 16-byte alignment take the scalar path: same results
    t = [torch.tensor(x, device="cuda") for x in (mb, mg, eb, eg)]
    ml2, err2 = gk.ml_from_colour(*[x[1:] for x in t], a, b, s)
    assert np.array_equal(ml2.cpu().numpy(), ml[1:], equal_nan=True)
    assert np.array_equal(err2.cpu().numpy(), err[1:])
    for m in (1, 2, 3, 5):                                  # tails shorter than one vector
        mm, ee = gk.ml_from_colour(*[x[:m] for x in t], a, b, s)
        assert np.array_equal(mm.cpu().numpy(), ml[:m], equal_nan=True)


def test_brightness_errors_match_oracle(gk):
    rng = np.random.default_rng(12)
    B = rng.lognormal(5.0, 1.5, 90001).astype(np.float32)
    B[::211] = 0.0
    B[3::307] = np.nan
    e = gk.brightness_errors(torch.tensor(B, device="cuda"), 0.05, 0.1).cpu().numpy()
    ref = P.brightness_errors(B, 0.05, 0.1)
    np.testing.assert_array_equal(e == 0, ref == 0)
    np.testing.assert_allclose(e, ref, rtol=2e-6)
    with pytest.raises(gk.GalkinError):
        gk.brightness_errors(torch.tensor(B, device="cuda"), -1.0, 0.1)
