"""nlch_step_noalloc against nlch_step through the C ABI.  The allocation-free
entry point runs the same kernels on tables it writes into its static device
area, so its states and outputs of interest must equal nlch_step's bit for
bit.  Each case makes two calls in a row, the second on a smaller lattice, so
the area's contents from the first call must not leak into the second."""
import math

import numpy as np
import pytest

from paper_2310_10750_amd import nlch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TDT = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}
NPD = {"f64": np.float64, "f32": np.float32, "f16": np.float16}
ALGO = {"direct": nlch.NLCH_ALGO_DIRECT, "rowrun": nlch.NLCH_ALGO_ROWRUN,
        "auto": nlch.NLCH_ALGO_AUTO}


def _model(n, R2, kind, boundary=0, tau=0.05):
    delta = math.sqrt(R2 + 0.25) / n
    _, m, N, _ = nlch.nlch_disc(n, delta)
    sigma = delta / 3
    amp = 1.0253 * n * n / N if kind == 0 else 1.0253 / (math.pi * sigma * sigma)
    return nlch.make_model(n, delta, kind, amp, sigma, c_F=0.97, tau=tau, boundary=boundary)


def _side(md):
    if not md.boundary:
        return md.n
    _, m, _, _ = nlch.nlch_disc(md.n, md.delta)
    return md.n + 2 * m


def _pair(md, prec, algo, seed):
    """One step of the same input by nlch_step and by nlch_step_noalloc."""
    side = _side(md)
    u = np.random.default_rng(seed).uniform(-1.1, 1.1, side * side).astype(NPD[prec])
    x = torch.from_numpy(u).to(DEV)
    outs = []
    for fn in (nlch.nlch_step, nlch.nlch_step_noalloc):
        y = torch.full_like(x, 7.0)
        o = torch.full((2,), float("nan"), dtype=torch.float64, device=DEV)
        fn(md, nlch.PRECISIONS[prec], ALGO[algo], x, y, o)
        torch.cuda.synchronize()
        outs.append((y.cpu().numpy(), o.cpu().numpy()))
    return outs


CASES = [
    # (first call, second call on a smaller lattice): (n, R2, kernel, boundary), prec, algo
    (((512, 256, 0, 0), (96, 16, 0, 0)), "f32", "rowrun"),
    (((256, 64, 1, 0), (64, 9, 1, 0)), "f32", "auto"),
    (((128, 40, 1, 0), (48, 10, 1, 0)), "f64", "direct"),
    (((160, 30, 0, 0), (40, 5, 0, 0)), "f32", "direct"),
    (((128, 64, 0, 1), (64, 16, 0, 1)), "f16", "rowrun"),
    (((300, 1024, 0, 0), (70, 25, 1, 0)), "f16", "auto"),
]


@pytest.mark.parametrize("shapes,prec,algo", CASES)
def test_noalloc_equals_nlch_step_two_calls(shapes, prec, algo):
    print("noalloc", shapes, prec, algo, flush=True)
    for k, (n, R2, kind, bnd) in enumerate(shapes):
        md = _model(n, R2, kind, bnd)
        (ya, oa), (yb, ob) = _pair(md, prec, algo, seed=10 * n + k)
        assert np.array_equal(ya, yb), (n, R2)
        assert np.array_equal(oa, ob), (n, R2)
        assert np.all(np.abs(yb.astype(np.float64)) <= 1.0)


def test_noalloc_matches_oracle(orc):
    print("noalloc vs oracle", flush=True)
    n, R2 = 96, 16
    md = _model(n, R2, 0)
    u = np.random.default_rng(5).uniform(-1, 1, (n, n))
    x = torch.from_numpy(u.reshape(-1)).to(DEV)
    y = torch.empty_like(x)
    o = torch.zeros(2, dtype=torch.float64, device=DEV)
    nlch.nlch_step_noalloc(md, nlch.NLCH_F64, nlch.NLCH_ALGO_AUTO, x, y, o)
    torch.cuda.synchronize()
    ref = orc.step(u, n, md.delta, md.kernel, md.kernel_amp, md.kernel_sigma, md.c_F,
                   md.beta1, md.tau)
    got = y.cpu().numpy().reshape(n, n)
    assert np.max(np.abs(got - ref)) <= 1e-13
    assert abs(o[0].item() - float(np.mean(ref))) <= 1e-13


def test_noalloc_rejects_beyond_its_area():
    """A lattice whose chunk sums do not fit the static area, and beta2 > 0,
    are rejected before any device work (the output stays untouched)."""
    md = _model(20000, 4, 0)
    x = torch.zeros(16, device=DEV)
    y = torch.full_like(x, 3.0)
    o = torch.zeros(2, dtype=torch.float64, device=DEV)
    with pytest.raises(nlch.NlchError) as e:
        nlch.nlch_step_noalloc(md, nlch.NLCH_F32, nlch.NLCH_ALGO_AUTO, x, y, o)
    assert e.value.code == nlch.NLCH_EUNSUPPORTED
    assert "static area" in str(e.value)
    mb = nlch.make_model(64, 4 / 64, 0, 1.0, beta2=0.05)
    with pytest.raises(nlch.NlchError) as e:
        nlch.nlch_step_noalloc(mb, nlch.NLCH_F32, nlch.NLCH_ALGO_AUTO, x, y, o)
    assert e.value.code == nlch.NLCH_EUNSUPPORTED
    torch.cuda.synchronize()
    assert torch.all(y == 3.0)
