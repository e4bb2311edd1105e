"""Basis kernel (eq. 1, eq. 6) against the oracle's closed forms."""
import numpy as np
import pytest

from oracle import model
import synth
from tests.gpu_util import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu

ULP_REL = {"f32": 2.0 ** -24, "bf16": 2.0 ** -8, "f16": 2.0 ** -11}


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("basis", ["power", "chebyshev", "legendre", "trig"])
def test_basis_matches_oracle(basis, dtype):
    torch = require_gpu()
    from paper_1211_5481_amd import Config, build_basis
    N, F, D = 1001, 3, 7
    X = np.random.default_rng(1).uniform(-1, 1, (N, F))
    X[:3] = [[-1.0, 0.0, 1.0], [0.5, -0.5, 0.25], [1.0, 1.0, -1.0]]
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis=basis, dtype=dtype, pop_size=4)
    io = torch.float64 if dtype == "f64" else torch.float32
    Xq = X if dtype == "f64" else X.astype(np.float32).astype(np.float64)
    ref = model.design_matrix(Xq, basis, D)
    M = ref.shape[1]
    announce(f"basis {basis} {dtype} N={N} F={F} D={D}")
    phi = build_basis(cfg, dev(X, io), ld=M + 5)
    got = host(phi.to(torch.float64))
    assert np.all(got[:, M:] == 0.0), "pad columns must be zero"
    got = got[:, :M]
    if dtype == "f64":
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)
    else:
        q = model.quantize(ref, dtype)
        diff = np.abs(got - q)
        # a value within 1e-15 of a rounding boundary may round the other way
        assert np.all(diff <= ULP_REL[dtype] * 2 * np.maximum(np.abs(q), 2.0 ** -14) + 1e-12)
        assert np.mean(diff == 0) > 0.999


def test_basis_c3_shape_rows_sampled():
    torch = require_gpu()
    from paper_1211_5481_amd import Config, build_basis
    N, F, D = 1_000_000, 16, 8
    X, _ = synth.classification_dataset(N, F, seed=synth.data_seed(3))
    cfg = Config(n_patterns=N, n_features=F, degree=D, basis="legendre", dtype="f32", pop_size=8)
    announce("basis legendre f32 N=1e6 F=16 D=8")
    phi = build_basis(cfg, dev(X, torch.float32))
    rows = np.random.default_rng(0).choice(N, 2000, replace=False)
    rows = np.concatenate([rows, [0, N - 1]])
    got = host(phi[torch.from_numpy(rows).cuda()].double())
    ref = model.quantize(model.design_matrix(X[rows].astype(np.float32).astype(np.float64),
                                             "legendre", D), "f32")
    np.testing.assert_allclose(got, ref, rtol=2 ** -23, atol=1e-14)
