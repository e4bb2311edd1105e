"""Pins of the oracle's model (basis, pattern output, error, fitness) against
values and routines that do not come from the oracle itself."""
import json
import math
import os

import numpy as np
import pytest
import scipy.special
from numpy.polynomial import chebyshev as npcheb
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly
from sklearn.metrics import mean_squared_error

from oracle import model
import synth


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as fh:
        return json.load(fh)


def test_basis_hand_values(golden_dir):
    ref = _load(golden_dir, "basis_hand_values.json")
    x = np.array(ref["x"])
    for fam in ("chebyshev", "legendre", "power"):
        for k, vals in ref[fam].items():
            got = model.basis_column(fam, 8, int(k) - 1, x)
            np.testing.assert_allclose(got, vals, rtol=0, atol=1e-14, err_msg=f"{fam} {k}")
    p8 = model.basis_column("legendre", 8, 7, np.array([0.0]))[0]
    assert abs(p8 - ref["legendre_8_at_0"]) < 1e-15


@pytest.mark.parametrize("degree", [1, 3, 8, 12])
def test_basis_matches_numpy_polynomial_library(degree):
    x = np.random.default_rng(degree).uniform(-1, 1, 257)
    x = np.concatenate([x, [-1.0, 0.0, 1.0]])
    for k in range(degree):
        e = np.zeros(k + 2)
        e[k + 1] = 1.0
        np.testing.assert_allclose(model.basis_column("chebyshev", degree, k, x),
                                   npcheb.chebval(x, e), atol=1e-13)
        np.testing.assert_allclose(model.basis_column("legendre", degree, k, x),
                                   npleg.legval(x, e), atol=1e-13)
        np.testing.assert_allclose(model.basis_column("power", degree, k, x),
                                   nppoly.polyval(x, e), atol=1e-14)


def test_trig_columns_order_and_values():
    d = 3
    x = np.array([0.0, 0.3, -0.7, 1.0])
    cols = [model.basis_column("trig", d, k, x) for k in range(2 * d)]
    for m in range(1, d + 1):
        np.testing.assert_allclose(cols[m - 1], [math.cos(m * v) for v in x], atol=1e-15)
        np.testing.assert_allclose(cols[d + m - 1], [math.sin(m * v) for v in x], atol=1e-15)
    assert cols[0][0] == 1.0 and cols[d][0] == 0.0


def test_design_matrix_layout_feature_major():
    X = np.array([[0.25, -0.5, 0.75]])
    Phi = model.design_matrix(X, "legendre", 4)
    assert Phi.shape == (1, 12)
    for i in range(3):
        e = np.zeros(5)
        for k in range(4):
            e[:] = 0
            e[k + 1] = 1
            assert abs(Phi[0, i * 4 + k] - npleg.legval(X[0, i], e)) < 1e-15


def test_worked_fitness_example(golden_dir):
    ref = _load(golden_dir, "worked_fitness.json")
    X, t, G = np.array(ref["X"]), np.array(ref["t"]), np.array(ref["G"])
    r = model.evaluate(X, t, G, ref["basis"], ref["degree"], "regression")
    np.testing.assert_allclose(r["z"][:, 0], ref["z"], atol=1e-15)
    assert abs(r["mse"][0] - ref["regression"]["mse"]) < 1e-15
    assert abs(r["fitness"][0] - ref["regression"]["fitness"]) < 1e-15
    c = model.evaluate(X, t, G, ref["basis"], ref["degree"], "classification")
    assert abs(c["mse"][0] - ref["classification"]["mse"]) < 1e-12
    assert c["miscls"][0] == ref["classification"]["miscls"]
    np.testing.assert_allclose(model.sigmoid(r["z"][:, 0]), ref["classification"]["sigmoid"], atol=1e-15)


def test_paper_worked_counts():
    # eq. (4) and (5) with the polytrigo example of Sec. 3: B = 2, N = 11 features, d = 3.
    assert model.paper_population_size(11, 2) == 23
    assert model.paper_gene_count(3, 2) == 7
    # per-feature gene counts of the workloads: Chebyshev F=8 D=4, trig F=10 D=6, Legendre F=16 D=8
    assert model.n_genes(8, "chebyshev", 4) == 32
    assert model.n_genes(10, "trig", 6) == 120
    assert model.n_genes(16, "legendre", 8) == 128
    assert model.n_genes(16, "legendre", 8, bias=1) == 129


def test_tied_coefficients_reproduce_shared_coefficient_model():
    # The paper's shared-coefficient polytrigo (eq. 7 and the serial code of Sec. 4):
    # out = a0 + sum_i sum_j [a_j cos(j x_i) + b_j sin(j x_i)].  Written here as a
    # direct double sum; the oracle gets the same model through tied per-feature genes.
    rng = np.random.default_rng(7)
    d, f = 3, 11
    v = rng.uniform(-1, 1, 2 * d + 1)          # [a0, a1..ad, b1..bd], 7 genes for d = 3
    X = rng.uniform(-1, 1, (200, f))            # 200 patterns x 11 features as in eq. (7)
    expect = np.array([v[0] + sum(v[j] * math.cos(j * xi) + v[j + d] * math.sin(j * xi)
                                  for xi in row for j in range(1, d + 1)) for row in X])
    G = np.concatenate([np.tile(v[1:], f), [v[0]]])  # per feature [a1..ad, b1..bd], bias last
    z = model.pattern_output(X, G, "trig", d, bias=1)[:, 0]
    np.testing.assert_allclose(z, expect, rtol=1e-13, atol=1e-13)
    # one literal value: F=2, x=(0.3,-0.7), d=1, v=(0.1, 0.5, -0.25)
    z1 = model.pattern_output(np.array([[0.3, -0.7]]), np.array([0.5, -0.25, 0.5, -0.25, 0.1]),
                              "trig", 1, bias=1)[0, 0]
    hand = 0.1 + 0.5 * (math.cos(0.3) + math.cos(-0.7)) - 0.25 * (math.sin(0.3) + math.sin(-0.7))
    assert abs(z1 - hand) < 1e-15 and abs(z1 - 1.0472637083) < 1e-9


def test_zero_chromosome_special_cases():
    X, t = synth.classification_dataset(1000, 5, seed=3)
    G = np.zeros((1, 5 * 4))
    c = model.evaluate(X, t, G, "chebyshev", 4, "classification")
    assert c["mse"][0] == 0.25                           # sigmoid(0) = 1/2 for every pattern
    assert c["miscls"][0] == np.mean(t == 0.0)           # z = 0 predicts class 1
    Xr, tr, _ = synth.regression_dataset(500, 3, 2, 0.05, seed=4)
    r = model.evaluate(Xr, tr, np.zeros(6), "power", 2, "regression")
    assert abs(r["mse"][0] - np.mean(tr ** 2)) < 1e-15
    assert r["miscls"][0] == 0.0


def test_unit_chromosomes_select_columns_and_linearity():
    rng = np.random.default_rng(11)
    X = rng.uniform(-1, 1, (64, 4))
    Phi = model.design_matrix(X, "trig", 2)
    M = Phi.shape[1]
    z = model.pattern_output(X, np.eye(M), "trig", 2)
    np.testing.assert_array_equal(z, Phi)
    G1, G2 = rng.uniform(-1, 1, (2, M))
    z12 = model.pattern_output(X, G1 + G2, "trig", 2)
    zs = model.pattern_output(X, G1, "trig", 2) + model.pattern_output(X, G2, "trig", 2)
    np.testing.assert_allclose(z12, zs, atol=1e-13)


def test_mse_against_library_routines():
    X, t = synth.classification_dataset(777, 6, seed=5)
    G = synth.random_population(9, 6 * 3, seed=6).astype(np.float64)
    c = model.evaluate(X, t, G, "legendre", 3, "classification")
    Phi = model.design_matrix(X, "legendre", 3)
    for p in range(9):
        out = scipy.special.expit(Phi @ G[p])
        assert abs(c["mse"][p] - mean_squared_error(t, out)) < 1e-14
        assert abs(c["fitness"][p] - (1 - mean_squared_error(t, out))) < 1e-14


def test_brute_force_loops_with_recurrences():
    # Pure-Python loops with the three-term recurrences (not the oracle's closed forms).
    rng = np.random.default_rng(2)
    N, F, D = 7, 3, 5
    X = rng.uniform(-1, 1, (N, F))
    t = rng.uniform(-1, 1, N)
    for basis in ("chebyshev", "legendre", "power", "trig"):
        K = 2 * D if basis == "trig" else D
        G = rng.uniform(-1, 1, F * K + 1)
        sse = 0.0
        for n in range(N):
            z = G[F * K]
            for i in range(F):
                x = X[n, i]
                if basis == "trig":
                    vals = [math.cos((k + 1) * x) for k in range(D)] + \
                           [math.sin((k + 1) * x) for k in range(D)]
                else:
                    prev, cur, vals = 1.0, x, [x]
                    for k in range(1, D):
                        if basis == "chebyshev":
                            nxt = 2 * x * cur - prev
                        elif basis == "legendre":
                            nxt = ((2 * k + 1) * x * cur - k * prev) / (k + 1)
                        else:
                            nxt = cur * x
                        prev, cur = cur, nxt
                        vals.append(cur)
                for k in range(K):
                    z += G[i * K + k] * vals[k]
            sse += (t[n] - z) ** 2
        r = model.evaluate(X, t, G, basis, D, "regression", bias=1)
        assert abs(r["mse"][0] - sse / N) < 1e-12, basis


def test_regression_ols_bound_and_hidden_polynomial():
    X, t, g_star = synth.regression_dataset(1000, 8, 4, 0.05, seed=synth.data_seed(1))
    Phi = model.design_matrix(X, "chebyshev", 4)
    coef, *_ = np.linalg.lstsq(Phi, t, rcond=None)
    ols_mse = np.mean((t - Phi @ coef) ** 2)
    G = synth.random_population(50, 32, seed=1).astype(np.float64)
    r = model.evaluate(X, t, np.vstack([G, g_star]), "chebyshev", 4, "regression")
    assert np.all(r["mse"] >= ols_mse - 1e-12)
    # the hidden chromosome leaves only the noise: mse ~ 0.05^2 (std err ~ 0.0025*sqrt(2/1000))
    assert abs(r["mse"][-1] - 0.0025) < 5 * 0.0025 * math.sqrt(2 / 1000)


def test_quantize_round_to_nearest_even():
    v = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, 0.1])
    bf = model.quantize(v, "bf16")
    assert bf[0] == 1.0 and bf[1] == 1.0 + 2.0 ** -6     # ties to even
    h = model.quantize(v, "f16")
    assert h[2] == 1.0 and h[3] == 1.0 + 2.0 ** -9
    assert model.quantize(v, "f32")[4] == float(np.float32(0.1))


def test_classification_compares_with_class_labels():
    # classification scores the sigmoid output against the label [t >= 0.5]
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, (50, 3))
    t_soft = rng.uniform(0, 1, 50)
    t_lab = (t_soft >= 0.5).astype(np.float64)
    G = rng.uniform(-1, 1, (4, 6))
    a = model.evaluate(X, t_soft, G, "legendre", 2, "classification")
    b = model.evaluate(X, t_lab, G, "legendre", 2, "classification")
    np.testing.assert_array_equal(a["mse"], b["mse"])
    np.testing.assert_array_equal(a["miscls"], b["miscls"])


def test_metrics_against_sklearn_and_a_hand_example():
    from sklearn import metrics as skm
    # hand example: four patterns, power basis D = 1, one feature, gene 1 -> z = x
    X = np.array([[0.5], [-0.2], [0.0], [-0.7]])
    t = np.array([1.0, 1.0, 0.0, 0.0])
    m = model.metrics(X, t, [1.0], "power", 1, "classification")
    # predictions z >= 0: [1, 0, 1, 0] -> TP 1, FN 1, FP 1, TN 1
    assert (m["tp"], m["fn"], m["fp"], m["tn"]) == (1, 1, 1, 1)
    assert m["accuracy"] == 0.5 and m["completeness"] == 0.5 and m["contamination"] == 0.5
    s = 1.0 / (1.0 + np.exp(-X[:, 0]))
    assert abs(m["mse"] - np.mean((t - s) ** 2)) < 1e-15
    # random set against scikit-learn's confusion matrix, recall and precision
    X, t = synth.classification_dataset(3000, 4, seed=13)
    g = synth.random_population(1, 4 * 2 * 3, seed=2)[0]
    m = model.metrics(X, t, g, "trig", 3, "classification")
    pred = model.predict(X, g, "trig", 3, "classification") >= 0.5
    lab = t >= 0.5
    tn, fp, fn, tp = skm.confusion_matrix(lab, pred).ravel()
    assert (m["tp"], m["fp"], m["tn"], m["fn"]) == (tp, fp, tn, fn)
    assert abs(m["accuracy"] - skm.accuracy_score(lab, pred)) < 1e-15
    assert abs(m["completeness"] - skm.recall_score(lab, pred)) < 1e-15
    assert abs(m["contamination"] - (1.0 - skm.precision_score(lab, pred))) < 1e-15
    # regression: RMSE from scikit-learn, no confusion counts
    X, t, _ = synth.regression_dataset(500, 3, 2, 0.05, seed=3)
    g = synth.random_population(1, 3 * 4, seed=4)[0]
    m = model.metrics(X, t, g, "legendre", 4, "regression")
    y = model.predict(X, g, "legendre", 4, "regression")
    assert abs(m["rmse"] - np.sqrt(skm.mean_squared_error(t, y))) < 1e-12
    assert m["tp"] == m["fp"] == m["tn"] == m["fn"] == 0 and math.isnan(m["accuracy"])


def test_shared_coefficient_form_is_the_literal_polytrigo():
    # eq. (7): out = a0 + sum_i sum_j [a_j cos(j x_i) + b_j sin(j x_i)], genes
    # stored [a1..ad, b1..bd, a0]; written out directly as a double sum
    rng = np.random.default_rng(11)
    d, f = 3, 11
    a0, a, b = rng.uniform(-1, 1), rng.uniform(-1, 1, d), rng.uniform(-1, 1, d)
    X = rng.uniform(-1, 1, (200, f))
    expect = np.array([a0 + sum(a[j - 1] * math.cos(j * xi) + b[j - 1] * math.sin(j * xi)
                                for xi in row for j in range(1, d + 1)) for row in X])
    g = np.concatenate([a, b, [a0]])
    z = model.pattern_output(X, g, "trig", d, bias=1, shared=True)[:, 0]
    np.testing.assert_allclose(z, expect, rtol=1e-13, atol=1e-13)
    # it is the per-feature model with coefficients tied across features
    G = np.concatenate([np.tile(g[:-1], f), [a0]])
    np.testing.assert_allclose(model.pattern_output(X, G, "trig", d, bias=1)[:, 0], z,
                               rtol=1e-13, atol=1e-13)
    # eq. (5): B * d + 1 genes
    assert g.size == model.paper_gene_count(d, 2) == 7
    # the other bases sum Chebyshev / Legendre / power columns the same way
    for basis in ("chebyshev", "legendre", "power"):
        Ps = model.design_matrix_shared(X[:5, :4], basis, 4)
        Pf = model.design_matrix(X[:5, :4], basis, 4)
        np.testing.assert_allclose(Ps, Pf.reshape(5, 4, 4).sum(axis=1), rtol=1e-14, atol=1e-14)
