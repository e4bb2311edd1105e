"""Oracle for the GAME model: basis, pattern output, error and fitness.

Test infrastructure only (see the package docstring).  Plain float64.

Paper passages followed (Sec. 3 unless noted):
  * eq. (1): each feature f_i is expanded as a polynomial sequence in g(f_i);
  * eq. (2): the pattern output is the sum over features of those expansions;
  * eq. (6): the trigonometric ("polytrigo") expansion uses cos(m x) and
    sin(m x) for m = 1..d, so it carries two coefficient groups (B = 2);
  * eq. (3): the per-pattern error is the squared difference to the target;
    the dataset error is the mean of those (MSE), and the fitness is the
    complement 1 - error, to be maximised.

Readings taken where the paper is silent (each listed in the design notes):
  * coefficients are per feature (gene index i*K + k, K = B*D basis columns per
    feature); the paper's shared-coefficient model is the special case of
    coefficients tied across features;
  * the constant a_0 is an optional bias gene stored after the M basis genes;
  * Chebyshev T_k, Legendre P_k and powers x^k use k = 1..D (no constant
    column, which would be collinear with the bias);
  * trigonometric columns of a feature are cos(1x)..cos(Dx) then
    sin(1x)..sin(Dx), following the serial loop of Sec. 4 (coefficient j
    multiplies cos, coefficient j + d multiplies sin);
  * classification maps the output through the logistic sigmoid and compares
    it with the class label l = [t >= 0.5] (t itself for 0/1 targets); a
    pattern is predicted class 1 iff z >= 0; for regression the
    misclassification rate is reported as 0.
"""
from __future__ import annotations

import math

import numpy as np

BASES = ("power", "chebyshev", "legendre", "trig")
TASKS = ("regression", "classification")


def basis_width(basis: str, degree: int) -> int:
    """K = B * D: number of basis columns per feature (B = 2 for trig, eq. 6)."""
    if basis not in BASES:
        raise ValueError(f"unknown basis {basis!r}")
    if degree < 1:
        raise ValueError("degree must be >= 1")
    return (2 if basis == "trig" else 1) * degree


def n_genes(n_features: int, basis: str, degree: int, bias: int = 0) -> int:
    """L = F * B * D (+1 when the bias gene a_0 is present)."""
    return n_features * basis_width(basis, degree) + (1 if bias else 0)


def paper_population_size(n_features: int, b_factor: int) -> int:
    """eq. (4): number of chromosomes = B * N + 1 (N = number of features)."""
    return b_factor * n_features + 1


def paper_gene_count(degree: int, b_factor: int) -> int:
    """eq. (5): genes of the paper's shared-coefficient chromosome = B * d + 1."""
    return b_factor * degree + 1


# --- basis functions: closed forms, deliberately not the recurrences the GPU uses

def chebyshev_T(k: int, x: np.ndarray) -> np.ndarray:
    """T_k(x) = cos(k arccos x) on [-1, 1]; cosh form outside."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1.0
    out[inside] = np.cos(k * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.sign(xo) ** k * np.cosh(k * np.arccosh(np.abs(xo)))
    return out


def legendre_P(k: int, x: np.ndarray) -> np.ndarray:
    """Explicit sum P_k(x) = 2^-k sum_m (-1)^m C(k,m) C(2k-2m,k) x^(k-2m)."""
    x = np.asarray(x, dtype=np.float64)
    acc = np.zeros_like(x)
    for m in range(k // 2 + 1):
        c = (-1) ** m * math.comb(k, m) * math.comb(2 * k - 2 * m, k)
        acc = acc + c * x ** (k - 2 * m)
    return acc / 2.0 ** k


def basis_column(basis: str, degree: int, k: int, x: np.ndarray) -> np.ndarray:
    """Column k (0-based, k < K) of one feature's expansion, phi_{k+1}(x)."""
    x = np.asarray(x, dtype=np.float64)
    if basis == "power":
        return x ** (k + 1)
    if basis == "chebyshev":
        return chebyshev_T(k + 1, x)
    if basis == "legendre":
        return legendre_P(k + 1, x)
    if basis == "trig":
        if k < degree:
            return np.cos((k + 1) * x)
        return np.sin((k - degree + 1) * x)
    raise ValueError(f"unknown basis {basis!r}")


def design_matrix(X: np.ndarray, basis: str, degree: int) -> np.ndarray:
    """Phi[n, i*K + k] = phi_{k+1}(X[n, i])   (eq. 1 expanded per feature)."""
    X = np.asarray(X, dtype=np.float64)
    n, f = X.shape
    K = basis_width(basis, degree)
    Phi = np.empty((n, f * K))
    for i in range(f):
        for k in range(K):
            Phi[:, i * K + k] = basis_column(basis, degree, k, X[:, i])
    return Phi


def design_matrix_shared(X: np.ndarray, basis: str, degree: int) -> np.ndarray:
    """The paper's literal form (eq. 2, eq. 7 and the serial code of Sec. 4):
    one coefficient per basis function, shared by all features, so the
    pattern's basis value is summed over its features,
    Phi_s[n, k] = sum_i phi_{k+1}(X[n, i])  (features added in order)."""
    X = np.asarray(X, dtype=np.float64)
    n, f = X.shape
    K = basis_width(basis, degree)
    Phi = np.zeros((n, K))
    for k in range(K):
        for i in range(f):
            Phi[:, k] += basis_column(basis, degree, k, X[:, i])
    return Phi


def pattern_output(X, G, basis: str, degree: int, bias: int = 0, Phi=None, shared: bool = False):
    """z[n, p] = bias_p + sum_i sum_k G[p, i*K+k] phi_{k+1}(X[n, i])   (eq. 2);
    shared: z[n, p] = bias_p + sum_k G[p, k] sum_i phi_{k+1}(X[n, i])."""
    G = np.asarray(G, dtype=np.float64)
    if G.ndim == 1:
        G = G[None, :]
    if Phi is None:
        Phi = design_matrix_shared(X, basis, degree) if shared else design_matrix(X, basis, degree)
    M = Phi.shape[1]
    if G.shape[1] != M + (1 if bias else 0):
        raise ValueError(f"chromosome length {G.shape[1]} != {M} + bias {bias}")
    z = Phi @ G[:, :M].T
    if bias:
        z = z + G[:, M][None, :]
    return z


def sigmoid(z):
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-np.asarray(z, dtype=np.float64)))


def evaluate(X, t, G, basis: str, degree: int, task: str = "regression",
             bias: int = 0, Phi=None, shared: bool = False):
    """Fitness of every chromosome (row of G) over all patterns.

    Returns dict(mse, miscls, fitness, z):
      regression:     err = (t_n - z)^2
      classification: err = (l_n - sigmoid(z))^2,  l_n = [t_n >= 0.5]
      mse[p]  = mean_n err[n, p]                  (eq. 3, then MSE)
      fitness = 1 - mse                           (complement of the error)
      miscls  = mean_n [(z >= 0) != l_n]          (classification only, else 0)
    """
    if task not in TASKS:
        raise ValueError(f"unknown task {task!r}")
    t = np.asarray(t, dtype=np.float64)
    z = pattern_output(X, G, basis, degree, bias, Phi, shared)
    if task == "classification":
        err = ((t >= 0.5).astype(np.float64)[:, None] - sigmoid(z)) ** 2
    else:
        err = (t[:, None] - z) ** 2
    mse = err.mean(axis=0)
    if task == "classification":
        miscls = ((z >= 0.0) != (t[:, None] >= 0.5)).mean(axis=0)
    else:
        miscls = np.zeros(z.shape[1])
    return dict(mse=mse, miscls=miscls, fitness=1.0 - mse, z=z)


def predict(X, genes, basis: str, degree: int, task: str = "regression", bias: int = 0,
            Phi=None, shared: bool = False) -> np.ndarray:
    """Model output of one chromosome on new patterns (the paper's test and
    validation use, Sec. 4): z for regression, sigmoid(z) for classification."""
    z = pattern_output(X, np.asarray(genes, dtype=np.float64)[None, :], basis, degree, bias,
                       Phi, shared)[:, 0]
    return sigmoid(z) if task == "classification" else z


def metrics(X, t, genes, basis: str, degree: int, task: str = "regression", bias: int = 0,
            Phi=None, shared: bool = False) -> dict:
    """Quality of one chromosome on a pattern set: MSE (eq. 3) and its root;
    for classification the confusion counts with class 1 as the positive class
    (predicted 1 iff z >= 0, label l = [t >= 0.5]) and the rates the paper
    reports (Sec. 5): accuracy = (TP + TN) / N, completeness = TP / (TP + FN),
    contamination = FP / (TP + FP) (NaN when a denominator is 0)."""
    g = np.asarray(genes, dtype=np.float64)[None, :]
    r = evaluate(X, t, g, basis, degree, task, bias, Phi, shared)
    mse = float(r["mse"][0])
    out = dict(mse=mse, rmse=math.sqrt(mse), tp=0, fp=0, tn=0, fn=0, accuracy=math.nan,
               completeness=math.nan, contamination=math.nan)
    if task == "classification":
        pred = r["z"][:, 0] >= 0.0
        lab = np.asarray(t, dtype=np.float64) >= 0.5
        tp = int(np.sum(pred & lab))
        fp = int(np.sum(pred & ~lab))
        tn = int(np.sum(~pred & ~lab))
        fn = int(np.sum(~pred & lab))
        n = tp + fp + tn + fn
        out.update(tp=tp, fp=fp, tn=tn, fn=fn, accuracy=(tp + tn) / n,
                   completeness=tp / (tp + fn) if tp + fn else math.nan,
                   contamination=fp / (tp + fp) if tp + fp else math.nan)
    return out


def quantize(a, kind: str) -> np.ndarray:
    """Round to a storage type and back to float64 (round to nearest even).

    'f32' rounds once to float32; 'bf16' and 'f16' round the float32 value
    to bfloat16 / float16 (the GPU stores float32-rounded basis values and
    rounds those).  Uses PyTorch CPU casts (library primitives).
    """
    a32 = np.asarray(a, dtype=np.float64).astype(np.float32)
    if kind == "f32":
        return a32.astype(np.float64)
    import torch
    tt = torch.from_numpy(np.ascontiguousarray(a32))
    if kind == "bf16":
        return tt.to(torch.bfloat16).to(torch.float64).numpy()
    if kind == "f16":
        return tt.to(torch.float16).to(torch.float64).numpy()
    raise ValueError(kind)
