"""GPU checks of mixed-precision TUXV (rq_tuxv_mixed: the sketch, the
per-block Y2^T A of TRQRCP and Z = A V on the FP32 matrix cores from an FP32
copy of A; everything else FP64).  Its pivots may differ from the FP64
oracle's where two sample norms lie within FP32 rounding of each other, so
parity is stated against the FP64 oracle through properties: the truncation
error within 1.05x the oracle's and never below the Eckart-Young optimum,
the same error as the FP64 GPU path to 1e-3 relative (the FP32 products
perturb the approximation by ~ sqrt(n) 6e-8 relative, orders of magnitude
below the errors these inputs have), and orthonormal factors at the FP64
bar (they come from FP64 QR and Jacobi)."""

import os

import numpy as np
import pytest
import scipy.linalg.lapack as lapack
import torch

import oracle
from paper_1509_06820_amd import binding, inputs
from test_gpu_parity import dev, host, orth_tol, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,k,b,p,seed", [
    (400, 300, 40, 16, 8, 1),
    (700, 500, 64, 32, 8, 2),
    (300, 420, 33, 8, 4, 3),
    (1200, 900, 96, 64, 8, 4),
])
def test_tuxv_mixed_error_against_fp64_oracle(m, n, k, b, p, seed):
    say(f"tuxv_mixed {m}x{n} k={k} b={b}")
    sig = inputs.sigma_decade(min(m, n), 6)
    A = inputs.with_spectrum(seed, m, n, sig)
    nrm = np.linalg.norm(A)
    ref = oracle.tuxv(A, k, b, p, seed=seed)
    e_ref = np.linalg.norm(A - (ref["U"] * ref["s"]) @ ref["VT"]) / nrm
    U, s, VT, info = [host(x) for x in binding.rq_tuxv(dev(A), k, b, p, seed, mixed=True)]
    assert info[0] == 0
    e = np.linalg.norm(A - (U * s) @ VT) / nrm
    U6, s6, VT6, _ = [host(x) for x in binding.rq_tuxv(dev(A), k, b, p, seed)]
    e6 = np.linalg.norm(A - (U6 * s6) @ VT6) / nrm
    say(f"mixed {e:.6e} fp64 {e6:.6e} oracle {e_ref:.6e}")
    assert inputs.optimal_truncation_error(sig, k) * (1 - 1e-9) <= e <= 1.05 * e_ref
    assert abs(e - e6) <= 1e-3 * e6
    assert np.linalg.norm(U.T @ U - np.eye(k)) <= orth_tol(k)
    assert np.linalg.norm(VT @ VT.T - np.eye(k)) <= orth_tol(k)
    assert np.all(np.diff(s) <= 0) and s[-1] >= 0


def test_tuxv_mixed_c3_full_size():
    """20000 x 10000, sigma_i = 0.9^(i/10), k = 256 (the benchmark launch):
    error within 1.05x the FP64 oracle's stored error and within 1e-3 of the
    FP64 GPU path's."""
    say("tuxv_mixed c3 20000x10000 k=256")
    A, prm = inputs.config_matrix("c3")
    At = dev(A)
    del A
    k, b, p, seed = prm["k"], prm["b"], prm["p"], prm["seed"]
    nrm = torch.linalg.norm(At)
    U, s, VT, info = binding.rq_tuxv(At, k, b, p, seed, mixed=True)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    e = (torch.linalg.norm(At - (U * s) @ VT) / nrm).item()
    eye = torch.eye(k, dtype=torch.float64, device="cuda")
    assert torch.linalg.norm(U.T @ U - eye).item() <= orth_tol(k)
    assert torch.linalg.norm(VT @ VT.T - eye).item() <= orth_tol(k)
    del U, VT
    U6, s6, VT6, _ = binding.rq_tuxv(At, k, b, p, seed)
    e6 = (torch.linalg.norm(At - (U6 * s6) @ VT6) / nrm).item()
    gold = {}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_tuxv_oracle_error.txt")) as f:
        for ln in f:
            if ":" in ln and not ln.startswith("#"):
                key, val = ln.split(":", 1)
                gold[key.strip()] = float(val)
    opt = inputs.optimal_truncation_error(inputs.sigma_power(10000, 0.9, 10.0), k)
    say(f"c3 mixed error {e:.6f} fp64 {e6:.6f} oracle {gold['oracle_error']:.6f} optimum {opt:.6f}")
    assert opt * (1 - 1e-9) <= e <= 1.05 * gold["oracle_error"]
    assert abs(e - e6) <= 1e-3 * e6


@pytest.mark.parametrize("m,n,k,b,p,seed", [
    (600, 500, 100, 32, 8, 1),
    (300, 400, 37, 16, 6, 2),
    (1200, 900, 128, 64, 8, 3),
])
def test_trqrcp_mixed_against_fp64_oracle(m, n, k, b, p, seed):
    """rq_trqrcp_mixed: pivots of the FP64 oracle up to its first relative
    gap below 1e-5 (FP32 products perturb sample norms by ~1e-7 relative);
    when all k agree, R within 1e-5 ||A|| of the oracle's; the first k
    columns factor with residual 1e-5 and an FP64-orthonormal Q; the block
    A(k:, k:) holds the permuted original entries bit for bit."""
    say(f"trqrcp_mixed {m}x{n} k={k} b={b} p={p}")
    A = inputs.with_spectrum(seed, m, n, inputs.sigma_decade(min(m, n), 8))
    ref = oracle.trqrcp(A, k, b, p, seed=seed)
    F, tau, jpvt, info = [host(x) for x in binding.rq_trqrcp(dev(A), k, b, p, seed, mixed=True)]
    assert info[0] == 0
    assert sorted(jpvt.tolist()) == list(range(n))
    gaps = np.asarray(ref["gaps"][:k])
    bad = np.nonzero(gaps < 1e-5)[0]
    t = int(bad[0]) if len(bad) else k
    assert np.array_equal(jpvt[:t], ref["jpvt"][:t])
    nrm = np.linalg.norm(A)
    if t == k:
        assert np.abs(np.triu(F[:k]) - np.triu(ref["F"][:k])).max() <= 1e-5 * nrm
    Q, _, _ = lapack.dorgqr(np.asfortranarray(F[:, :k]).copy(), tau)
    R11 = np.triu(F[:k, :k])
    assert np.linalg.norm(A[:, jpvt[:k]] - Q @ R11) <= 1e-5 * nrm
    assert np.linalg.norm(Q.T @ Q - np.eye(k)) <= 1e-13
    assert np.array_equal(F[k:, k:], A[k:, :][:, jpvt[k:]])
