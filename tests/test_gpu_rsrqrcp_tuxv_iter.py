"""GPU parity for RSRQRCP (Alg. 5) and TUXV with j_max > 1 (Alg. 7), through
the C ABI, against the CPU oracle on the same seeded inputs.  Bars as for
RQRCP and TUXV (pivots up to the first oracle near-tie, residual 1e-12,
orthogonality, R and the approximation within 1e-12 of the oracle's)."""

import numpy as np
import pytest
import torch

import oracle
from paper_1509_06820_amd import binding, inputs
from test_gpu_parity import dev, host, orth_tol, qr_checks, say, trusted_prefix

pytestmark = pytest.mark.gpu


def compare_rsrqrcp(A, b, p, seed):
    m, n = A.shape
    k = min(m, n)
    ref = oracle.rsrqrcp(A, b, p, seed=seed)
    F, tau, jpvt, info = [host(x) for x in binding.rq_rsrqrcp(dev(A), b, p, seed)]
    assert info[0] == 0
    assert sorted(jpvt.tolist()) == list(range(n))
    t = trusted_prefix(ref["gaps"], k)
    assert np.array_equal(jpvt[:t], ref["jpvt"][:t]), f"pivots differ before step {t}"
    res, orth = qr_checks(A, F, tau, jpvt, k)
    assert res <= 1e-12, res
    assert orth <= 1e-13, orth
    if t == k:
        assert np.array_equal(jpvt, ref["jpvt"])
        nrm = np.linalg.norm(A)
        assert np.abs(np.triu(F[:k]) - np.triu(ref["F"][:k])).max() <= 1e-12 * nrm
    return jpvt, ref


def test_rsrqrcp_512_configuration():
    say("rsrqrcp 512x512 b=32 p=8 seed=1")
    A, prm = inputs.config_matrix("c1")
    compare_rsrqrcp(A, prm["b"], prm["p"], prm["seed"])


@pytest.mark.parametrize("m,n,b,p,seed", [
    (300, 200, 24, 8, 4),      # tall, b does not divide k
    (150, 260, 16, 5, 5),      # wide
    (97, 97, 64, 3, 6),        # ragged last block
    (64, 40, 1, 4, 7),         # b = 1, sample taller than late trailing blocks
    (1000, 700, 64, 8, 8),     # several panel and sample workgroups
])
def test_rsrqrcp_shapes(m, n, b, p, seed):
    say(f"rsrqrcp {m}x{n} b={b} p={p} seed={seed}")
    A = inputs.with_spectrum(seed, m, n, inputs.sigma_decade(min(m, n), 8))
    compare_rsrqrcp(A, b, p, seed)


def test_rsrqrcp_first_block_equals_rqrcp():
    """Block 0 samples with the Omega of Alg. 4, so both GPU paths make the
    same first b pivot choices."""
    say("rsrqrcp vs rqrcp first block 400x300 b=32")
    A = inputs.with_spectrum(12, 400, 300, inputs.sigma_decade(300, 8))
    _, _, jr, _ = binding.rq_rsrqrcp(dev(A), 32, 8, 12)
    _, _, jq, _ = binding.rq_rqrcp(dev(A), 32, 8, 12)
    assert np.array_equal(host(jr)[:32], host(jq)[:32])


def test_rsrqrcp_8192_full_size_gaussian():
    """8192 x 8192 i.i.d. N(0,1), b = 64, p = 8, seed 2 (the benchmark launch):
    the pivots of the first two blocks against the oracle run to k = 128,
    residual and orthogonality of the whole GPU factorization on the GPU."""
    say("rsrqrcp 8192x8192 gaussian b=64 p=8 seed=2")
    A, prm = inputs.config_matrix("c2_iid")
    At = dev(A)
    F, tau, jpvt, info = binding.rq_rsrqrcp(At, prm["b"], prm["p"], prm["seed"])
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    ref = oracle.rsrqrcp(A, prm["b"], prm["p"], seed=prm["seed"], k=128)
    jp = host(jpvt)
    t = trusted_prefix(ref["gaps"], 128)
    assert np.array_equal(jp[:t], ref["jpvt"][:t])
    assert sorted(jp.tolist()) == list(range(8192))
    Q = torch.linalg.householder_product(F, tau)
    R = torch.triu(F)
    res = (torch.linalg.norm(At[:, jpvt] - Q @ R) / torch.linalg.norm(At)).item()
    orth = torch.linalg.norm(Q.T @ Q - torch.eye(8192, dtype=torch.float64, device="cuda")).item()
    say(f"rsrqrcp 8192 residual {res:.3e} orthogonality {orth:.3e}")
    assert res <= 1e-12
    assert orth <= 1e-12


def test_rsrqrcp_rank_deficient_zero_and_nan():
    """Exact rank 20: the first 20 pivots are the oracle's and the trailing
    block of R vanishes; a zero matrix factors to zeros with the identity
    permutation; a NaN entry is reported through info."""
    say("rsrqrcp rank-20 120x90 / zero / nan")
    A = inputs.rank_r(21, 120, 90, 20)
    ref = oracle.rsrqrcp(A, 8, 6, seed=3)
    F, tau, jpvt, info = [host(x) for x in binding.rq_rsrqrcp(dev(A), 8, 6, 3)]
    assert info[0] == 0
    assert list(jpvt[:20]) == list(ref["jpvt"][:20])
    R = np.triu(F[:90])
    assert np.linalg.norm(R[20:, 20:]) <= 1e-13 * np.linalg.norm(A)
    res, orth = qr_checks(A, F, tau, jpvt, 90)
    assert res <= 1e-12 and orth <= 1e-13
    F, tau, jpvt, info = [host(x) for x in binding.rq_rsrqrcp(dev(np.zeros((50, 40))), 8, 4, 1)]
    assert np.all(F == 0) and np.all(tau == 0) and list(jpvt) == list(range(40)) and info[0] == 0
    A = inputs.gaussian(1, 50, 40)
    A[3, 7] = np.nan
    F, tau, jpvt, info = [host(x) for x in binding.rq_rsrqrcp(dev(A), 8, 4, 1)]
    assert info[0] > 0


def test_tuxv_iter_converges_to_optimum_with_gap():
    """sigma_{k+1} / sigma_k = 0.1: nine LQ/QR steps are a converged subspace
    iteration, so the GPU reaches the Eckart-Young error and the leading
    singular values (the oracle's pin of the same property)."""
    say("tuxv_iter gap spectrum 300x200 k=12 jmax=9")
    m, n, k = 300, 200, 12
    sig = np.concatenate([np.linspace(2.0, 1.0, k), 0.1 * np.linspace(1.0, 0.5, n - k)])
    A = inputs.with_spectrum(5, m, n, sig)
    U, s, VT, info = [host(x) for x in binding.rq_tuxv(dev(A), k, 8, 4, 5, jmax=9)]
    assert info[0] == 0
    e = np.linalg.norm(A - (U * s) @ VT) / np.linalg.norm(A)
    e_opt = inputs.optimal_truncation_error(sig, k)
    assert abs(e - e_opt) <= 1e-10 * e_opt
    assert np.abs(s - sig[:k]).max() <= 1e-10


@pytest.mark.parametrize("m,n,k,b,p,seed,jmax", [
    (400, 300, 40, 16, 8, 1, 2),
    (700, 500, 64, 32, 8, 2, 3),
    (300, 420, 33, 8, 4, 3, 4),
    (260, 200, 17, 8, 4, 4, 7),
])
def test_tuxv_iter_matches_oracle(m, n, k, b, p, seed, jmax):
    say(f"tuxv_iter {m}x{n} k={k} b={b} jmax={jmax}")
    sig = inputs.sigma_power(min(m, n), 0.97)
    A = inputs.with_spectrum(seed, m, n, sig)
    ref = oracle.tuxv(A, k, b, p, seed=seed, jmax=jmax)
    U, s, VT, info = [host(x) for x in binding.rq_tuxv(dev(A), k, b, p, seed, jmax=jmax)]
    assert info[0] == 0
    nrm = np.linalg.norm(A)
    assert np.abs(s - ref["s"]).max() <= 1e-12 * ref["s"][0]
    approx = (U * s) @ VT
    assert np.linalg.norm(approx - (ref["U"] * ref["s"]) @ ref["VT"]) <= 1e-12 * nrm
    assert np.linalg.norm(U.T @ U - np.eye(k)) <= orth_tol(k)
    assert np.linalg.norm(VT @ VT.T - np.eye(k)) <= orth_tol(k)
    # the iterations improve on j_max = 1 and stay above Eckart-Young
    U1, s1, VT1, _ = [host(x) for x in binding.rq_tuxv(dev(A), k, b, p, seed)]
    e1 = np.linalg.norm(A - (U1 * s1) @ VT1) / nrm
    e = np.linalg.norm(A - approx) / nrm
    assert inputs.optimal_truncation_error(sig, k) * (1 - 1e-9) <= e <= e1 * (1 + 1e-12)


def test_tuxv_iter_one_is_tuxv():
    say("tuxv_iter jmax=1 vs tuxv 300x250 k=20")
    A = inputs.with_spectrum(6, 300, 250, inputs.sigma_decade(250, 6))
    a = [host(x) for x in binding.rq_tuxv(dev(A), 20, 8, 4, 6)]
    w = binding.workspace(binding.RQ_OP_TUXV, 300, 250, 20, 8, 4, torch.device("cuda"))
    Af = dev(A)
    U = torch.empty((20, 300), dtype=torch.float64, device="cuda").t()
    VT = torch.empty((250, 20), dtype=torch.float64, device="cuda").t()
    sg = torch.empty(20, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = binding.load().rq_tuxv_iter(None, 300, 250, 20, Af.data_ptr(), 300, 8, 4, 6, 1, U.data_ptr(), 300,
                                     sg.data_ptr(), VT.data_ptr(), 20, w.data_ptr(), w.numel(), info.data_ptr())
    assert rc == 0
    assert np.array_equal(host(sg), a[1])
    assert np.array_equal(host(U), a[0])
    assert np.array_equal(host(VT), a[2])


def test_tuxv_iter_c3_full_size():
    """20000 x 10000 with sigma_i = 0.9^(i/10), k = 256: j_max = 2 and 3 lower
    the error of j_max = 1 monotonically and stay above the Eckart-Young
    optimum; both bases orthonormal."""
    say("tuxv_iter c3 20000x10000 k=256 jmax=1,2,3")
    A, prm = inputs.config_matrix("c3")
    At = dev(A)
    del A
    k, b, p, seed = prm["k"], prm["b"], prm["p"], prm["seed"]
    sig = inputs.sigma_power(10000, 0.9, 10.0)
    e_opt = inputs.optimal_truncation_error(sig, k)
    nrm = torch.linalg.norm(At)
    errs = []
    for jmax in (1, 2, 3):
        U, s, VT, info = binding.rq_tuxv(At, k, b, p, seed, jmax=jmax)
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        errs.append((torch.linalg.norm(At - (U * s) @ VT) / nrm).item())
        eye = torch.eye(k, dtype=torch.float64, device="cuda")
        assert torch.linalg.norm(U.T @ U - eye).item() <= orth_tol(k)
        assert torch.linalg.norm(VT @ VT.T - eye).item() <= orth_tol(k)
        del U, VT
    say(f"c3 errors by jmax {errs} optimum {e_opt:.6e}")
    assert errs[0] >= errs[1] * (1 - 1e-12) >= errs[2] * (1 - 2e-12)
    assert errs[2] >= e_opt * (1 - 1e-9)
