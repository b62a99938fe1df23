"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bars:
* pivots: identical to the oracle's up to the first step whose oracle gap
  between the two best sample norms is below 1e-9 (rounding order may flip
  a near tie), and identical everywhere when no such step exists;
* ||A P - Q R||_F / ||A||_F <= 1e-12 and ||Q^T Q - I||_F <= 1e-13 (fp64 path);
* R entries within 1e-12 ||A||_F of the oracle's (while pivots agree);
* quantities that are pure data movement (permuted original entries of
  TRQRCP) bit-exact.
"""

import os
import sys

import numpy as np
import pytest
import scipy.linalg.lapack as lapack
import torch

import oracle
from paper_1509_06820_amd import binding, inputs

pytestmark = pytest.mark.gpu

TIE = 1e-9
EPS = np.finfo(np.float64).eps


def orth_tol(k):
    """Orthogonality bar for factors accumulated from ~10 sweeps of k-1
    plane rotations per column: ||V^T V - I||_F grows like k * eps."""
    return max(1e-13, 20 * k * EPS)


def dev(A):
    return torch.from_numpy(np.asfortranarray(A)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def trusted_prefix(gaps, k):
    bad = np.nonzero(np.asarray(gaps[:k]) < TIE)[0]
    return int(bad[0]) if len(bad) else k


def qr_checks(A, F, tau, jpvt, k):
    F = np.asfortranarray(F)
    Q, _, info = lapack.dorgqr(F[:, :k].copy(order="F"), tau)
    assert info == 0
    R = np.triu(F[:k, :])
    nrm = np.linalg.norm(A)
    res = np.linalg.norm(A[:, jpvt] - Q @ R) / nrm
    orth = np.linalg.norm(Q.T @ Q - np.eye(k))
    return res, orth


def compare_rqrcp(A, b, p, seed, Omega=None):
    m, n = A.shape
    k = min(m, n)
    ref = oracle.rqrcp(A, b, p, seed=seed, Omega=Omega)
    F, tau, jpvt, info = binding.rq_rqrcp(dev(A), b, p, seed, Omega=None if Omega is None else dev(Omega))
    F, tau, jpvt, info = host(F), host(tau), host(jpvt), host(info)
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
    return F, tau, jpvt, ref


# ---------------------------------------------------------------- components
@pytest.mark.parametrize("seed,l,m", [(1, 40, 512), (2, 72, 1000), (2**40 + 3, 7, 5), (0, 1, 3), (9, 128, 333)])
def test_omega_matches_oracle(seed, l, m):
    say(f"omega seed={seed} l={l} m={m}")
    Om = host(binding.rq_omega(seed, l, m))
    ref = oracle.omega(seed, l, m)
    # same Philox words; the transcendental functions may differ in the last ulp
    assert np.abs(Om - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())


def test_sketch_matches_oracle():
    say("sketch 300x200 l=40")
    A = inputs.gaussian(5, 300, 200)
    B = host(binding.rq_sketch(dev(A), 40, 5))
    ref = oracle.omega(5, 40, 300) @ A
    assert np.linalg.norm(B - ref) <= 1e-14 * np.linalg.norm(ref) * 10


@pytest.mark.parametrize("l,n,bs", [
    (40, 512, 32),      # the 512 x 512 configuration's first sample
    (72, 300, 64),      # one workgroup
    (72, 5000, 64),     # several workgroups, candidate rounds
    (72, 16384, 64),    # 64 workgroups
    (72, 20000, 64),    # several columns per scan thread
    (16, 20, 16),       # bsteps = l
    (9, 9, 9),          # square, every column pivoted
    (33, 40, 1),        # one step
    (44, 900, 40),      # l in (40, 48]: the 48-row tile
    (48, 5000, 48),     # l = 48, every row a pivot row
    (80, 3000, 64),     # l in (72, 80]
    (128, 700, 64),     # largest l (b + p = 128)
    (128, 65536, 64),   # largest l and n: 256 workgroups
])
def test_sample_qrcp_matches_oracle(l, n, bs):
    say(f"sample_qrcp l={l} n={n} b={bs}")
    rng = np.random.default_rng(l * 1000 + n)
    B = rng.standard_normal((l, n)) * rng.uniform(0.2, 2.0, size=n)
    ref = oracle.sample_qrcp(B, bs)
    S, piv, info = binding.rq_sample_qrcp(dev(B), bs)
    S, piv = host(S), host(piv)
    t = trusted_prefix(ref["gaps"], bs)
    assert list(piv[:t]) == ref["piv"][:t]
    if t == bs:
        assert np.abs(S - ref["S"]).max() <= 1e-13 * np.abs(B).max() * np.sqrt(l)


def test_sample_qrcp_exact_ties_take_lowest_position():
    say("sample_qrcp ties")
    rng = np.random.default_rng(3)
    base = rng.standard_normal((12, 40))
    B = np.concatenate([base, base[:, ::-1]], axis=1)  # every column appears twice
    ref = oracle.sample_qrcp(B, 8)
    S, piv, _ = binding.rq_sample_qrcp(dev(B), 8)
    assert list(host(piv)[:1]) == ref["piv"][:1]


@pytest.mark.parametrize("k", [1, 2, 17, 64, 129, 300, 700])
def test_small_svd_matches_lapack(k):
    """k = 300 and 700 take the 8- and 16-rows-per-lane sweep kernels.  There
    the bars follow the rounding of ~10 sweeps of k - 1 rotations per column:
    entries like k eps, and the orthogonality of the accumulated V, whose
    k^2 entries each take a random walk of ~10 k rounding errors, like
    k * sqrt(10 k) eps (4 k^1.5 eps)."""
    say(f"small_svd k={k}")
    rng = np.random.default_rng(k)
    X = np.triu(rng.standard_normal((k, k)))
    U, s, V = binding.rq_small_svd(dev(X))
    U, s, V = host(U), host(s), host(V)
    s_ref = np.linalg.svd(X, compute_uv=False)
    bar = 1e-13 if k <= 256 else orth_tol(k)
    assert np.abs(s - s_ref).max() <= bar * s_ref[0]
    assert np.linalg.norm(U @ np.diag(s) @ V.T - X) <= bar * np.linalg.norm(X)
    obar = orth_tol(k) if k <= 256 else max(orth_tol(k), 4 * k ** 1.5 * EPS)
    assert np.linalg.norm(V.T @ V - np.eye(k)) <= obar
    assert np.linalg.norm(U.T @ U - np.eye(k)) <= obar


# ---------------------------------------------------------------- RQRCP
def test_rqrcp_512_configuration():
    say("rqrcp 512x512 b=32 p=8 seed=1")
    A, prm = inputs.config_matrix("c1")
    compare_rqrcp(A, prm["b"], prm["p"], prm["seed"])


@pytest.mark.parametrize("seed", [2, 3, 4, 5])
def test_rqrcp_512_more_seeds(seed):
    say(f"rqrcp 512x512 seed={seed}")
    A, prm = inputs.config_matrix("c1", seed)
    compare_rqrcp(A, prm["b"], prm["p"], seed)


@pytest.mark.parametrize("m,n,b,p,seed", [
    (300, 200, 24, 8, 4),      # tall, b does not divide k
    (150, 260, 16, 5, 5),      # wide
    (97, 97, 64, 3, 6),        # ragged last block
    (64, 40, 1, 4, 7),         # b = 1
    (1000, 700, 64, 8, 8),     # two panel workgroups, three sample workgroups
    (2100, 1300, 32, 8, 9),    # five panel workgroups, six sample workgroups
    (600, 500, 64, 64, 10),    # largest oversampling, l = b + p = 128
    (10, 300, 64, 8, 11),      # fewer rows than b and than l: one block of 10 steps
    (5000, 3, 64, 8, 12),      # tall and three columns
    (900, 700, 40, 8, 13),     # l = 48: the 48-row sample tile
    (700, 650, 36, 8, 14),     # l = 44 in the 48-row tile, ragged last block
])
def test_rqrcp_shapes(m, n, b, p, seed):
    say(f"rqrcp {m}x{n} b={b} p={p} seed={seed}")
    A = inputs.with_spectrum(seed, m, n, inputs.sigma_decade(min(m, n), 8))
    compare_rqrcp(A, b, p, seed)


def test_rqrcp_given_omega():
    say("rqrcp_omega 400x300")
    A = inputs.gaussian(11, 400, 300)
    Om = np.random.default_rng(12).standard_normal((40, 400))
    compare_rqrcp(A, 32, 8, 0, Omega=Om)


def test_rqrcp_gaussian_is_deterministic():
    say("rqrcp determinism 1000x800")
    A = dev(inputs.gaussian(13, 1000, 800))
    r1 = [host(x) for x in binding.rq_rqrcp(A, 64, 8, 13)[:3]]
    r2 = [host(x) for x in binding.rq_rqrcp(A, 64, 8, 13)[:3]]
    for x, y in zip(r1, r2):
        assert np.array_equal(x, y)


def test_rqrcp_rank_deficient():
    say("rqrcp rank-20 120x90")
    A = inputs.rank_r(21, 120, 90, 20)
    ref = oracle.rqrcp(A, 8, 6, seed=3)
    F, tau, jpvt, info = [host(x) for x in binding.rq_rqrcp(dev(A), 8, 6, 3)]
    assert list(jpvt[:20]) == list(ref["jpvt"][:20])
    R = np.triu(F[:90])
    assert np.linalg.norm(R[20:, 20:]) <= 1e-13 * np.linalg.norm(A)
    res, orth = qr_checks(A, F, tau, jpvt, 90)
    assert res <= 1e-12 and orth <= 1e-13


def test_rqrcp_zero_and_nan():
    say("rqrcp zero / nan")
    F, tau, jpvt, info = [host(x) for x in binding.rq_rqrcp(dev(np.zeros((50, 40))), 8, 4, 1)]
    assert np.all(F == 0) and np.all(tau == 0) and list(jpvt) == list(range(40)) and info[0] == 0
    A = inputs.gaussian(1, 50, 40)
    A[3, 7] = np.nan
    F, tau, jpvt, info = [host(x) for x in binding.rq_rqrcp(dev(A), 8, 4, 1)]
    assert info[0] > 0


# ---------------------------------------------------------------- unpivoted QR
@pytest.mark.parametrize("m,n,b", [(700, 500, 32), (300, 300, 64), (129, 257, 16)])
def test_unpivoted_qr_matches_oracle(m, n, b):
    say(f"unpivoted_qr {m}x{n} b={b}")
    A = inputs.gaussian(m + n, m, n)
    F, tau, info = [host(x) for x in binding.rq_unpivoted_qr(dev(A), b)]
    Fr, tr = oracle.unpivoted_qr(A, b)
    nrm = np.linalg.norm(A)
    assert np.abs(np.triu(F) - np.triu(Fr)).max() <= 1e-12 * nrm
    assert np.abs(tau - tr).max() <= 1e-12
    res, orth = qr_checks(A, F, tau, np.arange(n), min(m, n))
    assert res <= 1e-12 and orth <= 1e-13


# ---------------------------------------------------------------- TRQRCP
@pytest.mark.parametrize("m,n,k,b,p,seed", [
    (600, 500, 100, 32, 8, 1),
    (300, 400, 37, 16, 6, 2),
    (1200, 900, 128, 64, 8, 3),
    (200, 150, 150, 64, 8, 4),   # k = min(m, n)
    (500, 400, 96, 32, 16, 5),   # l = 48 (the 48-row sample tile)
])
def test_trqrcp_matches_oracle(m, n, k, b, p, seed):
    say(f"trqrcp {m}x{n} k={k} b={b} p={p}")
    A = inputs.with_spectrum(seed, m, n, inputs.sigma_decade(min(m, n), 8))
    ref = oracle.trqrcp(A, k, b, p, seed=seed)
    F, tau, jpvt, info = [host(x) for x in binding.rq_trqrcp(dev(A), k, b, p, seed)]
    assert info[0] == 0
    t = trusted_prefix(ref["gaps"], k)
    assert np.array_equal(jpvt[:t], ref["jpvt"][:t])
    if t < k:
        return
    assert np.array_equal(jpvt, ref["jpvt"])
    nrm = np.linalg.norm(A)
    assert np.abs(np.triu(F[:k]) - np.triu(ref["F"][:k])).max() <= 1e-12 * nrm
    # the untouched block holds the permuted original entries, bit for bit
    assert np.array_equal(F[k:, k:], A[k:, :][:, jpvt[k:]])
    Qk, _, _ = lapack.dorgqr(np.asfortranarray(F[:, :k]).copy(), tau)
    assert np.linalg.norm(Qk.T @ Qk - np.eye(k)) <= 1e-13
    assert np.linalg.norm(Qk @ np.triu(F[:k, :k]) - A[:, jpvt[:k]]) <= 1e-12 * nrm


# ---------------------------------------------------------------- TUXV
@pytest.mark.parametrize("m,n,k,b,p,seed", [
    (400, 300, 40, 16, 8, 1),
    (700, 500, 64, 32, 8, 2),
    (300, 420, 33, 8, 4, 3),
])
def test_tuxv_matches_oracle(m, n, k, b, p, seed):
    say(f"tuxv {m}x{n} k={k} b={b}")
    sig = inputs.sigma_decade(min(m, n), 6)
    A = inputs.with_spectrum(seed, m, n, sig)
    ref = oracle.tuxv(A, k, b, p, seed=seed)
    U, s, VT, info = [host(x) for x in binding.rq_tuxv(dev(A), k, b, p, seed)]
    assert info[0] == 0
    nrm = np.linalg.norm(A)
    assert np.abs(s - ref["s"]).max() <= 1e-12 * ref["s"][0]
    approx = U @ np.diag(s) @ VT
    ref_approx = ref["U"] @ np.diag(ref["s"]) @ ref["VT"]
    assert np.linalg.norm(approx - ref_approx) <= 1e-12 * nrm
    assert np.linalg.norm(U.T @ U - np.eye(k)) <= orth_tol(k)
    assert np.linalg.norm(VT @ VT.T - np.eye(k)) <= orth_tol(k)
    e = np.linalg.norm(A - approx) / nrm
    assert inputs.optimal_truncation_error(sig, k) * (1 - 1e-9) <= e


# ---------------------------------------------------------------- full size
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_pivot_golden(name):
    """(jpvt, gaps, |R_jj|, header lines) of a golden written by
    tests/golden/make_full_size_goldens.py (oracle only)."""
    path = os.path.join(GOLDEN, name)
    header = [ln[1:].strip() for ln in open(path) if ln.startswith("#")]
    rows = np.loadtxt(path, comments="#")
    return rows[:, 1].astype(np.int64), rows[:, 2], rows[:, 3], header


def gpu_residual_orth(At, F, tau, jpvt, k=None):
    """||A P - Q R||_F / ||A||_F and ||Q^T Q - I||_F on the GPU (Q formed
    from the reflectors by torch.linalg.householder_product)."""
    n = At.shape[1]
    k = min(At.shape) if k is None else k
    Q = torch.linalg.householder_product(F[:, :k], tau[:k])
    R = torch.triu(F[:k, :])
    res = (torch.linalg.norm(At[:, jpvt] - Q @ R) / torch.linalg.norm(At)).item()
    orth = torch.linalg.norm(Q.T @ Q - torch.eye(k, dtype=torch.float64, device="cuda")).item()
    del Q, R
    return res, orth


def test_rqrcp_8192_full_size_gaussian():
    """8192 x 8192 i.i.d. N(0,1), b = 64, p = 8, seed 2 (the benchmark
    launch), the whole factorization against the oracle's full RQRCP
    (tests/golden/c2_iid_rqrcp.txt): every pivot up to the oracle's first
    near tie (there is none: its smallest gap is 2.3e-6), |R_jj| for all
    8192 steps within 1e-12 ||A||_F, rows 0..127 of R element by element
    against the oracle's TRQRCP(128) (which forms the same rows), residual
    and orthogonality on the GPU."""
    say("rqrcp 8192x8192 gaussian b=64 p=8 seed=2")
    A, prm = inputs.config_matrix("c2_iid")
    gj, gg, grd, _ = load_pivot_golden("c2_iid_rqrcp.txt")
    At = dev(A)
    F, tau, jpvt, info = binding.rq_rqrcp(At, prm["b"], prm["p"], prm["seed"])
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    jp = host(jpvt)
    t = trusted_prefix(gg, 8192)
    say(f"c2 trusted prefix {t}")
    assert np.array_equal(jp[:t], gj[:t])
    assert sorted(jp.tolist()) == list(range(8192))
    nrm = np.linalg.norm(A)
    rd = np.abs(host(torch.diagonal(F)))
    assert np.abs(rd[:t] - grd[:t]).max() <= 1e-12 * nrm
    # rows 0..127 of R compared un-permuted (R P^T): past column 127 the two
    # runs order the remaining columns differently (TRQRCP(128) stops after
    # two blocks of swaps, RQRCP applies 126 more)
    ref = oracle.trqrcp(A, 128, prm["b"], prm["p"], seed=prm["seed"])
    assert np.array_equal(ref["jpvt"][:128], gj[:128])
    Zg = np.zeros((128, 8192))
    Zg[:, jp] = np.triu(host(F[:128, :]))
    Zo = np.zeros((128, 8192))
    Zo[:, ref["jpvt"]] = np.triu(ref["F"][:128])
    assert np.abs(Zg - Zo).max() <= 1e-12 * nrm
    res, orth = gpu_residual_orth(At, F, tau, jpvt)
    say(f"8192 residual {res:.3e} orthogonality {orth:.3e}")
    assert res <= 1e-12
    assert orth <= 1e-12


def test_rqrcp_8192_rank512_plus_noise():
    """8192 x 8192 rank-512 product of Gaussians + 1e-8 N(0,1), b = 64,
    p = 8, seed 2 (the second input family of the benchmark): the first 512
    pivots equal the oracle's (tests/golden/c2_lr_trqrcp640.txt; its
    smallest gap among them is 2.6e-8, no near tie), as do |R_jj| for
    j < 512; the numerical rank #{j : |R_jj| > 1e-6 |R_00|} is exactly 512;
    residual and orthogonality at the FP64 bar.  Past the rank the sample
    holds noise of relative size 1e-8 / ||A|| ~ 4e-13, below the rounding of
    the first 512 steps, so later pivots are not compared."""
    say("rqrcp 8192x8192 rank-512 + 1e-8 noise b=64 p=8 seed=2")
    A, prm = inputs.config_matrix("c2_lr")
    gj, gg, grd, hdr = load_pivot_golden("c2_lr_trqrcp640.txt")
    assert any("numerical rank" in h and h.endswith(": 512") for h in hdr)
    assert trusted_prefix(gg, 512) == 512
    At = dev(A)
    nrm = np.linalg.norm(A)
    del A
    F, tau, jpvt, info = binding.rq_rqrcp(At, prm["b"], prm["p"], prm["seed"])
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    jp = host(jpvt)
    assert np.array_equal(jp[:512], gj[:512])
    assert sorted(jp.tolist()) == list(range(8192))
    rd = np.abs(host(torch.diagonal(F)))
    assert np.abs(rd[:512] - grd[:512]).max() <= 1e-12 * nrm
    rank = int(np.sum(rd > 1e-6 * rd[0]))
    say(f"c2_lr numerical rank {rank}, |R_511| {rd[511]:.3e} |R_512| {rd[512]:.3e}")
    assert rank == 512
    res, orth = gpu_residual_orth(At, F, tau, jpvt)
    say(f"c2_lr residual {res:.3e} orthogonality {orth:.3e}")
    assert res <= 1e-12
    assert orth <= 1e-12


def test_trqrcp_tuxv_c3_full_size():
    """20000 x 10000, sigma_i = 0.9^(i/10), k = 256, b = 64, p = 8, seed 3
    (the benchmark's TRQRCP/TUXV launch): all 256 pivots and |R_jj| against
    the oracle's TRQRCP(256) (tests/golden/c3_trqrcp256.txt, smallest gap
    1e-4); on the GPU, the residual of the k factored columns, the
    orthonormality of U and V, and the truncation error of TUXV within 1.05x
    of the oracle's (tests/golden/c3_tuxv_oracle_error.txt) and not below the
    Eckart-Young optimum."""
    say("trqrcp/tuxv 20000x10000 k=256 b=64 p=8 seed=3")
    A, prm = inputs.config_matrix("c3")
    k, b, p, seed = prm["k"], prm["b"], prm["p"], prm["seed"]
    gj, gg, grd, _ = load_pivot_golden("c3_trqrcp256.txt")
    At = dev(A)
    nrm = torch.linalg.norm(At).item()
    del A
    F, tau, jpvt, info = binding.rq_trqrcp(At, k, b, p, seed)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    jp = host(jpvt)
    t = trusted_prefix(gg, k)
    assert t == k
    assert np.array_equal(jp[:k], gj)
    assert sorted(jp.tolist()) == list(range(At.shape[1]))
    rd = np.abs(host(torch.diagonal(F[:k, :k])))
    assert np.abs(rd - grd).max() <= 1e-12 * nrm
    Qk = torch.linalg.householder_product(F[:, :k], tau)
    res = (torch.linalg.norm(At[:, jpvt[:k]] - Qk @ torch.triu(F[:k, :k])) / nrm).item()
    say(f"c3 trqrcp residual {res:.3e}")
    assert res <= 1e-12
    del Qk, F
    U, s, VT, info = binding.rq_tuxv(At, k, b, p, seed)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    eye = torch.eye(k, dtype=torch.float64, device="cuda")
    assert torch.linalg.norm(U.T @ U - eye).item() <= orth_tol(k)
    assert torch.linalg.norm(VT @ VT.T - eye).item() <= orth_tol(k)
    sh = host(s)
    assert np.all(np.diff(sh) <= 0) and sh[-1] >= 0
    e = (torch.linalg.norm(At - (U * s) @ VT) / nrm).item()
    opt = inputs.optimal_truncation_error(inputs.sigma_power(10000, 0.9, 10.0), k)
    gold = {}
    with open(os.path.join(GOLDEN, "c3_tuxv_oracle_error.txt")) as f:
        for ln in f:
            if ":" in ln and not ln.startswith("#"):
                key, val = ln.split(":", 1)
                gold[key.strip()] = float(val)
    say(f"c3 tuxv error {e:.6f} oracle {gold['oracle_error']:.6f} optimum {opt:.6f}")
    assert opt * (1 - 1e-9) <= e <= 1.05 * gold["oracle_error"]


def test_empty_matrices():
    """m = 0 or n = 0: the factorizations write the identity permutation and
    info = 0 and nothing else; the sketch of an empty A is zero."""
    say("empty matrices 0x5 / 5x0 / sketch 0x7")
    L = binding.load()
    for m, n in ((0, 5), (5, 0), (0, 0)):
        A = torch.empty((m, n), dtype=torch.float64, device="cuda")
        jpvt = torch.full((max(n, 1),), -7, dtype=torch.int64, device="cuda")
        tau = torch.empty(1, dtype=torch.float64, device="cuda")
        info = torch.full((1,), 77, dtype=torch.int32, device="cuda")
        work = binding.workspace(binding.RQ_OP_RQRCP, m, n, 0, 8, 4, torch.device("cuda"))
        for fn in (L.rq_rqrcp, L.rq_rsrqrcp):
            jpvt.fill_(-7)
            info.fill_(77)
            prec = (binding.RQ_FP64,) if fn is L.rq_rqrcp else ()
            rc = fn(None, m, n, A.data_ptr(), max(1, m), 8, 4, 1, *prec, jpvt.data_ptr(), tau.data_ptr(),
                    work.data_ptr(), work.numel(), info.data_ptr())
            assert rc == 0
            torch.cuda.synchronize()
            assert host(jpvt)[:n].tolist() == list(range(n))
            assert int(info.item()) == 0
        info.fill_(77)
        rc = L.rq_unpivoted_qr(None, m, n, A.data_ptr(), max(1, m), 8, tau.data_ptr(), work.data_ptr(), work.numel(),
                               info.data_ptr())
        assert rc == 0 and int(info.item()) == 0
    B = torch.full((4, 7), 3.0, dtype=torch.float64, device="cuda").t().contiguous().t()
    work = binding.workspace(binding.RQ_OP_RQRCP, 0, 7, 0, 4, 0, torch.device("cuda"))
    A = torch.empty((0, 7), dtype=torch.float64, device="cuda")
    rc = L.rq_sketch(None, 0, 7, A.data_ptr(), 1, 4, 5, binding.RQ_FP64, B.data_ptr(), 4, work.data_ptr(),
                     work.numel())
    assert rc == 0
    assert np.all(host(B) == 0.0)


def test_rqrcp_lookahead_is_bitwise_sequential():
    """The look-ahead (the bulk of each trailing update in the next sample
    QRCP's launch, on workgroups of its own that walk several tiles each:
    about 900 tiles of 128 x 64 on fewer than 256 workgroups) gives the
    factorization of the sequential order bit for bit."""
    say("rqrcp look-ahead on/off 3000x2500 b=64")
    A = dev(inputs.with_spectrum(17, 3000, 2500, inputs.sigma_decade(2500, 8)))
    prev = binding.rq_set_lookahead(True)
    try:
        on = [host(x) for x in binding.rq_rqrcp(A, 64, 8, 17)]
        binding.rq_set_lookahead(False)
        off = [host(x) for x in binding.rq_rqrcp(A, 64, 8, 17)]
    finally:
        binding.rq_set_lookahead(prev)
    for x, y in zip(on, off):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("n", [60000, 65536])
def test_rqrcp_wide_sample_fills_the_device(n):
    """Samples so wide that the sample QRCP's workgroups (one per 256
    columns: 235 and 256) leave few or no CUs for the previous block's
    trailing update in the same launch: the update gets what is left, or
    runs right after the sample QRCP.  Pivots against the oracle, and the
    factorization bit for bit the one without look-ahead."""
    m, b, p, seed = 200, 64, 8, 21
    say(f"rqrcp wide sample {m}x{n} b={b}")
    A = inputs.with_spectrum(seed, m, n, inputs.sigma_decade(m, 8))
    F, tau, jpvt, _ = compare_rqrcp(A, b, p, seed)
    prev = binding.rq_set_lookahead(False)
    try:
        off = [host(x) for x in binding.rq_rqrcp(dev(A), b, p, seed)]
    finally:
        binding.rq_set_lookahead(prev)
    for x, y in zip((F, tau, jpvt), off[:3]):
        assert np.array_equal(x, y)


def test_tuxv_rank_one_and_full_rank():
    """k = 1 against the oracle; k = min(m, n): TUXV spans all of A, so it
    is A's SVD (singular values of LAPACK, approximation error at rounding)."""
    say("tuxv k=1 300x200 / k=min 260x200")
    A = inputs.with_spectrum(41, 300, 200, inputs.sigma_decade(200, 6))
    ref = oracle.tuxv(A, 1, 8, 4, seed=41)
    U, s, VT, info = [host(x) for x in binding.rq_tuxv(dev(A), 1, 8, 4, 41)]
    assert info[0] == 0
    assert abs(s[0] - ref["s"][0]) <= 1e-12 * ref["s"][0]
    nrm = np.linalg.norm(A)
    assert np.linalg.norm(np.outer(U[:, 0], VT[0]) * s[0] - np.outer(ref["U"][:, 0], ref["VT"][0]) * ref["s"][0]) \
        <= 1e-12 * nrm
    A = inputs.with_spectrum(42, 260, 200, inputs.sigma_decade(200, 6))
    U, s, VT, info = [host(x) for x in binding.rq_tuxv(dev(A), 200, 32, 8, 42)]
    assert info[0] == 0
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.abs(s - sv).max() <= 1e-12 * sv[0]
    assert np.linalg.norm(A - (U * s) @ VT) <= 1e-12 * np.linalg.norm(A)
    assert np.linalg.norm(U.T @ U - np.eye(200)) <= orth_tol(200)
    assert np.linalg.norm(VT @ VT.T - np.eye(200)) <= orth_tol(200)


@pytest.mark.xfail(strict=False, reason="open issue: with the look-ahead on, repeated b = 32 factorizations of this "
                   "matrix sometimes differ (every result a valid factorization): from a bit-identical "
                   "sample, one fused sample-QRCP launch picked a different first pivot; not seen at "
                   "b = 64 or with the look-ahead off; cause not found")
def test_rqrcp_lookahead_repeatable_at_b32():
    """The look-ahead factorization at b = 32 repeats bit for bit."""
    m, n, b, p, seed = 2100, 1300, 32, 8, 9
    say(f"rqrcp look-ahead repeatability {m}x{n} b={b}")
    A = dev(inputs.with_spectrum(seed, m, n, inputs.sigma_decade(min(m, n), 8)))
    prev = binding.rq_set_lookahead(True)
    try:
        runs = [[host(x) for x in binding.rq_rqrcp(A, b, p, seed)] for _ in range(6)]
    finally:
        binding.rq_set_lookahead(prev)
    for r in runs[1:]:
        for x, y in zip(runs[0], r):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("m,n,b,p,seed,lookahead", [
    (2100, 1300, 32, 8, 9, True),
    (2100, 1300, 32, 8, 9, False),
    (1000, 700, 64, 8, 8, True),
])
def test_rqrcp_result_does_not_depend_on_workspace_contents(m, n, b, p, seed, lookahead):
    """Every buffer the factorization reads from its workspace is written
    first: a workspace full of NaNs, one full of zeros and one full of
    ones give the same factorization bit for bit."""
    say(f"rqrcp workspace contents {m}x{n} b={b} lookahead={lookahead}")
    A = dev(inputs.with_spectrum(seed, m, n, inputs.sigma_decade(min(m, n), 8)))
    nbytes = binding.rq_workspace_bytes(binding.RQ_OP_RQRCP, m, n, 0, b, p)
    prev = binding.rq_set_lookahead(lookahead)
    try:
        outs = []
        for fill in (float("nan"), 0.0, 1.0):
            work = torch.full(((nbytes + 7) // 8,), fill, dtype=torch.float64, device="cuda").view(torch.uint8)
            outs.append([host(x) for x in binding.rq_rqrcp(A, b, p, seed, work=work)])
    finally:
        binding.rq_set_lookahead(prev)
    assert outs[0][3][0] == 0
    for other in outs[1:]:
        for x, y in zip(outs[0], other):
            assert np.array_equal(x, y)
