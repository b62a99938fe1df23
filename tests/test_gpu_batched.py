"""GPU checks of the batched TRQRCP + TUXV engine (rq_batch_plan_create /
rq_tuxv_batched): every matrix of an uneven batch against the FP64 oracle's
TUXV with the same seed (pivots up to the oracle's first near tie, sigma
and U diag(sigma) VT to 1e-12 in FP64; with FP32 products the truncation
error within 1.05x the oracle's), the batched result against the
single-matrix entry point, each result the same alone and in the batch
(bit for bit), and HIP graph capture replayed several times.

The batched engine forms its orthogonal factors explicitly (Gram-Schmidt
and shifted CholeskyQR) where the single-matrix path uses Householder
reflectors, so the two agree to rounding, not bit for bit; singular vectors
are compared through U diag(sigma) VT."""

import numpy as np
import pytest
import torch

import oracle
from paper_1509_06820_amd import binding, inputs
from test_gpu_parity import dev, host, orth_tol, say, trusted_prefix

pytestmark = pytest.mark.gpu


def uneven_batch(count, seed, k, mmin=None, mmax=600):
    rng = np.random.default_rng(seed)
    mats = []
    for i in range(count):
        m = int(rng.integers(mmin or 2 * k, mmax))
        n = int(rng.integers(k, m + 1))
        sig = 10.0 ** (-6.0 * np.arange(min(m, n)) / n)
        mats.append(inputs.with_spectrum(seed * 1000 + i, m, n, sig))
    return mats


def run_batch(mats, k, b, p, seeds, precision="fp64", tile=0):
    bt = binding.BatchTUXV([dev(A) for A in mats], k, b, p, seeds, precision=precision, tile=tile)
    bt.run()
    torch.cuda.synchronize()
    out = [(host(bt.U[i]), host(bt.sigma[i]), host(bt.VT[i]), host(bt.jpvt[i])) for i in range(len(mats))]
    info = host(bt.info)[:len(mats)]
    bt.close()
    return out, info


@pytest.mark.parametrize("k,b,p,tile", [(16, 8, 8, 0), (16, 16, 8, 1), (32, 16, 8, 2), (24, 8, 4, 0)])
def test_batched_fp64_matches_oracle(k, b, p, tile):
    say(f"batched tuxv fp64 k={k} b={b} p={p} tile={tile}")
    mats = uneven_batch(10, 11 + k + b, k)
    seeds = [100 + i for i in range(len(mats))]
    out, info = run_batch(mats, k, b, p, seeds, tile=tile)
    assert np.all(info == 0), info
    for A, sd, (U, s, VT, jp) in zip(mats, seeds, out):
        ref = oracle.tuxv(A, k, b, p, seed=sd)
        tq = oracle.trqrcp(A, k, b, p, seed=sd)
        t = trusted_prefix(tq["gaps"], k)
        assert np.array_equal(jp[:t], tq["jpvt"][:t])
        nrm = np.linalg.norm(A)
        assert np.abs(s - ref["s"]).max() <= 1e-12 * ref["s"][0]
        approx = (U * s) @ VT
        assert np.linalg.norm(approx - (ref["U"] * ref["s"]) @ ref["VT"]) <= 1e-12 * nrm
        assert np.linalg.norm(U.T @ U - np.eye(k)) <= orth_tol(k)
        assert np.linalg.norm(VT @ VT.T - np.eye(k)) <= orth_tol(k)
        assert np.all(np.diff(s) <= 0) and s[-1] >= 0


def test_batched_mixed_error_against_oracle():
    say("batched tuxv mixed k=32 b=16")
    k, b, p = 32, 16, 8
    mats = uneven_batch(12, 5, k, mmax=900)
    seeds = [7 + i for i in range(len(mats))]
    out, info = run_batch(mats, k, b, p, seeds, precision="mixed")
    assert np.all(info == 0), info
    for A, sd, (U, s, VT, jp) in zip(mats, seeds, out):
        ref = oracle.tuxv(A, k, b, p, seed=sd)
        nrm = np.linalg.norm(A)
        e = np.linalg.norm(A - (U * s) @ VT) / nrm
        e_ref = np.linalg.norm(A - (ref["U"] * ref["s"]) @ ref["VT"]) / nrm
        assert e <= 1.05 * e_ref, (e, e_ref)
        assert np.linalg.norm(U.T @ U - np.eye(k)) <= orth_tol(k)
        assert np.linalg.norm(VT @ VT.T - np.eye(k)) <= orth_tol(k)


def test_batched_equals_single_entry_point():
    say("batched vs rq_tuxv k=16 b=8")
    k, b, p = 16, 8, 8
    mats = uneven_batch(6, 3, k)
    seeds = [40 + i for i in range(len(mats))]
    out, info = run_batch(mats, k, b, p, seeds)
    assert np.all(info == 0)
    for A, sd, (U, s, VT, jp) in zip(mats, seeds, out):
        U1, s1, VT1, inf1 = [host(x) for x in binding.rq_tuxv(dev(A), k, b, p, sd)]
        assert inf1[0] == 0
        assert np.abs(s - s1).max() <= 1e-12 * s1[0]
        assert np.linalg.norm((U * s) @ VT - (U1 * s1) @ VT1) <= 1e-12 * np.linalg.norm(A)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_result_same_alone_and_in_the_batch(precision):
    """Each matrix's work touches only its own buffers and its tiles do not
    depend on the rest of the batch: a matrix factored alone gives the bits
    it gets inside a batch."""
    say(f"batched alone vs in the batch ({precision})")
    k, b, p = 16, 8, 8
    mats = uneven_batch(7, 21, k)
    seeds = [300 + i for i in range(len(mats))]
    out, _ = run_batch(mats, k, b, p, seeds, precision=precision)
    for i in (0, 3, 6):
        alone, _ = run_batch([mats[i]], k, b, p, [seeds[i]], precision=precision)
        for x, y in zip(alone[0], out[i]):
            assert np.array_equal(x, y)


def test_batched_graph_capture_replays():
    """The batch captured in a HIP graph: three replays, with eager work on
    the same stream between them (the outputs wiped), each equal bit for bit
    to the eager run."""
    say("batched graph capture")
    k, b, p = 16, 8, 8
    mats = uneven_batch(9, 33, k)
    seeds = [500 + i for i in range(len(mats))]
    bt = binding.BatchTUXV([dev(A) for A in mats], k, b, p, seeds)
    bt.run()
    torch.cuda.synchronize()
    ref = [(host(bt.U[i]), host(bt.sigma[i]), host(bt.VT[i])) for i in range(len(mats))]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bt.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for i in range(len(mats)):
            bt.U[i].fill_(float("nan"))
            bt.sigma[i].zero_()
            bt.VT[i].fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(mats)):
            assert np.array_equal(host(bt.U[i]), ref[i][0]), (rep, i)
            assert np.array_equal(host(bt.sigma[i]), ref[i][1]), (rep, i)
            assert np.array_equal(host(bt.VT[i]), ref[i][2]), (rep, i)
    del g
    bt.close()


def test_batched_zero_matrix_reports_breakdown():
    """An all-zero matrix has no column space: CholeskyQR meets a zero pivot
    and the matrix's info word says so (-4); the other matrices of the batch
    are unaffected."""
    say("batched zero matrix")
    k, b, p = 8, 8, 4
    mats = uneven_batch(3, 44, k, mmax=200)
    mats[1] = np.zeros_like(mats[1])
    out, info = run_batch(mats, k, b, p, [1, 2, 3])
    assert info[1] == -4 and info[0] == 0 and info[2] == 0
    ref = oracle.tuxv(mats[0], k, b, p, seed=1)
    assert np.abs(out[0][1] - ref["s"]).max() <= 1e-12 * ref["s"][0]


def test_batched_c4_workload_subsample():
    """The 512-matrix workload (m log-uniform on [64, 2048], n uniform on
    [64, m], sigma_j = 10^(-6 j / n), k = 32, p = 8) with FP32 products, in
    the tile and block size the tuned plan uses by default (b = 16, 64 x 64
    tiles): all info words 0, and on 24 matrices spread over the batch the
    truncation error within 1.05x the FP64 oracle's."""
    say("batched c4 512 matrices, mixed, oracle on 24")
    batch = inputs.batch_c4(512)
    mats = [A for A, _ in batch]
    seeds = [prm["seed"] for _, prm in batch]
    out, info = run_batch(mats, 32, 16, 8, seeds, precision="mixed")
    assert np.all(info == 0), np.nonzero(info)
    for i in range(0, 512, 512 // 24):
        A = mats[i]
        U, s, VT, _ = out[i]
        ref = oracle.tuxv(A, 32, 16, 8, seed=seeds[i])
        nrm = np.linalg.norm(A)
        e = np.linalg.norm(A - (U * s) @ VT) / nrm
        e_ref = np.linalg.norm(A - (ref["U"] * ref["s"]) @ ref["VT"]) / nrm
        assert e <= 1.05 * e_ref, (i, e, e_ref)
