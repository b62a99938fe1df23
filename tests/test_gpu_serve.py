"""GPU checks of the continuous-batching TUXV server (paper_1509_06820_amd.
serve): a mixed stream of requests (uneven sizes, ranks 16..128, FP64 and
mixed precision, staggered arrivals) completes within the HBM budget; every
result equals, bit for bit, the result of the same request served alone;
and the truncation errors stay within 1.05x the FP64 oracle's."""

import numpy as np
import pytest
import torch

import oracle
from paper_1509_06820_amd import binding, serve
from test_gpu_parity import host, say

pytestmark = pytest.mark.gpu


def make_requests(count, seed, ks=(16, 32, 64, 128), smin=200, smax=900, gap=2e-4):
    rng = np.random.default_rng(seed)
    reqs, t = [], 0.0
    for i in range(count):
        a, b = np.exp(rng.uniform(np.log(smin), np.log(smax), size=2))
        m, n = int(max(a, b)), int(min(a, b))
        k = int(min(n, rng.choice(ks)))
        prec = binding.RQ_MIXED if rng.uniform() < 0.5 else binding.RQ_FP64
        A = serve.serving_matrix_device(i, m, n, seed=seed)
        reqs.append(serve.Request(i, A, k, prec, seed=1000 + i, arrival=t))
        t += float(rng.exponential(gap))
    return reqs


def test_server_mixed_stream_matches_alone_and_oracle():
    say("server: 24 mixed requests")
    reqs = make_requests(24, 3)
    budget = 4 * max(serve.TuxvServer(1).footprint(r) for r in reqs)
    srv = serve.TuxvServer(budget, streams=3)
    stats = srv.serve(reqs)
    say(f"server stats {stats}")
    assert stats["requests"] == 24 and stats["max_hbm_bytes"] <= budget
    assert stats["batched"] > 0 and stats["single"] > 0
    for r in reqs:
        assert int(host(r.info)[0]) == 0, r.id
    # the same requests served one at a time
    for r in reqs[::3]:
        alone = serve.Request(r.id, r.A, r.k, r.precision, r.seed, 0.0)
        serve.TuxvServer(budget, streams=1).serve([alone])
        for x, y in ((alone.U, r.U), (alone.sigma, r.sigma), (alone.VT, r.VT)):
            assert np.array_equal(host(x), host(y)), r.id
    # truncation error against the FP64 oracle (same block size and seed)
    for r in reqs[:6]:
        A = host(r.A)
        b = serve.block_size(r.k, r.batched)
        ref = oracle.tuxv(A, r.k, b, 8, seed=r.seed)
        nrm = np.linalg.norm(A)
        e = np.linalg.norm(A - (host(r.U) * host(r.sigma)) @ host(r.VT)) / nrm
        e_ref = np.linalg.norm(A - (ref["U"] * ref["s"]) @ ref["VT"]) / nrm
        assert e <= 1.05 * e_ref, (r.id, e, e_ref)


def test_server_admission_respects_the_budget():
    """With room for about two requests at a time, requests wait for memory
    and all of them still complete."""
    say("server: tight HBM budget")
    reqs = make_requests(10, 7, ks=(16, 32), gap=0.0)
    fp = [serve.TuxvServer(1).footprint(r) for r in reqs]
    budget = 2.2 * max(fp)
    srv = serve.TuxvServer(budget, streams=4)
    stats = srv.serve(reqs)
    assert stats["max_hbm_bytes"] <= budget
    assert all(r.t_done is not None for r in reqs)
    for r in reqs:
        assert int(host(r.info)[0]) == 0
