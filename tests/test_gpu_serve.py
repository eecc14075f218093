"""Serving on the GPU: the device genotype generator equals the host one bit
for bit; a job's results are the same alone and batched with other jobs;
a job that cannot be factored fails alone."""
import sys

import numpy as np
import pytest

from oracle import gls_oracle as orc
from paper_1210_7325_amd import datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def serve():
    from paper_1210_7325_amd import gls, serve
    gls.lib()
    dg._dlib()
    return serve


@pytest.mark.parametrize("n,p_R,snp0,nsnp", [(1000, 1, 0, 300), (1501, 4, 17, 33), (63, 2, 5, 9)])
def test_device_generator_bitwise_equal_to_host(serve, n, p_R, snp0, nsnp):
    say("device generator", n, p_R)
    w = dg.SMALL.replace(n=n, p_R=p_R, seed=dg.MASTER_SEED + n)
    out = torch.full((nsnp * p_R + 3, n), -1, dtype=torch.int8, device="cuda").t()
    dg.make_XR_device(w, snp0, nsnp, out, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got[:, :nsnp * p_R], dg.make_XR(w, snp0, nsnp, use_c=False))
    assert np.all(got[:, nsnp * p_R:] == -1)  # nothing written past the columns asked for


def mix_jobs(serve):
    specs = [(300, 4, 3000, 0.3), (700, 7, 2500, 0.5), (1000, 12, 2000, 0.7), (500, 4, 4000, 0.6)]
    return [serve.Job(id=i, arrival=0.002 * i, n=n, p=p, m=m, h=h, seed=dg.MASTER_SEED + 700 + i,
                      block=512) for i, (n, p, m, h) in enumerate(specs)]


def run_jobs(serve, jobs, precision, phi):
    ex = serve.GpuExecutor(precision=precision, phi=phi, keep_results=True)
    stats = serve.Scheduler(ex, budget_bytes=64 << 30).run(jobs)
    return stats, ex.results


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_alone_equals_mix(serve, precision):
    say("serve alone vs mix", precision)
    phi = {}
    jobs = mix_jobs(serve)
    stats, mixed = run_jobs(serve, jobs, precision, phi)
    assert stats["done"] == len(jobs)
    assert stats["items_per_round"] > 1.5          # blocks of different jobs share launches
    for j in mix_jobs(serve):
        _, alone = run_jobs(serve, [j], precision, phi)
        assert np.array_equal(alone[j.id][0], mixed[j.id][0]), j.id
        assert np.all(mixed[j.id][1] == 0)
    # and the mix against the oracle (sampled problems of every job)
    tol = 1e-10 if precision == "fp64" else 1e-8
    for j in jobs:
        w = j.workload()
        phih = phi[j.n].cpu().numpy()
        M = dg.make_M(w, phi=phih, h=j.h)
        idx = np.unique(np.linspace(0, j.m - 1, 40).astype(int))
        XR = np.concatenate([dg.make_XR(w, int(i), 1) for i in idx], axis=1)
        ref = orc.gls_sequence(M, dg.make_XL(w), XR, dg.make_Y(w), 1)
        err = orc.relative_error(mixed[j.id][0][idx], ref)
        say("job", j.id, "n", j.n, "p", j.p, "max rel err", err.max())
        assert err.max() < tol


def test_failed_job_does_not_disturb_the_mix(serve):
    say("serve failure isolation")
    phi = {}
    jobs = mix_jobs(serve)
    jobs[1].h = 1.5            # M = 1.5 Phi - 0.5 I + 1e-3 I is indefinite
    stats, res = run_jobs(serve, jobs, "fp64", phi)
    assert jobs[1].state == "failed" and "positive definite" in jobs[1].error
    assert stats["done"] == len(jobs) - 1
    ref_jobs = mix_jobs(serve)
    for k in (0, 2, 3):
        _, alone = run_jobs(serve, [ref_jobs[k]], "fp64", phi)
        assert np.array_equal(alone[k][0], res[k][0])
