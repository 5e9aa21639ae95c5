"""Continuous batching on the GPU: every served job's result equals the FP64
oracle's run of the same job (within 1e-12 in FP64, 2e-6 in FP32 shifted
storage) and its own solo run bitwise; jobs overlap on the device, the memory
budget forces queueing, and a diverging job is reported without disturbing
the others."""
import numpy as np
import pytest

import oracle
import sc_inputs
from gpu_common import maxabs, say

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32_shifted": 2e-6}
_ORACLE = {}


def _oracle(job):
    """Oracle populations of a served job after its steps (cached per job)."""
    key = (job.lattice, job.nx, job.ny, job.nz, job.tau, job.G, job.steps, job.kind,
           job.radius, job.seed)
    if key not in _ORACLE:
        fl = job.fields()
        _ORACLE[key] = oracle.run(oracle.init(job.lattice, fl.rho_A, fl.rho_B), job.tau,
                                  job.tau, job.G, job.steps, all_cores=True)
    return _ORACLE[key]


def _jobs(n, seed, rate, step_range=(40, 400)):
    return sc_inputs.serving_jobs(n, seed=seed, rate=rate, step_range=step_range, l2=(32, 160),
                                  l3=(16, 40), frac_3d=0.35)


@pytest.mark.parametrize("precision,mode,policy,sat", [
    ("fp32_shifted", "persistent", "srpt", 4_000_000),
    ("fp64", "fused", "srpt", 4_000_000),
    ("fp32_shifted", "fused", "srpt", 20_000),     # lone large jobs step by themselves
    ("fp64", "persistent", "all", 4_000_000),
])
def test_served_results_equal_solo_runs(precision, mode, policy, sat):
    from paper_1112_5547_amd import Lattice
    from paper_1112_5547_amd.serve import GpuBackend, Server
    # runs short enough that the oracle bounds hold pointwise: the spinodal
    # jobs amplify rounding differences by exp(growth rate x steps) (about
    # 0.056 per step at G = 1.6, tau = 1), so 60 steps at most; several
    # 16-step epochs per job keep jobs joining and leaving the batch
    jobs = _jobs(14, seed=31, rate=2000.0, step_range=(20, 60))
    be = GpuBackend(precision=precision)
    budget = sum(sorted(be.bytes_needed(j) for j in jobs)[-4:])  # forces queueing
    say(f"serve 14 jobs {precision} {mode} {policy} sat {sat}, budget {budget}")
    rep = Server(hbm_budget=budget, epoch_steps=16, mode=mode, backend=be,
                 keep_populations=True, policy=policy, sat_sites=sat).run(jobs)
    s = rep.summary()
    assert s["jobs"] == len(jobs) and s["nonfinite"] == 0 and s["refused"] == 0
    assert s["max_resident"] >= 2
    for r in rep.results:
        job = jobs[r.job_id]
        say(f"solo job {job.job_id} q={job.lattice} {job.nx}x{job.ny}x{job.nz} {job.steps} steps")
        lat = Lattice(job.lattice, job.nx, job.ny, job.nz, tau_A=job.tau, G=job.G,
                      precision=precision)
        fl = job.fields()
        lat.init(fl.rho_A, fl.rho_B)
        lat.step(job.steps)
        assert np.array_equal(r.populations, lat.get_populations()), job
        lat.close()
        err = maxabs(r.populations, _oracle(job))
        assert err <= TOL[precision], (job, err)


def test_diverging_job_is_evicted_and_others_finish():
    from paper_1112_5547_amd.serve import GpuBackend, Server
    jobs = _jobs(6, seed=32, rate=1000.0)
    jobs[3].G, jobs[3].tau, jobs[3].steps = 40.0, 0.51, 200
    say("serve 6 jobs with one diverging")
    rep = Server(hbm_budget=0, epoch_steps=50, mode="persistent",
                 backend=GpuBackend("fp32_shifted")).run(jobs)
    by_id = {r.job_id: r for r in rep.results}
    assert by_id[3].status == "nonfinite"
    assert all(r.status == "ok" for r in rep.results if r.job_id != 3)
