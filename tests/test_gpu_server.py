"""The job server: jobs that arrive while others run are admitted as memory
frees up, share batched launches, and finish with exactly the fields they
have when run alone (marked gpu)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def flb():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1708_01613_amd import foamlbm

    return foamlbm


def _say(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def _jobs():
    rng = np.random.default_rng(21)
    jobs = []
    for k in range(7):
        d3 = k % 3 == 2
        if d3:
            n = int(rng.integers(24, 40))
            p = dict(lattice=1, storage="f32", nx=n, ny=n + 3, nz=n - 2)
            nuc = [[float(rng.uniform(0, n)), float(rng.uniform(0, n)), float(rng.uniform(0, n - 2)),
                    float(rng.uniform(3, 6))] for _ in range(4)]
        else:
            n = int(rng.integers(48, 120))
            p = dict(lattice=0, storage="f32", nx=n, ny=n - 5)
            nuc = [[float(rng.uniform(0, n)), float(rng.uniform(0, n - 5)), 0.0, float(rng.uniform(3, 9))]
                   for _ in range(5)]
        p.update(G=float(rng.uniform(-6.0, -4.8)), rho_liquid=2.3, rho_gas=0.11, seed=100 + k,
                 film_on=int(k % 2 == 0), k_own=5, rupture_warmup=30)
        steps = int(rng.integers(20, 90))
        jobs.append((p, nuc, steps))
    return jobs


@pytest.mark.parametrize("policy", ["fifo", "shortest"])
def test_jobs_in_the_mix_equal_jobs_alone(flb, policy):
    jobs = _jobs()
    _say(f"server ({policy}) with {len(jobs)} mixed jobs, staggered arrivals, small pool")
    # a pool that holds about three of these jobs at once, so later jobs wait;
    # with shortest-first, a cell budget below the resident cells leaves some
    # resident jobs out of some rounds
    pol = flb.FLB_SERVE_FIFO if policy == "fifo" else flb.FLB_SERVE_SHORTEST
    srv = flb.Server(pool_bytes=3 * 40 * 1024 * 1024, chunk_steps=16, graph_steps=8, policy=pol,
                     max_cells=None if policy == "fifo" else 20000)
    ids = []
    for k, (p, nuc, steps) in enumerate(jobs):
        ids.append(srv.submit(steps, nuc, **p))
        if k % 2 == 1:
            srv.pump()  # jobs arrive while others run
    rounds = 0
    while True:
        running, queued, done = srv.pump()
        rounds += 1
        assert rounds < 1000
        if running == 0 and queued == 0:
            break
    assert done == len(jobs)
    used, pool = srv.usage()
    assert used == 0
    for k, (p, nuc, steps) in enumerate(jobs):
        st, sd = srv.state(ids[k])
        assert st == flb.FLB_JOB_DONE and sd == steps
        rho, stats = srv.result(ids[k])
        solo = flb.Sim(**p)
        solo.set_nuclei(nuc)
        solo.step(steps)
        assert np.array_equal(rho, solo.density()), k
        assert stats["step"] == steps
        srv.release(ids[k])


def test_shortest_first_finishes_short_jobs_first(flb):
    # a long job resident first, then short ones: with shortest-first the
    # short jobs finish while the long one waits, and the long one still ends
    _say("shortest-first ordering: one long job, four short ones")
    srv = flb.Server(chunk_steps=10, graph_steps=0, policy=flb.FLB_SERVE_SHORTEST, max_cells=9000)
    long_id = srv.submit(400, [[40, 40, 0, 8]], lattice=0, storage="f32", nx=90, ny=90, G=-5.5)
    srv.pump()
    short = [srv.submit(30, [[20, 20, 0, 6]], lattice=0, storage="f32", nx=60, ny=60, G=-5.5, seed=k)
             for k in range(4)]
    finished = []
    for _ in range(200):
        running, queued, _ = srv.pump()
        for jid in [long_id] + short:
            if jid not in finished and srv.state(jid)[0] == flb.FLB_JOB_DONE:
                finished.append(jid)
        if running == 0 and queued == 0:
            break
    assert finished[-1] == long_id and sorted(finished[:-1]) == sorted(short)
    rho, st = srv.result(long_id)
    solo = flb.Sim(lattice=0, storage="f32", nx=90, ny=90, G=-5.5)
    solo.set_nuclei([[40, 40, 0, 8]])
    solo.step(400)
    assert st["step"] == 400 and np.array_equal(rho, solo.density())


def test_job_larger_than_pool_is_refused(flb):
    srv = flb.Server(pool_bytes=1 << 20)
    with pytest.raises(flb.FlbError) as e:
        srv.submit(10, [[8, 8, 0, 3]], lattice=0, storage="f32", nx=256, ny=256)
    assert e.value.code == flb.FLB_EBUSY


def test_zero_step_job_finishes(flb):
    srv = flb.Server()
    jid = srv.submit(0, [[16, 16, 0, 5]], lattice=0, storage="f32", nx=40, ny=40)
    srv.pump()
    st, sd = srv.state(jid)
    assert st == flb.FLB_JOB_DONE and sd == 0
    rho, _ = srv.result(jid)
    s = flb.Sim(lattice=0, storage="f32", nx=40, ny=40)
    s.set_nuclei([[16, 16, 0, 5]])
    assert np.array_equal(rho, s.density())


def _solo(flb, p, nuc, steps):
    s = flb.Sim(**p)
    s.set_nuclei(nuc)
    s.step(steps)
    return s.density()


@pytest.mark.parametrize("policy", ["fifo", "shortest"])
def test_unstable_job_fails_early_and_others_are_unchanged(flb, policy):
    # G = -20 is far past the stable range of the pseudopotential force: the
    # mass turns non-finite within a few steps.  The job must leave the server
    # as failed after its first round, while the jobs sharing its launches
    # finish with exactly their solo fields.
    _say(f"server ({policy}): two stable jobs and one whose mass blows up")
    pol = flb.FLB_SERVE_FIFO if policy == "fifo" else flb.FLB_SERVE_SHORTEST
    srv = flb.Server(chunk_steps=10, graph_steps=5, policy=pol)
    good = [(dict(lattice=0, storage="f32", nx=64, ny=56, G=-5.5, rho_liquid=2.3, rho_gas=0.11, seed=4,
                  film_on=1, k_own=5, rupture_warmup=10), [[30, 28, 0, 7], [12, 10, 0, 5]], 60),
            (dict(lattice=0, storage="f32", nx=48, ny=48, G=-5.0, rho_liquid=2.3, rho_gas=0.11, seed=5),
             [[24, 24, 0, 8]], 45)]
    bad = dict(lattice=0, storage="f32", nx=40, ny=36, G=-20.0, rho_liquid=2.3, rho_gas=0.11, seed=3,
               film_on=1, k_own=5, rupture_warmup=0)
    ids = [srv.submit(steps, nuc, **p) for p, nuc, steps in good]
    bad_id = srv.submit(200, [[20, 18, 0, 6]], **bad)
    running, _, _ = srv.pump()
    assert running == 2
    st, sd = srv.state(bad_id)
    assert st == flb.FLB_JOB_FAILED and sd == 10
    with pytest.raises(flb.FlbError) as e:
        srv.result(bad_id)
    assert e.value.code == flb.FLB_ENUMERIC
    for _ in range(100):
        running, queued, done = srv.pump()
        if running == 0 and queued == 0:
            break
    assert done == 3 and srv.usage()[0] == 0
    for jid, (p, nuc, steps) in zip(ids, good):
        assert srv.state(jid) == (flb.FLB_JOB_DONE, steps)
        rho, stats = srv.result(jid)
        assert np.array_equal(rho, _solo(flb, p, nuc, steps))
    srv.release(bad_id)


def test_cancel_queued_and_running_jobs(flb):
    # one resident job at a time: A runs, B and C wait; B is cancelled while
    # queued, A while running, and C -- of another size, admitted into the
    # slot A held -- still finishes with its solo field
    _say("server: cancel a queued job and a running one")
    srv = flb.Server(max_jobs=1, chunk_steps=8, graph_steps=4)
    pa = dict(lattice=0, storage="f32", nx=72, ny=60, G=-5.5, seed=1)
    pc = dict(lattice=0, storage="f32", nx=40, ny=52, G=-5.2, seed=2, film_on=1, k_own=5, rupture_warmup=10)
    a = srv.submit(100, [[36, 30, 0, 9]], **pa)
    b = srv.submit(50, [[20, 20, 0, 6]], **pa)
    c = srv.submit(37, [[20, 26, 0, 7], [8, 8, 0, 4]], **pc)
    assert srv.pump()[:2] == (1, 2)
    srv.cancel(b)
    assert srv.state(b)[0] == flb.FLB_JOB_CANCELLED
    srv.pump()
    srv.cancel(a)
    assert srv.state(a) == (flb.FLB_JOB_CANCELLED, 16)
    assert srv.usage()[0] == 0
    for jid in (a, b):
        with pytest.raises(flb.FlbError) as e:
            srv.cancel(jid)
        assert e.value.code == flb.FLB_EINVAL
        with pytest.raises(flb.FlbError):
            srv.result(jid)
    for _ in range(100):
        running, queued, done = srv.pump()
        if running == 0 and queued == 0:
            break
    assert done == 3
    assert srv.state(c) == (flb.FLB_JOB_DONE, 37)
    rho, _ = srv.result(c)
    assert np.array_equal(rho, _solo(flb, pc, [[20, 26, 0, 7], [8, 8, 0, 4]], 37))
    for jid in (a, b, c):
        srv.release(jid)


@pytest.mark.parametrize("use_torch_memory", [True, False])
def test_back_to_back_jobs_of_different_sizes(flb, use_torch_memory):
    # one resident job at a time, so each new job's context may land at the
    # host address of the one just retired; each must still run on its own
    # tables and equal its solo field
    _say(f"server: single-slot jobs of different sizes (torch memory {use_torch_memory})")
    srv = flb.Server(max_jobs=1, chunk_steps=12, graph_steps=6, use_torch_memory=use_torch_memory)
    jobs = [(dict(lattice=0, storage="f32", nx=40 + 12 * k, ny=36 + 8 * k, G=-5.5, seed=10 + k,
                  film_on=k % 2, k_own=5, rupture_warmup=10), [[18 + 4 * k, 16 + 3 * k, 0, 6]], 24 + 5 * k)
            for k in range(4)]
    ids = [srv.submit(steps, nuc, **p) for p, nuc, steps in jobs]
    for _ in range(100):
        running, queued, done = srv.pump()
        if running == 0 and queued == 0:
            break
    assert done == len(jobs)
    for jid, (p, nuc, steps) in zip(ids, jobs):
        rho, stats = srv.result(jid)
        assert stats["step"] == steps
        assert np.array_equal(rho, _solo(flb, p, nuc, steps))
