"""GPU parity of the batched engine: every job of a batch against the oracle
(small batches) and, at the full 1024-point 3x3 scan, every point against
the single-state complex128 path plus sampled points against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2108_13410_amd import workloads, z2h

from helpers import (compare_observables, fidelity_loss, gpu_run, oracle_observables, oracle_run,
                     to_oracle_order)

pytestmark = pytest.mark.gpu


def run_batch(jobs, dtype, inits=None, orders=None, renorm=None):
    scheds, Lx, Ly, H = [], [], [], []
    for i, j in enumerate(jobs):
        scheds.append(z2h.schedule(j["c0"], j["c1"], j["M"], j["T"] / max(j["M"], 1),
                                   order=(orders[i] if orders else 0),
                                   renorm=(renorm if renorm is not None else (1 if dtype == z2h.Z2H_C64 else 0))))
        Lx.append(j["Lx"])
        Ly.append(j["Ly"])
        H.append(j["c1"])
    inits = inits or [z2h.Z2H_INIT_PSI1] * len(jobs)
    b = z2h.z2h_batch_create(Lx, Ly, scheds, inits, H, dtype)
    states = torch.empty(b.states_bytes, dtype=torch.uint8, device="cuda")
    ws = torch.empty(b.ws_bytes, dtype=torch.uint8, device="cuda")
    obs = torch.zeros(len(jobs) * z2h.Z2H_OBS_DOUBLES, dtype=torch.float64, device="cuda")
    z2h.z2h_batch_run(b, states, ws, obs)
    torch.cuda.synchronize()
    return b, states, obs.cpu().numpy().reshape(len(jobs), -1)


def row_to_obs(r):
    return {"norm": r[0], "energy": r[1], "sumA": r[2], "sumB": r[3], "mx": r[4], "mz": r[5],
            "zloop": list(r[6:14]), "xloop": list(r[14:22]), "dos": list(r[22:55]), "xnorm": r[55]}


def state_of(b, states, j, n, dtype):
    nbytes = (16 if dtype == z2h.Z2H_C128 else 8) << n
    off = int(b.offsets[j])
    raw = states[off:off + nbytes]
    t = raw.view(torch.complex128 if dtype == z2h.Z2H_C128 else torch.complex64)
    return t.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("dtype", [z2h.Z2H_C128, z2h.Z2H_C64])
def test_mixed_batch_against_oracle(dtype):
    """Uneven lattices and step counts, both step orders, all initial states."""
    rng = np.random.default_rng(7)
    jobs, inits, orders = [], [], []
    for (Lx, Ly) in ((2, 2), (2, 3), (3, 3), (2, 2), (3, 3), (2, 3), (3, 3)):
        hx, hz = rng.uniform(0, 0.6, 2)
        M = int(rng.integers(5, 40))
        jobs.append(dict(Lx=Lx, Ly=Ly, c0=workloads.TORIC, c1=(1.0, 0.9, hx, hz), T=0.08 * M, M=M))
        inits.append(int(rng.integers(0, 4)))
        orders.append(int(rng.integers(0, 2)))
    jobs.append(dict(Lx=3, Ly=3, c0=workloads.TORIC, c1=(1, 1, .2, .2), T=0.0, M=0))
    inits.append(0)
    orders.append(0)
    print(f"case mixed batch dtype={dtype}", flush=True)
    b, states, obs = run_batch(jobs, dtype, inits, orders)
    init_fn = {0: lambda L, M: oracle.init_psi1(L, M), 1: lambda L, M: oracle.init_psi1p(L, M)}
    for j, job in enumerate(jobs):
        Lx, Ly, n = job["Lx"], job["Ly"], 2 * job["Lx"] * job["Ly"]
        if inits[j] in init_fn:
            o0 = init_fn[inits[j]](Lx, Ly)
        elif inits[j] == 2:
            o0 = oracle.state(n)
            o0[0] = 1
        else:
            o0 = np.full(1 << n, 2.0 ** (-n / 2), np.complex128)
        o = oracle_run(Lx, Ly, job["c0"], job["c1"], job["M"], job["T"] / max(job["M"], 1), init=o0,
                       order=orders[j])
        g = to_oracle_order(Lx, Ly, state_of(b, states, j, n, dtype))
        loss = fidelity_loss(o, g)
        oo = oracle_observables(Lx, Ly, o, job["c1"])
        if dtype == z2h.Z2H_C128:
            assert loss < 1e-12, (j, loss)
            compare_observables(row_to_obs(obs[j]), oo, 1e-10, n)
        else:
            assert loss < 1e-5, (j, loss)
            compare_observables(row_to_obs(obs[j]), oo, 1e-5, n)


def test_batch_equals_single_state_bitwise():
    """A job inside a batch runs exactly the kernels of the single-state path."""
    jobs = workloads.scan_3x3(side=3, M=50)
    b, states, obs = run_batch(jobs, z2h.Z2H_C64)
    for j in (0, 4, 8):
        g, ob, _ = gpu_run(3, 3, z2h.Z2H_C64, jobs[j]["c0"], jobs[j]["c1"], 50, jobs[j]["T"] / 50, renorm=1)
        s = state_of(b, states, j, 18, z2h.Z2H_C64)
        assert np.array_equal(s, g)
        assert obs[j][1] == ob["energy"]


@pytest.mark.slow
def test_full_scan_1024_points():
    """Full 32 x 32 scan of the 3x3 torus, complex64, M = 1000: every point's
    energy and Wilson loops against the plain complex128 path (itself
    oracle-checked) within 1e-5, and the four corners against the oracle."""
    jobs = workloads.scan_3x3()
    print("case full scan 1024 x 3x3 c64", flush=True)
    b, states, obs = run_batch(jobs, z2h.Z2H_C64)
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    sz = z2h.z2h_plan_sizes(plan)
    psi = z2h.alloc_state(plan)
    ws = z2h.alloc_bytes(max(sz["ws_evolve"], sz["ws_observe"]))
    from helpers import standard_loops_lib
    zl, xl = standard_loops_lib(3, 3)
    worst = {"energy/n": 0, "zloop0": 0, "zloop1": 0}
    ref = {}
    for j, job in enumerate(jobs):
        z2h.z2h_state_init(plan, psi, z2h.Z2H_INIT_PSI1)
        z2h.z2h_evolve(plan, psi, ws, z2h.schedule(job["c0"], job["c1"], 1000, 0.02))
        r = z2h.z2h_observe(plan, psi, ws, job["c1"], zl, xl)
        ref[j] = r
        worst["energy/n"] = max(worst["energy/n"], abs(r["energy"] - obs[j][1]) / 18)
        worst["zloop0"] = max(worst["zloop0"], abs(r["zloop"][0] - obs[j][6]))
        worst["zloop1"] = max(worst["zloop1"], abs(r["zloop"][1] - obs[j][7]))
    print("worst c64-vs-c128 errors over 1024 points:", worst, flush=True)
    assert all(v <= 1e-5 for v in worst.values()), worst
    for j in (0, 31, 992, 1023):
        job = jobs[j]
        o = oracle_run(3, 3, job["c0"], job["c1"], 1000, 0.02)
        oo = oracle_observables(3, 3, o, job["c1"])
        assert abs(oo["energy"] - ref[j]["energy"]) < 1e-10
        compare_observables(row_to_obs(obs[j]), oo, 1e-5, 18)


@pytest.mark.parametrize("dtype", [z2h.Z2H_C128, z2h.Z2H_C64])
def test_traced_batch_against_oracle(dtype):
    """z2h_batch_run_trace on a mixed batch (2x2, 2x3, 3x3; uneven step
    counts): every sample of every job equals the oracle's observables after
    the same steps (observed with the couplings of the point reached; a job
    that has finished repeats its final state), and the final record equals
    the untraced run's to rounding."""
    rng = np.random.default_rng(11)
    jobs = []
    for (Lx, Ly) in ((3, 3), (2, 2), (2, 3), (3, 3), (2, 3), (2, 2)):
        hx, hz = rng.uniform(0, 0.6, 2)
        M = int(rng.integers(8, 30))
        jobs.append(dict(Lx=Lx, Ly=Ly, c0=workloads.TORIC, c1=(1.0, 1.0, hx, hz), T=0.06 * M, M=M))
    every = 6
    print(f"case traced batch dtype={dtype}", flush=True)
    b, states, obs_plain = run_batch(jobs, dtype)
    ns, wsb = z2h.z2h_batch_trace_sizes(b, every)
    assert ns == -(-max(j["M"] for j in jobs) // every)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    obs = torch.zeros(len(jobs) * z2h.Z2H_OBS_DOUBLES, dtype=torch.float64, device="cuda")
    trace = torch.zeros(ns * len(jobs) * z2h.Z2H_OBS_DOUBLES, dtype=torch.float64, device="cuda")
    for _ in range(2):  # graph recorded, then replayed
        z2h.z2h_batch_run_trace(b, states, ws, obs, every, trace)
    torch.cuda.synchronize()
    tr = trace.cpu().numpy().reshape(ns, len(jobs), -1)
    ob = obs.cpu().numpy().reshape(len(jobs), -1)
    tol = 1e-10 if dtype == z2h.Z2H_C128 else 1e-5
    for j, job in enumerate(jobs):
        n = 2 * job["Lx"] * job["Ly"]
        psi = oracle.init_psi1(job["Lx"], job["Ly"])
        a, c = np.array(job["c0"], float), np.array(job["c1"], float)
        M, dt = job["M"], job["T"] / job["M"]
        done = 0
        for s in range(ns):
            k1 = min((s + 1) * every, M)
            if k1 > done:
                ks = np.arange(done, k1)
                sv = (ks + 0.5) / M
                oracle.evolve(job["Lx"], job["Ly"], psi, tuple(a), tuple(c), k1 - done, dt, sZ=sv, sX=sv)
                done = k1
            ref = oracle_observables(job["Lx"], job["Ly"], psi, tuple(a + (k1 / M) * (c - a)))
            compare_observables(row_to_obs(tr[s, j]), ref, tol, n)
        assert tr[ns - 1, j, 1] == ob[j, 1]
        compare_observables(row_to_obs(ob[j]), row_to_obs(obs_plain[j]), tol, n)


@pytest.mark.parametrize("dtype", [z2h.Z2H_C128, z2h.Z2H_C64])
def test_workspace_reuse_between_runs(dtype):
    """The batch workspace holds only per-run scratch: filling it with other
    bytes between runs (as a caller reusing it, or torch's allocator handing
    it out, would) leaves plain and traced runs bitwise unchanged, also
    after the trace interval changes and returns."""
    rng = np.random.default_rng(23)
    jobs = []
    for (Lx, Ly) in ((3, 3), (2, 3), (2, 2), (3, 3)):
        hx, hz = rng.uniform(0, 0.6, 2)
        M = int(rng.integers(8, 24))
        jobs.append(dict(Lx=Lx, Ly=Ly, c0=workloads.TORIC, c1=(1.0, 1.0, hx, hz), T=0.05 * M, M=M))
    print(f"case workspace reuse dtype={dtype}", flush=True)
    b, states, obs0 = run_batch(jobs, dtype)
    ns5, wsb = z2h.z2h_batch_trace_sizes(b, 5)
    assert wsb == b.ws_bytes
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    obs = torch.zeros(len(jobs) * z2h.Z2H_OBS_DOUBLES, dtype=torch.float64, device="cuda")
    z2h.z2h_batch_run(b, states, ws, obs)
    torch.cuda.synchronize()
    first = obs.cpu().numpy().copy()
    ws.fill_(0xFF)
    obs.zero_()
    z2h.z2h_batch_run(b, states, ws, obs)
    torch.cuda.synchronize()
    assert np.array_equal(obs.cpu().numpy(), first)

    def traced(every):
        ns, _ = z2h.z2h_batch_trace_sizes(b, every)
        tr = torch.zeros(ns * len(jobs) * z2h.Z2H_OBS_DOUBLES, dtype=torch.float64, device="cuda")
        z2h.z2h_batch_run_trace(b, states, ws, obs, every, tr)
        torch.cuda.synchronize()
        return tr.cpu().numpy()

    t5 = traced(5)
    ws.fill_(0xA5)
    assert np.array_equal(traced(5), t5)
    t3 = traced(3)
    ws.fill_(0x00)
    assert np.array_equal(traced(5), t5)
    ws.fill_(0x7F)
    assert np.array_equal(traced(3), t3)


@pytest.mark.parametrize("dtype", [z2h.Z2H_C64, z2h.Z2H_C128])
def test_packed_levels_equal_level_synchronous(dtype):
    """Step counts that differ: jobs packed into slots (run back to back)
    give the observables of the level-synchronous launches bit for bit (same
    kernels per job), for several slot counts and the automatic choice."""
    import os
    rng = np.random.default_rng(41)
    jobs = []
    for k in range(11):
        Lx, Ly = ((3, 3), (2, 3), (3, 4) if dtype == z2h.Z2H_C64 else (3, 3))[k % 3]
        hx, hz = rng.uniform(0, 0.6, 2)
        M = int(rng.integers(3, 30))
        jobs.append(dict(Lx=Lx, Ly=Ly, c0=workloads.TORIC, c1=(1.0, 1.0, hx, hz), T=0.06 * M, M=M))
    outs = []
    try:
        for tv in ("slots=0", "slots=3", "slots=2", "slots=5", "chunk=0"):
            os.environ["Z2H_TUNE"] = tv
            print(f"case packed batch dtype={dtype} {tv}", flush=True)
            outs.append(run_batch(jobs, dtype)[2])
    finally:
        os.environ.pop("Z2H_TUNE", None)
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("dtype", [z2h.Z2H_C64, z2h.Z2H_C128])
def test_precomputed_batch_tables_bitwise(dtype):
    """A cache-resident group (here 12 3x3 states, uneven step counts, packed
    into slots) gets every job's phase tables computed once at batch
    creation; the passes copy them. Same bits as the batch built with
    Z2H_TUNE=tables=0, whose workgroups build their own tables."""
    import os
    rng = np.random.default_rng(77)
    jobs = []
    for k in range(12):
        hx, hz = rng.uniform(0, 0.6, 2)
        M = int(rng.integers(5, 40))
        jobs.append(dict(Lx=3, Ly=3, c0=workloads.TORIC, c1=(1.0, 1.0, hx, hz), T=0.05 * M, M=M))
    outs = []
    try:
        for tv in ("tables=0", ""):
            os.environ["Z2H_TUNE"] = tv
            print(f"case batch tables dtype={dtype} '{tv}'", flush=True)
            b, states, o = run_batch(jobs, dtype)
            outs.append((states.cpu().numpy(), o))
    finally:
        os.environ.pop("Z2H_TUNE", None)
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
