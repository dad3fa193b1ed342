"""Serving on the GPU: requests on two resident lattices with continuous
batching; every result equals (bitwise) the same request solved alone, and
meets the 1e-10 true residual by the oracle's operator."""
import numpy as np
import pytest

import lattice_inputs as li
from gpu_util import dev, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wd():
    from paper_1207_2223_amd import wd
    wd.lib()
    return wd


def _requests(lattices, n, seed):
    from paper_1207_2223_amd.serve import Request
    rng = np.random.default_rng(seed)
    reqs = []
    names = list(lattices)
    for i in range(n):
        name = names[i % len(names)]
        Vh = li.volume(lattices[name]["dims"]) // 2
        nrhs = int(rng.integers(1, 4))
        phi = li.gaussian_spinor(Vh, seed=seed * 100 + i, nrhs=nrhs)
        reqs.append(Request(rid=i, lattice=name, phi=phi, kappa=list(rng.uniform(0.14, 0.157, nrhs)),
                            arrival=0.002 * i))
    return reqs


def _solve_alone(wd, spec, params, req, k):
    from paper_1207_2223_amd.serve import SLOT_DONE, GpuExecutor
    ex = GpuExecutor(spec["dims"], spec["U"], params, max_slots=req.nrhs)
    try:
        slots = ex.add(req)
        req.slots = slots
        for _ in range(10000):
            ex.step(k)
            states, stats = ex.poll()
            if all(states[s] == SLOT_DONE for s in slots):
                break
        return ex.take(req), [stats[s] for s in slots]
    finally:
        ex.close()


def test_results_same_alone_and_in_the_mix(wd, oracle):
    import torch
    from paper_1207_2223_amd.serve import Admission, GpuExecutor, Server
    lattices = {"a": {"dims": (8, 8, 8, 8), "U": li.random_su3_field((8, 8, 8, 8), 0.5, seed=1003)},
                "b": {"dims": (6, 4, 4, 6), "U": li.random_su3_field((6, 4, 4, 6), 0.5, seed=1004)}}
    params = wd.solver_params(prec=wd.WD_F16, tol=1e-10, maxiter=5000)
    k = 8
    ex = {n: GpuExecutor(s["dims"], s["U"], params, max_slots=6) for n, s in lattices.items()}
    free = lambda: torch.cuda.mem_get_info()[0]
    srv = Server(ex, Admission(8 << 30, free_fn=free), k_iters=k)
    reqs = _requests(lattices, 10, seed=7)
    summ = srv.run(reqs)
    for e in ex.values():
        e.close()
    note(f"serving summary: {summ}")
    assert summ["completed"] == len(reqs)
    assert max(summ["max_batch"].values()) > 1
    for r in reqs:
        assert all(s["status"] == wd.WD_OK for s in r.stats)
        x_alone, st_alone = _solve_alone(wd, lattices[r.lattice], params, r, k)
        assert [s["iters"] for s in st_alone] == [s["iters"] for s in r.stats]
        assert np.array_equal(x_alone, r.x), r.rid
        dims, U = lattices[r.lattice]["dims"], lattices[r.lattice]["U"]
        for j in range(r.nrhs):
            res = r.phi[j] - oracle.mhatdag_mhat(dims, U, r.kappa[j], r.x[j])
            assert np.linalg.norm(res) / np.linalg.norm(r.phi[j]) <= 1.01e-10


def test_session_errors(wd):
    import torch
    dims = (4, 4, 4, 4)
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(li.random_su3_field(dims, 0.5, seed=9)))
    s = wd.wd_session_create(lat.ctx, 2, wd.solver_params(prec=wd.WD_F32))
    phi = dev(li.gaussian_spinor(128, seed=1, nrhs=3))
    with pytest.raises(wd.WDError) as e:
        wd.wd_session_add(s, phi, [0.15] * 3)
    assert e.value.status == wd.WD_ERR_OOM
    slots = wd.wd_session_add(s, phi[:2].contiguous(), [0.15, 0.15])
    x = torch.empty((128, 4, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(wd.WDError) as e:
        wd.wd_session_take(s, slots[0], x)
    assert e.value.status == wd.WD_ERR_STATE
    for _ in range(200):
        wd.wd_session_step(s, 8)
        states, stats = wd.wd_session_poll(s, 2)
        if all(v == 2 for v in states):
            break
    wd.wd_session_take(s, slots[0], x)
    states, _ = wd.wd_session_poll(s, 2)
    assert states[slots[0]] == 0 and states[slots[1]] == 2
    # the context refuses to go while a session on it is open, and the
    # session still works afterwards
    with pytest.raises(wd.WDError) as e:
        wd.wd_destroy(lat.ctx)
    assert e.value.status == wd.WD_ERR_STATE
    wd.wd_session_take(s, slots[1], x)
    wd.wd_session_destroy(s)
    lat.close()


def test_resize_keeps_running_slots_bitwise(wd):
    """A session grown while a slot runs, and shrunk while another runs,
    gives bitwise the results of a session that never changed size."""
    import torch
    dims = (6, 4, 4, 6)
    Vh = li.volume(dims) // 2
    lat = wd.Lattice(dims)
    lat.gauge_load(dev(li.random_su3_field(dims, 0.5, seed=1004)), recon=12)
    params = wd.solver_params(prec=wd.WD_F16, tol=1e-10, maxiter=4000)
    phi = dev(li.gaussian_spinor(Vh, seed=11, nrhs=2))
    kap = [0.150, 0.153]

    def run_to_done(s, slots):
        for _ in range(1000):
            wd.wd_session_step(s, 8)
            states, stats = wd.wd_session_poll(s)
            if all(states[q] == 2 for q in slots):
                return stats
        raise AssertionError("session did not finish")

    ref = wd.wd_session_create(lat.ctx, 2, params)
    slots = wd.wd_session_add(ref, phi, kap)
    st_ref = run_to_done(ref, slots)
    x_ref = torch.empty_like(phi)
    for j, q in enumerate(slots):
        wd.wd_session_take(ref, q, x_ref[j])
    wd.wd_session_destroy(ref)

    s = wd.wd_session_create(lat.ctx, 1, params)
    (q0,) = wd.wd_session_add(s, phi[:1].contiguous(), kap[:1])
    for _ in range(3):
        wd.wd_session_step(s, 8)
    wd.wd_session_resize(s, 4)
    assert wd.wd_session_capacity(s) == 4
    (q1,) = wd.wd_session_add(s, phi[1:].contiguous(), kap[1:])
    assert (q0, q1) == (0, 1)
    x = torch.empty_like(phi)
    stats = run_to_done(s, [q0])
    wd.wd_session_take(s, q0, x[0])
    states, _ = wd.wd_session_poll(s)
    if states[q1] == 1:
        with pytest.raises(wd.WDError) as e:
            wd.wd_session_resize(s, 1)
        assert e.value.status == wd.WD_ERR_STATE
    wd.wd_session_resize(s, 2)
    stats2 = run_to_done(s, [q1])
    wd.wd_session_take(s, q1, x[1])
    wd.wd_session_resize(s, 1)
    assert wd.wd_session_capacity(s) == 1
    wd.wd_session_destroy(s)
    torch.cuda.synchronize()
    note(f"resize: iters {stats[q0]['iters']}, {stats2[q1]['iters']} vs {st_ref[0]['iters']}, {st_ref[1]['iters']}")
    assert stats[q0]["iters"] == st_ref[slots[0]]["iters"] and stats2[q1]["iters"] == st_ref[slots[1]]["iters"]
    assert torch.equal(x, x_ref)
    lat.close()
