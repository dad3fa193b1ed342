"""GPU parity of the MD force and the HMC trajectory (Sec. 2 eq. 5; Sec. 3
kernels 2-4 and the three steps of a trajectory) against the oracle on the
same Philox draws."""
import numpy as np
import pytest

import lattice_inputs as li
from gpu_util import dev, host, note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wd():
    from paper_1207_2223_amd import wd
    wd.lib()
    return wd


def test_draws_match_oracle(wd, oracle):
    import torch
    dims = (4, 4, 2, 6)
    V = li.volume(dims)
    lat = wd.Lattice(dims)
    P = torch.empty((V, 4, 3, 3), dtype=torch.complex128, device="cuda")
    chi = torch.empty((V // 2, 4, 3), dtype=torch.complex128, device="cuda")
    for seed, traj in [(77, 3), (2 ** 40 + 5, 0)]:
        wd.wd_hmc_draw(lat.ctx, P, chi, seed, traj)
        Po = oracle.draw_momenta(dims, seed, traj)
        co = oracle.draw_chi(V // 2, seed, traj)
        assert np.allclose(host(P), Po, rtol=0, atol=1e-13)
        assert np.allclose(host(chi), co, rtol=0, atol=1e-13)
    lat.close()


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 4, 6)])
def test_md_force_matches_oracle(wd, oracle, dims):
    import torch
    V = li.volume(dims)
    U = li.random_su3_field(dims, 0.5, seed=5)
    phi = li.gaussian_spinor(V // 2, seed=6)
    kappa, beta = 0.15, 5.6
    lat = wd.Lattice(dims)
    F = torch.empty((V, 4, 3, 3), dtype=torch.complex128, device="cuda")
    it = wd.wd_md_force(lat.ctx, F, dev(U), dev(phi), kappa, beta, wd.solver_params(tol=1e-13))
    Fo, ito = oracle.md_force(dims, U, beta, kappa, phi, eo=True, tol=1e-13)
    Fg = host(F)
    err = np.abs(Fg - Fo).max() / np.abs(Fo).max()
    note(f"force {dims}: {it} iters, max rel err {err:.2e}")
    assert err <= 1e-9
    lat.close()


def test_trajectory_matches_oracle(wd, oracle):
    dims = (4, 4, 4, 4)
    U0 = li.random_su3_field(dims, 0.5, seed=50)
    beta, kappa, tau, n = 5.6, 0.12, 0.5, 10
    tight = wd.solver_params(tol=1e-13)
    lat = wd.Lattice(dims)
    Ud = dev(U0)
    hp = wd.hmc_params(beta, kappa, tau, n, seed=51, traj=0, force=tight, h=tight)
    r = wd.hmc_trajectory(lat.ctx, Ud, hp)
    Uo, ro = oracle.hmc_trajectory(dims, U0, beta, kappa, tau, n, seed=51, traj=0, eo=True,
                                   tol_force=1e-13, tol_h=1e-13)
    note(f"gpu dH {r['dH']:.10f} oracle {ro['dH']:.10f}; accepted {r['accepted']} / {ro['accepted']}")
    assert r["status"] == wd.WD_OK
    assert abs(r["H_old"] - ro["H_old"]) <= 1e-9 * abs(ro["H_old"])
    assert abs(r["dH"] - ro["dH"]) <= 1e-6
    assert r["u"] == ro["u"]
    assert bool(r["accepted"]) == ro["accepted"]
    assert np.abs(host(Ud) - Uo).max() <= 1e-10
    assert abs(r["plaquette"] - ro["plaquette"]) <= 1e-12
    lat.close()


def test_mixed_precision_force_solver(wd, oracle):
    dims = (4, 4, 4, 4)
    U0 = li.random_su3_field(dims, 0.5, seed=60)
    lat = wd.Lattice(dims)
    Ud = dev(U0)
    hp = wd.hmc_params(5.6, 0.12, 0.5, 10, seed=61, traj=2,
                       force=wd.solver_params(tol=1e-9, prec=wd.WD_F16),
                       h=wd.solver_params(tol=1e-12))
    r = wd.hmc_trajectory(lat.ctx, Ud, hp)
    _, ro = oracle.hmc_trajectory(dims, U0, 5.6, 0.12, 0.5, 10, seed=61, traj=2, eo=True,
                                  tol_force=1e-12, tol_h=1e-12)
    note(f"mixed-force dH {r['dH']:.8f} vs oracle {ro['dH']:.8f}")
    assert r["status"] == wd.WD_OK
    assert abs(r["dH"] - ro["dH"]) <= 1e-4 * max(1.0, abs(ro["dH"]))
    lat.close()


def test_reject_leaves_field_and_context_unchanged(wd):
    import torch
    dims = (4, 4, 4, 4)
    V = li.volume(dims)
    U0 = li.random_su3_field(dims, 0.5, seed=70)
    lat = wd.Lattice(dims)
    Ud = dev(U0)
    hp = wd.hmc_params(5.6, 0.12, 6.0, 2, seed=71, traj=0,
                       force=wd.solver_params(tol=1e-10), h=wd.solver_params(tol=1e-10))
    r = wd.hmc_trajectory(lat.ctx, Ud, hp)
    assert not r["accepted"]
    assert np.array_equal(host(Ud), U0)
    # the context's packed links still hold U0
    psi = li.gaussian_spinor(V // 2, seed=72)
    out = torch.empty((V // 2, 4, 3), dtype=torch.complex128, device="cuda")
    lat.dslash(out, dev(psi), wd.WD_EVEN, 0, wd.WD_F64)
    lat2 = wd.Lattice(dims)
    lat2.gauge_load(dev(U0))
    out2 = torch.empty_like(out)
    lat2.dslash(out2, dev(psi), wd.WD_EVEN, 0, wd.WD_F64)
    assert torch.equal(out, out2)
    lat.close()
    lat2.close()


def test_md_trajectory_without_metropolis_takes_the_proposal(wd, oracle):
    """metropolis = 0 accepts the leapfrog proposal whatever dH is: with
    three steps for tau = 1 the oracle's dH is about 175 (a certain
    rejection under the test), and the field returned is the oracle's leapfrog
    result from the same Philox draws."""
    dims = (4, 4, 4, 4)
    V = li.volume(dims)
    U0 = li.random_su3_field(dims, 0.5, seed=70)
    beta, kappa, tau, n, seed, traj = 5.6, 0.12, 1.0, 3, 71, 0
    tight = wd.solver_params(tol=1e-13)
    lat = wd.Lattice(dims)
    Ud = dev(U0)
    hp = wd.hmc_params(beta, kappa, tau, n, seed=seed, traj=traj, force=tight, h=tight, metropolis=False)
    r = wd.hmc_trajectory(lat.ctx, Ud, hp)
    assert r["status"] == wd.WD_OK and r["accepted"] == 1
    assert r["dH"] > 100
    P = oracle.draw_momenta(dims, seed, traj)
    chi = oracle.draw_chi(V // 2, seed, traj)
    phi = oracle.mhat(dims, U0, kappa, chi, dagger=True)
    Uo, _, _ = oracle.leapfrog(dims, U0, P, beta, kappa, phi, tau, n, eo=True, tol=1e-13)
    err = np.abs(host(Ud) - Uo).max()
    note(f"MD trajectory dH {r['dH']:.3f}, accepted {r['accepted']}, |U - U_oracle| {err:.2e}")
    assert err <= 1e-9
    assert abs(r["plaquette"] - oracle.plaquette(dims, Uo)) <= 1e-11
    lat.close()


def test_chronological_force_solves(wd, oracle):
    """chrono = 1 (each force solve starts from the previous step's solution)
    and 2 (linear extrapolation of the last two): fewer CG iterations per
    trajectory, and with tight force solves the same dH and field as the
    oracle's trajectory (x0 = 0) to solver tolerance."""
    dims = (4, 4, 4, 4)
    U0 = li.random_su3_field(dims, 0.5, seed=50)
    beta, kappa, tau, n = 5.6, 0.12, 0.5, 10
    tight = wd.solver_params(tol=1e-13)
    res = {}
    for chrono in (0, 1, 2):
        lat = wd.Lattice(dims)
        Ud = dev(U0)
        hp = wd.hmc_params(beta, kappa, tau, n, seed=51, traj=0, force=tight, h=tight, chrono=chrono)
        res[chrono] = (wd.hmc_trajectory(lat.ctx, Ud, hp), host(Ud))
        lat.close()
    _, ro = oracle.hmc_trajectory(dims, U0, beta, kappa, tau, n, seed=51, traj=0, eo=True,
                                  tol_force=1e-13, tol_h=1e-13)
    r0 = res[0][0]
    note(f"chrono: cg iters {r0['cg_iters']} -> {res[1][0]['cg_iters']} (previous) / {res[2][0]['cg_iters']} "
         f"(extrapolated), dH {r0['dH']:.10f} / {res[1][0]['dH']:.10f} / {res[2][0]['dH']:.10f} "
         f"(oracle {ro['dH']:.10f})")
    for ch in (1, 2):
        r1 = res[ch][0]
        assert r1["status"] == wd.WD_OK and r1["cg_iters"] < r0["cg_iters"]
        assert abs(r1["dH"] - ro["dH"]) <= 1e-6
        assert bool(r1["accepted"]) == ro["accepted"]
        assert np.abs(res[ch][1] - res[0][1]).max() <= 1e-10


@pytest.mark.parametrize("prec,chrono", [("F64", 0), ("F16", 1)])
def test_exp_minus_dh_averages_to_one(wd, prec, chrono):
    """Area preservation and reversibility of the GPU trajectory (the
    Metropolis step is exact only if both hold): <exp(-dH)> = 1 within three
    standard errors over 190 trajectories of a 4^4 chain, with FP64 force
    solves from zero and with FP16 mixed-precision force solves started
    from the previous solution (the production settings)."""
    dims = (4, 4, 4, 4)
    U = dev(li.random_su3_field(dims, 0.5, seed=70))
    lat = wd.Lattice(dims)
    code = {"F64": wd.WD_F64, "F16": wd.WD_F16}[prec]
    vals, acc = [], 0
    for traj in range(200):
        hp = wd.hmc_params(5.6, 0.12, 0.5, 20, seed=73, traj=traj,
                           force=wd.solver_params(tol=1e-10, prec=code),
                           h=wd.solver_params(tol=1e-12), chrono=chrono)
        r = wd.hmc_trajectory(lat.ctx, U, hp)
        assert r["status"] == wd.WD_OK
        if traj >= 10:
            vals.append(np.exp(-r["dH"]))
            acc += int(r["accepted"])
    vals = np.array(vals)
    m, se = vals.mean(), vals.std(ddof=1) / np.sqrt(len(vals))
    note(f"{prec} chrono {chrono}: <exp(-dH)> = {m:.4f} +- {se:.4f}, acceptance {acc / len(vals):.2f}")
    assert abs(m - 1) < max(3 * se, 0.02), (m, se)
    lat.close()
