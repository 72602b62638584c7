"""Mutation check of the oracle's pins (CPU only).

Each entry below plants one plausible mistake (a flipped sign, a swapped
index, a dropped factor or term, a wrong operator) in a copy of the oracle
written to a temporary directory; the pin suite then runs against that copy in
a subprocess and must fail.  An unmodified copy must pass, so that a broken
harness cannot pass for a caught mistake.  The repository's oracle file is
never modified."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "afc_oracle.py")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")

MUTATIONS = {
    "unmodified": None,
    # SSP fluxes of eq. (20): sign of the diffusive part
    "ssp_flux_d_sign": ("r = P.m_ij * (udot[i] - udot[j]) + d * (u[j] - u[i])  # eq. (20)",
                        "r = P.m_ij * (udot[i] - udot[j]) - d * (u[j] - u[i])  # eq. (20)"),
    # Zalesak step 4: R+ paired with R- of the other node
    "zalesak_alpha_index": ("alpha = np.where(r > 0.0, np.minimum(Rp[i], Rm[j]), np.minimum(Rm[i], Rp[j]))",
                            "alpha = np.where(r > 0.0, np.minimum(Rp[i], Rp[j]), np.minimum(Rm[i], Rm[j]))"),
    # Zalesak step 3 without the lumped mass
    "zalesak_R_no_mass": ("Rp[nzp] = np.minimum(1.0, P.m[nzp] * Qp[nzp] / (dt * Pp[nzp]))",
                          "Rp[nzp] = np.minimum(1.0, Qp[nzp] / (dt * Pp[nzp]))"),
    # Zalesak step 2 over N_i including i, shifted
    "zalesak_Q_self": ("Qp = np.maximum(0.0, P.row_max(np.where(P.offd, diff, -np.inf)))",
                       "Qp = np.maximum(0.0, P.row_max(diff)) + 0.01"),
    # CN fluxes of eq. (12): mass term transposed
    "cn_flux_mass_sign": ("r = P.m_ij / dt * (du[i] - du[j]) + 0.5 * d * (su[j] - su[i])",
                          "r = P.m_ij / dt * (du[j] - du[i]) + 0.5 * d * (su[j] - su[i])"),
    # CN predictor of eq. (14): a full step instead of a half step
    "cn_predictor_full_step": ("ut = u_old - 0.5 * dt * (P.matvec(AL, u_old) - F_old) / P.m",
                               "ut = u_old - dt * (P.matvec(AL, u_old) - F_old) / P.m"),
    # eq. (5): diagonal of D with the wrong sign
    "diffusion_diagonal_sign": ("d[P.diag_pos] = -P.row_sum(d)", "d[P.diag_pos] = P.row_sum(d)"),
    # MCL bar state of eq. (22): sign of the convective part
    "mcl_bar_state_sign": ("S_ij = d * (u[i] + u[j]) + c * (u[j] - u[i])  # 2 d_ij ubar_ij",
                           "S_ij = d * (u[i] + u[j]) - c * (u[j] - u[i])  # 2 d_ij ubar_ij"),
    # MCL bound of the neighbour taken at node i
    "mcl_bound_index": ("two_d * umin[j] - S_ji", "two_d * umin[i] - S_ji"),
    # GMRES update without the right preconditioner
    "gmres_no_preconditioner": ("x = x + dinv * (V[:k_used].T @ y)", "x = x + (V[:k_used].T @ y)"),
    # linear Zal+CN: fluxes at the predictor instead of 2 u~ - u^{n-1}
    "linear_cn_extrapolation": ("u_star = 2.0 * ut - u_old", "u_star = ut"),
    # MU ownership (Sec. 3.2, steps 1 and 4) reversed
    "mu_edge_owner": ("owns = P.offd & (aT <= a)", "owns = P.offd & (aT >= a)"),
    # MU ties (a_ji = a_ij): the larger of the two nodes' factors
    "mu_tie_larger_factor": ("np.where(aT > a, abarT, np.minimum(abar, abarT))",
                             "np.where(aT > a, abarT, np.maximum(abar, abarT))"),
    # MU step 2: Q from the fluxes of the other sign
    "mu_Q_sign": ("    Qp = -P.row_sum(rm)\n    Qm = -P.row_sum(rp)", "    Qp = P.row_sum(rp)\n    Qm = P.row_sum(rm)"),
    # MCL bar state of the reverse edge with c_ij instead of c_ji
    "mcl_reverse_bar_state": ("S_ji = d * (u[i] + u[j]) + c[P.tpos] * (u[i] - u[j])",
                              "S_ji = d * (u[i] + u[j]) + c * (u[i] - u[j])"),
    # MC schemes: D from the full A instead of the convective part (Remark 1)
    "mc_diffusion_operator": ("    d = artificial_diffusion(P, P.c)\n    return d, low_order_operator(P, P.a, d)",
                              "    d = artificial_diffusion(P, P.a)\n    return d, low_order_operator(P, P.a, d)"),
    # MC fluxes of eq. (20): mass term transposed
    "mc_flux_mass_sign": ("P.m_ij * (udot[i] - udot[j]) + d * (u[j] - u[i]), 0.0)",
                          "P.m_ij * (udot[j] - udot[i]) + d * (u[j] - u[i]), 0.0)"),
    # MC+CN: the old level's correction without its factor 1/2
    "mc_cn_old_half": ("        + 0.5 * mc_correction(P, u_old, udot_old, d, alpha_mode)",
                       "        + mc_correction(P, u_old, udot_old, d, alpha_mode)"),
    # Shu-Osher SSP-RK3: second-stage weights swapped
    "rk3_stage2_weights": ("u2 = 0.75 * u + 0.25 * fe_ssp_stage(P, u1, F, dt, alpha_mode)",
                           "u2 = 0.25 * u + 0.75 * fe_ssp_stage(P, u1, F, dt, alpha_mode)"),
    # Shu-Osher SSP-RK3: final weights swapped
    "rk3_final_weights": ("return (1.0 / 3.0) * u + (2.0 / 3.0) * fe_ssp_stage(P, u2, F, dt, alpha_mode)",
                          "return (2.0 / 3.0) * u + (1.0 / 3.0) * fe_ssp_stage(P, u2, F, dt, alpha_mode)"),
    # Heun's form of Sec. 2.1.2: not the plain average of u^{n,0} and u^{n,2}
    "heun_average_weights": ("return 0.5 * (u + u2)", "return 0.4 * u + 0.6 * u2"),
    # MC SSP-RK3: second-stage weights swapped
    "mc_rk3_stage2_weights": ("u2 = 0.75 * u + 0.25 * mc_ssp_stage(P, u1, F, dt, alpha_mode)",
                              "u2 = 0.25 * u + 0.75 * mc_ssp_stage(P, u1, F, dt, alpha_mode)"),
    # dynamic damping: a different floor
    "damping_floor": ("return max(omega * 0.5, 1.0 / 64.0)", "return max(omega * 0.5, 1.0 / 32.0)"),
    # dynamic damping: a different growth factor
    "damping_growth": ("return min(1.0, omega * 1.25)", "return min(1.0, omega * 1.5)"),
    # dynamic damping: growth when the residual grew
    "damping_direction": ("    if R > R_prev:\n        return max(", "    if R < R_prev:\n        return max("),
    # relaxation applied to the wrong iterate
    "relaxation_form": ("return u + omega * (w - u)", "return w + omega * (w - u)"),
}


def _run(tmp, src, name, change):
    d = os.path.join(tmp, name, "oracle")
    os.makedirs(d)
    with open(os.path.join(d, "__init__.py"), "w"):
        pass
    text = src
    if change is not None:
        old, new = change
        assert src.count(old) == 1, name
        text = src.replace(old, new)
    with open(os.path.join(d, "afc_oracle.py"), "w") as f:
        f.write(text)
    env = dict(os.environ, PYTHONPATH=os.pathsep.join([os.path.join(tmp, name), ROOT]))
    probe = subprocess.run([sys.executable, "-c", "import oracle.afc_oracle as m; print(m.__file__)"],
                           capture_output=True, text=True, env=env, cwd=tmp)
    assert probe.stdout.strip().startswith(os.path.join(tmp, name)), (name, probe.stdout, probe.stderr)
    p = subprocess.run([sys.executable, "-m", "pytest", PINS, "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"],
                       capture_output=True, text=True, env=env, cwd=tmp)
    return name, p.returncode, (p.stdout.strip().splitlines() or [""])[-1]


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin(tmp_path):
    with open(SRC) as f:
        src = f.read()
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda kv: _run(str(tmp_path), src, kv[0], kv[1]), MUTATIONS.items()))
    for name, rc, last in results:
        print("%-28s rc=%d  %s" % (name, rc, last))
    by = {name: rc for name, rc, _ in results}
    assert by.pop("unmodified") == 0
    missed = [name for name, rc in by.items() if rc == 0]
    assert not missed, missed
