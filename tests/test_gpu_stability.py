"""Numerical stability at low viscosity (Sec. 4.1, Fig. VisCompare): the comparison the paper
uses to show that the modified model is more stable than a lattice-BGK model whose
relaxation times set the viscosity and the diffusivity.

The paper compares its model at tau_f = 1 with an earlier LBGK scheme at tau_f = 0.5009
in the mixed-convection channel of Sec. 4.1 (32 x 32 lattice, Re = 5, Ra = 100, Pr = 1,
eps = 0.6, Da = 0.01) at nu = 9.375e-6 and 9.375e-7 (delta_x = delta_t = 1/32, i.e.
lattice viscosities 3e-4 and 3e-5), and reports that the LBGK scheme becomes unstable by
t = 46000 while the modified model stays stable and agrees with the closed form.  The
earlier scheme is not part of this library; its stand-in is the same kernel with A = B = 0,
which is a BGK model whose relaxation times alone set nu_e and alpha_e
(tau = 1/2 + 3 nu).  Re = 5 with the stated viscosity fixes the injection speed
v0 = Re nu / H (the paper's v0 = 0.01 of its accuracy study would give Re of about 1e3
here; it is run as a third pair).  The channel is uniform in x, so a two-dimensional
disturbance is seeded: the closed-form state plus small random velocity and temperature
noise.  Both forms run in one FP64 batch; the non-finite detector is read every 1000
steps."""
import numpy as np
import pytest

from closed_forms import E, mixed_convection_cfg
import workloads as W  # noqa: F401  (the seeded inputs live with the closed forms)

pytestmark = pytest.mark.gpu

CHECK_EVERY = 1000
PAPER_T = 46000


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1505_02976_amd import lbm
    lbm.lib()
    return lbm


def _channel(nu, model, seed, Re=5.0, nx=32, ny=33):
    """The Sec. 4.1 channel at lattice viscosity nu (Pr = 1, so alpha_e = nu), either the
    modified model at tau = 1 (A = B = 1/2 - 3 nu) or its BGK form A = B = 0 at
    tau = 1/2 + 3 nu; the closed-form state plus a seeded disturbance."""
    if model == "bgk":
        tau, A = 0.5 + 3 * nu, 0.0
    else:
        tau, A = 1.0, 0.5 - 3 * nu
    cfg, _, exact = mixed_convection_cfg(ny, tau, Re=Re, A=A)
    ua, Ta, _, _, v0 = exact
    rng = np.random.default_rng(seed)
    cfg["nx"] = nx
    T = np.repeat(Ta[:, None], nx, axis=1)
    T[1:-1] += 1e-4 * rng.uniform(-1, 1, size=(ny - 2, nx))
    cfg["T_init"] = T
    cfg["ux_init"] = np.repeat(ua[:, None], nx, axis=1) + 1e-2 * v0 * rng.uniform(-1, 1, size=(ny, nx))
    cfg["uy_init"] = v0 + 1e-2 * v0 * rng.uniform(-1, 1, size=(ny, nx))
    cfg["storage"] = "f64"
    return cfg, exact


def _spread(f, v0):
    """Largest departure along x from the row mean: of u_x (in units of v0) and of T."""
    su = float(np.abs(f["ux"] - f["ux"].mean(axis=1, keepdims=True)).max()) / v0
    sT = float(np.abs(f["T"] - f["T"].mean(axis=1, keepdims=True)).max())
    return su, sT


def test_modified_model_stable_where_bgk_form_diverges(gpu):
    cases = []
    for nu, Re in ((3e-4, 5.0), (3e-5, 5.0), (3e-4, 32 * 0.01 / 3e-4)):
        for model in ("bgk", "modified"):
            cfg, exact = _channel(nu, model, seed=1, Re=Re)
            cases.append((nu, Re, model, cfg, exact))
    _say("case: Sec. 4.1 channel 32 x 33, FP64 batch of " + ", ".join(
        f"nu {nu:g} Re {Re:.3g} {m} (tau_f {c['tau_f']:.5f})" for nu, Re, m, c, _ in cases))
    batch = gpu.Batch([c for *_, c, _ in cases])
    first_nonfinite = [None] * len(cases)
    spread46 = {}
    end = 200000
    for s in range(CHECK_EVERY, end + CHECK_EVERY, CHECK_EVERY):
        batch.step(CHECK_EVERY)
        for k, flag in enumerate(batch.check()):
            if flag and first_nonfinite[k] is None:
                first_nonfinite[k] = s
        if s == PAPER_T:
            for k, (nu, Re, model, cfg, exact) in enumerate(cases):
                if model == "modified" and first_nonfinite[k] is None:
                    spread46[k] = _spread({q: v.cpu().numpy() for q, v in batch[k].fields().items()}, exact[4])
    for (nu, Re, model, cfg, exact), t in zip(cases, first_nonfinite):
        _say(f"  nu {nu:g} Re {Re:.3g} {model}: " + ("finite through step %d" % end if t is None
                                                     else f"non-finite by step {t}"))
    for k, ((nu, Re, model, cfg, exact), t) in enumerate(zip(cases, first_nonfinite)):
        if model == "bgk":
            # the paper's LBGK becomes unstable by t = 46000
            assert t is not None and t <= PAPER_T, (nu, Re, t)
            continue
        assert t is None, (nu, Re, t)
        f = {q: v.cpu().numpy() for q, v in batch[k].fields().items()}
        ua, Ta, _, _, v0 = exact
        su, sT = _spread(f, v0)
        su46, sT46 = spread46[k]
        eu, eT = E(ua, f["ux"].mean(axis=1)), E(Ta, f["T"].mean(axis=1))
        _say(f"  nu {nu:g} Re {Re:.3g} modified: disturbance along x {su46:.1e} v0 / {sT46:.1e} at step "
             f"{PAPER_T}, {su:.1e} v0 / {sT:.1e} at step {end}; E(u_x) {eu:.2e}, E(T) {eT:.2e} "
             f"against the closed form")
        if Re < 10:
            # the seeded disturbance decays, and the profiles stay near the closed form (at this
            # tau - A - 1/2 of 1e-3 or 1e-4 the model's error is a few percent, and the diffusive
            # time H^2 / nu is 3.4e6 steps or more); at Re of about 1e3 the 33-node channel does
            # not resolve the closed form's boundary layers, and only stability is asserted
            assert su < su46 and sT < sT46, (nu, Re)
            assert eu < 5e-2 and eT < 1e-2, (nu, Re, eu, eT)
