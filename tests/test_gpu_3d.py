"""The 3-D (D3Q19) HIP path through the C interface against the 3-D oracle: populations and
every field of seeded random problems (walled and periodic z, walls in x and in y with and
without z walls, closed boxes, isothermal and prescribed-gradient walls, moving walls, porosity fields, ragged
sizes, the smallest walled nx and nz), FP64 within
1e-10 and FP32 within 1e-5 relative L2, the exact conduction fixed point, a larger
layer heated from below, the porous cavity's wall Nusselt numbers."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def gpu3():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1505_02976_amd import lbm3d
    lbm3d.lib()
    return lbm3d


def _perm(gpu3):
    """Index of each library population in the oracle's lattice order."""
    import oracle.oracle3 as O3
    c_o, _ = O3.lattice()
    order = [tuple(int(v) for v in c) for c in c_o]
    return [order.index(c) for c in gpu3.lattice()]


def _compare(gpu3, cfg, steps, tol_pop, tol_field):
    import oracle.oracle3 as O3
    sim = gpu3.Sim3(cfg)
    sim.step(steps)
    ref = O3.Oracle3(cfg)
    ref.step(steps)
    perm = _perm(gpu3)
    f, g = [t.cpu().numpy() for t in sim.populations()]
    fo, go = ref.populations()
    dpop = max(np.abs(f - fo[perm]).max(), np.abs(g - go[perm]).max())
    a = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    b = ref.fields()
    dfield = {k: float(np.abs(a[k] - b[k]).max()) for k in b}
    return dpop, dfield, a, b


CASES = [
    # (seed, nx, ny, nz, periodic_z, porosity field)
    (1, 20, 12, 9, 0, False),
    (2, 17, 5, 4, 0, False),       # smallest walled nz, ragged x
    (3, 9, 14, 11, 1, False),      # periodic z
    (4, 33, 3, 7, 0, False),
    (5, 16, 9, 8, 0, True),        # porosity field, walls
    (6, 11, 7, 10, 1, True),       # porosity field, periodic z
]


@pytest.mark.parametrize("seed,nx,ny,nz,pz,ef", CASES)
def test_fp64_parity(gpu3, seed, nx, ny, nz, pz, ef):
    cfg = W.random_case3d(seed, nx, ny, nz, periodic_z=pz, eps_field=ef)
    _say(f"case: 3-D FP64 seed {seed} {nx}x{ny}x{nz} periodic_z {pz} porosity field {ef}, walls "
         f"{[w['kind'] for w in cfg['walls']]}, 200 steps")
    dpop, dfield, _, _ = _compare(gpu3, cfg, 200, 1e-10, 1e-10)
    _say(f"  max |populations| diff {dpop:.2e}; fields {max(dfield.values()):.2e}")
    assert dpop < 1e-10
    assert all(v < 1e-10 for v in dfield.values()), dfield


@pytest.mark.parametrize("seed", [1, 3, 5])
def test_fp32_parity(gpu3, seed):
    cfg = W.random_case3d(seed, 20, 12, 9, periodic_z=1 if seed == 3 else 0, storage="f32", eps_field=seed == 5)
    _say(f"case: 3-D FP32 seed {seed}, 200 steps")
    _, _, a, b = _compare(gpu3, cfg, 200, None, None)
    # the velocity as one vector field (between walls u_z is small, and its own relative
    # error says little), and the temperature
    du = np.sqrt(sum(np.linalg.norm(a[k] - b[k]) ** 2 for k in ("ux", "uy", "uz")))
    nu = np.sqrt(sum(np.linalg.norm(b[k]) ** 2 for k in ("ux", "uy", "uz")))
    rel = {"u": du / nu, "T": np.linalg.norm(a["T"] - b["T"]) / np.linalg.norm(b["T"])}
    _say(f"  rel L2: u {rel['u']:.2e}, T {rel['T']:.2e}")
    assert rel["u"] < 1e-5 and rel["T"] < 1e-5, rel


@pytest.mark.parametrize("kind", ["dirichlet", "neumann"])
def test_conduction_fixed_point(gpu3, kind):
    nz = 24
    slope = 0.8 / (nz - 1)
    z = np.arange(nz, dtype=float)
    walls = [{"kind": "T", "T": 0.1}, {"kind": "T", "T": 0.9}]
    if kind == "neumann":
        walls[0] = {"kind": "dTdn", "dTdn": slope}
    cfg = {"nx": 4, "ny": 3, "nz": nz, "periodic_z": 0, "walls": walls, "Da": 1e-2, "Ra": 0.0, "Pr": 1.0,
           "J": 1.0, "Ma": 0.1, "sigma": 1.0, "Q": 0.0, "tau_f": 0.9, "tau_T": 0.9, "A": 0.05, "B": -0.1,
           "eps": 0.6, "a": (0.0, 0.0, 0.0), "T_hot": 1.0, "T_cold": 0.0, "F_eps": None, "storage": "f64",
           "T_init": np.broadcast_to((0.1 + slope * z)[:, None, None], (nz, 3, 4)).copy()}
    sim = gpu3.Sim3(cfg)
    sim.step(2000)
    f = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    assert np.abs(f["T"] - (0.1 + slope * z)[:, None, None]).max() < 1e-12
    assert np.abs(f["dTdz"] - slope).max() < 1e-12


def test_heated_layer_against_oracle(gpu3):
    """A 64 x 64 x 32 porous layer heated from below (Ra 1e4, Da 1e-2), 20 steps, FP64;
    with the average Nusselt numbers of both walls (FP64 reduction) against the oracle's."""
    import oracle.oracle3 as O3
    cfg = W.layer3d(64, 64, 32, Ra=1e4, Da=1e-2)
    _say("case: 3-D FP64 heated layer 64x64x32, 20 steps")
    sim = gpu3.Sim3(cfg)
    sim.step(20)
    ref = O3.Oracle3(cfg)
    ref.step(20)
    for w in (0, 1):
        a, b = sim.nusselt(w), ref.nusselt(w)
        _say(f"  Nusselt number of wall {w}: {a:.12f} (oracle {b:.12f})")
        assert abs(a - b) < 1e-10 * max(1.0, abs(b))
    dpop, dfield, _, _ = _compare(gpu3, cfg, 20, 1e-10, 1e-10)
    _say(f"  max |populations| diff {dpop:.2e}; fields {max(dfield.values()):.2e}")
    assert dpop < 1e-10
    assert all(v < 1e-10 for v in dfield.values()), dfield


def test_brinkman_between_plates(gpu3):
    """The 3-D path against the Brinkman closed form between plates at rest (eps 0.5,
    Da 1e-2, tau 0.8, A = B = 0.1, F_eps = 0, force along x), second order in the plate
    distance, FP64."""
    from closed_forms import E, brinkman_profile, order, poiseuille_cfg
    ns = (17, 33, 65)
    errs = []
    for nz in ns:
        cfg2, c = poiseuille_cfg(nz, 0.1, F_eps=0.0)
        cfg = {"nx": 4, "ny": 4, "nz": nz, "periodic_z": 0,
               "walls": [{"kind": "T", "T": 0.0}, {"kind": "T", "T": 0.0}],
               "Da": cfg2["Da"], "Ra": 0.0, "Pr": 1.0, "J": 1.0, "Ma": 0.1, "sigma": 1.0, "Q": 0.0,
               "tau_f": cfg2["tau_f"], "tau_T": cfg2["tau_T"], "A": cfg2["A"], "B": cfg2["B"],
               "eps": cfg2["eps"], "a": (c["a"], 0.0, 0.0), "T_hot": 0.0, "T_cold": 0.0, "F_eps": 0.0,
               "storage": "f64"}
        sim = gpu3.Sim3(cfg)
        sim.step(int(6 * (nz - 1) ** 2 / c["nu"]))
        ua, _ = brinkman_profile(np.arange(nz, dtype=float), c)
        errs.append(E(ua, sim.fields()["ux"].cpu().numpy()[:, 1, 1]))
    _say(f"  Brinkman between plates, E(u) at nz {ns}: {[f'{e:.3e}' for e in errs]}")
    assert errs[-1] < 2e-3, errs
    assert order(errs[1], errs[2], ns[1], ns[2]) > 1.7, errs


@pytest.mark.parametrize("storage,A", [("f64", 0.3), ("f32", -0.2)])
def test_shear_wave_decay(gpu3, storage, A):
    """A shear wave u_x = u0 sin(k y) in a periodic 4 x 64 x 4 box decays at nu_e k^2,
    nu_e = cs^2 (tau_f - A - 1/2) (Sec. 3.1)."""
    n = 64
    k = 2 * np.pi / n
    y = np.arange(n, dtype=float)
    u = np.zeros((3, 4, n, 4))
    u[0] = (1e-3 * np.sin(k * y))[None, :, None]
    cfg = {"nx": 4, "ny": n, "nz": 4, "periodic_z": 1, "walls": [{}, {}], "Da": 1e30, "Ra": 0.0, "Pr": 1.0,
           "J": 1.0, "Ma": 0.1, "sigma": 1.0, "Q": 0.0, "tau_f": 1.0, "tau_T": 1.0, "A": A, "B": 0.0, "eps": 1.0,
           "a": (0.0, 0.0, 0.0), "T_hot": 1.0, "T_cold": 0.0, "F_eps": 0.0, "u_init": u, "storage": storage}
    sim = gpu3.Sim3(cfg)
    nu_e = (1.0 - A - 0.5) / 3.0
    t1, t2 = int(0.1 / (nu_e * k * k)), int(0.6 / (nu_e * k * k))
    sim.step(t1)
    a1 = 2 / n * (sim.fields()["ux"].cpu().numpy()[0, :, 0] * np.sin(k * y)).sum()
    sim.step(t2 - t1)
    a2 = 2 / n * (sim.fields()["ux"].cpu().numpy()[0, :, 0] * np.sin(k * y)).sum()
    rate = np.log(a1 / a2) / (t2 - t1) / (nu_e * k * k)
    _say(f"  {storage} A {A}: decay rate / nu_e k^2 = {rate:.6f}")
    assert abs(rate - 1) < 2e-3


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_bench_size_against_oracle(gpu3, storage):
    """The bench's 3-D workload at its full size (192 x 192 x 96 heated layer, the launches
    the bench times), 5 steps: every field against the oracle (FP64 within 1e-10, FP32
    within 1e-5 relative L2)."""
    cfg = W.layer3d(192, 192, 96, Ra=1e4, Da=1e-2, storage=storage)
    _say(f"case: 3-D {storage} bench layer 192x192x96, 5 steps")
    _, dfield, a, b = _compare(gpu3, cfg, 5, None, None)
    if storage == "f64":
        _say(f"  max |fields| diff {max(dfield.values()):.2e}")
        assert all(v < 1e-10 for v in dfield.values()), dfield
    else:
        rel = {k: float(np.linalg.norm(a[k] - b[k]) / np.linalg.norm(b[k])) for k in ("T", "p")}
        du = np.sqrt(sum(np.linalg.norm(a[k] - b[k]) ** 2 for k in ("ux", "uy", "uz")))
        rel["u"] = float(du / np.sqrt(sum(np.linalg.norm(b[k]) ** 2 for k in ("ux", "uy", "uz"))))
        _say(f"  rel L2 {rel}")
        assert rel["u"] < 1e-5 and rel["T"] < 1e-5, rel


XCASES = [
    # (seed, nx, ny, nz, periodic_z, porosity field): walls at x = 0 and x = nx - 1
    (11, 13, 5, 9, 0, False),      # x and z walls, edges
    (12, 4, 6, 7, 1, False),       # smallest walled nx, periodic z
    (13, 10, 3, 4, 0, True),       # smallest walled nz, porosity field
    (14, 9, 7, 12, 0, True),
]


@pytest.mark.parametrize("seed,nx,ny,nz,pz,ef", XCASES)
def test_fp64_parity_x_walls(gpu3, seed, nx, ny, nz, pz, ef):
    cfg = W.random_case3d(seed, nx, ny, nz, periodic_z=pz, eps_field=ef, periodic_x=0)
    _say(f"case: 3-D FP64 x walls seed {seed} {nx}x{ny}x{nz} periodic_z {pz} porosity field {ef}, walls "
         f"{[w['kind'] for w in cfg['walls']]}, 200 steps")
    dpop, dfield, _, _ = _compare(gpu3, cfg, 200, 1e-10, 1e-10)
    _say(f"  max |populations| diff {dpop:.2e}; fields {max(dfield.values()):.2e}")
    assert dpop < 1e-10
    assert all(v < 1e-10 for v in dfield.values()), dfield


def test_fp32_parity_x_walls(gpu3):
    cfg = W.random_case3d(11, 13, 5, 9, storage="f32", periodic_x=0)
    _say("case: 3-D FP32 x walls seed 11, 200 steps")
    _, _, a, b = _compare(gpu3, cfg, 200, None, None)
    du = np.sqrt(sum(np.linalg.norm(a[k] - b[k]) ** 2 for k in ("ux", "uy", "uz")))
    nu = np.sqrt(sum(np.linalg.norm(b[k]) ** 2 for k in ("ux", "uy", "uz")))
    rel = {"u": du / nu, "T": np.linalg.norm(a["T"] - b["T"]) / np.linalg.norm(b["T"])}
    _say(f"  rel L2: u {rel['u']:.2e}, T {rel['T']:.2e}")
    assert rel["u"] < 1e-5 and rel["T"] < 1e-5, rel


def test_cavity_nusselt_against_oracle_and_paper(gpu3):
    """The porous cavity of Sec. 4.2 on the 3-D lattice (hot x = 0, cold x = nx - 1,
    adiabatic z walls, 40 x 2 x 40, Ra 1e3, Da 1e-2, eps 0.6): the four wall Nusselt numbers
    after 300 steps against the oracle's (FP64), then the hot wall's at 12000 steps within
    half a percent of Table Tab:Square1's 1.012."""
    import oracle.oracle3 as O3
    cfg = W.cavity3d(40, 2, eps=0.6, Da=1e-2, Ra=1e3)
    _say("case: 3-D FP64 cavity 40x2x40 Ra 1e3, 300 then 12000 steps")
    sim = gpu3.Sim3(cfg)
    sim.step(300)
    ref = O3.Oracle3(cfg)
    ref.step(300)
    for w in range(4):
        a, b = sim.nusselt(w), ref.nusselt(w)
        _say(f"  Nusselt number of wall {w}: {a:.12f} (oracle {b:.12f})")
        assert abs(a - b) < 1e-10 * max(1.0, abs(b))
    sim.step(12000 - 300)
    nu = sim.nusselt(2)
    _say(f"  hot wall at 12000 steps: {nu:.5f} (paper 1.012)")
    assert abs(nu - 1.012) < 0.005 * 1.012
    assert abs(sim.nusselt(3) - nu) < 0.002 * nu


YCASES = [
    # (seed, nx, ny, nz, periodic_x, periodic_z): walls at y = 0 and y = ny - 1
    (21, 11, 8, 10, 0, 0),         # closed box: edges and vertices
    (22, 7, 9, 5, 1, 0),           # y and z walls
    (26, 5, 4, 6, 0, 1),           # smallest walled ny, x walls, periodic z (a case that stays bounded)
    (24, 4, 4, 4, 0, 0),           # smallest closed box
]


@pytest.mark.parametrize("seed,nx,ny,nz,px,pz", YCASES)
def test_fp64_parity_y_walls(gpu3, seed, nx, ny, nz, px, pz):
    cfg = W.random_case3d(seed, nx, ny, nz, periodic_z=pz, eps_field=seed % 2 == 1, periodic_x=px, periodic_y=0)
    _say(f"case: 3-D FP64 y walls seed {seed} {nx}x{ny}x{nz} periodic_x {px} periodic_z {pz}, walls "
         f"{[w.get('kind') for w in cfg['walls']]}, 200 steps")
    dpop, dfield, _, _ = _compare(gpu3, cfg, 200, 1e-10, 1e-10)
    _say(f"  max |populations| diff {dpop:.2e}; fields {max(dfield.values()):.2e}")
    assert dpop < 1e-10
    assert all(v < 1e-10 for v in dfield.values()), dfield


@pytest.mark.parametrize("seed,steps", [(27, 400), (23, 100)])
def test_fp64_parity_thin_porous_cross_section(gpu3, seed, steps):
    """A 5 x 4 cross-section walled on both pairs (x and y), periodic z, with the random
    porosity field, whose smooth modes span the box so that the porosity jumps by up to 0.5
    between neighbours.  Seed 27 stays bounded: FP64 parity over 400 steps.  Seed 23 grows
    without bound after about 100 steps in the oracle as well (the model assumes a porosity
    that varies slowly on the lattice scale): parity over the first 100 steps, and both
    sides then leave the bounded regime together."""
    import oracle.oracle3 as O3
    cfg = W.random_case3d(seed, 5, 4, 6, periodic_z=1, eps_field=True, periodic_x=0, periodic_y=0)
    _say(f"case: 3-D FP64 thin porous cross-section seed {seed} 5x4x6, {steps} steps")
    dpop, dfield, _, _ = _compare(gpu3, cfg, steps, 1e-10, 1e-10)
    _say(f"  max |populations| diff {dpop:.2e}; fields {max(dfield.values()):.2e}")
    assert dpop < 1e-10
    assert all(v < 1e-10 for v in dfield.values()), dfield
    if seed == 23:
        sim = gpu3.Sim3(cfg)
        ref = O3.Oracle3(cfg)
        sim.step(400)
        ref.step(400)
        a = sim.fields()["ux"].cpu().numpy()
        b = ref.fields()["ux"]
        grew = lambda v: (not np.all(np.isfinite(v))) or np.abs(v).max() > 0.1
        assert grew(a) and grew(b), (np.abs(a).max(), np.abs(b).max())


def test_fp32_parity_closed_box(gpu3):
    cfg = W.random_case3d(21, 11, 8, 10, storage="f32", periodic_x=0, periodic_y=0)
    _say("case: 3-D FP32 closed box seed 21, 200 steps")
    _, _, a, b = _compare(gpu3, cfg, 200, None, None)
    du = np.sqrt(sum(np.linalg.norm(a[k] - b[k]) ** 2 for k in ("ux", "uy", "uz")))
    nu = np.sqrt(sum(np.linalg.norm(b[k]) ** 2 for k in ("ux", "uy", "uz")))
    rel = {"u": du / nu, "T": np.linalg.norm(a["T"] - b["T"]) / np.linalg.norm(b["T"])}
    _say(f"  rel L2: u {rel['u']:.2e}, T {rel['T']:.2e}")
    assert rel["u"] < 1e-5 and rel["T"] < 1e-5, rel


def test_closed_box_nusselt_numbers_against_oracle(gpu3):
    """A box closed on all six faces (the cavity of Sec. 4.2 between x walls, with y walls
    as well), 300 steps: the six wall Nusselt numbers against the oracle's (FP64)."""
    import oracle.oracle3 as O3
    cfg = W.cavity3d(20, 2, eps=0.6, Da=1e-2, Ra=1e4)
    cfg = dict(cfg, ny=6, periodic_y=0, T_init=np.repeat(cfg["T_init"][:, :1, :], 6, axis=1),
               walls=cfg["walls"] + [{"kind": "dTdn", "dTdn": 0.0}, {"kind": "T", "T": 0.5}])
    _say("case: 3-D FP64 closed box 20x6x20, 300 steps")
    sim = gpu3.Sim3(cfg)
    sim.step(300)
    ref = O3.Oracle3(cfg)
    ref.step(300)
    for w in range(6):
        a, b = sim.nusselt(w), ref.nusselt(w)
        _say(f"  Nusselt number of wall {w}: {a:.12f} (oracle {b:.12f})")
        assert abs(a - b) < 1e-10 * max(1.0, abs(b))


@pytest.mark.parametrize("case", ["layer", "closed_box"])
def test_fp16_against_fp64_oracle(gpu3, case):
    """FP16 storage (deviations scaled by 256, FP32 arithmetic): u and T within 5e-2
    relative L2 of the FP64 oracle after 200 steps, the bound the two-dimensional FP16
    storage meets on the cavity; the wall Nusselt numbers within 1e-2 of the oracle's."""
    import oracle.oracle3 as O3
    if case == "layer":
        cfg = W.layer3d(32, 24, 16, Ra=1e4, Da=1e-2, storage="f16")
    else:
        cfg = W.random_case3d(21, 11, 8, 10, storage="f16", periodic_x=0, periodic_y=0)
    _say(f"case: 3-D FP16 {case}, 200 steps")
    sim = gpu3.Sim3(cfg)
    sim.step(200)
    ref = O3.Oracle3(cfg)
    ref.step(200)
    a = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    b = ref.fields()
    du = np.sqrt(sum(np.linalg.norm(a[k] - b[k]) ** 2 for k in ("ux", "uy", "uz")))
    nu = np.sqrt(sum(np.linalg.norm(b[k]) ** 2 for k in ("ux", "uy", "uz")))
    rel = {"u": du / nu, "T": np.linalg.norm(a["T"] - b["T"]) / np.linalg.norm(b["T"])}
    _say(f"  rel L2: u {rel['u']:.2e}, T {rel['T']:.2e}")
    assert rel["u"] < 5e-2 and rel["T"] < 5e-2, rel
    for w in ((0, 1) if case == "layer" else range(6)):
        nu_a, nu_b = sim.nusselt(w), ref.nusselt(w)
        _say(f"  Nusselt number of wall {w}: {nu_a:.6f} (oracle {nu_b:.6f})")
        assert abs(nu_a - nu_b) < 1e-2 * max(1.0, abs(nu_b))


def test_fp16_bench_size_against_oracle(gpu3):
    """The bench's FP16 3-D workload at its full size (192 x 192 x 96), 5 steps: T and u
    within 5e-3 relative L2 of the FP64 oracle."""
    cfg = W.layer3d(192, 192, 96, Ra=1e4, Da=1e-2, storage="f16")
    _say("case: 3-D f16 bench layer 192x192x96, 5 steps")
    _, _, a, b = _compare(gpu3, cfg, 5, None, None)
    du = np.sqrt(sum(np.linalg.norm(a[k] - b[k]) ** 2 for k in ("ux", "uy", "uz")))
    rel = {"T": float(np.linalg.norm(a["T"] - b["T"]) / np.linalg.norm(b["T"])),
           "u": float(du / np.sqrt(sum(np.linalg.norm(b[k]) ** 2 for k in ("ux", "uy", "uz"))))}
    _say(f"  rel L2 {rel}")
    assert rel["u"] < 5e-3 and rel["T"] < 5e-3, rel


def test_cavity_table_square1_higher_ra(gpu3):
    """The porous cavity of Sec. 4.2 on the 3-D lattice at the paper's 120 x 120 (2 nodes in
    y, periodic), Da 1e-2, eps 0.6, Pr 1, FP64, 200000 steps as the two-dimensional test of
    the same rows: the hot-wall Nusselt numbers at Ra 1e4 and 1e5 within 0.5 % of Table
    Tab:Square1's 1.498 and 3.463 (the paper reports the hot wall), and the cold wall's
    within 1 % of the hot wall's (measured: 1.4941 and 3.4510; the cold wall 0.32 % and
    0.74 % below)."""
    for Ra, paper in ((1e4, 1.498), (1e5, 3.463)):
        _say(f"case: 3-D FP64 cavity 120x2x120 Ra {Ra:g}, 200000 steps")
        sim = gpu3.Sim3(W.cavity3d(120, 2, eps=0.6, Da=1e-2, Ra=Ra))
        sim.step(100000)
        _say("  100000 steps")
        sim.step(100000)
        hot, cold = sim.nusselt(2), sim.nusselt(3)
        _say(f"  Nu hot {hot:.4f}, cold {cold:.4f} (paper {paper})")
        sim.close()
        assert abs(hot - paper) <= 0.005 * paper, (Ra, hot)
        assert abs(cold - hot) <= 1e-2 * hot, (Ra, hot, cold)


def test_fp32_long_run_keeps_heat_and_nusselt(gpu3):
    """FP32 storage over long runs: the collision keeps the zeroth and first moments exact in
    the arithmetic type (rest population from the other 18, first-moment-exact weights, the
    relaxation factors summing to one exactly), so no heat creeps in step by step as it did
    with the rounded D3Q19 weights (about 1.5e-8 sigma T / tau_T per node and step).  The 3-D
    cavity of Sec. 4.2 (Da 1e-2, eps 0.6) in FP32 against FP64: at 40 x 2 x 40, Ra 1e3, after
    12000 steps the wall Nusselt numbers within 1e-4 (measured: 6e-6 and 4e-5); at
    120 x 2 x 120, Ra 1e5, after 100000 steps within 1e-3 (measured 3.5e-4 and 3.7e-4; the
    two-dimensional path: 8e-5) and the mean temperature within 1e-4 (measured 2.5e-5, where
    the rounded weights would have added about 6e-4 by 200000 steps)."""
    for n, Ra, steps, tol_nu, tol_T in ((40, 1e3, 12000, 1e-4, 1e-5), (120, 1e5, 100000, 1e-3, 1e-4)):
        out = {}
        for storage in ("f64", "f32"):
            _say(f"case: 3-D {storage} cavity {n}x2x{n} Ra {Ra:g}, {steps} steps")
            sim = gpu3.Sim3(W.cavity3d(n, 2, eps=0.6, Da=1e-2, Ra=Ra, storage=storage))
            done = 0
            while done < steps:
                k = min(50000, steps - done)
                sim.step(k)
                done += k
                _say(f"  {done} steps")
            out[storage] = (sim.nusselt(2), sim.nusselt(3), float(sim.fields()["T"].double().mean()))
            sim.close()
            _say(f"  Nu hot {out[storage][0]:.6f}, cold {out[storage][1]:.6f}, mean T {out[storage][2]:.9f}")
        a, b = out["f32"], out["f64"]
        assert abs(a[0] - b[0]) < tol_nu and abs(a[1] - b[1]) < tol_nu, (n, a, b)
        assert abs(a[2] - b[2]) < tol_T, (n, a, b)
