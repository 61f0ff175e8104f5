"""Pins of the oracle's single-collision physics outside the null-collision
core (section 3.4.3 and the ion model read from section 3.4): attachment,
excitation loss with the sub-threshold ionisation fallback, isotropic ion
scattering in the centre-of-mass frame, and charge exchange to a thermal
(Maxwellian) velocity.

Each collision is driven through the oracle's own transport step with a test
gas in which one process is the only real channel, no field and one flight
with a collision (max_coll = 1), so a particle's velocity after the step is
its velocity right after the collision.  The checks are closed forms and
conservation laws that do not restate the oracle's formulas: momentum carried
onto a molecule at rest, kinetic energy conserved in an elastic encounter,
the Maxwell-Boltzmann moments of the gas, isotropy of directions.

The second half plants a mistake in a copy of oracle.c (on the CPU), builds
it, and checks that the pin of that part fails for it."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from paper_2110_09214_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_C = os.path.join(os.path.dirname(HERE), "oracle", "oracle.c")


def _params(**kw):
    p = dict(dt=1e-12, step=0, seed=7, max_coll=1, max_ion_per_step=4, ion_v_cap=2e4,
             box_lo=(-1.0, -1.0, -1.0), box_hi=(1.0, 1.0, 1.0))
    p.update(kw)
    return p


def _electron_gas(orc, proc, rate=1e16):
    """Only process `proc` (0 elastic .. 4 attachment) with collision
    frequency `rate` at the nodes (cross section ∝ 1/v): the first flight
    ends within 1 ps except with probability exp(-1e4), and in a real
    collision of that kind unless the draw falls in the 0.3 % margin of the
    bound nu_max (a null collision)."""
    k = orc.constants()
    gas = W.synthetic_ar_co2()
    v_nodes = np.sqrt(2 * gas.energies * k["e"] / k["m_e"])
    gas.xs[:] = 0.0
    gas.xs[proc] = rate / (gas.density * v_nodes)
    return gas


def _collided(v0, v1, count, n):
    """Particles whose first flight ended in a real collision (one flight
    per step: the bound nu_max exceeds the real rate of a 1/v cross section
    on the log-spaced nodes by 0.3 %, so a few end in a null collision and
    keep their velocity)."""
    hit = np.any(v1 != v0, axis=1)
    assert hit.sum() == count and count >= 0.99 * n
    return hit


def _unit(v):
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _isotropic_ok(d, nsig=5.0):
    """Unit vectors d (n, 3) uniform on the sphere: zero mean (each component
    has variance 1/3) and second moments I/3 (d_k^2 has variance 4/45)."""
    n = len(d)
    m1 = d.mean(axis=0)
    m2 = (d[:, :, None] * d[:, None, :]).mean(axis=0)
    ok1 = np.all(np.abs(m1) <= nsig * np.sqrt(1.0 / (3 * n)))
    ok2 = np.all(np.abs(np.diag(m2) - 1.0 / 3.0) <= nsig * np.sqrt(4.0 / 45.0 / n))
    # off-diagonal d_j d_k: variance 1/15
    off = m2[np.triu_indices(3, 1)]
    ok3 = np.all(np.abs(off) <= nsig * np.sqrt(1.0 / 15.0 / n))
    return bool(ok1 and ok2 and ok3)


# ---------------------------------------------------------------------------
# the pins, as functions of the oracle module (run on the real oracle below,
# and on copies with a planted mistake further down)
# ---------------------------------------------------------------------------
def check_attachment(orc):
    """Attachment (section 3.4.3): the electron becomes a negative ion and
    its momentum is conserved (the molecule at rest takes it in), so the
    velocity scales by m_e / m_anion; the anion then flies ballistically to
    the end of the step (no further collision, even with ion cross
    sections present)."""
    k = orc.constants()
    gas = _electron_gas(orc, 4)
    gas.ion_xs_iso = gas.ion_xs_back = 1e-12         # ions would collide at once if allowed
    n = 400
    rng = np.random.default_rng(1)
    v0 = rng.normal(size=(n, 3)) * 4e5
    x, v = np.zeros((n, 3)), v0.copy()
    sp, ids = np.zeros(n, np.int8), np.arange(n, dtype=np.int64)
    st, hit, nch, cx, cv, cnt = orc.mc_step(x, v, sp, ids, np.zeros((n, 3)), gas, _params(max_coll=64))
    assert np.all(sp == 2), "attached electrons become anions"
    assert cnt[4] == n and cnt[6] == 0, "one attachment each, then no collision for the rest of the step"
    p0 = k["m_e"] * v0
    p1 = gas.m_anion * v
    assert np.allclose(p1, p0, rtol=1e-13, atol=1e-13 * np.abs(p0).max()), "momentum conserved"


def check_excitation(orc):
    """Excitation (section 3.4.3): the electron loses exactly the threshold
    T_k and leaves in an isotropic direction; no child."""
    k = orc.constants()
    for proc, T in ((1, 11.55), (2, 13.0)):
        gas = _electron_gas(orc, proc)
        n = 6000
        e0 = 20.0 + 5.0 * np.random.default_rng(proc).random(n)       # eV, above both thresholds
        d0 = _unit(np.random.default_rng(10 + proc).normal(size=(n, 3)))
        v = d0 * np.sqrt(2 * e0 * k["e"] / k["m_e"])[:, None]
        x, sp, ids = np.zeros((n, 3)), np.zeros(n, np.int8), np.arange(n, dtype=np.int64)
        v0 = v.copy()
        st, hit, nch, cx, cv, cnt = orc.mc_step(x, v, sp, ids, np.zeros((n, 3)), gas, _params())
        hit = _collided(v0, v, cnt[proc], n)
        assert np.all(nch == 0)
        e1 = 0.5 * k["m_e"] * np.sum(v[hit] ** 2, axis=1) / k["e"]
        assert np.allclose(e1, e0[hit] - T, rtol=1e-12), f"excitation {proc} loses T = {T} eV"
        assert _isotropic_ok(_unit(v[hit])), "excited electrons leave isotropically"


def check_subthreshold_ionisation(orc):
    """An ionising collision with E_res = E - E_ioni - 3/2 kT <= 0 (section
    3.4.3 leaves no energy for the pair) is taken as an excitation of E_ioni:
    the electron keeps E - 15.7 eV, no pair is created."""
    k = orc.constants()
    gas = _electron_gas(orc, 3)
    eth = 1.5 * k["k_B"] * gas.temperature / k["e"]                   # 0.0388 eV
    n = 500
    e0 = 15.7 + eth * np.linspace(0.05, 0.95, n)
    v = np.zeros((n, 3))
    v[:, 0] = np.sqrt(2 * e0 * k["e"] / k["m_e"])
    x, sp, ids = np.zeros((n, 3)), np.zeros(n, np.int8), np.arange(n, dtype=np.int64)
    v0 = v.copy()
    st, hit, nch, cx, cv, cnt = orc.mc_step(x, v, sp, ids, np.zeros((n, 3)), gas, _params())
    assert np.all(nch == 0), "no pair below E_ioni + 3/2 kT"
    hit = _collided(v0, v, cnt[3], n)
    e1 = 0.5 * k["m_e"] * np.sum(v[hit] ** 2, axis=1) / k["e"]
    assert np.allclose(e1, e0[hit] - 15.7, rtol=1e-9, atol=1e-14), "loses exactly E_ioni"


def _ion_run(orc, species, iso, back, n=20000, speed=1.5e4, seed=3):
    """Ions of one species with speed `speed` in random directions, one
    flight in a gas where only the isotropic (iso) or the charge-exchange
    (back) ion channel is on; returns the gas and the velocities before and
    after of the ions whose first flight ended in a real collision."""
    gas = W.synthetic_ar_co2()
    gas.ion_xs_iso = 1e-13 if iso else 0.0
    gas.ion_xs_back = 1e-13 if back else 0.0
    rng = np.random.default_rng(seed)
    v0 = _unit(rng.normal(size=(n, 3))) * speed
    v = v0.copy()
    x = np.zeros((n, 3))
    sp = np.full(n, species, np.int8)
    ids = np.arange(n, dtype=np.int64)
    *_, cnt = orc.mc_step(x, v, sp, ids, np.zeros((n, 3)), gas, _params())
    moved = np.any(v != v0, axis=1)
    assert moved.sum() == cnt[6] and cnt[6] > 0.3 * n, "real ion collisions (the rest are null)"
    return gas, v0[moved], v[moved]


def check_ion_isotropic(orc):
    """Isotropic ion scattering off a molecule at rest, elastic (reading of
    the ion model, section 3.4): per collision, with M the molecule's mass and
    U' = m (v - v') / M its recoil velocity, momentum and kinetic energy are
    conserved; the direction is isotropic in the centre-of-mass frame, so the
    mean outgoing velocity is m/(m + M) v and |v'|^2 is uniform between
    ((m - M)/(m + M))^2 |v|^2 and |v|^2."""
    for species in (1, 2):
        gas, v0, v1 = _ion_run(orc, species, iso=True, back=False)
        m = gas.m_cation if species == 1 else gas.m_anion
        M = gas.m_gas
        U = m * (v0 - v1) / M
        ke0 = 0.5 * m * np.sum(v0 ** 2, axis=1)
        ke1 = 0.5 * m * np.sum(v1 ** 2, axis=1) + 0.5 * M * np.sum(U ** 2, axis=1)
        assert np.allclose(ke1, ke0, rtol=1e-10), f"species {species}: kinetic energy conserved"
        vcm = m / (m + M) * v0
        assert _isotropic_ok(_unit(v1 - vcm)), "isotropic in the centre-of-mass frame"
        n = len(v0)
        # mean outgoing velocity along the incoming direction
        par = np.einsum("ij,ij->i", v1, _unit(v0))
        sd = np.std(par) / np.sqrt(n)
        assert abs(par.mean() - m / (m + M) * np.linalg.norm(v0[0])) <= 5 * sd
        s2 = np.sum(v1 ** 2, axis=1) / np.sum(v0 ** 2, axis=1)
        lo, hi = ((m - M) / (m + M)) ** 2, 1.0
        assert s2.min() >= lo - 1e-12 and s2.max() <= hi + 1e-12
        # uniform on [lo, hi]: mean (lo + hi) / 2, variance (hi - lo)^2 / 12
        assert abs(s2.mean() - 0.5 * (lo + hi)) <= 5 * (hi - lo) / np.sqrt(12 * n)


def check_charge_exchange(orc):
    """Charge exchange (reading of the ion model): the ion takes the velocity
    of a gas molecule, Maxwell-Boltzmann at T: each component normal with
    mean 0 and variance k_B T / M_gas (the molecule's mass, not the ion's),
    components independent, independent of the incoming velocity."""
    k = orc.constants()
    for species in (1, 2):
        gas, v0, v1 = _ion_run(orc, species, iso=False, back=True, n=40000)
        n = len(v1)
        var = k["k_B"] * gas.temperature / gas.m_gas
        sd = np.sqrt(var)
        assert np.all(np.abs(v1.mean(axis=0)) <= 5 * sd / np.sqrt(n))
        assert np.all(np.abs(v1.var(axis=0) / var - 1.0) <= 5 * np.sqrt(2.0 / n))
        z = v1 / sd
        kurt = np.mean(z ** 4, axis=0)
        assert np.all(np.abs(kurt - 3.0) <= 5 * np.sqrt(96.0 / n)), "normal components"
        c = np.corrcoef(np.concatenate([v1, v0], axis=1).T)
        assert np.all(np.abs(c[np.triu_indices(6, 1)]) <= 5 / np.sqrt(n)), "independent components"


PINS = [check_attachment, check_excitation, check_subthreshold_ionisation, check_ion_isotropic,
        check_charge_exchange]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_collision_pin(orc, pin):
    pin(orc)


# ---------------------------------------------------------------------------
# planted mistakes: each must fail its pin
# ---------------------------------------------------------------------------
MUTANTS = [
    # (pin, original text in oracle.c, planted text)
    (check_attachment, "Vv[d] *= me / g->m_anion;", "Vv[d] *= me / g->m_cation;"),
    (check_attachment, "          sp = 2;\n          ballistic = 1;", "          sp = 2;\n          ballistic = 0;"),
    (check_excitation, "double e2 = eps - g->thr[proc];", "double e2 = eps - 0.5 * g->thr[proc];"),
    (check_excitation, "      isotropic(u2, u3, dir);\n      double s = sqrt(2.0 * e2 * qe / me);",
     "      isotropic(0.5 * u2, u3, dir);\n      double s = sqrt(2.0 * e2 * qe / me);"),
    (check_subthreshold_ionisation, "if (proc != 3 || e_res <= 0.0) {", "if (proc != 3 || e_res <= -1.0) {"),
    (check_ion_isotropic, "double fm = mion / (mion + g->m_gas), fM = g->m_gas / (mion + g->m_gas);",
     "double fm = g->m_gas / (mion + g->m_gas), fM = mion / (mion + g->m_gas);"),
    (check_ion_isotropic, "Vv[d] = fm * Vv[d] + fM * vm * dir[d];", "Vv[d] = fm * Vv[d] + fm * vm * dir[d];"),
    (check_charge_exchange, "double sd = sqrt((double)KB * g->temperature / g->m_gas);",
     "double sd = sqrt((double)KB * g->temperature / (sp == 1 ? g->m_cation : g->m_anion));"),
    (check_charge_exchange, "double r1 = sqrt(-2.0 * log(u01(w2[0]))), r2 = sqrt(-2.0 * log(u01(w2[2])));",
     "double r1 = sqrt(-2.0 * log(u01(w2[0]))), r2 = sqrt(-3.0 * log(u01(w2[2])));"),
    (check_charge_exchange, "Vv[1] = sd * r1 * sin(2.0 * M_PI * u01(w2[1]));",
     "Vv[1] = sd * r1 * cos(2.0 * M_PI * u01(w2[1]));"),
]


@pytest.mark.parametrize("pin,orig,planted", MUTANTS, ids=[f"{m[0].__name__}-{i}" for i, m in enumerate(MUTANTS)])
def test_planted_mistake_fails_its_pin(orc, tmp_path, monkeypatch, pin, orig, planted):
    src = open(ORACLE_C).read()
    assert src.count(orig) == 1, "the mutated line must exist once in oracle.c"
    path = tmp_path / "mut.c"
    path.write_text(src.replace(orig, planted))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-std=gnu11", "-O1", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                    "-ffp-contract=off", str(path), "-o", str(so), "-lm"], check=True)
    monkeypatch.setattr(orc, "_lib", C.CDLL(str(so)))
    with pytest.raises(AssertionError):
        pin(orc)
