"""Mixed-precision transport against the oracle, statistically (sections 3.3.5
and 3.4): electrons released at rest in a uniform field (a constant field
map, so only the field of the charges themselves is summed directly) drift
for 200 steps of 1 ps with the null-collision Monte Carlo.  The GPU step in
mixed precision and the oracle's FP64 step run 8 seeds each, with different
random streams (Philox seeds 1..8 on the GPU, 101..108 in the oracle), so
the two are independent samples of the same physics.  Compared within 3
standard errors: the drift velocity (eq. vd), the transverse and
longitudinal spreads of the displacement (eq. diffusion), and the
ionisation, attachment and excitation counts per released electron
(section 4, multiplication)."""
import numpy as np
import pytest
import torch

from paper_2110_09214_amd import binding as B
from paper_2110_09214_amd import workloads as W
from gpu_helpers import dev, host

pytestmark = pytest.mark.gpu

N_E = 1000
STEPS = 200
DT = 1e-12
EZ = -2e6          # V/m: electrons drift towards +z
SEEDS = 8
LO, H, NN = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0), (3, 3, 3)


def _params(step, seed, prec):
    return dict(dt=DT, step=step, seed=seed, max_coll=64, max_ion_per_step=4, ion_v_cap=2e4,
                box_lo=(-1.0, -1.0, -1.0), box_hi=(1.0, 1.0, 1.0), soft=1e-7, r_rec=1e-12, capacity=10 ** 5,
                precision=prec)


def _start(k):
    x = np.random.default_rng(k).normal(size=(N_E, 3)) * 1e-4
    return x, np.zeros((N_E, 3)), np.zeros(N_E, np.int8), np.arange(N_E, dtype=np.int64)


def _summary(x0, ids, x, species, v):
    """Per-electron samples of the primaries still electrons at the end."""
    keep = (ids < N_E) & (species == 0)
    d = x[keep] - x0[ids[keep]]
    en = 0.5 * W.M_ELECTRON * (v[species == 0] ** 2).sum(1) / W.E_CHARGE
    return d, en


def _gpu_run(ctx, seed, gas_s, fmap):
    x0, v0, sp0, id0 = _start(seed)
    parts = B.Particles(10 ** 5, "cuda", dev(x0), dev(v0), dev(sp0, torch.int8), dev(id0, torch.int64), N_E)
    cnt = np.zeros(5, np.int64)
    for s in range(STEPS):
        st = B.track_step(ctx, None, parts, gas_s, _params(s, seed, B.OBEM_MIXED), None, None, fmap=fmap)
        cnt += np.array(st["real_collisions"])
    g = parts.state()
    d, en = _summary(x0, host(g["id"]), host(g["x"]), host(g["species"]), host(g["v"]))
    return d, en, cnt


def _oracle_run(orc, seed, gas, Emap):
    x0, v0, sp0, id0 = _start(seed - 100)
    state = dict(x=x0.copy(), v=v0, species=sp0, id=id0, next_id=N_E)
    counts = np.zeros(0, np.int64)
    cnt = np.zeros(5, np.int64)
    for s in range(STEPS):
        state, _, counts, so, _ = orc.track_step(state, None, None, gas, _params(s, seed, B.OBEM_FP64), counts,
                                                 field_map=(Emap, LO, H))
        cnt += np.array([so[k] for k in ("elastic", "exc1", "exc2", "ionisation", "attachment")])
    d, en = _summary(x0, state["id"], state["x"], state["species"], state["v"])
    return d, en, cnt


def _stats(runs):
    """(value, standard error) of each compared quantity over the seeds."""
    d = np.concatenate([r[0] for r in runs])
    en = np.concatenate([r[1] for r in runs])
    T = STEPS * DT
    out = {}
    out["drift_velocity"] = (d[:, 2].mean() / T, d[:, 2].std() / np.sqrt(len(d)) / T)
    rt = (d[:, :2] ** 2).sum(1)
    out["transverse_var"] = (rt.mean(), rt.std() / np.sqrt(len(rt)))
    rl = (d[:, 2] - d[:, 2].mean()) ** 2
    out["longitudinal_var"] = (rl.mean(), rl.std() / np.sqrt(len(rl)))
    out["mean_energy_eV"] = (en.mean(), en.std() / np.sqrt(len(en)))
    per = np.array([r[2] for r in runs], np.float64) / N_E      # per released electron, per seed
    for k, name in ((3, "ionisations"), (4, "attachments")):
        tot = per[:, k].sum() * N_E
        se = max(per[:, k].std(ddof=1) / np.sqrt(len(runs)), np.sqrt(tot) / (N_E * len(runs)))
        out[name] = (per[:, k].mean(), se)
    exc = per[:, 1] + per[:, 2]
    out["excitations"] = (exc.mean(), max(exc.std(ddof=1) / np.sqrt(len(runs)),
                                          np.sqrt(exc.sum() * N_E) / (N_E * len(runs))))
    return out


def test_mixed_transport_matches_oracle_statistically(ctx, orc):
    gas = W.synthetic_ar_co2()
    gas_s, keep = B.gas_struct(gas, "cuda")
    Emap = np.zeros(NN + (3,))
    Emap[..., 2] = EZ
    fmap = B.FieldMap(LO, H, NN)
    fmap.e[2].fill_(EZ)
    g = _stats([_gpu_run(ctx, s, gas_s, fmap) for s in range(1, SEEDS + 1)])
    o = _stats([_oracle_run(orc, s, gas, Emap) for s in range(101, 101 + SEEDS)])
    bad = []
    for k in g:
        (a, sa), (b, sb) = g[k], o[k]
        z = abs(a - b) / np.hypot(sa, sb)
        print(f"{k}: GPU mixed {a:.5g} +- {sa:.2g}, oracle {b:.5g} +- {sb:.2g} ({z:.2f} sigma)")
        if z > 3.0:
            bad.append(k)
    assert not bad, bad
    # the run is a real avalanche start: ionisation and attachment both occur
    assert g["ionisations"][0] > 0.1 and g["attachments"][0] > 0.1
