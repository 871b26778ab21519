"""Pins of the oracle's physiologically structured consumer (Supplementary
S2: resource consumption, somatic growth, reproduction, mortality, two
dynamic resources; neonate mass Omega = exp(z) the evolving trait).

One time step is recomputed here from the state before it -- masses,
phenotypes, sexes and resource densities read from the oracle -- with
numpy, independently of the oracle's C loops, and checked against what
the step produced:

* mass balance X' + Y' + G = X + Y + dW, irreversible mass never falling,
  a surplus shared min(1, kappa Y/X) to X, a deficit drawn from Y;
* gonads only at breeding steps and only of mature individuals, leaving
  Y' = q_A X';
* the resource update max(0, r' R/(1 + R/K) - consumption) with the
  step's growth-rate deviate;
* survival frequency against (1 - exp(-beta_s Y/X)) / (1 + exp(-beta_2 (X
  - beta_1))), and death without reserves;
* the eggs F, the recruits floor(kappa1 F / (1 + (F/kappa2)^kappa3)) up to
  the capacity, none without a mature male;
* mothers in proportion to their eggs and fathers to X (v = 1), by a chi-
  square over the parents of many recruits; a recruit's body X = Omega of
  its mother, Y = q_J X;
* starvation of the whole population without food.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle

ST_RESOURCE = 19

PHY = dict(alpha=0.3, gamma=0.75, delta=0.1, attack=2.0, handling=1.0, K=[6000.0, 6000.0], growth=[2.0, 2.0],
           growth_sd=[0.1, 0.1], R0=[6000.0, 6000.0], steepness=5.0, switch_frac=0.5, w_max=8.0, kappa=1.0,
           qJ=0.2, qA=0.4, beta1=0.05, beta2=20.0, beta_s=20.0, maturity=1.0, v_f=1.0, v_m=1.0,
           kappa1=0.5, kappa2=2000.0, kappa3=1.0, breed_every=5)
L = 16


def pop(n0=2000, cap=20000, seed=3, **phy):
    p = dict(PHY)
    p.update(phy)
    return oracle.OraclePop(seed=seed, replicate_id=1, regime=3, n0=n0, capacity=cap, n_loci=L, mu=1e-3, r=0.5,
                            genetics=1, allele_mean=-2.3 / L, allele_sd=0.02, mut_sd_factor=0.2, noise_sd=0.05,
                            exp_transform=1, physiology=p), p


def grow_np(X, Y, R, p, breeding):
    """One step of consumption and growth, vectorised."""
    h = [p["attack"] * R[j] / p["K"][j] for j in (0, 1)]
    h = [x / (1.0 + p["handling"] * x) for x in h]
    W = X + Y
    pi1 = 1.0 / (1.0 + np.exp(-p["steepness"] * (np.cbrt(W) - p["switch_frac"] * np.cbrt(p["w_max"]))))
    intake = p["alpha"] * W ** p["gamma"]
    e1, e2 = h[0] * pi1 * intake, h[1] * (1.0 - pi1) * intake
    dW = e1 + e2 - p["delta"] * W
    f = np.minimum(1.0, p["kappa"] * Y / X)
    Xn = np.where(dW > 0, X + f * dW, X)
    Yn = np.where(dW > 0, Y + (1.0 - f) * dW, Y + dW)
    G = np.zeros_like(X)
    if breeding:
        mature = Xn >= p["maturity"]
        G = np.where(mature, np.maximum(0.0, Yn - p["qA"] * Xn), 0.0)
        Yn = Yn - G
    return Xn, Yn, G, dW, e1.sum(), e2.sum()


def step_and_read(o, p):
    X, Y = o.body()
    z = o.phenotypes_f().astype(np.float64)
    sex = o.sexes()
    st0 = o.stats()
    t = o.generation
    R = st0["resource"]
    breeding = t % p["breed_every"] == p["breed_every"] - 1
    o.step(1)
    return dict(X=X, Y=Y, z=z, sex=sex, R=R, t=t, breeding=breeding, S=o.survivors(), st=o.stats())


def test_growth_mass_balance_and_allocation():
    o, p = pop()
    o.step(3)  # a few steps in, masses spread out
    s = step_and_read(o, p)
    Xn, Yn, G, dW, _, _ = grow_np(s["X"], s["Y"], s["R"], p, s["breeding"])
    X1, Y1 = o.body()
    ns = s["S"].size
    # survivors come first in the new census, in ascending order
    assert np.allclose(X1[:ns], Xn[s["S"]], rtol=1e-12)
    assert np.allclose(Y1[:ns], Yn[s["S"]], rtol=1e-12, atol=1e-15)
    # mass balance and the irreversible mass's monotonicity
    assert np.allclose(Xn + Yn + G, s["X"] + s["Y"] + dW, rtol=1e-12)
    assert np.all(Xn >= s["X"])
    grew = dW > 0
    assert np.allclose((Xn - s["X"])[grew], (np.minimum(1.0, p["kappa"] * s["Y"] / s["X"]) * dW)[grew], rtol=1e-9)


def test_resource_update_with_the_steps_growth_deviate():
    o, p = pop()
    o.step(2)
    s = step_and_read(o, p)
    _, _, _, _, c1, c2 = grow_np(s["X"], s["Y"], s["R"], p, s["breeding"])
    c3 = (1 << 12) | 0
    for j, c in enumerate((c1, c2)):
        r = p["growth"][j] + p["growth_sd"][j] * oracle.normals(3, c3, 0, ST_RESOURCE, s["t"], j, 1)[0]
        want = max(0.0, r * s["R"][j] / (1.0 + s["R"][j] / p["K"][j]) - c)
        assert s["st"]["resource"][j] == pytest.approx(want, rel=1e-11)


def test_survival_law_and_death_without_reserves():
    o, p = pop(n0=20000, cap=40000, beta1=0.3, beta2=8.0)
    s = step_and_read(o, p)
    Xn, Yn, _, _, _, _ = grow_np(s["X"], s["Y"], s["R"], p, s["breeding"])
    prob = np.where(Yn > 0, (1.0 - np.exp(-p["beta_s"] * Yn / Xn)) / (1.0 + np.exp(-p["beta2"] * (Xn - p["beta1"]))),
                    0.0)
    ns = s["S"].size
    assert abs(ns - prob.sum()) < 4.0 * math.sqrt((prob * (1 - prob)).sum())
    # survivors by size class follow the size logistic
    small = Xn < np.median(Xn)
    surv = np.zeros(Xn.size, bool)
    surv[s["S"]] = True
    for m in (small, ~small):
        assert abs(surv[m].sum() - prob[m].sum()) < 4.0 * math.sqrt((prob[m] * (1 - prob[m])).sum()) + 1


def breeding_run(seed=3, **phy):
    o, p = pop(seed=seed, **phy)
    while o.generation % p["breed_every"] != p["breed_every"] - 1 or o.generation < 20:
        o.step(1)
    return o, p, step_and_read(o, p)


def test_gonads_eggs_and_recruits():
    o, p, s = breeding_run()
    assert s["breeding"]
    Xn, Yn, G, _, _, _ = grow_np(s["X"], s["Y"], s["R"], p, True)
    mature = Xn >= p["maturity"]
    assert np.all(G[~mature] == 0.0)
    assert np.all(Yn[mature] <= p["qA"] * Xn[mature] * (1 + 1e-12) + 1e-15)
    surv = np.zeros(Xn.size, bool)
    surv[s["S"]] = True
    fem = surv & mature & (s["sex"] == 0)
    eggs = (G[fem] / (s["z"][fem] + p["qJ"] * s["z"][fem])).sum()
    assert s["st"]["eggs"] == pytest.approx(eggs, rel=1e-10)
    phi = p["kappa1"] * eggs / (1.0 + (eggs / p["kappa2"]) ** p["kappa3"])
    recruits = s["st"]["n"] - s["S"].size
    assert recruits == min(math.floor(phi), 20000 - s["S"].size)
    assert recruits > 50
    # a recruit's body: its mother's neonate mass, reserves q_J of it
    mom, dad = o.parents()
    X1, Y1 = o.body()
    assert np.array_equal(X1[s["S"].size:], s["z"][mom])
    assert np.allclose(Y1[s["S"].size:], p["qJ"] * s["z"][mom], rtol=0, atol=0)
    assert np.all(s["sex"][mom] == 0) and np.all(s["sex"][dad] == 1)
    assert np.all(mature[mom]) and np.all(mature[dad])


def test_parents_in_proportion_to_eggs_and_size():
    o, p, s = breeding_run(kappa1=2.0, kappa2=1e9, n0=4000, cap=200000)
    Xn, _, G, _, _, _ = grow_np(s["X"], s["Y"], s["R"], p, True)
    mom, dad = o.parents()
    surv = np.zeros(Xn.size, bool)
    surv[s["S"]] = True
    mature = Xn >= p["maturity"]
    fem = np.flatnonzero(surv & mature & (s["sex"] == 0))
    mal = np.flatnonzero(surv & mature & (s["sex"] == 1))
    eggs = G[fem] / (s["z"][fem] + p["qJ"] * s["z"][fem])
    for who, idx, w in (("mothers", fem, eggs), ("fathers", mal, Xn[mal])):
        drawn = mom if who == "mothers" else dad
        obs = np.array([np.sum(drawn == i) for i in idx], dtype=float)
        exp = w / w.sum() * drawn.size
        # pool into ten weight deciles for the chi-square
        order = np.argsort(w)
        bins = np.array_split(order, 10)
        o_b = np.array([obs[b].sum() for b in bins])
        e_b = np.array([exp[b].sum() for b in bins])
        assert stats.chisquare(o_b, e_b).pvalue > 1e-4, who


def test_no_recruits_off_breeding_steps_and_starvation():
    o, p = pop(breed_every=1000)
    for _ in range(5):
        n_before = o.stats()["n"]
        o.step(1)
        st = o.stats()
        assert st["n"] == st["n_survivors"] <= n_before and st["eggs"] == 0.0
    # no food at all: reserves run out, every consumer dies
    o2, _ = pop(R0=[0.0, 0.0], growth=[0.0, 0.0], growth_sd=[0.0, 0.0])
    for _ in range(60):
        o2.step(1)
        X, Y = o2.body()
        if o2.n == 0:
            break
    assert o2.n == 0 and o2.stats()["extinct"] == 1


def test_rejections():
    with pytest.raises(ValueError):
        oracle.OraclePop(regime=3, n0=10, n_loci=4, genetics=0, physiology=PHY)
    with pytest.raises(ValueError):
        oracle.OraclePop(regime=3, n0=10, n_loci=4, genetics=1, exp_transform=0, physiology=PHY)
    bad = dict(PHY)
    bad["gamma"] = 1.5
    with pytest.raises(ValueError):
        oracle.OraclePop(regime=3, n0=10, n_loci=4, genetics=1, exp_transform=1, physiology=bad)
