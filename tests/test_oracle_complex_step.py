"""Pins of the oracle's complex-step reference derivatives (oracle/complex_step.py).

The complex-step module is a second, vectorised numpy rendering of the
oracle step for the differentiation setting (hydrogen only, one group,
GLF, periodic).  It is pinned to things other than itself:
  - its rates equal the C oracle's App. E rates, and its analytic d/dT
    equal the complex-step derivatives of the rate values;
  - the real part of a run equals the C oracle run (state and the per-cell
    substep counts of every step);
  - its directional derivatives equal central finite differences of the C
    oracle's loss (brute force), for source rates, one cell's density and a
    random direction over all densities, isothermal and with T evolving.
"""
import numpy as np
import pytest

import oracle
import rt_inputs as ri
from oracle import complex_step as cs
from oracle import physics

TEMPS = np.logspace(1.0, 8.0, 29)


def test_rates_equal_c_oracle_rates():
    for T in TEMPS:
        for name, f in (("beta_HI", cs.beta_HI), ("alphaB_HII", cs.alphaB_HII)):
            v, d = oracle.rate(name, T)
            cv, cd = f(np.complex128(T))
            assert abs(cv.real - v) <= 1e-13 * abs(v) + 1e-300, (name, T)
            assert abs(cd.real - d) <= 1e-12 * abs(d) + 1e-300, (name, T)
        # hydrogen-only cooling: ne = nHI = nHII = 1 picks out the rate sum
        L, dL = cs.cooling_H(np.complex128(T), 1.0, 1.0, 1.0, 1.0)
        parts = [oracle.rate(k, T) for k in ("zeta_HI", "psi_HI", "etaB_HII", "theta")]
        cv, cd = oracle.rate("varpi", T, 1.0)
        Lr = sum(p[0] for p in parts) + cv
        dLr = sum(p[1] for p in parts) + cd
        assert abs(L.real - Lr) <= 1e-13 * abs(Lr)
        assert abs(dL.real - dLr) <= 1e-12 * abs(dLr)


def test_analytic_T_derivatives_are_the_derivatives_of_the_values():
    eps = 1e-30
    for T in TEMPS:
        z = np.complex128(T + 1j * eps)
        for f in (cs.beta_HI, cs.alphaB_HII):
            v, d = f(z)
            assert abs(v.imag / eps - d.real) <= 1e-12 * abs(d.real) + 1e-300
        L, dL = cs.cooling_H(z, 0.3, 0.7, 0.3, 1.0)
        assert abs(L.imag / eps - dL.real) <= 1e-12 * abs(dL.real)


def small_case(iso, n=12, steps=8, ns=4, seed=1):
    w = ri.grey_box(n, 3.3 * n / 64, ns, steps, seed=seed, isothermal=iso)
    sN, sE, eb, _ = physics.spectrum_attributes(w.spectrum)
    p = cs.CSParams(w.n, w.dx, w.c_r, sN[0][0], sE[0][0], eb[0], iso, X=w.X, gamma=w.gamma, a_exp=w.a_exp,
                    x_min=w.x_min)
    o = oracle.OracleRT.for_workload(w)
    st = ri.initial_state(w)
    ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
    s0 = {"N": st["N"][0], "F": st["F"][0], "xHII": st["xHII"], "T": st["T"]}
    return w, p, o, st, s0, ijk, nd


def c_oracle_run(o, st, dt, steps, ijk, lnnd, lnnH):
    so = oracle.copy_state(st)
    so["nH"] = np.exp(lnnH)
    nd = np.exp(lnnd)[:, None]
    counts = []
    for _ in range(steps):
        _, na, _ = o.step(so, dt, ijk, nd, want_counts=True)
        counts.append(na.ravel())
    return so, counts


@pytest.mark.parametrize("iso", [True, False])
def test_real_part_is_the_c_oracle_run(iso):
    w, p, o, st, s0, ijk, nd = small_case(iso)
    dt = o.courant_dt()
    fin, counts = cs.run(p, s0, dt, w.steps, ijk, np.log(nd), np.log(st["nH"]))
    so, cts = c_oracle_run(o, st, dt, w.steps, ijk, np.log(nd), np.log(st["nH"]))
    assert all(np.array_equal(a, b) for a, b in zip(counts, cts))
    assert max(c.max() for c in cts) > 10  # the run subcycles
    for a, b in ((fin["N"], so["N"][0]), (fin["F"], so["F"][0]), (fin["xHII"], so["xHII"]), (fin["T"], so["T"])):
        assert np.max(np.abs(a.imag)) == 0.0
        assert np.max(np.abs(a.real - b)) <= 1e-13 * np.max(np.abs(b))


@pytest.mark.parametrize("iso", [True, False])
def test_complex_step_equals_central_differences_of_the_c_oracle(iso):
    w, p, o, st, s0, ijk, nd = small_case(iso, steps=10)
    dt = o.courant_dt()
    lnnd, lnnH = np.log(nd), np.log(st["nH"])
    tfin, _ = cs.run(p, s0, dt, w.steps, ijk, ri.perturbed_log_rates(nd, w.seed), lnnH)
    target = tfin["xHII"].real
    rng = np.random.default_rng(5)
    cell = np.zeros(st["nH"].shape)
    i, j, k = ijk[0]
    cell[k, j, (i + 1) % w.n[0]] = 1.0
    dirs = [(np.eye(len(nd))[0], None), (np.eye(len(nd))[2], None), (None, rng.standard_normal(st["nH"].shape)),
            (None, cell)]
    h = 1e-5
    for vs, vc in dirs:
        dcs = cs.directional_derivative(p, s0, dt, w.steps, ijk, lnnd, lnnH, target, vs, vc)
        lp = lm = None
        for sgn in (1.0, -1.0):
            a = lnnd + (sgn * h * vs if vs is not None else 0.0)
            b = lnnH + (sgn * h * vc if vc is not None else 0.0)
            so, _ = c_oracle_run(o, st, dt, w.steps, ijk, a, b)
            v = float(np.sum((so["xHII"] - target) ** 2))
            if sgn > 0:
                lp = v
            else:
                lm = v
        fd = (lp - lm) / (2 * h)
        assert abs(fd - dcs) <= 1e-6 * abs(dcs), (vs is not None, fd, dcs)
