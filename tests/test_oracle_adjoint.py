"""Pin of the oracle's adjoint: its gradients equal central finite differences
of the oracle's own forward objective J = |sum_n dt exp(-i 2 pi f0 n dt) s_n|^2
(the derivative is a mathematical identity, independent of how either is coded)."""
import numpy as np
import pytest

from oracle.oracle import OracleSim
from paper_2305_13419_amd import workloads

MU0 = 1.25663706212e-6


def build(wl, maps, f0, src=True):
    pml = wl["pml"]
    o = OracleSim(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], pml=[0 if p is None else 1 for p in pml],
                  npml=[(0, 0) if p is None else p for p in pml])
    o.set_materials(*maps)
    E, H, J = wl["fields"]
    o.set_fields(E, [h * MU0 for h in H], J)
    if src:
        o.add_source(1, (5, 6, 0, wl["shape"][1], 2, 5), 1.0, 2, 3e14, 1e-15, 5e-16)
    pid = o.add_probe(1, (8, 9, 0, wl["shape"][1], 0, wl["shape"][2]), 1, [f0])
    return o, pid


@pytest.mark.parametrize("pml,theta", [(((3, 3), None, (2, 2)), 0.7), ((None, None, None), 1.0),
                                       ((None, (2, 2), None), 0.5)])
def test_oracle_adjoint_matches_central_differences(pml, theta):
    f0, N = 2.5e14, 50
    wl = workloads.random_medium((12, 6, 8), seed=31, pml=pml, theta=theta)
    o, pid = build(wl, wl["maps"], f0)
    J, F, gl, gs = o.adjoint(N, pid, f0)
    assert abs(J - abs(F) ** 2) <= 1e-14 * J
    rng = np.random.default_rng(5)
    for g, mi, ref in ((gl, 2, 1e14), (gs, 1, 1e4)):
        m = wl["maps"][mi]
        big = np.argwhere(np.abs(g) >= 1e-2 * np.abs(g).max())
        for c in big[rng.choice(len(big), min(8, len(big)), replace=False)]:
            c = tuple(c)
            h = 1e-6 * max(abs(m[c]), ref)
            vals = []
            for sgn in (1, -1):
                maps = [x.copy() for x in wl["maps"]]
                maps[mi][c] += sgn * h
                o2, p2 = build(wl, maps, f0)
                o2.step(N)
                vals.append(abs(o2.probe(p2)[1][0]) ** 2)
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(g[c] - fd) <= 1e-5 * abs(fd), (mi, c, g[c], fd)
    # cells without superconductivity get no inv_lambda2 gradient (fixed classification)
    assert np.all(gl[wl["maps"][2] == 0] == 0.0)


@pytest.mark.parametrize("pml,theta,N", [((None, None, None), 1.0, 1), ((None, None, None), 0.5, 1),
                                         ((None, None, None), 0.7, 23), (((0, 0), None, (0, 0)), 1.0, 17)])
def test_oracle_adjoint_dot_product(pml, theta, N):
    """Dot-product test of the reverse sweep over one step and over N steps: without sources F is linear
    in the initial state x = (E^0, B^0, Js^0), so the adjoint g = dJ/dx at x0 must satisfy
    <g, d> = 2 Re(conj(F(x0)) F(d)) for any direction d, F(d) being a forward run started from d.  This
    is the transpose identity <M^T y, d> = <y, M d> of the whole linear map, exact up to rounding (no
    finite-difference error); periodic grids and PEC walls (the CPML transpose is covered by the
    finite-difference test above)."""
    f0 = 2.5e14
    wl = workloads.random_medium((11, 6, 9), seed=37, pml=pml, theta=theta)
    o, pid = build(wl, wl["maps"], f0, src=False)
    J, F0, gl, gs, aE, aB, aJ = o.adjoint_state(N, pid, f0)
    assert abs(J - abs(F0) ** 2) <= 1e-14 * J
    rng = np.random.default_rng(9)
    sc = [np.asarray(e) > 0 for e in o.edge_materials()[2]]
    for trial in range(3):
        dE = [rng.standard_normal(o.shape3) for _ in range(3)]
        dB = [rng.standard_normal(o.shape3) * MU0 / 377.0 for _ in range(3)]
        dJ = [np.where(sc[c], 1e3 * rng.standard_normal(o.shape3), 0.0) for c in range(3)]
        o2 = OracleSim(wl["shape"], wl["spacing"], wl["dt"], wl["theta"],
                       pml=[0 if p is None else 1 for p in pml], npml=[(0, 0) if p is None else p for p in pml])
        o2.set_materials(*wl["maps"])
        o2.set_fields(dE, dB, dJ)
        p2 = o2.add_probe(1, (8, 9, 0, wl["shape"][1], 0, wl["shape"][2]), 1, [f0])
        o2.step(N)
        Fd = o2.probe(p2)[1][0]
        lhs = sum(float(np.sum(a * b)) for a, b in zip(aE + aB + aJ, dE + dB + dJ))
        rhs = 2.0 * (np.conj(F0) * Fd).real
        terms = sum(float(np.sum(np.abs(a * b))) for a, b in zip(aE + aB + aJ, dE + dB + dJ))
        assert abs(lhs - rhs) <= 1e-13 * terms, (trial, lhs, rhs, terms)
        assert abs(rhs) > 1e-6 * terms  # the identity is not trivially 0 = 0
