"""Adjoint (reverse-time) gradients of the HIP path against the oracle's adjoint
and against central finite differences of the HIP FP64 forward."""
import numpy as np
import pytest

from oracle.oracle import OracleSim
from paper_2305_13419_amd import workloads
from tests.helpers import MU0, WAVE_KIND, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def gpu_adjoint(wl, objective, N, seg, dtype, maps=None, edge_classes=True, fused=True):
    from paper_2305_13419_amd import Simulation
    npdt = np.float64 if dtype == torch.float64 else np.float32
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype, wl["pml"], edge_classes=edge_classes,
                     fused=fused)
    sim.set_materials(*[np.asarray(m, dtype=npdt) for m in (maps or wl["maps"])])
    if wl["fields"] is None:
        z = [np.zeros(sim.shape3, dtype=npdt)] * 3
        sim.set_fields(z, z, z)
    else:
        sim.set_fields(*[[np.asarray(a, dtype=npdt) for a in grp] for grp in wl["fields"]])
    for s in wl["sources"]:
        sim.add_source(**s)
    ckpt, snap, work = sim.adjoint_buffers(N, seg)
    F = sim.forward_checkpointed(objective, N, seg, ckpt)
    gl, gs = sim.adjoint(objective, N, seg, ckpt, F, snap, work)
    torch.cuda.synchronize()
    out = F, gl.cpu().numpy(), gs.cpu().numpy()
    sim.close()
    return out


def oracle_adjoint(wl, objective, N, npdt=np.float64):
    pml = wl["pml"]
    o = OracleSim(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], pml=[0 if p is None else 1 for p in pml],
                  npml=[(0, 0) if p is None else p for p in pml])
    o.set_materials(*[np.asarray(m, dtype=npdt).astype(np.float64) for m in wl["maps"]])
    sh = o.shape3
    if wl["fields"] is None:
        z = [np.zeros(sh)] * 3
        o.set_fields(z, z, z)
    else:
        E, H, J = [[np.asarray(a, dtype=npdt).astype(np.float64) for a in grp] for grp in wl["fields"]]
        o.set_fields(E, [h * MU0 for h in H], J)
    for s in wl["sources"]:
        o.add_source(s["comp"], s["box"], s["amplitude"], WAVE_KIND[s["waveform"]], s.get("freq", 0.0),
                     s.get("t0", 0.0), s.get("tw", 1.0))
    comp, box, f0 = objective
    pid = o.add_probe(comp, box, 1, [f0])
    return o.adjoint(N, pid, f0)


CASES = [
    dict(shape=(40, 9, 36), pml=(None, None, None), theta=1.0, fields=True, N=37, seg=8),
    dict(shape=(34, 12, 40), pml=((5, 5), None, (4, 4)), theta=0.5, fields=False, N=40, seg=40),
    dict(shape=(30, 14, 33), pml=((4, 3), (3, 4), (5, 2)), theta=0.7, fields=True, N=25, seg=1),
    dict(shape=(70, 6, 35), pml=((6, 6), None, None), theta=1.0, fields=True, N=30, seg=7),
]


def make_case(c, seed=41):
    wl = workloads.random_medium(c["shape"], seed=seed, pml=c["pml"], theta=c["theta"])
    if not c["fields"]:
        wl["fields"] = None
    nx, ny, nz = c["shape"]
    wl["sources"] = [dict(comp=1, box=(nx // 3, nx // 3 + 1, 0, ny, nz // 4, nz // 2), amplitude=2.0,
                          waveform="mod_gauss", freq=3e14, t0=1.5e-15, tw=6e-16)]
    objective = (1, (2 * nx // 3, 2 * nx // 3 + 1, 0, ny, 0, nz), 2.5e14)
    return wl, objective


@pytest.mark.parametrize("case", range(len(CASES)))
def test_adjoint_fp64_matches_oracle_adjoint(case):
    c = CASES[case]
    wl, obj = make_case(c)
    print(f"case {case}: {c}", flush=True)
    F, gl, gs = gpu_adjoint(wl, obj, c["N"], c["seg"], torch.float64)
    Jo, Fo, glo, gso = oracle_adjoint(wl, obj, c["N"])
    print(f"  F rel {abs(F - Fo) / abs(Fo):.2e}  grad ell {rel_l2(gl, glo):.2e}  grad sigma {rel_l2(gs, gso):.2e}",
          flush=True)
    assert abs(F - Fo) <= 1e-12 * abs(Fo)
    assert rel_l2(gl, glo) <= 1e-10
    assert rel_l2(gs, gso) <= 1e-10
    assert np.all(gl[wl["maps"][2] == 0] == 0.0)


def test_adjoint_fp32_close_to_oracle():
    c = CASES[0]
    wl, obj = make_case(c)
    F, gl, gs = gpu_adjoint(wl, obj, c["N"], c["seg"], torch.float32)
    Jo, Fo, glo, gso = oracle_adjoint(wl, obj, c["N"], np.float32)
    print(f"FP32: F rel {abs(F - Fo) / abs(Fo):.2e} grad ell {rel_l2(gl, glo):.2e} grad sigma {rel_l2(gs, gso):.2e}",
          flush=True)
    assert abs(F - Fo) <= 1e-5 * abs(Fo)
    assert rel_l2(gl, glo) <= 1e-4
    assert rel_l2(gs, gso) <= 1e-4


def test_autograd_function_and_finite_differences():
    """TwoFluidObjective returns J and, in backward, the adjoint gradients; they match central
    differences of the HIP FP64 forward on superconducting cells (ell) and on any cell (sigma)."""
    from paper_2305_13419_amd import AdjointProblem, TwoFluidObjective
    c = CASES[1]
    wl, obj = make_case(c)
    eps, sig, ell = wl["maps"]
    prob = AdjointProblem(wl["shape"], wl["spacing"], wl["dt"], eps, obj, c["N"], seg=10, theta=c["theta"],
                          pml=c["pml"], sources=wl["sources"])
    L = torch.tensor(ell, device="cuda", requires_grad=True)
    S = torch.tensor(sig, device="cuda", requires_grad=True)
    J = TwoFluidObjective.apply(L, S, prob)
    J.backward()
    gl, gs = L.grad.cpu().numpy(), S.grad.cpu().numpy()
    Jo, Fo, glo, gso = oracle_adjoint(wl, obj, c["N"])
    assert abs(J.item() / Jo - 1) < 1e-12
    assert rel_l2(gl, glo) <= 1e-10 and rel_l2(gs, gso) <= 1e-10
    rng = np.random.default_rng(4)
    worst = 0.0
    for g, m, ref, mi in ((gl, ell, 1e14, 0), (gs, sig, 1e4, 1)):
        # cells whose map value stays non-negative under -h (sigma = 0 cells are excluded)
        big = np.argwhere((np.abs(g) >= 1e-2 * np.abs(g).max()) & (m > 2e-6 * np.maximum(m, ref)))
        for cell in big[rng.choice(len(big), 6, replace=False)]:
            cell = tuple(cell)
            h = 1e-6 * max(abs(m[cell]), ref)
            vals = []
            for sgn in (1, -1):
                mm = [ell.copy(), sig.copy()]
                mm[mi][cell] += sgn * h
                vals.append(prob.forward(torch.tensor(mm[0], device="cuda"), torch.tensor(mm[1], device="cuda")))
            fd = (vals[0] - vals[1]) / (2 * h)
            worst = max(worst, abs(g[cell] - fd) / abs(fd))
    print(f"max relative FD error {worst:.2e}", flush=True)
    assert worst <= 1e-4


@pytest.mark.parametrize("seg,seg2", [(16, 5), (40, 40), (9, 1)])
def test_nested_schedule_equals_two_level(seg, seg2):
    """Three-level checkpointing recomputes the same forward states: gradients equal the two-level ones
    bit for bit, and the oracle adjoint to 1e-10."""
    from paper_2305_13419_amd import Simulation
    c = CASES[2]
    wl, obj = make_case(c)
    N = 37
    F, gl, gs = gpu_adjoint(wl, obj, N, seg, torch.float64)
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], torch.float64, wl["pml"])
    sim.set_materials(*wl["maps"])
    sim.set_fields(*wl["fields"])
    for s in wl["sources"]:
        sim.add_source(**s)
    ckpt, ckpt2, snap, work = sim.adjoint_nested_buffers(N, seg, seg2)
    F2 = sim.forward_checkpointed(obj, N, seg, ckpt)
    gl2, gs2 = sim.adjoint_nested(obj, N, seg, seg2, ckpt, F2, ckpt2, snap, work)
    gl2, gs2 = gl2.cpu().numpy(), gs2.cpu().numpy()
    sim.close()
    assert F2 == F
    assert np.array_equal(gl2, gl) and np.array_equal(gs2, gs)
    Jo, Fo, glo, gso = oracle_adjoint(wl, obj, N)
    assert rel_l2(gl2, glo) <= 1e-10 and rel_l2(gs2, gso) <= 1e-10


def test_adjoint_rejects_stale_checkpoints():
    """A checkpointed run is invalidated by new maps or sources, and its reverse sweep needs the same
    objective: each mismatch returns TFL_E_STATE instead of a gradient of another run."""
    from paper_2305_13419_amd import Simulation, _lib as L
    c = CASES[0]
    wl, obj = make_case(c)
    N, seg = 12, 4
    sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], torch.float64, wl["pml"])

    def fresh_run():
        sim.set_materials(*wl["maps"])
        sim.set_fields(*wl["fields"])
        return sim.forward_checkpointed(obj, N, seg, ckpt)

    for s in wl["sources"]:
        sim.add_source(**s)
    ckpt, snap, work = sim.adjoint_buffers(N, seg)
    F = fresh_run()
    gl, gs = sim.adjoint(obj, N, seg, ckpt, F, snap, work)  # the matching call works
    assert np.isfinite(gl.cpu().numpy()).all()

    def expect_state(fn):
        with pytest.raises(L.TflError) as err:
            fn()
        assert err.value.code == L.TFL_E_STATE, err.value

    # another objective frequency, box or component
    for other in ((obj[0], obj[1], obj[2] * 1.01), (obj[0], (0, 1) + tuple(obj[1][2:]), obj[2]),
                  ((obj[0] + 1) % 3, obj[1], obj[2])):
        expect_state(lambda: sim.adjoint(other, N, seg, ckpt, F, snap, work))
    # new maps after the run
    F = fresh_run()
    sim.set_materials(*wl["maps"])
    expect_state(lambda: sim.adjoint(obj, N, seg, ckpt, F, snap, work))
    # a new source after the run
    F = fresh_run()
    sim.add_source(**wl["sources"][0])
    expect_state(lambda: sim.adjoint(obj, N, seg, ckpt, F, snap, work))
    # sources cleared after the run
    F = fresh_run()
    sim._call("tfl_clear_sources_probes")
    expect_state(lambda: sim.adjoint(obj, N, seg, ckpt, F, snap, work))
    sim.close()


def test_autograd_rejects_backward_after_a_later_forward():
    """Two applies on one AdjointProblem: the later graph's backward gives the oracle gradient of its
    own maps; the earlier graph's backward raises instead of returning the later run's gradient."""
    from paper_2305_13419_amd import AdjointProblem, TwoFluidObjective
    c = CASES[1]
    wl, obj = make_case(c)
    eps, sig, ell = wl["maps"]
    prob = AdjointProblem(wl["shape"], wl["spacing"], wl["dt"], eps, obj, c["N"], seg=10, theta=c["theta"],
                          pml=c["pml"], sources=wl["sources"])
    L1 = torch.tensor(ell, device="cuda", requires_grad=True)
    S1 = torch.tensor(sig, device="cuda", requires_grad=True)
    J1 = TwoFluidObjective.apply(L1, S1, prob)
    ell2 = ell * 1.1
    L2 = torch.tensor(ell2, device="cuda", requires_grad=True)
    S2 = torch.tensor(sig, device="cuda", requires_grad=True)
    J2 = TwoFluidObjective.apply(L2, S2, prob)
    J2.backward()
    wl2 = dict(wl)
    wl2["maps"] = (eps, sig, ell2)
    Jo, Fo, glo, gso = oracle_adjoint(wl2, obj, c["N"])
    assert abs(J2.item() / Jo - 1) < 1e-12
    assert rel_l2(L2.grad.cpu().numpy(), glo) <= 1e-10 and rel_l2(S2.grad.cpu().numpy(), gso) <= 1e-10
    with pytest.raises(RuntimeError, match="another forward pass"):
        J1.backward()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_two_step_sweep_in_checkpointed_forward_and_nested_recomputation(dtype):
    """Where the two-step sweep runs (forced here on a small CPML grid with edge classes) it serves the
    checkpointed forward, the objective probe folded into it, and the three-level schedule's outer
    recomputation, with the sources only: objective and gradients equal those of the fused sweep bit
    for bit."""
    from paper_2305_13419_amd import Simulation
    c = dict(shape=(130, 20, 40), pml=((5, 4), None, (3, 6)), theta=1.0, fields=True)
    wl, obj = make_case(c)
    wl["maps"] = workloads.roofline_grid(c["shape"])["maps"]  # few distinct materials: edge classes bind
    npdt = np.float64 if dtype == torch.float64 else np.float32
    N, seg, seg2 = 40, 20, 8
    res = {}
    for sweep in ("two_step", "fused"):
        print(f"case: checkpointed forward and nested adjoint, sweep={sweep}, {dtype}", flush=True)
        sim = Simulation(wl["shape"], wl["spacing"], wl["dt"], wl["theta"], dtype, wl["pml"])
        sim.set_materials(*[np.asarray(m, dtype=npdt) for m in wl["maps"]])
        assert sim.edge_classes > 0
        sim.set_fields(*[[np.asarray(a, dtype=npdt) for a in grp] for grp in wl["fields"]])
        for s in wl["sources"]:
            sim.add_source(**s)
        sim.set_sweep(sweep)
        ckpt, ckpt2, snap, work = sim.adjoint_nested_buffers(N, seg, seg2)
        F = sim.forward_checkpointed(obj, N, seg, ckpt)
        forward_counts = sim.sweep_counts()
        gl, gs = sim.adjoint_nested(obj, N, seg, seg2, ckpt, F, ckpt2, snap, work)
        torch.cuda.synchronize()
        res[sweep] = (F, gl.cpu().numpy(), gs.cpu().numpy(), forward_counts, sim.sweep_counts())
        sim.close()
    two, fused = res["two_step"], res["fused"]
    assert two[3][2] == N and fused[3][2] == 0, (two[3], fused[3])  # the forward's segments, 5 x 4 steps each
    assert two[4][2] > two[3][2], two[4]  # the outer recomputation too
    assert two[0] == fused[0]
    assert np.array_equal(two[1], fused[1]) and np.array_equal(two[2], fused[2])
