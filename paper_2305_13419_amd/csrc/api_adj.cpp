// C ABI of the adjoint: checkpointed forward run and the reverse sweep.
// All device work runs in kernels_fwd.hip and kernels_adj.hip.
#include <cmath>
#include <cstring>

#include "sim_internal.h"

using namespace tfl;
using namespace tfl::detail;

namespace {

struct AdjLayout {
    size_t field = 0;   // bytes of one field component, 256-aligned
    size_t grad = 0;    // bytes of one FP64 per-edge accumulator, 256-aligned
    size_t psi = 0;     // bytes of the PML adjoint variables
    size_t total = 0;
};

AdjLayout adj_layout(const tfl_sim *s)
{
    AdjLayout L;
    L.field = round256((size_t)s->N * s->esz);
    L.grad = round256((size_t)s->N * 8);
    for (int a = 0; a < 3; ++a) L.psi += round256(4 * s->psi_count[a] * s->esz);
    L.total = (9 + 3 * kGradWindow) * L.field + L.psi + 6 * L.grad;
    return L;
}

size_t state_bytes(const tfl_sim *s) { return 9 * round256((size_t)s->N * s->esz) + round256(s->work_bytes); }

int check_obj(tfl_sim *s, const tfl_objective *o)
{
    if (!o) return fail(s, TFL_E_INVAL, "null objective");
    if (o->comp < 0 || o->comp > 2) return fail(s, TFL_E_INVAL, "objective component must be 0..2");
    if (!box_ok(s->cfg, o->box)) return fail(s, TFL_E_INVAL, "objective box outside the grid or empty");
    if (!std::isfinite(o->f0)) return fail(s, TFL_E_INVAL, "objective frequency must be finite");
    return TFL_OK;
}

// The objective of the reverse sweep must be the one the checkpointed run accumulated F for.
bool same_objective(const tfl_objective &a, const tfl_objective &b)
{
    if (a.comp != b.comp || a.f0 != b.f0) return false;
    for (int q = 0; q < 6; ++q)
        if (a.box[q] != b.box[q]) return false;
    return true;
}

ProbeDesc objective_probe(const tfl_objective *o, double *dft)
{
    ProbeDesc d{};
    d.comp = o->comp;
    d.i0 = (int)o->box[0]; d.i1 = (int)o->box[1];
    d.j0 = (int)o->box[2]; d.j1 = (int)o->box[3];
    d.k0 = (int)o->box[4]; d.k1 = (int)o->box[5];
    d.series = nullptr;
    d.cap = 0;
    d.nfreq = 1;
    d.freq[0] = o->f0;
    d.dft = dft;
    return d;
}

template <typename T>
int forward_ckpt(tfl_sim *s, const tfl_objective *o, int64_t nsteps, int64_t seg, void *ckpt, double F[2],
                 hipStream_t st)
{
    double *dft = s->scratch + kObjectiveSlot;
    hipError_t e = launch_fill_zero(dft, 2 * sizeof(double), st);
    if (e != hipSuccess) return hip_fail(s, e, "objective clear");
    const int64_t n0 = s->step;
    const bool first = (n0 == 0 && !s->sampled0);
    s->probe.push_back(objective_probe(o, dft));
    s->probes_dirty = true;
    // sample at n0: every probe if this is the first sample of the run, else the objective only
    {
        int rc0 = upload_probes(s, st);
        ProbeArgs<T> pa{};
        const StepArgs<T> a = make_args<T>(s);
        pa.g = a.g;
        for (int q = 0; q < 3; ++q) pa.E[q] = a.E[q];
        pa.dt = s->cfg.dt;
        pa.n = n0;
        pa.p = (const ProbeDesc *)((const char *)s->scratch + kProbeDescOffset);
        const int np = (int)s->probe.size();
        pa.first = first ? 0 : np - 1;
        if (rc0 == TFL_OK && (e = launch_probes<T>(pa, first ? np : 1, st)) != hipSuccess)
            rc0 = hip_fail(s, e, "objective sample");
        if (rc0 != TFL_OK) {
            s->probe.pop_back();
            s->probes_dirty = true;
            return rc0;
        }
        s->sampled0 = true;
    }
    const size_t sb = state_bytes(s);
    int rc = TFL_OK;
    const int64_t nseg = (nsteps + seg - 1) / seg;
    for (int64_t g = 0; g < nseg && rc == TFL_OK; ++g) {
        rc = copy_state(s, (char *)ckpt + (size_t)g * sb, nullptr, true, st);
        if (rc != TFL_OK) break;
        const int64_t len = std::min(seg, nsteps - g * seg);
        rc = do_step<T>(s, len, st);
    }
    s->probe.pop_back();
    s->probes_dirty = true;
    if (rc != TFL_OK) return rc;
    e = hipMemcpyAsync(F, dft, 2 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(s, e, "objective readback");
    s->ckpt_valid = true;
    s->ckpt_obj = *o;
    s->ckpt_n0 = n0;
    s->ckpt_nsteps = nsteps;
    s->ckpt_seg = seg;
    return TFL_OK;
}

template <typename T>
struct Reverse {
    tfl_sim *s;
    const tfl_objective *o;
    const double *F;
    AdjArgs<T> A;
    void *snap;
    size_t fb;
    int64_t n0, nend;
    hipStream_t st;

    T *snapE(int64_t t, int q) const { return (T *)((char *)snap + ((size_t)t * 3 + q) * fb); }
    static T *snapIn(void *buf, size_t fb, int64_t t, int q) { return (T *)((char *)buf + ((size_t)t * 3 + q) * fb); }

    // mu of the edge sweeps, one set of three fields per step of a window; the window's sigma
    // gradient is added when it is full and at the end of every range (before the snapshots are
    // overwritten)
    char *mu_base = nullptr;
    size_t field = 0;
    GradSigmaArgs<T> G{};

    void set_mu_slot(int w)
    {
        for (int q = 0; q < 3; ++q) A.mu[q] = (T *)(mu_base + ((size_t)w * 3 + q) * field);
    }

    int flush_grad_sigma()
    {
        hipError_t e = launch_adj_grad_sigma<T>(G, st);
        G.nwin = 0;
        if (e != hipSuccess) return hip_fail(s, e, "sigma gradient");
        return TFL_OK;
    }

    double objective_coef(int64_t n) const
    {
        const double ph = kTwoPi * o->f0 * (double)n * s->cfg.dt;
        return 2.0 * s->cfg.dt * (F[0] * std::cos(ph) - F[1] * std::sin(ph));
    }

    // Reverse sweep over the forward steps [s0, s0 + len) from the saved state at s0: recompute the
    // range writing E^{s0+t} into snapshot t, then the adjoint sweeps CA(s0+len) [with doC unless the
    // range ends the run], (B(n), CA(n)) for n = s0+len-1 .. s0+1, and B(s0); the range starting the
    // run also does CA(n0) (no edge-local part) and the initial half-kick gradient.  CA(s0) of a later
    // range is the first kernel of the range before it.
    int range(int64_t s0, int64_t len, const void *state_s0)
    {
        const int rc = recompute(s0, len, state_s0, snap, st);
        return rc != TFL_OK ? rc : reverse(s0, len);
    }

    // The recomputation of the forward steps [s0, s0 + len) from the saved state at s0 on stream rs,
    // writing E^{s0+t} into snapshot t of buf.
    int recompute(int64_t s0, int64_t len, const void *state_s0, void *buf, hipStream_t rs)
    {
        hipError_t e;
        int rc = copy_state(s, nullptr, state_s0, false, rs);
        if (rc != TFL_OK) return rc;
        for (int q = 0; q < 3; ++q) {
            e = hipMemcpyAsync(snapIn(buf, fb, 0, q), s->E[q], (size_t)s->N * s->esz, hipMemcpyDeviceToDevice, rs);
            if (e != hipSuccess) return hip_fail(s, e, "snapshot");
        }
        StepArgs<T> f = make_args<T>(s);
        source_boxes(s, f.side);
        const double dt = s->cfg.dt;
        // With the fused buffer bound the recomputation runs the fused sweep: E goes from snapshot t
        // to snapshot t + 1 as in the two passes, H and the H-side CPML variables alternate between
        // the bound set (even t) and the buffer (odd t).
        const bool fused = s->fused != nullptr;
        StepArgs<T> fo = f, fe = f;  // odd t: buffer -> bound set; even t: bound set -> buffer
        if (fused) {
            size_t psi_at[3];
            const size_t fst = fused_layout(s, psi_at);
            for (int q = 0; q < 3; ++q) {
                T *hb = (T *)((char *)s->fused + (3 + q) * fst);
                fe.Hout[q] = hb;
                fo.H[q] = hb;
                fo.Hout[q] = f.H[q];
            }
            for (int ax = 0; ax < 3; ++ax) {
                if (!f.pml[ax].on || s->psi_count[ax] == 0) continue;
                T *pb = (T *)((char *)s->fused + psi_at[ax]);
                const size_t m = s->psi_count[ax];
                fe.pml[ax].psiHo[0] = pb;
                fe.pml[ax].psiHo[1] = pb + m;
                fo.pml[ax].psiH[0] = pb;
                fo.pml[ax].psiH[1] = pb + m;
                fo.pml[ax].psiHo[0] = f.pml[ax].psiH[0];
                fo.pml[ax].psiHo[1] = f.pml[ax].psiH[1];
            }
        }
        for (int64_t t = 0; t < len; ++t) {
            StepArgs<T> &g = fused ? ((t & 1) ? fo : fe) : f;
            for (int q = 0; q < 3; ++q) {
                g.E[q] = snapIn(buf, fb, t, q);
                g.Eout[q] = snapIn(buf, fb, t + 1, q);
            }
            source_values(s, g.side, (double)(s0 + t + 1) * dt);
            if (fused) {
                if ((e = launch_fused_step<T>(g, rs)) != hipSuccess) return hip_fail(s, e, "recompute fused step");
            } else {
                if ((e = launch_h_pass<T>(g, rs)) != hipSuccess) return hip_fail(s, e, "recompute h_pass");
                if ((e = launch_e_pass<T>(g, rs)) != hipSuccess) return hip_fail(s, e, "recompute e_pass");
            }
        }
        s->step = s0 + len;
        return TFL_OK;
    }

    // The adjoint sweeps over the recomputed range [s0, s0 + len) (snapshots in snap) on stream st.
    int reverse(int64_t s0, int64_t len)
    {
        hipError_t e;
        int rc = TFL_OK;
        const double dt = s->cfg.dt;
        const int64_t end = s0 + len;
        for (int64_t n = end; n >= s0 + 1; --n) {
            if (n != end && (e = launch_adj_faces<T>(A, st)) != hipSuccess) return hip_fail(s, e, "adjoint faces");
            if (G.nwin == kGradWindow && (rc = flush_grad_sigma()) != TFL_OK) return rc;
            source_values(s, A.f.side, (double)n * dt);
            A.doC = (n != nend);
            A.doA = 1;
            A.obj = 1;
            A.og = objective_coef(n);
            for (int q = 0; q < 3; ++q) A.En[q] = snapE(n - 1 - s0, q);
            // this step's mu goes to slot nwin of the window, read by the next face sweep and then by
            // the window's sigma gradient together with E^{m+1}, E^m and the step's source values
            const int w = G.nwin++;
            set_mu_slot(w);
            for (int q = 0; q < 3; ++q) {
                G.mu[w][q] = A.mu[q];
                G.Ep[w][q] = snapE(n - s0, q);
                G.En[w][q] = (A.f.theta == T(1)) ? nullptr : snapE(n - 1 - s0, q);
            }
            for (int p = 0; p < G.nsrc; ++p) G.sg[w][p] = A.f.side.sg[p];
            if ((e = launch_adj_edges<T>(A, st)) != hipSuccess) return hip_fail(s, e, "adjoint edges");
        }
        if ((e = launch_adj_faces<T>(A, st)) != hipSuccess) return hip_fail(s, e, "adjoint faces");
        if ((rc = flush_grad_sigma()) != TFL_OK) return rc;
        if (s0 == n0) {
            A.doC = 1;
            A.doA = 0;
            A.obj = 1;
            A.og = objective_coef(n0);
            if ((e = launch_adj_edges<T>(A, st)) != hipSuccess) return hip_fail(s, e, "adjoint edges");
            for (int q = 0; q < 3; ++q) A.En[q] = snapE(0, q);
            if ((e = launch_adj_initial_kick<T>(A, st)) != hipSuccess) return hip_fail(s, e, "adjoint kick");
        }
        return TFL_OK;
    }
};

template <typename T>
int make_reverse(tfl_sim *s, const tfl_objective *o, const double F[2], void *snap, void *adj, hipStream_t st,
                 Reverse<T> &R)
{
    const AdjLayout L = adj_layout(s);
    hipError_t e = launch_fill_zero(adj, L.total, st);
    if (e != hipSuccess) return hip_fail(s, e, "adjoint clear");
    R.s = s;
    R.o = o;
    R.F = F;
    R.snap = snap;
    R.st = st;
    R.fb = round256((size_t)s->N * s->esz);
    R.n0 = s->ckpt_n0;
    R.nend = s->ckpt_n0 + s->ckpt_nsteps;
    AdjArgs<T> &A = R.A;
    A = AdjArgs<T>{};
    A.f = make_args<T>(s);
    char *p = (char *)adj;
    for (int q = 0; q < 3; ++q) { A.lE[q] = (T *)p; p += L.field; }
    for (int q = 0; q < 3; ++q) { A.lH[q] = (T *)p; p += L.field; }
    for (int q = 0; q < 3; ++q) { A.lJ[q] = (T *)p; p += L.field; }
    R.mu_base = p;
    R.field = L.field;
    R.set_mu_slot(0);
    p += (size_t)kGradWindow * 3 * L.field;
    for (int a = 0; a < 3; ++a) {
        const size_t m = s->psi_count[a] * s->esz;
        if (s->cfg.bc[a] == TFL_CPML) {
            A.lpsiH[a][0] = (T *)p; A.lpsiH[a][1] = (T *)(p + m);
            A.lpsiE[a][0] = (T *)(p + 2 * m); A.lpsiE[a][1] = (T *)(p + 3 * m);
        }
        p += round256(4 * m);
    }
    for (int q = 0; q < 3; ++q) { A.gL[q] = (double *)p; p += L.grad; }
    for (int q = 0; q < 3; ++q) { A.gS[q] = (double *)p; p += L.grad; }
    A.ocomp = o->comp;
    for (int q = 0; q < 6; ++q) A.ob[q] = (int)o->box[q];
    source_boxes(s, A.f.side);
    GradSigmaArgs<T> &G = R.G;
    G = GradSigmaArgs<T>{};
    G.g = A.f.g;
    for (int q = 0; q < 3; ++q) G.gS[q] = A.gS[q];
    G.theta = (double)A.f.theta;
    G.nsrc = A.f.side.nsrc;
    for (int q = 0; q < G.nsrc; ++q)
        for (int c = 0; c < 7; ++c) G.sbox[q][c] = A.f.side.sbox[q][c];
    return TFL_OK;
}

template <typename T>
int adjoint(tfl_sim *s, const tfl_objective *o, int64_t nsteps, int64_t seg, const void *ckpt, const double F[2],
            void *snap, void *adj, double *grad_ell, double *grad_sig, hipStream_t st)
{
    Reverse<T> R;
    int rc = make_reverse<T>(s, o, F, snap, adj, st, R);
    if (rc != TFL_OK) return rc;
    const size_t sb = state_bytes(s);
    const int64_t nseg = (nsteps + seg - 1) / seg;
    // Two snapshot sets: segment g's recomputation (into set g mod 2, on a second stream) runs while
    // the adjoint sweeps of segment g + 1 (on `st`) read the other set.  The recomputation of g waits
    // for the sweeps of g + 2 (same set); the sweeps of g wait for the recomputation of g.
    const size_t set_bytes = (size_t)(std::min(seg, nsteps) + 1) * 3 * R.fb;
    auto set = [&](int64_t g) { return (void *)((char *)snap + (size_t)(g & 1) * set_bytes); };
    auto state = [&](int64_t g) { return (const void *)((const char *)ckpt + (size_t)g * sb); };
    auto first = [&](int64_t g) { return R.n0 + g * seg; };
    auto length = [&](int64_t g) { return std::min(seg, R.nend - first(g)); };
    hipStream_t rs = nullptr;
    hipEvent_t ev[5] = {};  // recomputation of set 0 / 1 done, sweeps over set 0 / 1 done, `st` ready
    hipError_t e = hipStreamCreateWithFlags(&rs, hipStreamNonBlocking);
    for (int q = 0; q < 5 && e == hipSuccess; ++q) e = hipEventCreateWithFlags(&ev[q], hipEventDisableTiming);
    // everything issued on `st` so far (the cleared workspace, the caller's state) before the second stream
    if (e == hipSuccess) e = hipEventRecord(ev[4], st);
    if (e == hipSuccess) e = hipStreamWaitEvent(rs, ev[4], 0);
    if (e != hipSuccess) rc = hip_fail(s, e, "recomputation stream");
    if (rc == TFL_OK) rc = R.recompute(first(nseg - 1), length(nseg - 1), state(nseg - 1), set(nseg - 1), rs);
    if (rc == TFL_OK && (e = hipEventRecord(ev[(nseg - 1) & 1], rs)) != hipSuccess) rc = hip_fail(s, e, "event");
    for (int64_t g = nseg - 1; g >= 0 && rc == TFL_OK; --g) {
        if (g >= 1) {  // the next recomputation, once the sweeps that last read its set are done
            if (g + 1 <= nseg - 1 && (e = hipStreamWaitEvent(rs, ev[2 + ((g + 1) & 1)], 0)) != hipSuccess) {
                rc = hip_fail(s, e, "event");
                break;
            }
            if ((rc = R.recompute(first(g - 1), length(g - 1), state(g - 1), set(g - 1), rs)) != TFL_OK) break;
            if ((e = hipEventRecord(ev[(g - 1) & 1], rs)) != hipSuccess) {
                rc = hip_fail(s, e, "event");
                break;
            }
        }
        if ((e = hipStreamWaitEvent(st, ev[g & 1], 0)) != hipSuccess) {
            rc = hip_fail(s, e, "event");
            break;
        }
        R.snap = set(g);
        if ((rc = R.reverse(first(g), length(g))) != TFL_OK) break;
        if ((e = hipEventRecord(ev[2 + (g & 1)], st)) != hipSuccess) rc = hip_fail(s, e, "event");
    }
    // `st` has waited for every recomputation (the last one before the last sweeps); on an error, the
    // second stream's work is waited for before its stream and events go
    if (rc != TFL_OK && rs) (void)hipStreamSynchronize(rs);
    if (rs) (void)hipStreamDestroy(rs);
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (rc != TFL_OK) return rc;
    e = launch_adj_edge_to_cell<T>(R.A, grad_ell, grad_sig, st);
    if (e != hipSuccess) return hip_fail(s, e, "gradient to cells");
    return TFL_OK;
}

// Three levels: the outer checkpoints of the forward run every seg steps; each outer segment is
// recomputed saving inner checkpoints every seg2 steps into ckpt2; each inner segment is recomputed
// into the snapshots and swept backwards.
template <typename T>
int adjoint_nested(tfl_sim *s, const tfl_objective *o, int64_t nsteps, int64_t seg, const void *ckpt,
                   const double F[2], int64_t seg2, void *ckpt2, void *snap, void *adj, double *grad_ell,
                   double *grad_sig, hipStream_t st)
{
    Reverse<T> R;
    int rc = make_reverse<T>(s, o, F, snap, adj, st, R);
    if (rc != TFL_OK) return rc;
    const size_t sb = state_bytes(s);
    const int64_t nseg = (nsteps + seg - 1) / seg;
    for (int64_t g = nseg - 1; g >= 0; --g) {
        const int64_t s0 = R.n0 + g * seg;
        const int64_t len = std::min(seg, R.nend - s0);
        const int64_t nin = (len + seg2 - 1) / seg2;
        if ((rc = copy_state(s, nullptr, (const char *)ckpt + (size_t)g * sb, false, st)) != TFL_OK) return rc;
        s->step = s0;
        for (int64_t h = 0; h < nin; ++h) {
            if ((rc = copy_state(s, (char *)ckpt2 + (size_t)h * sb, nullptr, true, st)) != TFL_OK) return rc;
            const int64_t l2 = std::min(seg2, len - h * seg2);
            if (h + 1 < nin && (rc = do_step<T>(s, l2, st, nullptr, false)) != TFL_OK) return rc;
        }
        for (int64_t h = nin - 1; h >= 0; --h) {
            const int64_t m0 = s0 + h * seg2;
            const int64_t l2 = std::min(seg2, len - h * seg2);
            if ((rc = R.range(m0, l2, (const char *)ckpt2 + (size_t)h * sb)) != TFL_OK) return rc;
        }
    }
    hipError_t e = launch_adj_edge_to_cell<T>(R.A, grad_ell, grad_sig, st);
    if (e != hipSuccess) return hip_fail(s, e, "gradient to cells");
    return TFL_OK;
}

}  // namespace

extern "C" {

int tfl_adjoint_sizes(const tfl_sim *s, int64_t nsteps, int64_t seg, size_t *ckpt_bytes, size_t *snap_bytes,
                      size_t *adj_bytes)
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    if (nsteps < 1 || seg < 1) return fail(const_cast<tfl_sim *>(s), TFL_E_INVAL, "nsteps and seg must be >= 1");
    const int64_t nseg = (nsteps + seg - 1) / seg;
    const int64_t sl = std::min(seg, nsteps);
    if (ckpt_bytes) *ckpt_bytes = (size_t)nseg * state_bytes(s);
    // two snapshot sets: one segment's recomputation overlaps the previous segment's adjoint sweeps
    if (snap_bytes) *snap_bytes = 2 * (size_t)(sl + 1) * 3 * round256((size_t)s->N * s->esz);
    if (adj_bytes) *adj_bytes = adj_layout(s).total;
    return TFL_OK;
}

int tfl_forward_checkpointed(tfl_sim *s, const tfl_objective *obj, int64_t nsteps, int64_t seg, void *ckpt,
                             double F[2], void *stream)
{
    int rc = check_bound(s, true);
    if (rc != TFL_OK) return rc;
    if ((rc = check_obj(s, obj)) != TFL_OK) return rc;
    if (nsteps < 1 || seg < 1) return fail(s, TFL_E_INVAL, "nsteps and seg must be >= 1");
    if (!ckpt || !aligned(ckpt) || !F) return fail(s, TFL_E_INVAL, "checkpoint buffer must be aligned, F non-null");
    s->ckpt_valid = false;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = nonfinite_begin(s, st)) != TFL_OK) return rc;
    rc = s->esz == 8 ? forward_ckpt<double>(s, obj, nsteps, seg, ckpt, F, st)
                     : forward_ckpt<float>(s, obj, nsteps, seg, ckpt, F, st);
    const int rc2 = nonfinite_end(s, st);
    if (rc2 != TFL_OK) s->ckpt_valid = false;  // no gradient of a run that went non-finite
    return rc != TFL_OK ? rc : rc2;
}

int tfl_adjoint_nested_sizes(const tfl_sim *s, int64_t nsteps, int64_t seg, int64_t seg2, size_t *ckpt_bytes,
                             size_t *ckpt2_bytes, size_t *snap_bytes, size_t *adj_bytes)
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    if (nsteps < 1 || seg < 1 || seg2 < 1 || seg2 > seg)
        return fail(const_cast<tfl_sim *>(s), TFL_E_INVAL, "need nsteps, seg >= 1 and 1 <= seg2 <= seg");
    const int64_t sl = std::min(seg, nsteps), s2 = std::min(seg2, sl);
    if (ckpt_bytes) *ckpt_bytes = (size_t)((nsteps + seg - 1) / seg) * state_bytes(s);
    if (ckpt2_bytes) *ckpt2_bytes = (size_t)((sl + seg2 - 1) / seg2) * state_bytes(s);
    if (snap_bytes) *snap_bytes = (size_t)(s2 + 1) * 3 * round256((size_t)s->N * s->esz);
    if (adj_bytes) *adj_bytes = adj_layout(s).total;
    return TFL_OK;
}

int tfl_adjoint_nested(tfl_sim *s, const tfl_objective *obj, int64_t nsteps, int64_t seg, const void *ckpt,
                       const double F[2], int64_t seg2, void *ckpt2, void *snap, void *adj, double *grad_ell,
                       double *grad_sigma, void *stream)
{
    int rc = check_bound(s, true);
    if (rc != TFL_OK) return rc;
    if ((rc = check_obj(s, obj)) != TFL_OK) return rc;
    if (!s->ckpt_valid || s->ckpt_nsteps != nsteps || s->ckpt_seg != seg)
        return fail(s, TFL_E_STATE,
                    "no checkpointed forward run with these nsteps and seg since the maps or sources last changed");
    if (!same_objective(s->ckpt_obj, *obj))
        return fail(s, TFL_E_STATE, "objective differs from the one of the checkpointed forward run");
    if (seg2 < 1 || seg2 > seg) return fail(s, TFL_E_INVAL, "seg2 must lie in [1, seg]");
    if (!ckpt || !ckpt2 || !snap || !adj || !grad_ell || !grad_sigma || !F)
        return fail(s, TFL_E_INVAL, "null buffer");
    if (!aligned(ckpt) || !aligned(ckpt2) || !aligned(snap) || !aligned(adj) || !aligned(grad_ell) ||
        !aligned(grad_sigma))
        return fail(s, TFL_E_INVAL, "device buffers must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    return s->esz == 8
               ? adjoint_nested<double>(s, obj, nsteps, seg, ckpt, F, seg2, ckpt2, snap, adj, grad_ell, grad_sigma, st)
               : adjoint_nested<float>(s, obj, nsteps, seg, ckpt, F, seg2, ckpt2, snap, adj, grad_ell, grad_sigma, st);
}

int tfl_adjoint(tfl_sim *s, const tfl_objective *obj, int64_t nsteps, int64_t seg, const void *ckpt,
                const double F[2], void *snap, void *adj, double *grad_ell, double *grad_sigma, void *stream)
{
    int rc = check_bound(s, true);
    if (rc != TFL_OK) return rc;
    if ((rc = check_obj(s, obj)) != TFL_OK) return rc;
    if (!s->ckpt_valid || s->ckpt_nsteps != nsteps || s->ckpt_seg != seg)
        return fail(s, TFL_E_STATE,
                    "no checkpointed forward run with these nsteps and seg since the maps or sources last changed");
    if (!same_objective(s->ckpt_obj, *obj))
        return fail(s, TFL_E_STATE, "objective differs from the one of the checkpointed forward run");
    if (!ckpt || !snap || !adj || !grad_ell || !grad_sigma || !F)
        return fail(s, TFL_E_INVAL, "null buffer");
    if (!aligned(ckpt) || !aligned(snap) || !aligned(adj) || !aligned(grad_ell) || !aligned(grad_sigma))
        return fail(s, TFL_E_INVAL, "device buffers must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    return s->esz == 8 ? adjoint<double>(s, obj, nsteps, seg, ckpt, F, snap, adj, grad_ell, grad_sigma, st)
                       : adjoint<float>(s, obj, nsteps, seg, ckpt, F, snap, adj, grad_ell, grad_sigma, st);
}

}  // extern "C"
