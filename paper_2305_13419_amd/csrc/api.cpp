// C ABI of the two-fluid FDTD library: validation, binding, the step loop and
// the CPML tables.  All device work is launched through kernels_fwd.hip;
// nothing of the time step runs on the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sim_internal.h"

using namespace tfl;


namespace tfl {
namespace detail {

thread_local std::string g_create_err;

int fail(tfl_sim *s, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (s) s->err = buf;
    else g_create_err = buf;
    return code;
}

int hip_fail(tfl_sim *s, hipError_t e, const char *where)
{
    return fail(s, TFL_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

bool aligned(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }


int64_t axis_n(const tfl_config &c, int a) { return a == 0 ? c.nx : (a == 1 ? c.ny : c.nz); }
double axis_d(const tfl_config &c, int a) { return a == 0 ? c.dx : (a == 1 ? c.dy : c.dz); }

// Convolutional PML (Roden and Gedney 2000) coefficients at position pos
// (in cells) of axis a: depth d in [0, 1] into the slab, polynomial grading.
void pml_coeff(const tfl_config &c, int a, double pos, double &b, double &cc, double &kinv)
{
    b = 1.0;
    cc = 0.0;
    kinv = 1.0;
    const double n = (double)axis_n(c, a);
    const double lo = c.pml_lo[a], hi = c.pml_hi[a];
    double depth = -1.0;
    if (lo > 0 && pos < lo) depth = (lo - pos) / lo;
    else if (hi > 0 && pos > n - hi) depth = (pos - (n - hi)) / hi;
    if (depth <= 0.0) return;
    const double eta0 = std::sqrt(kMu0 / kEps0);
    const double m = c.pml_order;
    const double smax = c.pml_scale * 0.8 * (m + 1.0) / (eta0 * axis_d(c, a));
    const double dm = std::pow(depth, m);
    const double sg = smax * dm;
    const double kp = 1.0 + (c.kappa_max - 1.0) * dm;
    const double al = c.alpha_max * (1.0 - depth);
    b = std::exp(-(sg / kp + al) * c.dt / kEps0);
    cc = (sg > 0.0) ? sg / (sg * kp + kp * kp * al) * (b - 1.0) : 0.0;
    kinv = 1.0 / kp;
}

size_t slab_elems(const tfl_config &c, int a)
{
    const size_t P = (size_t)(c.pml_lo[a] + c.pml_hi[a]);
    if (a == 0) return (size_t)c.nz * c.ny * P;
    if (a == 1) return (size_t)c.nz * P * c.nx;
    return P * c.ny * c.nx;
}

size_t round256(size_t bytes) { return (bytes + 255) & ~size_t(255); }

size_t fused_layout(const tfl_sim *s, size_t psi_at[3], size_t *total)
{
    const size_t fb = round256((size_t)s->N * s->esz);
    size_t off = 9 * fb;  // second E, H and Js
    for (int ax = 0; ax < 3; ++ax) {  // second set of the axis's variables: H side (two), E side (two)
        psi_at[ax] = off;
        if (s->cfg.bc[ax] == TFL_CPML) off += round256(4 * s->psi_count[ax] * s->esz);
    }
    if (total) *total = off;
    return fb;
}

void layout_workspace(tfl_sim *s)
{
    const tfl_config &c = s->cfg;
    size_t off = 0;  // in elements
    const size_t per256 = 256 / s->esz;
    for (int a = 0; a < 3; ++a) {
        if (c.bc[a] != TFL_CPML) continue;
        s->table_off[a] = off;
        off += 6 * (size_t)axis_n(c, a);
        off = (off + per256 - 1) / per256 * per256;
    }
    for (int a = 0; a < 3; ++a) {
        if (c.bc[a] != TFL_CPML) continue;
        s->psi_count[a] = slab_elems(c, a);
        s->psi_off[a] = off;
        off += 4 * s->psi_count[a];
        off = (off + per256 - 1) / per256 * per256;
    }
    s->work_bytes = off * (size_t)s->esz;
}

template <typename T>
StepArgs<T> make_args(const tfl_sim *s)
{
    const tfl_config &c = s->cfg;
    StepArgs<T> a{};
    a.g.nx = (int)c.nx;
    a.g.ny = (int)c.ny;
    a.g.nz = (int)c.nz;
    a.g.sxy = (long long)c.nx * c.ny;
    for (int q = 0; q < 3; ++q) {
        a.E[q] = (T *)s->E[q];
        a.Eout[q] = (T *)s->E[q];
        a.H[q] = (T *)s->H[q];
        a.Hout[q] = (T *)s->H[q];
        a.J[q] = (T *)s->J[q];
        a.Jout[q] = (T *)s->J[q];
    }
    a.eps = (const T *)s->eps;
    a.sig = (const T *)s->sig;
    a.ell = (const T *)s->ell;
    const void *tab;
    class_pointers(s, a.cls, &tab);
    a.ctab = (const T *)tab;
    a.rd[0] = (T)(1.0 / c.dx);
    a.rd[1] = (T)(1.0 / c.dy);
    a.rd[2] = (T)(1.0 / c.dz);
    a.hdt = (T)(c.dt / kMu0);
    a.dt = (T)c.dt;
    a.theta = (T)c.theta;
    T *w = (T *)s->work;
    for (int ax = 0; ax < 3; ++ax) {
        PmlAxis<T> &p = a.pml[ax];
        p.on = c.bc[ax] == TFL_CPML;
        p.n = (int)axis_n(c, ax);
        if (!p.on) continue;
        p.lo = c.pml_lo[ax];
        p.hi = c.pml_hi[ax];
        p.P = p.lo + p.hi;
        const T *tb = w + s->table_off[ax];
        const size_t n = (size_t)p.n;
        p.bn = tb; p.cn = tb + n; p.kn = tb + 2 * n;
        p.bh = tb + 3 * n; p.ch = tb + 4 * n; p.kh = tb + 5 * n;
        T *ps = w + s->psi_off[ax];
        const size_t m = s->psi_count[ax];
        p.psiH[0] = ps; p.psiH[1] = ps + m; p.psiE[0] = ps + 2 * m; p.psiE[1] = ps + 3 * m;
        p.psiHo[0] = p.psiH[0]; p.psiHo[1] = p.psiH[1];
        p.psiEo[0] = p.psiE[0]; p.psiEo[1] = p.psiE[1];
    }
    return a;
}

template <typename T>
int do_step(tfl_sim *s, int64_t nsteps, hipStream_t st, hipEvent_t *ev, bool probes)
{
    StepArgs<T> a = make_args<T>(s);
    source_boxes(s, a.side);
    ProbeArgs<T> pa{};
    pa.g = a.g;
    for (int q = 0; q < 3; ++q) pa.E[q] = a.E[q];
    pa.dt = s->cfg.dt;
    const int np = probes ? (int)s->probe.size() : 0;
    if (np > 0) {
        const int rc = upload_probes(s, st);
        if (rc != TFL_OK) return rc;
    }
    pa.p = (const ProbeDesc *)((const char *)s->scratch + kProbeDescOffset);
    pa.first = 0;
    hipError_t e;
    if (np > 0 && s->step == 0 && !s->sampled0) {
        pa.n = 0;
        if ((e = launch_probes<T>(pa, np, st)) != hipSuccess) return hip_fail(s, e, "probe");
        s->sampled0 = true;
    }
    // Probes ride along with the sweeps when there are few enough and their boxes fit the copy
    // halves of scratch: each sweep copies its new E on the boxes to one half and first sums the
    // copies the previous sweep left in the other; one probe launch after the last step sums the
    // last copies.  Otherwise a probe launch follows every step.
    // A two-step sweep leaves two samples: its copies go to the two quarters of a half.
    size_t coff[kFoldProbes] = {};
    bool fold = np > 0 && np <= kFoldProbes;
    size_t copy_bytes = 0;
    for (int p = 0; p < np && fold; ++p) {
        const ProbeDesc &d = s->probe[p];
        coff[p] = copy_bytes;
        copy_bytes += round256((size_t)(d.i1 - d.i0) * (d.j1 - d.j0) * (d.k1 - d.k0) * sizeof(T));
        fold = copy_bytes <= kProbeCopyHalf;
    }
    const bool fold2 = fold && copy_bytes <= kProbeCopyHalf / 2;
    char *const copy_base = (char *)s->scratch + kProbeCopyOffset;
    auto copy_at = [&](int hf, int sample, int p) {
        return copy_base + hf * kProbeCopyHalf + sample * (kProbeCopyHalf / 2) + coff[p];
    };
    if (fold) {
        a.side.pdesc = pa.p;
        a.side.dt = s->cfg.dt;
        for (int p = 0; p < np; ++p) {
            const ProbeDesc &d = s->probe[p];
            const int bx[7] = {d.comp, d.i0, d.i1, d.j0, d.j1, d.k0, d.k1};
            for (int c = 0; c < 7; ++c) a.side.pbox[p][c] = bx[c];
        }
    }
    int half = 0;          // copy half the next sweep writes
    bool pending = false;  // copies of samples pending_n .. pending_n + pending_cnt - 1 wait in the other half
    int64_t pending_n = 0;
    int pending_cnt = 0;
    auto probes_of = [&](StepArgs<T> &g) {
        if (!fold) return;
        g.side.nprobe = np;
        g.side.nred = pending ? np : 0;
        g.side.nsamp = pending_cnt;
        g.side.rn = pending_n;
        for (int p = 0; p < np; ++p) {  // second samples only where two copies fit a half
            g.side.pcopy[p] = copy_at(half, 0, p);
            g.side.pcopy2[p] = fold2 ? copy_at(half, 1, p) : nullptr;
            g.side.rcopy[p] = copy_at(1 - half, 0, p);
            g.side.rcopy2[p] = fold2 ? copy_at(1 - half, 1, p) : nullptr;
        }
    };
    // the side work of the sweep of step s->step -> s->step + 1
    auto side = [&](StepArgs<T> g) {
        source_values(s, g.side, (double)(s->step + 1) * s->cfg.dt);
        probes_of(g);
        return g;
    };
    // after a sweep whose cnt samples start at index first
    auto side_done = [&](int64_t first, int cnt) {
        if (!fold) return;
        pending = true;
        pending_n = first;
        pending_cnt = cnt;
        half = 1 - half;
    };
    // With a fused buffer bound, steps go A -> B -> A in pairs through the fused sweep (A the bound
    // fields, B the buffer), so the state is back in A after every call; an odd last step runs the
    // two passes in place on A.
    StepArgs<T> ab = a, ba = a;
    const bool fused = s->fused != nullptr && s->sweep != TFL_SWEEP_TWO_PASS;
    // Two steps per sweep (grids with edge classes) where nothing but soft sources and folded probes
    // happens between the steps: no probe launches or non-finite checks.  Launches go A -> B -> A (E,
    // H, Js and the CPML variables), four steps per round trip, so the state is back in A; the
    // remaining steps take the paths below.
    const bool two_applies = fused && (np == 0 || fold2) && !(s->checking && s->check_every > 0) &&
                             a.cls[0] != nullptr;
    const bool two = two_applies && (s->sweep == TFL_SWEEP_TWO_STEP || (s->sweep == TFL_SWEEP_AUTO &&
                                                                        two_step_pays<T>(a)));
    StepArgs<T> ab2 = a, ba2 = a;
    if (fused) {
        size_t psi_at[3];
        const size_t fb = fused_layout(s, psi_at);
        for (int q = 0; q < 3; ++q) {
            T *eb = (T *)((char *)s->fused + q * fb), *hb = (T *)((char *)s->fused + (3 + q) * fb);
            ab.Eout[q] = eb;
            ab.Hout[q] = hb;
            ba.E[q] = eb;
            ba.H[q] = hb;
        }
        // CPML axes: the H-side variables go A -> B -> A with the fields (the E-side ones stay in place)
        for (int ax = 0; ax < 3; ++ax) {
            if (!a.pml[ax].on || s->psi_count[ax] == 0) continue;
            T *pb = (T *)((char *)s->fused + psi_at[ax]);
            const size_t m = s->psi_count[ax];
            ab.pml[ax].psiHo[0] = pb;
            ab.pml[ax].psiHo[1] = pb + m;
            ba.pml[ax].psiH[0] = pb;
            ba.pml[ax].psiH[1] = pb + m;
            ba.pml[ax].psiHo[0] = a.pml[ax].psiH[0];
            ba.pml[ax].psiHo[1] = a.pml[ax].psiH[1];
        }
    }
    int64_t it = 0;
    if (two) {
        size_t psi_at[3];
        const size_t fb = fused_layout(s, psi_at);
        for (int q = 0; q < 3; ++q) {
            T *eb = (T *)((char *)s->fused + q * fb), *hb = (T *)((char *)s->fused + (3 + q) * fb);
            T *jb = (T *)((char *)s->fused + (6 + q) * fb);
            ab2.Eout[q] = eb;
            ab2.Hout[q] = hb;
            ab2.Jout[q] = jb;
            ba2.E[q] = eb;
            ba2.H[q] = hb;
            ba2.J[q] = jb;
            ba2.Eout[q] = a.E[q];
            ba2.Hout[q] = a.H[q];
            ba2.Jout[q] = a.J[q];
        }
        // CPML axes: both sides' variables go A -> B -> A with the fields
        for (int ax = 0; ax < 3; ++ax) {
            if (!a.pml[ax].on || s->psi_count[ax] == 0) continue;
            T *pb = (T *)((char *)s->fused + psi_at[ax]);
            const size_t m = s->psi_count[ax];
            for (int c = 0; c < 2; ++c) {
                ab2.pml[ax].psiHo[c] = pb + c * m;
                ab2.pml[ax].psiEo[c] = pb + (2 + c) * m;
                ba2.pml[ax].psiH[c] = pb + c * m;
                ba2.pml[ax].psiE[c] = pb + (2 + c) * m;
                ba2.pml[ax].psiHo[c] = a.pml[ax].psiH[c];
                ba2.pml[ax].psiEo[c] = a.pml[ax].psiE[c];
            }
        }
        for (; it + 4 <= nsteps; it += 4) {
            for (int h = 0; h < 2; ++h) {
                if (ev && (e = hipEventRecord(ev[2 * (it + 2 * h)], st)) != hipSuccess) return hip_fail(s, e, "event");
                // the sources' values at the launch's two steps, the probes' copies of both
                StepArgs<T> g = h == 0 ? ab2 : ba2;
                source_values(s, g.side, (double)(s->step + 2 * h + 1) * s->cfg.dt);
                for (int q = 0; q < g.side.nsrc; ++q)
                    g.side.sg2[q] = source_value(s->src[q], (double)(s->step + 2 * h + 2) * s->cfg.dt);
                probes_of(g);
                if ((e = launch_two_step<T>(g, st)) != hipSuccess) return hip_fail(s, e, "two steps");
                side_done(s->step + 2 * h + 1, 2);
                // the two steps' events: the sweep in the first interval, the others empty
                for (int q = 1; q < 4 && ev; ++q)
                    if ((e = hipEventRecord(ev[2 * (it + 2 * h) + q], st)) != hipSuccess) return hip_fail(s, e, "event");
            }
            s->step += 4;
            s->sweep_counts[2] += 4;
        }
    }
    bool inB = false;
    for (; it < nsteps; ++it) {
        if (ev && (e = hipEventRecord(ev[2 * it], st)) != hipSuccess) return hip_fail(s, e, "event");
        if (fused && (inB || it + 1 < nsteps)) {
            if ((e = launch_fused_step<T>(side(inB ? ba : ab), st)) != hipSuccess) return hip_fail(s, e, "fused step");
            if (ev && (e = hipEventRecord(ev[2 * it + 1], st)) != hipSuccess) return hip_fail(s, e, "event");
            inB = !inB;
            s->sweep_counts[1] += 1;
        } else {
            s->sweep_counts[0] += 1;
            if ((e = launch_h_pass<T>(a, st)) != hipSuccess) return hip_fail(s, e, "h_pass");
            if (ev && (e = hipEventRecord(ev[2 * it + 1], st)) != hipSuccess) return hip_fail(s, e, "event");
            if ((e = launch_e_pass<T>(side(a), st)) != hipSuccess) return hip_fail(s, e, "e_pass");
        }
        for (int q = 0; q < 3; ++q) pa.E[q] = inB ? ab.Eout[q] : a.E[q];
        s->step += 1;
        side_done(s->step, 1);  // the sample index of the new E
        if (np > 0 && !fold) {
            pa.n = s->step;
            if ((e = launch_probes<T>(pa, np, st)) != hipSuccess) return hip_fail(s, e, "probe");
        }
        if (s->checking && s->check_every > 0 && s->step % s->check_every == 0) {
            NonfiniteArgs<T> na{};
            for (int q = 0; q < 3; ++q) {
                na.f[q] = pa.E[q];
                na.f[3 + q] = inB ? ab.Hout[q] : a.H[q];
                na.f[6 + q] = a.J[q];
            }
            na.n = a.g.sxy * a.g.nz;
            auto *ctr = (unsigned long long *)((char *)s->scratch + kNonfiniteOffset);
            if ((e = launch_nonfinite<T>(na, ctr, s->step, st)) != hipSuccess) return hip_fail(s, e, "non-finite check");
            s->checked = true;
        }
    }
    for (int r = 0; pending && r < pending_cnt; ++r) {  // the last sweep's copies
        pa.n = pending_n + r;
        for (int p = 0; p < np; ++p) pa.copy[p] = (const T *)copy_at(1 - half, r, p);
        if ((e = launch_probes<T>(pa, np, st)) != hipSuccess) return hip_fail(s, e, "probe");
    }
    if (ev && nsteps > 0 && (e = hipEventRecord(ev[2 * nsteps], st)) != hipSuccess) return hip_fail(s, e, "event");
    return TFL_OK;
}



int upload_probes(tfl_sim *s, hipStream_t st)
{
    if (!s->probes_dirty || s->probe.empty()) return TFL_OK;
    void *dst = (char *)s->scratch + kProbeDescOffset;
    hipError_t e = hipMemcpyAsync(dst, s->probe.data(), s->probe.size() * sizeof(ProbeDesc), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host vector may change after return
    if (e != hipSuccess) return hip_fail(s, e, "probe descriptor upload");
    s->probes_dirty = false;
    return TFL_OK;
}

int nonfinite_begin(tfl_sim *s, hipStream_t st)
{
    s->checking = s->check_every > 0;
    s->checked = false;
    if (!s->checking) return TFL_OK;
    hipError_t e = launch_nonfinite_reset((unsigned long long *)((char *)s->scratch + kNonfiniteOffset), st);
    if (e != hipSuccess) {
        s->checking = false;
        return hip_fail(s, e, "non-finite check reset");
    }
    return TFL_OK;
}

int nonfinite_end(tfl_sim *s, hipStream_t st)
{
    const bool ran = s->checking && s->checked;
    s->checking = false;
    s->checked = false;
    if (!ran) return TFL_OK;
    unsigned long long r[2];
    hipError_t e = hipMemcpyAsync(r, (char *)s->scratch + kNonfiniteOffset, sizeof(r), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(s, e, "non-finite check readback");
    if (r[0] != 0)
        return fail(s, TFL_E_NONFINITE, "%llu non-finite values in E, H and Js, first seen after step %llu", r[0],
                    r[1]);
    return TFL_OK;
}

int check_bound(tfl_sim *s, bool need_maps)
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    if (!s->state_bound) return fail(s, TFL_E_STATE, "state arrays not bound (tfl_bind_state)");
    if (!s->work_bound) return fail(s, TFL_E_STATE, "workspace not bound (tfl_bind_workspace)");
    if (need_maps && !s->maps_bound) return fail(s, TFL_E_STATE, "materials not bound (tfl_bind_materials)");
    return TFL_OK;
}

double source_value(const SourceDesc &d, double t)
{
    if (d.wave == TFL_WAVE_SIN) return d.amp * std::sin(kTwoPi * d.f * t);
    const double g = std::exp(-(t - d.t0) * (t - d.t0) / (2.0 * d.tw * d.tw));
    return d.amp * (d.wave == TFL_WAVE_GAUSS ? g : g * std::sin(kTwoPi * d.f * t));
}

void source_boxes(const tfl_sim *s, SideArgs &sd)
{
    sd.nsrc = (int)s->src.size();
    for (int q = 0; q < sd.nsrc; ++q) {
        const SourceDesc &d = s->src[q];
        const int bx[7] = {d.comp, d.i0, d.i1, d.j0, d.j1, d.k0, d.k1};
        for (int c = 0; c < 7; ++c) sd.sbox[q][c] = bx[c];
        sd.sg[q] = 0.0;
    }
}

void source_values(const tfl_sim *s, SideArgs &sd, double t)
{
    for (int q = 0; q < sd.nsrc; ++q) sd.sg[q] = source_value(s->src[q], t);
}

bool box_ok(const tfl_config &c, const int64_t *b)
{
    const int64_t n[3] = {c.nx, c.ny, c.nz};
    for (int a = 0; a < 3; ++a)
        if (b[2 * a] < 0 || b[2 * a + 1] > n[a] || b[2 * a] >= b[2 * a + 1]) return false;
    return true;
}

template <typename T>
static void fill_tables(const tfl_sim *s, std::vector<T> &host, int a)
{
    const tfl_config &c = s->cfg;
    const size_t n = (size_t)axis_n(c, a);
    host.assign(6 * n, T(0));
    for (size_t i = 0; i < n; ++i) {
        double b, cc, k;
        pml_coeff(c, a, (double)i, b, cc, k);
        host[i] = (T)b; host[n + i] = (T)cc; host[2 * n + i] = (T)k;
        pml_coeff(c, a, (double)i + 0.5, b, cc, k);
        host[3 * n + i] = (T)b; host[4 * n + i] = (T)cc; host[5 * n + i] = (T)k;
    }
}

template <typename T>
static int upload_tables(tfl_sim *s, hipStream_t st)
{
    for (int a = 0; a < 3; ++a) {
        if (s->cfg.bc[a] != TFL_CPML) continue;
        std::vector<T> host;
        fill_tables<T>(s, host, a);
        T *dst = (T *)s->work + s->table_off[a];
        hipError_t e = hipMemcpyAsync(dst, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(s, e, "upload PML tables");
        e = hipStreamSynchronize(st);  // host vector goes out of scope
        if (e != hipSuccess) return hip_fail(s, e, "upload PML tables");
    }
    return TFL_OK;
}

static int clear_psi(tfl_sim *s, hipStream_t st)
{
    for (int a = 0; a < 3; ++a) {
        if (s->cfg.bc[a] != TFL_CPML || s->psi_count[a] == 0) continue;
        char *p = (char *)s->work + s->psi_off[a] * s->esz;
        hipError_t e = launch_fill_zero(p, 4 * s->psi_count[a] * s->esz, st);
        if (e != hipSuccess) return hip_fail(s, e, "clear PML variables");
    }
    return TFL_OK;
}

int copy_state(tfl_sim *s, void *dst, const void *src, bool save, hipStream_t st)
{
    const size_t fb = (size_t)s->N * s->esz, stride = round256(fb);
    char *buf = save ? (char *)dst : (char *)const_cast<void *>(src);
    void *arrs[9] = {s->E[0], s->E[1], s->E[2], s->H[0], s->H[1], s->H[2], s->J[0], s->J[1], s->J[2]};
    for (int q = 0; q < 9; ++q) {
        hipError_t e = save ? hipMemcpyAsync(buf + q * stride, arrs[q], fb, hipMemcpyDeviceToDevice, st)
                            : hipMemcpyAsync(arrs[q], buf + q * stride, fb, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(s, e, "state copy");
    }
    if (s->work_bytes > 0) {
        hipError_t e = save ? hipMemcpyAsync(buf + 9 * stride, s->work, s->work_bytes, hipMemcpyDeviceToDevice, st)
                            : hipMemcpyAsync(s->work, buf + 9 * stride, s->work_bytes, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(s, e, "workspace copy");
    }
    return TFL_OK;
}

template StepArgs<double> make_args<double>(const tfl_sim *);
template StepArgs<float> make_args<float>(const tfl_sim *);
template int do_step<double>(tfl_sim *, int64_t, hipStream_t, hipEvent_t *, bool);
template int do_step<float>(tfl_sim *, int64_t, hipStream_t, hipEvent_t *, bool);

}  // namespace detail
}  // namespace tfl

using namespace tfl::detail;

extern "C" {

const char *tfl_last_error(const tfl_sim *sim) { return sim ? sim->err.c_str() : g_create_err.c_str(); }

int tfl_create(const tfl_config *cfg, tfl_sim **out)
{
    if (!cfg || !out) return fail(nullptr, TFL_E_INVAL, "null argument");
    *out = nullptr;
    const tfl_config &c = *cfg;
    if (c.nx < 1 || c.ny < 1 || c.nz < 1) return fail(nullptr, TFL_E_INVAL, "grid sizes must be >= 1");
    if (c.nx > (1LL << 30) || c.ny > (1LL << 30) || c.nz > (1LL << 30) || c.nx * c.ny * c.nz > (1LL << 40))
        return fail(nullptr, TFL_E_INVAL, "grid too large");
    // the sweeps address one x-y plane with 32-bit byte offsets
    if (c.nx * c.ny > (1LL << 29)) return fail(nullptr, TFL_E_INVAL, "nx * ny must not exceed 2^29");
    if (!(c.dx > 0) || !(c.dy > 0) || !(c.dz > 0) || !std::isfinite(c.dx) || !std::isfinite(c.dy) ||
        !std::isfinite(c.dz))
        return fail(nullptr, TFL_E_INVAL, "spacings must be finite and > 0");
    if (!(c.dt > 0) || !std::isfinite(c.dt)) return fail(nullptr, TFL_E_INVAL, "dt must be finite and > 0");
    if (!(c.theta >= 0.5 && c.theta <= 1.0)) return fail(nullptr, TFL_E_INVAL, "theta must lie in [0.5, 1]");
    if (c.dtype != TFL_F64 && c.dtype != TFL_F32) return fail(nullptr, TFL_E_INVAL, "dtype must be TFL_F64 or TFL_F32");
    for (int a = 0; a < 3; ++a) {
        if (c.bc[a] != TFL_PERIODIC && c.bc[a] != TFL_CPML) return fail(nullptr, TFL_E_INVAL, "bad bc on axis %d", a);
        if (c.bc[a] == TFL_CPML) {
            if (c.pml_lo[a] < 0 || c.pml_hi[a] < 0 || c.pml_lo[a] + c.pml_hi[a] > axis_n(c, a))
                return fail(nullptr, TFL_E_INVAL, "bad PML cell counts on axis %d", a);
            if (!(c.pml_order >= 0) || !(c.pml_scale >= 0) || !(c.kappa_max >= 1) || !(c.alpha_max >= 0))
                return fail(nullptr, TFL_E_INVAL, "bad PML grading parameters");
        }
    }
    tfl_sim *s = new (std::nothrow) tfl_sim();
    if (!s) return fail(nullptr, TFL_E_NOMEM, "host allocation failed");
    s->cfg = c;
    for (int a = 0; a < 3; ++a)
        if (c.bc[a] != TFL_CPML) s->cfg.pml_lo[a] = s->cfg.pml_hi[a] = 0;
    s->N = (long long)c.nx * c.ny * c.nz;
    s->esz = c.dtype == TFL_F64 ? 8 : 4;
    layout_workspace(s);
    *out = s;
    return TFL_OK;
}

int tfl_destroy(tfl_sim *sim)
{
    delete sim;
    return TFL_OK;
}

int tfl_buffer_sizes(const tfl_sim *s, size_t *workspace_bytes, size_t *scratch_bytes, size_t *state_bytes)
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    if (workspace_bytes) *workspace_bytes = s->work_bytes;
    if (scratch_bytes) *scratch_bytes = kScratchBytes;
    if (state_bytes) *state_bytes = 9 * round256((size_t)s->N * s->esz) + round256(s->work_bytes);
    return TFL_OK;
}

int tfl_bind_state(tfl_sim *s, void *const E[3], void *const H[3], void *const J[3])
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    if (!E || !H || !J) return fail(s, TFL_E_INVAL, "null array list");
    for (int q = 0; q < 3; ++q) {
        if (!E[q] || !H[q] || !J[q]) return fail(s, TFL_E_INVAL, "null state pointer (component %d)", q);
        if (!aligned(E[q]) || !aligned(H[q]) || !aligned(J[q]))
            return fail(s, TFL_E_INVAL, "state pointers must be 256-byte aligned (component %d)", q);
    }
    for (int q = 0; q < 3; ++q) {
        s->E[q] = E[q];
        s->H[q] = H[q];
        s->J[q] = J[q];
    }
    s->state_bound = true;
    return TFL_OK;
}

int tfl_bind_workspace(tfl_sim *s, void *workspace, void *scratch, void *stream)
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    if (s->work_bytes > 0 && (!workspace || !aligned(workspace)))
        return fail(s, TFL_E_INVAL, "workspace must be a 256-byte aligned device pointer of %zu bytes", s->work_bytes);
    if (!scratch || !aligned(scratch)) return fail(s, TFL_E_INVAL, "scratch must be a 256-byte aligned device pointer");
    s->work = workspace;
    s->scratch = (double *)scratch;
    hipStream_t st = (hipStream_t)stream;
    int rc = s->esz == 8 ? upload_tables<double>(s, st) : upload_tables<float>(s, st);
    if (rc != TFL_OK) return rc;
    rc = clear_psi(s, st);
    if (rc != TFL_OK) return rc;
    s->work_bound = true;
    return TFL_OK;
}


int tfl_fused_buffer_bytes(const tfl_sim *s, size_t *bytes)
{
    if (!s || !bytes) return fail(nullptr, TFL_E_INVAL, "null argument");
    size_t psi_at[3];
    fused_layout(s, psi_at, bytes);
    return TFL_OK;
}

int tfl_bind_fused_buffer(tfl_sim *s, void *buf)
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    if (buf && !aligned(buf)) return fail(s, TFL_E_INVAL, "fused buffer must be 256-byte aligned");
    s->fused = buf;
    return TFL_OK;
}

int tfl_bind_materials(tfl_sim *s, const void *eps_r, const void *sigma_n, const void *inv_lambda2, void *stream)
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    if (!s->work_bound) return fail(s, TFL_E_STATE, "bind the workspace (scratch) before the materials");
    s->cls = nullptr;  // edge classes are a snapshot of the previous maps
    s->ncls = 0;
    s->ckpt_valid = false;  // a checkpointed run of the previous maps no longer matches a recomputation
    if (!eps_r || !sigma_n || !inv_lambda2) return fail(s, TFL_E_INVAL, "null map pointer");
    if (!aligned(eps_r) || !aligned(sigma_n) || !aligned(inv_lambda2))
        return fail(s, TFL_E_INVAL, "map pointers must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = s->esz == 8
                       ? launch_map_stats<double>((const double *)eps_r, (const double *)sigma_n,
                                                  (const double *)inv_lambda2, s->N, s->scratch, kRedBlocks, st)
                       : launch_map_stats<float>((const float *)eps_r, (const float *)sigma_n,
                                                 (const float *)inv_lambda2, s->N, s->scratch, kRedBlocks, st);
    if (e != hipSuccess) return hip_fail(s, e, "map statistics");
    double r[5];
    e = hipMemcpyAsync(r, s->scratch, sizeof(r), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(s, e, "map statistics readback");
    if (r[4] != 0.0) return fail(s, TFL_E_INVAL, "material maps hold %.0f non-finite values", r[4]);
    if (!(r[0] > 0.0)) return fail(s, TFL_E_INVAL, "eps_r must be > 0 (min %g)", r[0]);
    if (r[1] < 0.0) return fail(s, TFL_E_INVAL, "sigma_n must be >= 0 (min %g)", r[1]);
    if (r[2] < 0.0) return fail(s, TFL_E_INVAL, "inv_lambda2 must be >= 0 (min %g)", r[2]);
    const double max_ell = -r[3];
    const tfl_config &c = s->cfg;
    const double c0 = 1.0 / std::sqrt(kEps0 * kMu0);
    const double dt_max =
        2.0 / (c0 * std::sqrt(4.0 / (c.dx * c.dx) + 4.0 / (c.dy * c.dy) + 4.0 / (c.dz * c.dz) + max_ell));
    if (c.dt > dt_max)
        return fail(s, TFL_E_UNSTABLE, "dt = %.6e s exceeds the stability bound %.6e s (max 1/lambda^2 = %.4e m^-2)",
                    c.dt, dt_max, max_ell);
    s->eps = eps_r;
    s->sig = sigma_n;
    s->ell = inv_lambda2;
    s->max_ell = max_ell;
    s->maps_bound = true;
    return TFL_OK;
}

int tfl_set_initial_integer_time(tfl_sim *s, void *stream)
{
    int rc = check_bound(s, true);
    if (rc != TFL_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    rc = clear_psi(s, st);
    if (rc != TFL_OK) return rc;
    hipError_t e;
    if (s->esz == 8) {
        StepArgs<double> a = make_args<double>(s);
        double *Ho[3] = {a.H[0], a.H[1], a.H[2]}, *Jo[3] = {a.J[0], a.J[1], a.J[2]};
        e = launch_half_kick<double>(a, 1.0, Ho, Jo, st);
    } else {
        StepArgs<float> a = make_args<float>(s);
        float *Ho[3] = {a.H[0], a.H[1], a.H[2]}, *Jo[3] = {a.J[0], a.J[1], a.J[2]};
        e = launch_half_kick<float>(a, 1.0f, Ho, Jo, st);
    }
    if (e != hipSuccess) return hip_fail(s, e, "half kick");
    s->step = 0;
    s->sampled0 = false;
    return TFL_OK;
}

int tfl_add_source(tfl_sim *s, const tfl_source *src, int *id)
{
    if (!s || !src) return fail(s, TFL_E_INVAL, "null argument");
    if ((int)s->src.size() >= TFL_MAX_SOURCES) return fail(s, TFL_E_INVAL, "too many sources");
    if (src->comp < 0 || src->comp > 2) return fail(s, TFL_E_INVAL, "source component must be 0..2");
    if (!box_ok(s->cfg, src->box)) return fail(s, TFL_E_INVAL, "source box outside the grid or empty");
    if (src->waveform < TFL_WAVE_SIN || src->waveform > TFL_WAVE_MOD_GAUSS)
        return fail(s, TFL_E_INVAL, "bad waveform");
    if (src->waveform != TFL_WAVE_SIN && !(src->tw > 0)) return fail(s, TFL_E_INVAL, "gaussian width must be > 0");
    SourceDesc d{};
    d.comp = src->comp;
    d.i0 = (int)src->box[0]; d.i1 = (int)src->box[1];
    d.j0 = (int)src->box[2]; d.j1 = (int)src->box[3];
    d.k0 = (int)src->box[4]; d.k1 = (int)src->box[5];
    d.amp = src->amplitude;
    d.wave = src->waveform;
    d.f = src->freq;
    d.t0 = src->t0;
    d.tw = src->tw;
    s->src.push_back(d);
    s->ckpt_valid = false;  // the recomputation of a checkpointed run would add this source
    if (id) *id = (int)s->src.size() - 1;
    return TFL_OK;
}

int tfl_add_probe(tfl_sim *s, const tfl_probe *p, int *id)
{
    if (!s || !p) return fail(s, TFL_E_INVAL, "null argument");
    if ((int)s->probe.size() >= TFL_MAX_PROBES) return fail(s, TFL_E_INVAL, "too many probes");
    if (p->comp < 0 || p->comp > 2) return fail(s, TFL_E_INVAL, "probe component must be 0..2");
    if (!box_ok(s->cfg, p->box)) return fail(s, TFL_E_INVAL, "probe box outside the grid or empty");
    if (p->nfreq < 0 || p->nfreq > TFL_MAX_FREQS) return fail(s, TFL_E_INVAL, "nfreq must be 0..%d", TFL_MAX_FREQS);
    if (p->capacity < 0) return fail(s, TFL_E_INVAL, "capacity must be >= 0");
    if (p->capacity > 0 && !p->series) return fail(s, TFL_E_INVAL, "series buffer missing");
    if (p->nfreq > 0 && (!p->dft || !p->freqs)) return fail(s, TFL_E_INVAL, "dft buffer or frequencies missing");
    ProbeDesc d{};
    d.comp = p->comp;
    d.i0 = (int)p->box[0]; d.i1 = (int)p->box[1];
    d.j0 = (int)p->box[2]; d.j1 = (int)p->box[3];
    d.k0 = (int)p->box[4]; d.k1 = (int)p->box[5];
    d.series = p->capacity > 0 ? p->series : nullptr;
    d.cap = p->capacity;
    d.nfreq = p->nfreq;
    for (int f = 0; f < p->nfreq; ++f) d.freq[f] = p->freqs[f];
    d.dft = p->dft;
    s->probe.push_back(d);
    s->probes_dirty = true;
    if (id) *id = (int)s->probe.size() - 1;
    return TFL_OK;
}

int tfl_clear_sources_probes(tfl_sim *s)
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    s->src.clear();
    s->probe.clear();
    s->probes_dirty = true;
    s->ckpt_valid = false;
    return TFL_OK;
}

int tfl_step(tfl_sim *s, int64_t nsteps, void *stream)
{
    int rc = check_bound(s, true);
    if (rc != TFL_OK) return rc;
    if (nsteps < 0) return fail(s, TFL_E_INVAL, "nsteps must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    if ((rc = nonfinite_begin(s, st)) != TFL_OK) return rc;
    for (auto &c : s->sweep_counts) c = 0;
    rc = s->esz == 8 ? do_step<double>(s, nsteps, st) : do_step<float>(s, nsteps, st);
    const int rc2 = nonfinite_end(s, st);
    return rc != TFL_OK ? rc : rc2;
}

int tfl_set_sweep(tfl_sim *s, int32_t sweep)
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    if (sweep < TFL_SWEEP_AUTO || sweep > TFL_SWEEP_TWO_STEP) return fail(s, TFL_E_INVAL, "bad sweep %d", sweep);
    s->sweep = sweep;
    return TFL_OK;
}

int tfl_sweep_counts(const tfl_sim *s, int64_t counts[3])
{
    if (!s || !counts) return fail(nullptr, TFL_E_INVAL, "null argument");
    for (int q = 0; q < 3; ++q) counts[q] = s->sweep_counts[q];
    return TFL_OK;
}

int tfl_set_nonfinite_check(tfl_sim *s, int64_t every)
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    if (every < 0) return fail(s, TFL_E_INVAL, "the check interval must be >= 0");
    s->check_every = every;
    return TFL_OK;
}

int tfl_profile_step(tfl_sim *s, int64_t nsteps, void *stream, double *h_ms, double *e_ms)
{
    int rc = check_bound(s, true);
    if (rc != TFL_OK) return rc;
    if (nsteps < 1 || nsteps > (1 << 20)) return fail(s, TFL_E_INVAL, "nsteps must be in [1, 2^20]");
    hipStream_t st = (hipStream_t)stream;
    std::vector<hipEvent_t> ev((size_t)(2 * nsteps + 1), nullptr);
    hipError_t e = hipSuccess;
    for (auto &x : ev)
        if ((e = hipEventCreate(&x)) != hipSuccess) break;
    if (e == hipSuccess) {
        for (auto &c : s->sweep_counts) c = 0;
        rc = s->esz == 8 ? do_step<double>(s, nsteps, st, ev.data()) : do_step<float>(s, nsteps, st, ev.data());
        if (rc == TFL_OK) {
            e = hipEventSynchronize(ev.back());
            double th = 0.0, te = 0.0;
            for (int64_t it = 0; it < nsteps && e == hipSuccess; ++it) {
                float a = 0.f, b = 0.f;
                e = hipEventElapsedTime(&a, ev[2 * it], ev[2 * it + 1]);
                if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[2 * it + 1], ev[2 * it + 2]);
                th += a;
                te += b;
            }
            if (h_ms) *h_ms = th;
            if (e_ms) *e_ms = te;
        }
    }
    for (auto &x : ev)
        if (x) (void)hipEventDestroy(x);
    if (rc != TFL_OK) return rc;
    if (e != hipSuccess) return hip_fail(s, e, "profile events");
    return TFL_OK;
}

int tfl_sync_integer_time(tfl_sim *s, void *const Hn[3], void *const Jn[3], void *stream)
{
    int rc = check_bound(s, true);
    if (rc != TFL_OK) return rc;
    for (int q = 0; q < 3; ++q) {
        if (Hn && (!Hn[q] || !aligned(Hn[q]))) return fail(s, TFL_E_INVAL, "Hn pointers must be aligned, non-null");
        if (Jn && (!Jn[q] || !aligned(Jn[q]))) return fail(s, TFL_E_INVAL, "Jn pointers must be aligned, non-null");
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (s->esz == 8) {
        StepArgs<double> a = make_args<double>(s);
        double *Ho[3], *Jo[3];
        for (int q = 0; q < 3; ++q) {
            Ho[q] = Hn ? (double *)Hn[q] : nullptr;
            Jo[q] = Jn ? (double *)Jn[q] : nullptr;
        }
        e = launch_half_kick<double>(a, -1.0, Hn ? Ho : nullptr, Jn ? Jo : nullptr, st);
    } else {
        StepArgs<float> a = make_args<float>(s);
        float *Ho[3], *Jo[3];
        for (int q = 0; q < 3; ++q) {
            Ho[q] = Hn ? (float *)Hn[q] : nullptr;
            Jo[q] = Jn ? (float *)Jn[q] : nullptr;
        }
        e = launch_half_kick<float>(a, -1.0f, Hn ? Ho : nullptr, Jn ? Jo : nullptr, st);
    }
    if (e != hipSuccess) return hip_fail(s, e, "sync half kick");
    return TFL_OK;
}

int tfl_energy(tfl_sim *s, double *energy, int64_t *nonfinite, void *stream)
{
    int rc = check_bound(s, true);
    if (rc != TFL_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = s->esz == 8 ? launch_energy<double>(make_args<double>(s), s->scratch, kRedBlocks, st)
                               : launch_energy<float>(make_args<float>(s), s->scratch, kRedBlocks, st);
    if (e != hipSuccess) return hip_fail(s, e, "energy");
    double r[2];
    e = hipMemcpyAsync(r, s->scratch, sizeof(r), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(s, e, "energy readback");
    if (energy) *energy = r[0];
    if (nonfinite) *nonfinite = (int64_t)r[1];
    return TFL_OK;
}

int tfl_energy_noalloc(tfl_sim *s, double *out, void *stream)
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    if (!s->state_bound) return fail(s, TFL_E_STATE, "state arrays not bound (tfl_bind_state)");
    if (!s->maps_bound) return fail(s, TFL_E_STATE, "materials not bound (tfl_bind_materials)");
    if (!out || (reinterpret_cast<uintptr_t>(out) & 7u) != 0)
        return fail(s, TFL_E_INVAL, "out must be an 8-byte aligned device pointer of 2 doubles");
    // the reduction uses kRedBlocks partial pairs, the same as tfl_energy (so the results are the same
    // bits); the fixed scratch holds kStaticScratchBlocks of them
    const int nblocks = kRedBlocks;
    if (nblocks > kStaticScratchBlocks)
        return fail(s, TFL_E_NOMEM, "the energy reduction needs %d block partials, the fixed scratch holds %d",
                    nblocks, kStaticScratchBlocks);
    double *part = nullptr;
    hipError_t e = static_scratch(&part);
    if (e != hipSuccess) return hip_fail(s, e, "fixed scratch address");
    hipStream_t st = (hipStream_t)stream;
    e = s->esz == 8 ? launch_energy<double>(make_args<double>(s), part, nblocks, st, out)
                    : launch_energy<float>(make_args<float>(s), part, nblocks, st, out);
    if (e != hipSuccess) return hip_fail(s, e, "energy");
    return TFL_OK;
}

int tfl_get_step(const tfl_sim *s, int64_t *step)
{
    if (!s || !step) return fail(nullptr, TFL_E_INVAL, "null argument");
    *step = s->step;
    return TFL_OK;
}

int tfl_set_step(tfl_sim *s, int64_t step)
{
    if (!s) return fail(nullptr, TFL_E_INVAL, "null handle");
    if (step < 0) return fail(s, TFL_E_INVAL, "step must be >= 0");
    s->step = step;
    s->sampled0 = step > 0;
    return TFL_OK;
}

int tfl_save_state(tfl_sim *s, void *dst, void *stream)
{
    int rc = check_bound(s, false);
    if (rc != TFL_OK) return rc;
    if (!dst || !aligned(dst)) return fail(s, TFL_E_INVAL, "destination must be a 256-byte aligned device pointer");
    return copy_state(s, dst, nullptr, true, (hipStream_t)stream);
}

int tfl_load_state(tfl_sim *s, const void *src, void *stream)
{
    int rc = check_bound(s, false);
    if (rc != TFL_OK) return rc;
    if (!src || !aligned(src)) return fail(s, TFL_E_INVAL, "source must be a 256-byte aligned device pointer");
    return copy_state(s, nullptr, src, false, (hipStream_t)stream);
}

}  // extern "C"
