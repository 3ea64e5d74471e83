// Forward kernels of the two-fluid FDTD step for gfx950.
//
// One time step (Algorithm 1, steps 1-5 of step n-1 fused with steps 1-2 of
// step n, Sec. 3) is two HBM-bound sweeps:
//   H pass:   H^{n+1/2} = H^{n-1/2} - dt/mu0 curl E^n                (Faraday)
//   E pass:   Js^{n+1/2} = Js^{n-1/2} + dt ell_e/mu0 E^n              (London)
//             E^{n+1} = a_e E^n + b_e (curl H^{n+1/2} - Js^{n+1/2})     (Ampere, theta scheme)
// with a_e = (eps_e - (1-theta) sigma_e dt)/(eps_e + theta sigma_e dt) and
// b_e = dt/(eps_e + theta sigma_e dt), i.e. Algorithm 1 step 3 multiplied out.
// Per-edge materials are formed on the fly from the per-cell maps, or read as
// one 16-bit class per edge and a coefficient table when classes are bound
// (the CLS template argument).  The two sweeps can be replaced by one
// (fused_step_kernel), which reads the old fields from one set of buffers and
// writes the new ones to another.
//
// Each block owns a column tile of the x-y plane (rows of 64 cells, one
// wavefront each, 4 or 8 rows; the FP32 fused sweep takes rows of 256 or 128
// cells when they divide nx) and marches 8-64 planes along z (chosen at launch
// from the grid size), so the z neighbour of every stencil comes from
// registers; x and y neighbours come from L1/L2.  Blocks are renumbered so that each XCD
// (blocks are dealt to the 8 XCDs round robin) receives a contiguous range of
// tiles, keeping the halo rows of neighbouring tiles in the same L2.  The soft
// sources and the probe samples of a step ride along with the sweep that
// writes E^{n+1} (SideArgs), so a step with sources and probes is one launch.
#include <mutex>

#include "fdtd_common.h"

namespace tfl {
namespace {

// ---------------------------------------------------------------------------
// H pass (Faraday's law)
// ---------------------------------------------------------------------------
template <typename T, int TY, int TZ, int W>
__global__ __launch_bounds__(kTileX *TY, TFL_MIN_WAVES) void h_pass_kernel(const StepArgs<T> a)
{
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    int i, j, k0, k1;
    if (!tile_of_w<TY, TZ, W>(nx, ny, nz, i, j, k0, k1)) return;
    const long long sxy = a.g.sxy;
    const int ip = (i + 1 == nx) ? 0 : i + 1;
    const int jp = (j + 1 == ny) ? 0 : j + 1;
    const long long r0 = (long long)j * nx, r1 = (long long)jp * nx;
    const T *__restrict__ Ex = a.E[0];
    const T *__restrict__ Ey = a.E[1];
    const T *__restrict__ Ez = a.E[2];
    T *__restrict__ Hx = a.H[0];
    T *__restrict__ Hy = a.H[1];
    T *__restrict__ Hz = a.H[2];
    const T rdx = a.rd[0], rdy = a.rd[1], rdz = a.rd[2], hdt = a.hdt;
    const PmlAxis<T> &px = a.pml[0], &py = a.pml[1], &pz = a.pml[2];
    const int sx = px.on ? slab_slot(i, px.lo, px.hi, nx) : -1;
    const int sy = py.on ? slab_slot(j, py.lo, py.hi, ny) : -1;

    T exk = Ex[(long long)k0 * sxy + r0 + i];
    T eyk = Ey[(long long)k0 * sxy + r0 + i];
    for (int k = k0; k < k1; ++k) {
        const int kp = (k + 1 == nz) ? 0 : k + 1;
        const long long b0 = (long long)k * sxy, b1 = (long long)kp * sxy;
        const long long c = b0 + r0 + i;
        const T exk1 = Ex[b1 + r0 + i];
        const T eyk1 = Ey[b1 + r0 + i];
        const T ez = Ez[c];
        const T ez_x = Ez[b0 + r0 + ip];
        const T ez_y = Ez[b0 + r1 + i];
        const T ey_x = Ey[b0 + r0 + ip];
        const T ex_y = Ex[b0 + r1 + i];
        T dyEz = (ez_y - ez) * rdy, dzEy = (eyk1 - eyk) * rdz;  // Hx
        T dzEx = (exk1 - exk) * rdz, dxEz = (ez_x - ez) * rdx;  // Hy
        T dxEy = (ey_x - eyk) * rdx, dyEx = (ex_y - exk) * rdy; // Hz
        if (sx >= 0) {
            const long long p = ((long long)k * ny + j) * px.P + sx;
            dxEz = stretch(dxEz, px.psiH[0], p, px.bh[i], px.ch[i], px.kh[i]);  // Hy
            dxEy = stretch(dxEy, px.psiH[1], p, px.bh[i], px.ch[i], px.kh[i]);  // Hz
        }
        if (sy >= 0) {
            const long long p = ((long long)k * py.P + sy) * nx + i;
            dyEx = stretch(dyEx, py.psiH[0], p, py.bh[j], py.ch[j], py.kh[j]);  // Hz
            dyEz = stretch(dyEz, py.psiH[1], p, py.bh[j], py.ch[j], py.kh[j]);  // Hx
        }
        if (pz.on) {
            const int sz = slab_slot(k, pz.lo, pz.hi, nz);
            if (sz >= 0) {
                const long long p = ((long long)sz * ny + j) * nx + i;
                dzEy = stretch(dzEy, pz.psiH[0], p, pz.bh[k], pz.ch[k], pz.kh[k]);  // Hx
                dzEx = stretch(dzEx, pz.psiH[1], p, pz.bh[k], pz.ch[k], pz.kh[k]);  // Hy
            }
        }
        Hx[c] = Hx[c] - hdt * (dyEz - dzEy);
        Hy[c] = Hy[c] - hdt * (dzEx - dxEz);
        Hz[c] = Hz[c] - hdt * (dxEy - dyEx);
        exk = exk1;
        eyk = eyk1;
    }
}

// ---------------------------------------------------------------------------
// E pass (London supercurrent + Ampere's law with the theta-weighted Ohmic term)
// ---------------------------------------------------------------------------
// Coefficients of one edge (EdgeCoef) from the four cells sharing it.
template <typename T>
__device__ __forceinline__ EdgeCoef<T> edge_coef(const T e[4], const T s[4], const T l[4], T dt, T theta, T hdt)
{
    T eps, sig, ell;
    edge_material(e, s, l, eps, sig, ell);
    const T sdt = sig * dt;
    const T inv = T(1) / (eps + theta * sdt);
    return {(eps - (T(1) - theta) * sdt) * inv, dt * inv, hdt * ell};
}

// ---------------------------------------------------------------------------
// Soft sources and probes (Sec. 4.2, 5), folded into the E update of a sweep
// ---------------------------------------------------------------------------
constexpr int kProbeThreads = 256;

// Sum of the cnt values of a probe box, load(idx) in box order (x fastest), formed as 256 lanes
// would: lane t adds idx = t, t + 256, ... in order, each wavefront of 64 such lanes folds its sums
// by shuffles, and the four wavefront sums are added in order.  A block of any whole number of
// wavefronts gives the same bits (its wavefronts take the four parts in turn); every thread gets
// the sum.
template <typename Load>
__device__ __forceinline__ double probe_sum(long long cnt, Load load)
{
    __shared__ double part[kProbeThreads / 64];
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int lane = tid & 63, nw = (int)(blockDim.x * blockDim.y) >> 6;
    for (int vw = tid >> 6; vw < kProbeThreads / 64; vw += nw) {
        double acc = 0.0;
        for (long long idx = vw * 64 + lane; idx < cnt; idx += kProbeThreads) acc += load(idx);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
        if (lane == 0) part[vw] = acc;
    }
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < kProbeThreads / 64; ++w) s += part[w];
    return s;
}

// Sample n of probe p: the series value and the running DFT sum_n s_n dt exp(-2 pi i f n dt).
__device__ __forceinline__ void probe_record(const ProbeDesc &p, double s, long long n, double dt)
{
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    if (tid == 0 && p.series != nullptr && n < p.cap) p.series[n] = s;
    if (tid < p.nfreq) {
        const double ph = kTwoPi * p.freq[tid] * (double)n * dt;
        p.dft[2 * tid] += s * dt * cos(ph);
        p.dft[2 * tid + 1] -= s * dt * sin(ph);
    }
}

// Side work a wavefront can meet: bit p (p < 32) for source p, bit 32 + p for probe p, set when the
// box holds an edge of some lane's column (i, j) within planes [k0, k1).  Uniform over the
// wavefront, so the sweep's planes skip the side work with one scalar test where the mask is empty
// (nearly everywhere).
__device__ __forceinline__ uint64_t side_mask(const SideArgs &sd, int i, int j, int k0, int k1)
{
    uint64_t m = 0;
    auto meets = [&](const int *b) {
        return __any(i >= b[1] && i < b[2] && j >= b[3] && j < b[4] && k0 < b[6] && b[5] < k1);
    };
    for (int p = 0; p < sd.nsrc; ++p)
        if (meets(sd.sbox[p])) m |= 1ull << p;
    for (int p = 0; p < sd.nprobe; ++p)
        if (meets(sd.pbox[p])) m |= 1ull << (32 + p);
    return m;
}

// Side work at the new E of edge (i, j, k), component q, after the PEC walls, for the sources and
// probes of mask m: the sources whose boxes hold the edge add their values in source order, and the
// probes whose boxes hold it receive a copy of the result.
template <typename T>
__device__ __forceinline__ T add_sources(const SideArgs &sd, const double *sg, uint64_t m, int q, int i, int j, int k,
                                         T v)
{
    for (uint32_t ms = (uint32_t)m; ms != 0; ms &= ms - 1) {
        const int *b = sd.sbox[__builtin_ctz(ms)];
        if (b[0] == q && k >= b[5] && k < b[6] && j >= b[3] && j < b[4] && i >= b[1] && i < b[2])
            v = (T)((double)v + sg[__builtin_ctz(ms)]);
    }
    return v;
}

template <typename T>
__device__ __forceinline__ void probe_copy(const SideArgs &sd, void *const *copy, uint64_t m, int q, int i, int j,
                                           int k, T v)
{
    for (uint32_t mp = (uint32_t)(m >> 32); mp != 0; mp &= mp - 1) {
        const int p = __builtin_ctz(mp);
        const int *b = sd.pbox[p];
        if (b[0] == q && k >= b[5] && k < b[6] && j >= b[3] && j < b[4] && i >= b[1] && i < b[2]) {
            const long long c = ((long long)(k - b[5]) * (b[4] - b[3]) + (j - b[3])) * (b[2] - b[1]) + (i - b[1]);
            ((T *)copy[p])[c] = v;
        }
    }
}

template <typename T>
__device__ __forceinline__ T side_e(const SideArgs &sd, uint64_t m, int q, int i, int j, int k, T v)
{
    v = add_sources(sd, sd.sg, m, q, i, j, k, v);
    probe_copy(sd, sd.pcopy, m, q, i, j, k, v);
    return v;
}

// First thing of a sweep: blocks 0 .. nred-1 record the previous sweep's probe samples rn (and rn + 1
// after a two-step sweep), one probe per block, from the copies it left, in sample order.
template <typename T>
__device__ __forceinline__ void side_reduce(const SideArgs &sd)
{
    if ((int)blockIdx.x >= sd.nred) return;
    const ProbeDesc &p = sd.pdesc[blockIdx.x];
    const long long cnt = (long long)(p.i1 - p.i0) * (p.j1 - p.j0) * (p.k1 - p.k0);
    for (int r = 0; r < sd.nsamp; ++r) {
        if (r > 0) __syncthreads();  // every wavefront has read the previous sum's partials
        const T *c = (const T *)(r == 0 ? sd.rcopy[blockIdx.x] : sd.rcopy2[blockIdx.x]);
        const double s = probe_sum(cnt, [c](long long idx) { return (double)c[idx]; });
        probe_record(p, s, sd.rn + r, sd.dt);
    }
}

template <typename T, int TY, int TZ, bool CLS, int W>
__global__ __launch_bounds__(kTileX *TY, TFL_MIN_WAVES) void e_pass_kernel(const StepArgs<T> a)
{
    side_reduce<T>(a.side);
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    int i, j, k0, k1;
    if (!tile_of_w<TY, TZ, W>(nx, ny, nz, i, j, k0, k1)) return;
    const uint64_t side = side_mask(a.side, i, j, k0, k1);
    const long long sxy = a.g.sxy;
    const int im = (i == 0) ? nx - 1 : i - 1;
    const int jm = (j == 0) ? ny - 1 : j - 1;
    // byte offsets inside one plane (a plane is below 4 GiB): each access is a uniform plane base in
    // scalar registers plus one of these four 32-bit lane offsets
    const uint32_t o00 = uint32_t(j * nx + i) * sizeof(T), o10 = uint32_t(j * nx + im) * sizeof(T);
    const uint32_t o01 = uint32_t(jm * nx + i) * sizeof(T), o11 = uint32_t(jm * nx + im) * sizeof(T);
    const T rdx = a.rd[0], rdy = a.rd[1], rdz = a.rd[2];
    const T dt = a.dt, theta = a.theta, hdt = a.hdt;
    const PmlAxis<T> &px = a.pml[0], &py = a.pml[1], &pz = a.pml[2];
    const int sx = px.on ? slab_slot(i, px.lo, px.hi, nx) : -1;
    const int sy = py.on ? slab_slot(j, py.lo, py.hi, ny) : -1;
    const bool wall_x = px.on && i == 0;
    const bool wall_y = py.on && j == 0;

    // Materials of plane k-1 at cells (i,j), (i-1,j), (i,j-1) are carried in registers and the edge
    // coefficients of a plane are formed one iteration ahead, so all loads of an iteration (Js on
    // superconducting edges, H, E, the maps of the next plane) are issued before the first wait.
    T pe00, pe10, pe01, ps00, ps10, ps01, pl00, pl10, pl01;
    EdgeCoef<T> cx, cy, cz;
    struct Maps {
        T e00, e10, e01, e11, s00, s10, s01, s11, l00, l10, l01, l11;
    };
    struct Classes {
        uint32_t x, y, z;
    };
    const uint32_t oc = uint32_t(j * nx + i) * 2u;  // byte offset into a class plane
    auto load_maps = [&](int kk) {
        const long long b = opaque_offset((long long)kk * sxy);
        if constexpr (CLS) {
            return Classes{ldp(a.cls[0] + b, oc), ldp(a.cls[1] + b, oc), ldp(a.cls[2] + b, oc)};
        } else {
            const T *me = a.eps + b, *ms = a.sig + b, *ml = a.ell + b;
            return Maps{ldp(me, o00), ldp(me, o10), ldp(me, o01), ldp(me, o11),
                        ldp(ms, o00), ldp(ms, o10), ldp(ms, o01), ldp(ms, o11),
                        ldp(ml, o00), ldp(ml, o10), ldp(ml, o01), ldp(ml, o11)};
        }
    };
    auto coefs = [&](const auto &m) {
        if constexpr (CLS) {
            cx = class_coef(a.ctab, m.x);
            cy = class_coef(a.ctab, m.y);
            cz = class_coef(a.ctab, m.z);
        } else {
            {   // Ex: cells (j,k), (j,k-1), (j-1,k), (j-1,k-1)
                const T e[4] = {m.e00, pe00, m.e01, pe01}, s[4] = {m.s00, ps00, m.s01, ps01},
                        l[4] = {m.l00, pl00, m.l01, pl01};
                cx = edge_coef(e, s, l, dt, theta, hdt);
            }
            {   // Ey: cells (k,i), (k,i-1), (k-1,i), (k-1,i-1)
                const T e[4] = {m.e00, m.e10, pe00, pe10}, s[4] = {m.s00, m.s10, ps00, ps10},
                        l[4] = {m.l00, m.l10, pl00, pl10};
                cy = edge_coef(e, s, l, dt, theta, hdt);
            }
            {   // Ez: cells (i,j), (i,j-1), (i-1,j), (i-1,j-1)
                const T e[4] = {m.e00, m.e01, m.e10, m.e11}, s[4] = {m.s00, m.s01, m.s10, m.s11},
                        l[4] = {m.l00, m.l01, m.l10, m.l11};
                cz = edge_coef(e, s, l, dt, theta, hdt);
            }
            pe00 = m.e00; pe10 = m.e10; pe01 = m.e01;
            ps00 = m.s00; ps10 = m.s10; ps01 = m.s01;
            pl00 = m.l00; pl10 = m.l10; pl01 = m.l01;
        }
    };
    const int km0 = (k0 == 0) ? nz - 1 : k0 - 1;
    T hx_km, hy_km;
    {
        const long long b = (long long)km0 * sxy;
        if constexpr (!CLS) {
            const Maps m = load_maps(km0);
            pe00 = m.e00; pe10 = m.e10; pe01 = m.e01;
            ps00 = m.s00; ps10 = m.s10; ps01 = m.s01;
            pl00 = m.l00; pl10 = m.l10; pl01 = m.l01;
        }
        hx_km = ldp(a.H[0] + b, o00);
        hy_km = ldp(a.H[1] + b, o00);
    }
    coefs(load_maps(k0));

    for (int k = k0; k < k1; ++k) {
        const long long b = opaque_offset((long long)k * sxy);
        T *Jx = a.J[0] + b, *Jy = a.J[1] + b, *Jz = a.J[2] + b;
        const EdgeCoef<T> qx = cx, qy = cy, qz = cz;
        T jx = T(0), jy = T(0), jz = T(0);
        if (qx.cj > T(0)) jx = ldp(Jx, o00);
        if (qy.cj > T(0)) jy = ldp(Jy, o00);
        if (qz.cj > T(0)) jz = ldp(Jz, o00);
        const T *Hx = a.H[0] + b, *Hy = a.H[1] + b, *Hz = a.H[2] + b;
        const T *Ex = a.E[0] + b, *Ey = a.E[1] + b, *Ez = a.E[2] + b;
        const T hx = ldp(Hx, o00), hy = ldp(Hy, o00), hz = ldp(Hz, o00);
        const T hz_xm = ldp(Hz, o10), hz_ym = ldp(Hz, o01);
        const T hy_xm = ldp(Hy, o10), hx_ym = ldp(Hx, o01);
        const T ex = ldp(Ex, o00), ey = ldp(Ey, o00), ez = ldp(Ez, o00);
        // materials of the next plane (the last iteration re-reads its own plane and discards them)
        const auto mn = load_maps(k + 1 < nz ? k + 1 : k);

        T dyHz = (hz - hz_ym) * rdy, dzHy = (hy - hy_km) * rdz;  // Ex
        T dzHx = (hx - hx_km) * rdz, dxHz = (hz - hz_xm) * rdx;  // Ey
        T dxHy = (hy - hy_xm) * rdx, dyHx = (hx - hx_ym) * rdy;  // Ez
        if (sx >= 0) {
            const long long p = ((long long)k * ny + j) * px.P + sx;
            dxHz = stretch(dxHz, px.psiE[0], p, px.bn[i], px.cn[i], px.kn[i]);  // Ey
            dxHy = stretch(dxHy, px.psiE[1], p, px.bn[i], px.cn[i], px.kn[i]);  // Ez
        }
        if (sy >= 0) {
            const long long p = ((long long)k * py.P + sy) * nx + i;
            dyHx = stretch(dyHx, py.psiE[0], p, py.bn[j], py.cn[j], py.kn[j]);  // Ez
            dyHz = stretch(dyHz, py.psiE[1], p, py.bn[j], py.cn[j], py.kn[j]);  // Ex
        }
        bool wall_z = false;
        if (pz.on) {
            wall_z = (k == 0);
            const int sz = slab_slot(k, pz.lo, pz.hi, nz);
            if (sz >= 0) {
                const long long p = ((long long)sz * ny + j) * nx + i;
                dzHy = stretch(dzHy, pz.psiE[0], p, pz.bn[k], pz.cn[k], pz.kn[k]);  // Ex
                dzHx = stretch(dzHx, pz.psiE[1], p, pz.bn[k], pz.cn[k], pz.kn[k]);  // Ey
            }
        }
        if (qx.cj > T(0)) { jx = jx + qx.cj * ex; stp(Jx, o00, jx); }
        if (qy.cj > T(0)) { jy = jy + qy.cj * ey; stp(Jy, o00, jy); }
        if (qz.cj > T(0)) { jz = jz + qz.cj * ez; stp(Jz, o00, jz); }
        const T nex = qx.ca * ex + qx.cb * ((dyHz - dzHy) - jx);
        const T ney = qy.ca * ey + qy.cb * ((dzHx - dxHz) - jy);
        const T nez = qz.ca * ez + qz.cb * ((dxHy - dyHx) - jz);
        // E and Eout are the same arrays except in the adjoint's recomputation; each lane reads E at
        // its own offset before writing Eout there and no other lane touches that word
        T vx = (wall_y || wall_z) ? T(0) : nex, vy = (wall_z || wall_x) ? T(0) : ney;
        T vz = (wall_x || wall_y) ? T(0) : nez;
        if (side != 0) {
            vx = side_e(a.side, side, 0, i, j, k, vx);
            vy = side_e(a.side, side, 1, i, j, k, vy);
            vz = side_e(a.side, side, 2, i, j, k, vz);
        }
        T *Exo = a.Eout[0] + b, *Eyo = a.Eout[1] + b, *Ezo = a.Eout[2] + b;
        stp(Exo, o00, vx);
        stp(Eyo, o00, vy);
        stp(Ezo, o00, vz);
        hx_km = hx;
        hy_km = hy;
        coefs(mn);
    }
}

// ---------------------------------------------------------------------------
// Fused step (H and E pass in one sweep)
// ---------------------------------------------------------------------------
// Each lane updates E at its own edges and H at its own faces.  The E update
// needs H^{n+1/2} also at the faces x-1 (Hz, Hy) and y-1 (Hz, Hx) of its cell,
// which belong to other lanes or blocks: the lane recomputes them from E^n and
// H^{n-1/2}, which the sweep only reads (the new fields go to the other pair of
// buffers), with the same arithmetic as the H pass.  H^{n+1/2} at z-1 is the
// lane's own value from the previous plane.  Per cell the sweep reads E, H, the
// maps and Js and writes E, H and Js once: 15 + 6 f_J words instead of the
// 21 + 6 f_J of the two passes (12 + 6 f_J words and three 16-bit classes with
// edge classes).  NT: the new E and H are stored with a
// nontemporal hint (chosen at launch for grids well beyond the infinity cache,
// where keeping them would only evict lines the sweep still reads).  PML: the
// CPML variant (an instantiation of its own, so periodic grids run the code
// without it): the H-side auxiliary variables go from psiH to psiHo (the faces
// recomputed at x-1 and y-1 read the old values), the E-side ones are updated
// in place, and tangential E is zeroed on the PEC walls, all with the
// arithmetic of the two passes.
template <typename T, int TY, int TZ, bool CLS, bool NT, int TX, bool PML>
__global__ __launch_bounds__(TX *TY, TFL_MIN_WAVES) void fused_step_kernel(const StepArgs<T> a)
{
    side_reduce<T>(a.side);
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    int i, j, k0, k1;
    if (!tile_of<TY, TZ, TX>(nx, ny, nz, i, j, k0, k1, PML && zmix_of(a.pml[2], nz))) return;
    const uint64_t side = side_mask(a.side, i, j, k0, k1);
    const long long sxy = a.g.sxy;
    const int im = (i == 0) ? nx - 1 : i - 1, ip = (i + 1 == nx) ? 0 : i + 1;
    const int jm = (j == 0) ? ny - 1 : j - 1, jp = (j + 1 == ny) ? 0 : j + 1;
    constexpr uint32_t w = sizeof(T);
    const uint32_t o00 = uint32_t(j * nx + i) * w, o10 = uint32_t(j * nx + im) * w;
    const uint32_t o01 = uint32_t(jm * nx + i) * w, o11 = uint32_t(jm * nx + im) * w;
    const uint32_t oxp = uint32_t(j * nx + ip) * w, oyp = uint32_t(jp * nx + i) * w;
    const uint32_t oxm_yp = uint32_t(jp * nx + im) * w, oxp_ym = uint32_t(jm * nx + ip) * w;
    const T rdx = a.rd[0], rdy = a.rd[1], rdz = a.rd[2];
    const T dt = a.dt, theta = a.theta, hdt = a.hdt;
    // loads at a plane base plus a lane offset (ldo on CPML grids, where the longer body would
    // otherwise keep 64-bit addresses live across the z loop)
    auto ld = [](const auto *base, uint32_t off) {
        if constexpr (PML) return ldo(base, off);
        else return ldp(base, off);
    };
    // CPML grids (PML): slab slots (-1 outside) of the lane's column and of column x-1, of the
    // row and of row y-1 (a wavefront is one row: those are scalar), and the PEC walls; the
    // auxiliary variables and coefficient tables are addressed as scalar bases plus these lane
    // byte offsets
    const PmlAxis<T> &px = a.pml[0], &py = a.pml[1], &pz = a.pml[2];
    [[maybe_unused]] int sx = -1, sxm = -1, sy = -1, sym = -1, jw = j, jmw = jm;
    [[maybe_unused]] bool wall_x = false, wall_y = false;
    [[maybe_unused]] uint32_t osx = 0, osxm = 0;
    [[maybe_unused]] const uint32_t oi = uint32_t(i) * w, oim = uint32_t(im) * w;
    if constexpr (PML) {
        jw = __builtin_amdgcn_readfirstlane(j);
        jmw = __builtin_amdgcn_readfirstlane(jm);
        sx = px.on ? slab_slot(i, px.lo, px.hi, nx) : -1;
        sxm = px.on ? slab_slot(im, px.lo, px.hi, nx) : -1;
        sy = py.on ? slab_slot(jw, py.lo, py.hi, ny) : -1;
        sym = py.on ? slab_slot(jmw, py.lo, py.hi, ny) : -1;
        osx = uint32_t(sx) * w;
        osxm = uint32_t(sxm) * w;
        wall_x = px.on && i == 0;
        wall_y = py.on && jw == 0;
    }
    // x slabs cut through the wavefronts of a row: their coefficients (the tables cover the whole
    // axis) are loaded once, and each plane's x-slab variables are loaded with the plane's other
    // loads at slots clamped into the slab, so that only arithmetic and stores depend on the lane
    // (only in the wavefronts whose columns, or their x-1 neighbours, lie in a slab)
    [[maybe_unused]] const bool xv = PML && px.on && px.P > 0 && __any(sx >= 0 || sxm >= 0);
    [[maybe_unused]] T xbh = T(0), xch = T(0), xkh = T(0), xbn = T(0), xcn = T(0), xkn = T(0);
    [[maybe_unused]] T xbhm = T(0), xchm = T(0), xkhm = T(0);
    [[maybe_unused]] uint32_t osxc = 0, osxmc = 0;
    if constexpr (PML) {
        if (xv) {
            xbh = ldo(px.bh, oi); xch = ldo(px.ch, oi); xkh = ldo(px.kh, oi);
            xbn = ldo(px.bn, oi); xcn = ldo(px.cn, oi); xkn = ldo(px.kn, oi);
            xbhm = ldo(px.bh, oim); xchm = ldo(px.ch, oim); xkhm = ldo(px.kh, oim);
            osxc = uint32_t(sx >= 0 ? sx : 0) * w;
            osxmc = uint32_t(sxm >= 0 ? sxm : 0) * w;
        }
    }

    T pe00, pe10, pe01, ps00, ps10, ps01, pl00, pl10, pl01;
    EdgeCoef<T> cx, cy, cz;
    struct Maps {
        T e00, e10, e01, e11, s00, s10, s01, s11, l00, l10, l01, l11;
    };
    struct Classes {
        uint32_t x, y, z;
    };
    const uint32_t oc = uint32_t(j * nx + i) * 2u;  // byte offset into a class plane
    auto load_maps = [&](int kk) {
        const long long b = opaque_offset((long long)kk * sxy);
        if constexpr (CLS) {
            return Classes{ld(a.cls[0] + b, oc), ld(a.cls[1] + b, oc), ld(a.cls[2] + b, oc)};
        } else {
            const T *me = a.eps + b, *ms = a.sig + b, *ml = a.ell + b;
            return Maps{ld(me, o00), ld(me, o10), ld(me, o01), ld(me, o11),
                        ld(ms, o00), ld(ms, o10), ld(ms, o01), ld(ms, o11),
                        ld(ml, o00), ld(ml, o10), ld(ml, o01), ld(ml, o11)};
        }
    };
    auto coefs = [&](const auto &m) {
        if constexpr (CLS) {
            cx = class_coef(a.ctab, m.x);
            cy = class_coef(a.ctab, m.y);
            cz = class_coef(a.ctab, m.z);
        } else {
            {   // Ex: cells (j,k), (j,k-1), (j-1,k), (j-1,k-1)
                const T e[4] = {m.e00, pe00, m.e01, pe01}, s[4] = {m.s00, ps00, m.s01, ps01},
                        l[4] = {m.l00, pl00, m.l01, pl01};
                cx = edge_coef(e, s, l, dt, theta, hdt);
            }
            {   // Ey: cells (k,i), (k,i-1), (k-1,i), (k-1,i-1)
                const T e[4] = {m.e00, m.e10, pe00, pe10}, s[4] = {m.s00, m.s10, ps00, ps10},
                        l[4] = {m.l00, m.l10, pl00, pl10};
                cy = edge_coef(e, s, l, dt, theta, hdt);
            }
            {   // Ez: cells (i,j), (i,j-1), (i-1,j), (i-1,j-1)
                const T e[4] = {m.e00, m.e01, m.e10, m.e11}, s[4] = {m.s00, m.s01, m.s10, m.s11},
                        l[4] = {m.l00, m.l01, m.l10, m.l11};
                cz = edge_coef(e, s, l, dt, theta, hdt);
            }
            pe00 = m.e00; pe10 = m.e10; pe01 = m.e01;
            ps00 = m.s00; ps10 = m.s10; ps01 = m.s01;
            pl00 = m.l00; pl10 = m.l10; pl01 = m.l01;
        }
    };
    // H^{n+1/2} (Hx, Hy) at plane k0-1 of the lane's own faces, and E^n of plane k0 that the
    // loop carries from one plane to the next: Ex at (i,j), (i-1,j); Ey at (i,j), (i,j-1)
    const int km0 = (k0 == 0) ? nz - 1 : k0 - 1;
    T hx_km, hy_km, ex0, exm, ey0, eym;
    {
        const long long bm = (long long)km0 * sxy, b = (long long)k0 * sxy;
        const T *Ex = a.E[0] + bm, *Ey = a.E[1] + bm, *Ez = a.E[2] + bm;
        const T exk = ld(Ex, o00), eyk = ld(Ey, o00), ez = ld(Ez, o00);
        const T exk1 = ld(a.E[0] + b, o00), eyk1 = ld(a.E[1] + b, o00);
        const T ez_x = ld(Ez, oxp), ez_y = ld(Ez, oyp);
        T dyEz = (ez_y - ez) * rdy, dzEy = (eyk1 - eyk) * rdz;
        T dzEx = (exk1 - exk) * rdz, dxEz = (ez_x - ez) * rdx;
        if constexpr (PML) {  // the H pass's stretching at plane k0-1, without storing (another tile does)
            if (sx >= 0)
                dxEz = stretch_virtual_o(dxEz, px.psiH[0] + ((long long)km0 * ny + jw) * px.P, osx, ldo(px.bh, oi),
                                         ldo(px.ch, oi), ldo(px.kh, oi));
            if (sy >= 0)
                dyEz = stretch_virtual_o(dyEz, py.psiH[1] + ((long long)km0 * py.P + sy) * nx, oi, py.bh[jw], py.ch[jw],
                                         py.kh[jw]);
            const int sz = pz.on ? slab_slot(km0, pz.lo, pz.hi, nz) : -1;
            if (sz >= 0) {
                const long long r = ((long long)sz * ny + jw) * nx;
                dzEy = stretch_virtual_o(dzEy, pz.psiH[0] + r, oi, pz.bh[km0], pz.ch[km0], pz.kh[km0]);
                dzEx = stretch_virtual_o(dzEx, pz.psiH[1] + r, oi, pz.bh[km0], pz.ch[km0], pz.kh[km0]);
            }
        }
        hx_km = ld(a.H[0] + bm, o00) - hdt * (dyEz - dzEy);
        hy_km = ld(a.H[1] + bm, o00) - hdt * (dzEx - dxEz);
        if constexpr (!CLS) {
            const Maps m = load_maps(km0);
            pe00 = m.e00; pe10 = m.e10; pe01 = m.e01;
            ps00 = m.s00; ps10 = m.s10; ps01 = m.s01;
            pl00 = m.l00; pl10 = m.l10; pl01 = m.l01;
        }
        ex0 = exk1;
        ey0 = eyk1;
        exm = ld(a.E[0] + b, o10);
        eym = ld(a.E[1] + b, o01);
    }
    coefs(load_maps(k0));

    for (int k = k0; k < k1; ++k) {
        const int kp = (k + 1 == nz) ? 0 : k + 1;
        const long long b = opaque_offset((long long)k * sxy), bp = opaque_offset((long long)kp * sxy);
        T *Jx = a.J[0] + b, *Jy = a.J[1] + b, *Jz = a.J[2] + b;
        const EdgeCoef<T> qx = cx, qy = cy, qz = cz;
        T jx = T(0), jy = T(0), jz = T(0);
        if (qx.cj > T(0)) jx = ld(Jx, o00);
        if (qy.cj > T(0)) jy = ld(Jy, o00);
        if (qz.cj > T(0)) jz = ld(Jz, o00);
        const T *Ex = a.E[0] + b, *Ey = a.E[1] + b, *Ez = a.E[2] + b;
        const T *Hx = a.H[0] + b, *Hy = a.H[1] + b, *Hz = a.H[2] + b;
        // E^n of this plane and the next
        const T ex_yp = ld(Ex, oyp), exm_yp = ld(Ex, oxm_yp), ex_ym = ld(Ex, o01);
        const T ey_xp = ld(Ey, oxp), ey_xm = ld(Ey, o10), eym_xp = ld(Ey, oxp_ym);
        const T ez = ld(Ez, o00), ez_xp = ld(Ez, oxp), ez_yp = ld(Ez, oyp), ez_xm = ld(Ez, o10), ez_ym = ld(Ez, o01);
        const T ex1 = ld(a.E[0] + bp, o00), exm1 = ld(a.E[0] + bp, o10);
        const T ey1 = ld(a.E[1] + bp, o00), eym1 = ld(a.E[1] + bp, o01);
        // H^{n-1/2}: own faces, Hz and Hy at x-1, Hz and Hx at y-1
        const T hx = ld(Hx, o00), hy = ld(Hy, o00), hz = ld(Hz, o00);
        const T hz_xm = ld(Hz, o10), hy_xm = ld(Hy, o10), hz_ym = ld(Hz, o01), hx_ym = ld(Hx, o01);
        const auto mn = load_maps(k + 1 < nz ? k + 1 : k);

        [[maybe_unused]] T qh0 = T(0), qh1 = T(0), qh1ym = T(0), qm0 = T(0), qm1 = T(0), qe0 = T(0), qe1 = T(0);
        if constexpr (PML) {
            if (xv) {
                const long long r = ((long long)k * ny + jw) * px.P, rym = ((long long)k * ny + jmw) * px.P;
                qh0 = ldo(px.psiH[0] + r, osxc);
                qh1 = ldo(px.psiH[1] + r, osxc);
                qh1ym = ldo(px.psiH[1] + rym, osxc);
                qm0 = ldo(px.psiH[0] + r, osxmc);
                qm1 = ldo(px.psiH[1] + r, osxmc);
                qe0 = ldo(px.psiE[0] + r, osxc);
                qe1 = ldo(px.psiE[1] + r, osxc);
            }
        }
        // z slabs (a plane is in one or not): the plane's auxiliary variables of the lane's column,
        // loaded with the plane's other loads (the H-side ones also at x-1 and y-1)
        [[maybe_unused]] int sz = -1;
        [[maybe_unused]] T zh0 = T(0), zh1 = T(0), zh1xm = T(0), zh0ym = T(0), ze0 = T(0), ze1 = T(0);
        if constexpr (PML) {
            sz = pz.on ? slab_slot(k, pz.lo, pz.hi, nz) : -1;
            if (sz >= 0) {
                const long long r = ((long long)sz * ny + jw) * nx, rym = ((long long)sz * ny + jmw) * nx;
                zh0 = ldo(pz.psiH[0] + r, oi);
                zh1 = ldo(pz.psiH[1] + r, oi);
                zh1xm = ldo(pz.psiH[1] + r, oim);
                zh0ym = ldo(pz.psiH[0] + rym, oi);
                ze0 = ldo(pz.psiE[0] + r, oi);
                ze1 = ldo(pz.psiE[1] + r, oi);
            }
        }

        // H^{n+1/2} with the H pass's arithmetic: own faces, Hz and Hy at x-1, Hz and Hx at y-1
        T nhx, nhy, nhz, nhz_xm, nhy_xm, nhz_ym, nhx_ym;
        if constexpr (!PML) {
            nhx = hx - hdt * ((ez_yp - ez) * rdy - (ey1 - ey0) * rdz);
            nhy = hy - hdt * ((ex1 - ex0) * rdz - (ez_xp - ez) * rdx);
            nhz = hz - hdt * ((ey_xp - ey0) * rdx - (ex_yp - ex0) * rdy);
            nhz_xm = hz_xm - hdt * ((ey0 - ey_xm) * rdx - (exm_yp - exm) * rdy);
            nhy_xm = hy_xm - hdt * ((exm1 - exm) * rdz - (ez - ez_xm) * rdx);
            nhz_ym = hz_ym - hdt * ((eym_xp - eym) * rdx - (ex0 - ex_ym) * rdy);
            nhx_ym = hx_ym - hdt * ((ez - ez_ym) * rdy - (eym1 - eym) * rdz);
        } else {
            T dyEz = (ez_yp - ez) * rdy, dzEy = (ey1 - ey0) * rdz;              // Hx
            T dzEx = (ex1 - ex0) * rdz, dxEz = (ez_xp - ez) * rdx;              // Hy
            T dxEy = (ey_xp - ey0) * rdx, dyEx = (ex_yp - ex0) * rdy;           // Hz
            T dxEy_xm = (ey0 - ey_xm) * rdx, dyEx_xm = (exm_yp - exm) * rdy;    // Hz at x-1
            T dzEx_xm = (exm1 - exm) * rdz, dxEz_xm = (ez - ez_xm) * rdx;       // Hy at x-1
            T dxEy_ym = (eym_xp - eym) * rdx, dyEx_ym = (ex0 - ex_ym) * rdy;    // Hz at y-1
            T dyEz_ym = (ez - ez_ym) * rdy, dzEy_ym = (eym1 - eym) * rdz;       // Hx at y-1
            // stretched differences: the lane's own faces update their variables (old set in,
            // new set out); the faces at x-1 and y-1 belong to other lanes and only read them
            if (sx >= 0) {
                const long long r = ((long long)k * ny + jw) * px.P;
                T p0, p1, pv;
                dxEz = stretch_v(dxEz, qh0, xbh, xch, xkh, p0);
                dxEy = stretch_v(dxEy, qh1, xbh, xch, xkh, p1);
                dxEy_ym = stretch_v(dxEy_ym, qh1ym, xbh, xch, xkh, pv);
                sto(px.psiHo[0] + r, osx, p0);
                sto(px.psiHo[1] + r, osx, p1);
            }
            if (sxm >= 0) {
                T pv;
                dxEy_xm = stretch_v(dxEy_xm, qm1, xbhm, xchm, xkhm, pv);
                dxEz_xm = stretch_v(dxEz_xm, qm0, xbhm, xchm, xkhm, pv);
            }
            if (sy >= 0) {
                const long long r = ((long long)k * py.P + sy) * nx;
                const T bh = py.bh[jw], ch = py.ch[jw], kh = py.kh[jw];
                dyEx = stretch_to_o(dyEx, py.psiH[0] + r, py.psiHo[0] + r, oi, bh, ch, kh);
                dyEz = stretch_to_o(dyEz, py.psiH[1] + r, py.psiHo[1] + r, oi, bh, ch, kh);
                dyEx_xm = stretch_virtual_o(dyEx_xm, py.psiH[0] + r, oim, bh, ch, kh);
            }
            if (sym >= 0) {
                const long long r = ((long long)k * py.P + sym) * nx;
                const T bh = py.bh[jmw], ch = py.ch[jmw], kh = py.kh[jmw];
                dyEx_ym = stretch_virtual_o(dyEx_ym, py.psiH[0] + r, oi, bh, ch, kh);
                dyEz_ym = stretch_virtual_o(dyEz_ym, py.psiH[1] + r, oi, bh, ch, kh);
            }
            if (sz >= 0) {
                const long long r = ((long long)sz * ny + jw) * nx;
                const T bh = pz.bh[k], ch = pz.ch[k], kh = pz.kh[k];
                T p0, p1, pv;
                dzEy = stretch_v(dzEy, zh0, bh, ch, kh, p0);
                dzEx = stretch_v(dzEx, zh1, bh, ch, kh, p1);
                sto(pz.psiHo[0] + r, oi, p0);
                sto(pz.psiHo[1] + r, oi, p1);
                dzEx_xm = stretch_v(dzEx_xm, zh1xm, bh, ch, kh, pv);
                dzEy_ym = stretch_v(dzEy_ym, zh0ym, bh, ch, kh, pv);
            }
            nhx = hx - hdt * (dyEz - dzEy);
            nhy = hy - hdt * (dzEx - dxEz);
            nhz = hz - hdt * (dxEy - dyEx);
            nhz_xm = hz_xm - hdt * (dxEy_xm - dyEx_xm);
            nhy_xm = hy_xm - hdt * (dzEx_xm - dxEz_xm);
            nhz_ym = hz_ym - hdt * (dxEy_ym - dyEx_ym);
            nhx_ym = hx_ym - hdt * (dyEz_ym - dzEy_ym);
        }
        T *Hxo = a.Hout[0] + b, *Hyo = a.Hout[1] + b, *Hzo = a.Hout[2] + b;
        stp_hint<NT>(Hxo, o00, nhx);
        stp_hint<NT>(Hyo, o00, nhy);
        stp_hint<NT>(Hzo, o00, nhz);

        // E^{n+1} with the E pass's arithmetic
        if constexpr (!PML) {
            const T dyHz = (nhz - nhz_ym) * rdy, dzHy = (nhy - hy_km) * rdz;  // Ex
            const T dzHx = (nhx - hx_km) * rdz, dxHz = (nhz - nhz_xm) * rdx;  // Ey
            const T dxHy = (nhy - nhy_xm) * rdx, dyHx = (nhx - nhx_ym) * rdy;  // Ez
            if (qx.cj > T(0)) { jx = jx + qx.cj * ex0; stp(Jx, o00, jx); }
            if (qy.cj > T(0)) { jy = jy + qy.cj * ey0; stp(Jy, o00, jy); }
            if (qz.cj > T(0)) { jz = jz + qz.cj * ez; stp(Jz, o00, jz); }
            T nex = qx.ca * ex0 + qx.cb * ((dyHz - dzHy) - jx);
            T ney = qy.ca * ey0 + qy.cb * ((dzHx - dxHz) - jy);
            T nez = qz.ca * ez + qz.cb * ((dxHy - dyHx) - jz);
            if (side != 0) {
                nex = side_e(a.side, side, 0, i, j, k, nex);
                ney = side_e(a.side, side, 1, i, j, k, ney);
                nez = side_e(a.side, side, 2, i, j, k, nez);
            }
            T *Exo = a.Eout[0] + b, *Eyo = a.Eout[1] + b, *Ezo = a.Eout[2] + b;
            stp_hint<NT>(Exo, o00, nex);
            stp_hint<NT>(Eyo, o00, ney);
            stp_hint<NT>(Ezo, o00, nez);
        } else {
            T dyHz = (nhz - nhz_ym) * rdy, dzHy = (nhy - hy_km) * rdz;  // Ex
            T dzHx = (nhx - hx_km) * rdz, dxHz = (nhz - nhz_xm) * rdx;  // Ey
            T dxHy = (nhy - nhy_xm) * rdx, dyHx = (nhx - nhx_ym) * rdy;  // Ez
            {  // E-side variables: only this lane touches them, in place
                if (sx >= 0) {
                    const long long r = ((long long)k * ny + jw) * px.P;
                    T p0, p1;
                    dxHz = stretch_v(dxHz, qe0, xbn, xcn, xkn, p0);  // Ey
                    dxHy = stretch_v(dxHy, qe1, xbn, xcn, xkn, p1);  // Ez
                    sto(px.psiE[0] + r, osx, p0);
                    sto(px.psiE[1] + r, osx, p1);
                }
                if (sy >= 0) {
                    const long long r = ((long long)k * py.P + sy) * nx;
                    dyHx = stretch_o(dyHx, py.psiE[0] + r, oi, py.bn[jw], py.cn[jw], py.kn[jw]);  // Ez
                    dyHz = stretch_o(dyHz, py.psiE[1] + r, oi, py.bn[jw], py.cn[jw], py.kn[jw]);  // Ex
                }
                if (sz >= 0) {
                    const long long r = ((long long)sz * ny + jw) * nx;
                    T p0, p1;
                    dzHy = stretch_v(dzHy, ze0, pz.bn[k], pz.cn[k], pz.kn[k], p0);  // Ex
                    dzHx = stretch_v(dzHx, ze1, pz.bn[k], pz.cn[k], pz.kn[k], p1);  // Ey
                    sto(pz.psiE[0] + r, oi, p0);
                    sto(pz.psiE[1] + r, oi, p1);
                }
            }
            if (qx.cj > T(0)) { jx = jx + qx.cj * ex0; stp(Jx, o00, jx); }
            if (qy.cj > T(0)) { jy = jy + qy.cj * ey0; stp(Jy, o00, jy); }
            if (qz.cj > T(0)) { jz = jz + qz.cj * ez; stp(Jz, o00, jz); }
            T nex = qx.ca * ex0 + qx.cb * ((dyHz - dzHy) - jx);
            T ney = qy.ca * ey0 + qy.cb * ((dzHx - dxHz) - jy);
            T nez = qz.ca * ez + qz.cb * ((dxHy - dyHx) - jz);
            {  // tangential E on the PEC walls
                const bool wall_z = pz.on && k == 0;
                nex = (wall_y || wall_z) ? T(0) : nex;
                ney = (wall_z || wall_x) ? T(0) : ney;
                nez = (wall_x || wall_y) ? T(0) : nez;
            }
            if (side != 0) {
                nex = side_e(a.side, side, 0, i, jw, k, nex);
                ney = side_e(a.side, side, 1, i, jw, k, ney);
                nez = side_e(a.side, side, 2, i, jw, k, nez);
            }
            T *Exo = a.Eout[0] + b, *Eyo = a.Eout[1] + b, *Ezo = a.Eout[2] + b;
            stp_hint<NT>(Exo, o00, nex);
            stp_hint<NT>(Eyo, o00, ney);
            stp_hint<NT>(Ezo, o00, nez);
        }
        hx_km = nhx;
        hy_km = nhy;
        ex0 = ex1;
        exm = exm1;
        ey0 = ey1;
        eym = eym1;
        coefs(mn);
    }
}

// ---------------------------------------------------------------------------
// Two time steps in one sweep (temporal blocking; grids with edge classes)
// ---------------------------------------------------------------------------
// A block covers a footprint of 64 x TY columns of the x-y plane (one wavefront per row) and marches
// along z, one plane per iteration, the second step one plane behind the first:
//   A  H^{n+1/2}(k) at the lane's own faces and at its x-1 and y-1 faces, from E^n and H^{n-1/2}
//      (the fused sweep's first half);
//   B  Js^{n+1/2}(k) and E^{n+1}(k), kept in registers, E^{n+1}(k) also written to LDS;
//   C  H^{n+3/2}(k-1) at the lane's own faces from E^{n+1}(k-1) (own, and x+1 / y+1 from LDS) and
//      E^{n+1}(k) (own), written to LDS;
//   D  Js^{n+3/2}(k-1) and E^{n+2}(k-1) from H^{n+3/2}(k-1) (own, and x-1 / y-1 from LDS) and
//      H^{n+3/2}(k-2) (own, from the previous iteration).
// Stage A reads E^n and H^{n-1/2} from LDS tiles of the footprint's 64 columns with the rows -1..TY
// (as each component's stencil needs), filled by asynchronous global-to-LDS loads issued two planes
// ahead, before the first barrier of a plane: E^n in a ring of four planes (stage A reads planes k and
// k+1, plane k+2 is in flight, plane k+3 is issued into the slot of plane k-1), H^{n-1/2} in a ring of
// three.  The wavefronts of a block meet at two barriers per plane that order LDS only (lds_barrier):
// a wavefront waits for its own tile loads of the previous plane just before the first barrier, so
// the loads stay in flight for a whole plane of compute, where __syncthreads would wait for them (and
// for every other outstanding global access) at once.  (Issuing after the first barrier into the
// slots of plane k, with rings of three and two, measured 4 % slower; so did loading Js^{n-1/2} one
// plane ahead.)  The tiles hold no columns beyond the footprint,
// so stages A and B are exact on lanes 1..62 (lanes 0 and 63 miss their x-1 or x+1 neighbour), stage
// C on lanes 1..61 and rows 0..TY-2 (the x+1 / y+1 neighbours), stage D on lanes 2..61 and rows
// 1..TY-2: a footprint's outputs are its 60 x (TY-2) interior cells, footprints overlap by four
// columns and two rows (those cells are computed by both), and along z a block computes the first
// step on two planes before its range.  Per cell the sweep reads E, H, Js (on superconducting edges)
// and the classes once and writes them once for two steps.  Every expression is the fused sweep's,
// so the results equal two fused steps bit for bit.
// Soft sources (both steps' values) and probe copies (of E^{n+1} and E^{n+2}) ride along in the SIDE
// instantiation.  On CPML grids (PML) the stages stretch their differences as the fused sweep does:
// A and B with the stored auxiliary variables, keeping the lane's new ones in registers, C and D with
// those; D stores the second step's variables for the footprint's interior to the other set (halo
// cells read the old ones).  No global load may be consumed between the issue of the tile loads and
// their wait (waiting for it would also wait for them): the slab coefficients come from LDS tables
// filled once per block, and the auxiliary variables are loaded one plane ahead with the Js.
static __device__ __forceinline__ int wrap_index(int v, int n)
{
    const int r = v % n;
    return r < 0 ? r + n : r;
}

constexpr int kTwoStepOX = kTileX - 4;  // output columns of a footprint
// s_waitcnt vmcnt(6) with expcnt and lgkmcnt left alone (gfx9 encoding: vmcnt bits 3:0 and 15:14,
// expcnt 6:4, lgkmcnt 11:8)
constexpr int kWaitVm6 = 0x0F76;
constexpr int kWaitLgkm0 = 0xC07F;  // s_waitcnt lgkmcnt(0)

// Barrier for LDS data only: this wavefront's LDS accesses complete before it and no LDS access moves
// across it, but global memory operations stay in flight (__syncthreads also waits for every
// outstanding global load and store of the wavefront).
static __device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// LDS pointer of the global-to-LDS loads (the instruction writes lane t's dword at this address + 4 t).
template <typename T>
static __device__ __forceinline__ __attribute__((address_space(3))) void *lds_ptr(T *p)
{
    return (__attribute__((address_space(3))) void *)p;
}


// Footprint tiles of the two-step sweep in LDS.
template <typename T, int TY>
struct TwoStepShared {
    static constexpr int RW = kTileX + 2, NR = TY + 2;  // a tile row (lane t at t + 1); rows -1..TY
    T e[4][3][NR][RW];          // E^n, ring of four planes
    T h[3][3][NR][RW];          // H^{n-1/2}, ring of three planes
    T e1[2][3][TY][kTileX];     // E^{n+1} of the last two planes
    T h2[3][TY][kTileX];        // H^{n+3/2} of the previous plane
};

template <typename T, int TY, int TZ, bool NT, bool SIDE, bool PML>
__global__ __launch_bounds__(kTileX *TY, 1) void two_step_kernel(const StepArgs<T> a)
{
    if constexpr (SIDE) side_reduce<T>(a.side);
    constexpr int OX = kTwoStepOX, OY = TY - 2;
    using S = TwoStepShared<T, TY>;
    constexpr int RW = S::RW, NR = S::NR;
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int ntx = (nx + OX - 1) / OX, nty = (ny + OY - 1) / OY, ntz = (nz + TZ - 1) / TZ;
    const int t = logical_block(blockIdx.x, ntx * nty * ntz);
    const int tx = t % ntx, tr = t / ntx;
    int ty, tz;
    tile_yz(tr, nty, ntz, PML && zmix_of(a.pml[2], nz), ty, tz);  // every XCD its share of the z-slab planes
    const int lane = threadIdx.x, row = threadIdx.y;
    const int wave = __builtin_amdgcn_readfirstlane(row);
    const int xo = tx * OX + lane - 2, yo = ty * OY + row - 1;  // the cell's output coordinates
    const int i = wrap_index(xo, nx), j = wrap_index(yo, ny);
    const bool out = lane >= 2 && lane <= OX + 1 && xo < nx && row >= 1 && row <= OY && yo < ny;
    const int k0 = tz * TZ, k1 = min(k0 + TZ, nz);
    // soft sources and probes whose boxes meet this wavefront's columns on the planes the run touches
    // (k0-1 .. k1, wrapped along z); SIDE: an instantiation of its own, so that the sweep without them
    // keeps its registers
    uint64_t side = 0;
    if constexpr (SIDE) {
        side = side_mask(a.side, i, j, max(k0 - 1, 0), min(k1 + 1, nz));
        if (k0 == 0) side |= side_mask(a.side, i, j, nz - 1, nz);
        if (k1 == nz) side |= side_mask(a.side, i, j, 0, 1);
    }
    const long long sxy = a.g.sxy;
    const int jp = (j + 1 == ny) ? 0 : j + 1, ip = (i + 1 == nx) ? 0 : i + 1;
    constexpr uint32_t w = sizeof(T);
    const uint32_t o00 = uint32_t(j * nx + i) * w;
    const uint32_t oxp = uint32_t(j * nx + ip) * w, oyp = uint32_t(jp * nx + i) * w;
    const uint32_t oc = uint32_t(j * nx + i) * 2u;
    const T rdx = a.rd[0], rdy = a.rd[1], rdz = a.rd[2], hdt = a.hdt;
    // CPML grids (PML): the slab slots (-1 outside) of the lane's column and of column x-1, of the row
    // and of row y-1 (uniform over a wavefront), and the PEC walls; the auxiliary variables are read
    // from the bound set and written to the other (a footprint's halo cells read the old values of
    // cells another footprint writes), and the new values of the first step stay in registers
    const PmlAxis<T> &px = a.pml[0], &py = a.pml[1], &pz = a.pml[2];
    const int jw = __builtin_amdgcn_readfirstlane(j);
    const int im = (i == 0) ? nx - 1 : i - 1, jmw = (jw == 0) ? ny - 1 : jw - 1;
    [[maybe_unused]] int sx = -1, sxm = -1, sy = -1, sym = -1;
    [[maybe_unused]] bool wall_x = false, wall_y = false;
    [[maybe_unused]] const uint32_t oi = uint32_t(i) * w, oim = uint32_t(im) * w;
    [[maybe_unused]] uint32_t osx = 0, osxm = 0;
    if constexpr (PML) {
        sx = px.on ? slab_slot(i, px.lo, px.hi, nx) : -1;
        sxm = px.on ? slab_slot(im, px.lo, px.hi, nx) : -1;
        sy = py.on ? slab_slot(jw, py.lo, py.hi, ny) : -1;
        sym = py.on ? slab_slot(jmw, py.lo, py.hi, ny) : -1;
        osx = uint32_t(sx) * w;
        osxm = uint32_t(sxm) * w;
        wall_x = px.on && i == 0;
        wall_y = py.on && jw == 0;
    }
    auto zslot = [&](int kk) { return (PML && pz.on) ? slab_slot(kk, pz.lo, pz.hi, nz) : -1; };
    // wavefronts with x-slab lanes (or x-1 neighbours in a slab): every wavefront of a block has the
    // same columns
    [[maybe_unused]] const bool xv = PML && px.on && px.P > 0 && __any(sx >= 0 || sxm >= 0);
    [[maybe_unused]] const uint32_t osxc = uint32_t(sx >= 0 ? sx : 0) * w, osxmc = uint32_t(sxm >= 0 ? sxm : 0) * w;
    // The auxiliary variables stage A and B read, loaded one plane ahead with the next plane's Js
    // (a load consumed in the plane that issues it would also wait for the tile loads in flight):
    // z slabs (the plane's): own faces, Hy's x-1 and Hx's y-1 neighbours, E side; x slabs (the
    // lane's column, clamped into the slab): the same with the x-1 column, in FP32 only (FP64 has
    // no registers left for them).  y slabs (and FP64 x slabs) read theirs in place.
    constexpr bool XPRE = sizeof(T) == 4;
    struct Psi {
        T zh0, zh1, zh1xm, zh0ym, ze0, ze1, qh0, qh1, qh1ym, qm0, qm1, qe0, qe1;
    };
    auto load_psi = [&](int kk) {
        Psi q{};
        if constexpr (PML) {
            const int sz = zslot(kk);
            if (sz >= 0) {
                const long long r = ((long long)sz * ny + jw) * nx, rym = ((long long)sz * ny + jmw) * nx;
                q.zh0 = ldo(pz.psiH[0] + r, oi);
                q.zh1 = ldo(pz.psiH[1] + r, oi);
                q.zh1xm = ldo(pz.psiH[1] + r, oim);
                q.zh0ym = ldo(pz.psiH[0] + rym, oi);
                q.ze0 = ldo(pz.psiE[0] + r, oi);
                q.ze1 = ldo(pz.psiE[1] + r, oi);
            }
            if (XPRE && xv) {
                const long long r = ((long long)kk * ny + jw) * px.P, rym = ((long long)kk * ny + jmw) * px.P;
                q.qh0 = ldo(px.psiH[0] + r, osxc);
                q.qh1 = ldo(px.psiH[1] + r, osxc);
                q.qh1ym = ldo(px.psiH[1] + rym, osxc);
                q.qm0 = ldo(px.psiH[0] + r, osxmc);
                q.qm1 = ldo(px.psiH[1] + r, osxmc);
                q.qe0 = ldo(px.psiE[0] + r, osxc);
                q.qe1 = ldo(px.psiE[1] + r, osxc);
            }
        }
        return q;
    };

    __shared__ S sh;
    // CPML: the slab coefficients (bh, ch, kh, bn, cn, kn), read once per block (loads of them in the
    // loop would wait for the tile loads in flight): x slabs of the lane's column and column x-1
    // (bh, ch, kh), y slabs of the wavefront's row and row y-1 (bh, ch, kh), z slabs of the block's
    // planes k0-2 .. k1 (entry t: plane k0-2+t)
    __shared__ T xcf[PML ? 9 : 1][kTileX];
    __shared__ T ycf[PML ? 9 : 1][TY];
    __shared__ T zcf[PML ? 6 : 1][TZ + 3];
    if constexpr (PML) {
        if (lane == 0 && py.on) {
            ycf[0][row] = py.bh[jw];
            ycf[1][row] = py.ch[jw];
            ycf[2][row] = py.kh[jw];
            ycf[3][row] = py.bn[jw];
            ycf[4][row] = py.cn[jw];
            ycf[5][row] = py.kn[jw];
            ycf[6][row] = py.bh[jmw];
            ycf[7][row] = py.ch[jmw];
            ycf[8][row] = py.kh[jmw];
        }
        if (row == 1 % TY && pz.on && lane < TZ + 3) {
            const int kk = wrap_index(k0 - 2 + lane, nz);
            zcf[0][lane] = pz.bh[kk];
            zcf[1][lane] = pz.ch[kk];
            zcf[2][lane] = pz.kh[kk];
            zcf[3][lane] = pz.bn[kk];
            zcf[4][lane] = pz.cn[kk];
            zcf[5][lane] = pz.kn[kk];
        }
        if (row == 0 && px.on) {
            xcf[0][lane] = ldo(px.bh, oi);
            xcf[1][lane] = ldo(px.ch, oi);
            xcf[2][lane] = ldo(px.kh, oi);
            xcf[3][lane] = ldo(px.bn, oi);
            xcf[4][lane] = ldo(px.cn, oi);
            xcf[5][lane] = ldo(px.kn, oi);
            xcf[6][lane] = ldo(px.bh, oim);
            xcf[7][lane] = ldo(px.ch, oim);
            xcf[8][lane] = ldo(px.kh, oim);
        }
    }
    const int lxp = min(lane + 1, kTileX - 1), lxm = max(lane - 1, 0);
    const int ryp = min(row + 1, TY - 1), rym = max(row - 1, 0);

    // ---- the tile loads of this wavefront: jobs (component, row slot) dealt to the wavefronts in
    // turn, E: Ex rows -1..TY, Ey rows -1..TY-1, Ez rows -1..TY; H (dealt on from where the E jobs
    // leave off): Hx rows -1..TY-1, Hy rows 0..TY-1, Hz rows -1..TY-1.  Row slot s is grid row
    // wrap(ty OY - 2 + s); lane t loads column wrap(tx OX - 2 + t) (FP64: two loads of 32 values).
    constexpr int NJE = 3 * NR - 1, NJH = 3 * NR - 4;
    constexpr int JE = (NJE + TY - 1) / TY, JH = (NJH + TY - 1) / TY;
    const int x0 = tx * OX - 2;
    const uint32_t cmain0 = sizeof(T) == 8 ? uint32_t(wrap_index(x0 + lane / 2, nx)) * w + 4u * (lane & 1)
                                           : uint32_t(wrap_index(x0 + lane, nx)) * w;
    const uint32_t cmain1 = uint32_t(wrap_index(x0 + 32 + lane / 2, nx)) * w + 4u * (lane & 1);
    auto row_of = [&](int sr) { return (long long)wrap_index(ty * OY - 2 + sr, ny) * nx; };
    const T *ebase[JE], *hbase[JH];
    int elds[JE], hlds[JH];
    int ne = 0, nh = 0;
#pragma unroll
    for (int m = 0; m < JE; ++m) {
        const int q = wave + m * TY;
        const int c = q < NR ? 0 : (q < 2 * NR - 1 ? 1 : 2);
        const int sr = q - (c == 0 ? 0 : (c == 1 ? NR : 2 * NR - 1));
        ebase[m] = a.E[c] + row_of(sr);
        elds[m] = (c * NR + sr) * RW + 1;
        ne += q < NJE;
    }
    const int hw = (wave + TY - NJE % TY) % TY;
#pragma unroll
    for (int m = 0; m < JH; ++m) {
        const int q = hw + m * TY;
        const int c = q < NR - 1 ? 0 : (q < 2 * NR - 3 ? 1 : 2);
        const int sr = c == 0 ? q : (c == 1 ? q - (NR - 1) + 1 : q - (2 * NR - 3));
        hbase[m] = a.H[c] + row_of(sr);
        hlds[m] = (c * NR + sr) * RW + 1;
        nh += q < NJH;
    }
    auto tile_row = [&](const T *src, T *dst) {
        __builtin_amdgcn_global_load_lds((const char *)src + cmain0, lds_ptr(dst), 4, 0, 0);
        if constexpr (sizeof(T) == 8)
            __builtin_amdgcn_global_load_lds((const char *)src + cmain1, lds_ptr(dst + 32), 4, 0, 0);
    };
    auto load_e = [&](int kk, int slot) {
        const long long b = (long long)kk * sxy;
#pragma unroll
        for (int m = 0; m < JE; ++m)
            if (m < ne) tile_row(ebase[m] + b, &sh.e[slot][0][0][0] + elds[m]);
    };
    auto load_h = [&](int kk, int slot) {
        const long long b = (long long)kk * sxy;
#pragma unroll
        for (int m = 0; m < JH; ++m)
            if (m < nh) tile_row(hbase[m] + b, &sh.h[slot][0][0][0] + hlds[m]);
    };

    struct Classes {
        uint32_t x, y, z;
    };
    auto load_cls = [&](int kk) {
        const long long b = opaque_offset((long long)kk * sxy);
        return Classes{ldp(a.cls[0] + b, oc), ldp(a.cls[1] + b, oc), ldp(a.cls[2] + b, oc)};
    };
    EdgeCoef<T> cx, cy, cz;
    auto coefs = [&](const Classes &m) {
        cx = class_coef(a.ctab, m.x);
        cy = class_coef(a.ctab, m.y);
        cz = class_coef(a.ctab, m.z);
    };

    // prologue: H^{n+1/2} (Hx, Hy) at plane k0-2 carried into the loop, and the first tiles
    const int p0 = k0 - 1;  // stage A plane of the first iteration
    const int nit = (k1 - k0) + 2;
    const int km0 = wrap_index(k0 - 2, nz), kb = wrap_index(p0, nz);
    T hx_km, hy_km;
    {
        const long long bm = (long long)km0 * sxy, b = (long long)kb * sxy;
        const T *Ex = a.E[0] + bm, *Ey = a.E[1] + bm, *Ez = a.E[2] + bm;
        const T exk = ldp(Ex, o00), eyk = ldp(Ey, o00), ez = ldp(Ez, o00);
        const T exk1 = ldp(a.E[0] + b, o00), eyk1 = ldp(a.E[1] + b, o00);
        const T ez_x = ldp(Ez, oxp), ez_y = ldp(Ez, oyp);
        T dyEz = (ez_y - ez) * rdy, dzEy = (eyk1 - eyk) * rdz;
        T dzEx = (exk1 - exk) * rdz, dxEz = (ez_x - ez) * rdx;
        if constexpr (PML) {  // the stretching at plane k0-2, without storing (another tile does)
            if (sx >= 0)
                dxEz = stretch_virtual_o(dxEz, px.psiH[0] + ((long long)km0 * ny + jw) * px.P, osx, ldo(px.bh, oi),
                                         ldo(px.ch, oi), ldo(px.kh, oi));
            if (sy >= 0)
                dyEz = stretch_virtual_o(dyEz, py.psiH[1] + ((long long)km0 * py.P + sy) * nx, oi, py.bh[jw], py.ch[jw],
                                         py.kh[jw]);
            const int sz = zslot(km0);
            if (sz >= 0) {
                const long long r = ((long long)sz * ny + jw) * nx;
                dzEy = stretch_virtual_o(dzEy, pz.psiH[0] + r, oi, pz.bh[km0], pz.ch[km0], pz.kh[km0]);
                dzEx = stretch_virtual_o(dzEx, pz.psiH[1] + r, oi, pz.bh[km0], pz.ch[km0], pz.kh[km0]);
            }
        }
        hx_km = ldp(a.H[0] + bm, o00) - hdt * (dyEz - dzEy);
        hy_km = ldp(a.H[1] + bm, o00) - hdt * (dzEx - dxEz);
    }
    for (int q = 0; q < 3 && q <= nit; ++q) load_e(wrap_index(p0 + q, nz), q);
    for (int q = 0; q < 2 && q < nit; ++q) load_h(wrap_index(p0 + q, nz), q);
    coefs(load_cls(kb));
    // Js^{n-1/2} of the stage A plane, loaded one plane ahead on every edge (the step writes it only
    // on superconducting edges: the others are masked to 0 where it is used)
    T jnx, jny, jnz;
    {
        const long long b = (long long)kb * sxy;
        jnx = ldp(a.J[0] + b, o00);
        jny = ldp(a.J[1] + b, o00);
        jnz = ldp(a.J[2] + b, o00);
    }
    [[maybe_unused]] Psi psn = load_psi(kb);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    // carried from the previous plane k-1: H^{n+1/2}, E^{n+1}, Js^{n+3/2} (the London update of the
    // second step, formed as soon as E^{n+1} exists), the E-update coefficients; and H^{n+3/2}(k-2)
    T phx = T(0), phy = T(0), phz = T(0), pex = T(0), pey = T(0), pez = T(0);
    T pjx = T(0), pjy = T(0), pjz = T(0);
    EdgeCoef<T> px_ = {T(0), T(0), T(0)}, py_ = px_, pz_ = px_;
    T qhx_km = T(0), qhy_km = T(0);
    // CPML: the first step's new variables of the previous plane, H side (x, y, z axis, two each) and
    // E side
    [[maybe_unused]] T pax0 = T(0), pax1 = T(0), pay0 = T(0), pay1 = T(0), paz0 = T(0), paz1 = T(0);
    [[maybe_unused]] T pbx0 = T(0), pbx1 = T(0), pby0 = T(0), pby1 = T(0), pbz0 = T(0), pbz1 = T(0);
    const int L = lane + 1, R = row + 1;  // the lane's column and row slots in the tiles

    for (int it = 0; it < nit; ++it) {
        const int kc = wrap_index(p0 + it, nz);
        const int kn = (kc + 1 == nz) ? 0 : kc + 1;
        // ---- stages A and B at plane kc (the fused sweep's periodic arithmetic)
        const EdgeCoef<T> qx = cx, qy = cy, qz = cz;
        // Js^{n-1/2} as loaded (masked to 0 off the superconducting edges in stage B, where the
        // coefficients are first needed: a test here would wait for their table loads at once)
        T jx = jnx, jy = jny, jz = jnz;
        // CPML: this plane's auxiliary variables, and the next plane's (issued before the six loads)
        [[maybe_unused]] const Psi ps = psn;
        if constexpr (PML) psn = load_psi(kn);
        // the next plane's Js and classes: exactly six loads, issued after every load the wait below
        // is for
        {
            const long long bn = opaque_offset((long long)kn * sxy);
            jnx = ldp(a.J[0] + bn, o00);
            jny = ldp(a.J[1] + bn, o00);
            jnz = ldp(a.J[2] + bn, o00);
        }
        const Classes mn = load_cls(kn);
        const auto &E0 = sh.e[it & 3], &E1 = sh.e[(it + 1) & 3];
        const auto &H0 = sh.h[it % 3];
        const T ex0 = E0[0][R][L], exm = E0[0][R][L - 1], ex_yp = E0[0][R + 1][L], exm_yp = E0[0][R + 1][L - 1];
        const T ex_ym = E0[0][R - 1][L];
        const T ey0 = E0[1][R][L], ey_xp = E0[1][R][L + 1], ey_xm = E0[1][R][L - 1], eym = E0[1][R - 1][L];
        const T eym_xp = E0[1][R - 1][L + 1];
        const T ez = E0[2][R][L], ez_xp = E0[2][R][L + 1], ez_yp = E0[2][R + 1][L], ez_xm = E0[2][R][L - 1];
        const T ez_ym = E0[2][R - 1][L];
        const T ex1 = E1[0][R][L], exm1 = E1[0][R][L - 1], ey1 = E1[1][R][L], eym1 = E1[1][R - 1][L];
        const T hx = H0[0][R][L], hx_ym = H0[0][R - 1][L];
        const T hy = H0[1][R][L], hy_xm = H0[1][R][L - 1];
        const T hz = H0[2][R][L], hz_xm = H0[2][R][L - 1], hz_ym = H0[2][R - 1][L];
        // nothing of the arithmetic below moves above the tile reads: a test of this plane's edge
        // coefficients scheduled next to their table loads would wait for them at once
        __builtin_amdgcn_sched_barrier(0);

        T nhx, nhy, nhz, nhz_xm, nhy_xm, nhz_ym, nhx_ym;
        [[maybe_unused]] T ax0 = T(0), ax1 = T(0), ay0 = T(0), ay1 = T(0), az0 = T(0), az1 = T(0);
        [[maybe_unused]] T bx0 = T(0), bx1 = T(0), by0 = T(0), by1 = T(0), bz0 = T(0), bz1 = T(0);
        [[maybe_unused]] const int szc = zslot(kc);
        if constexpr (!PML) {
            nhx = hx - hdt * ((ez_yp - ez) * rdy - (ey1 - ey0) * rdz);
            nhy = hy - hdt * ((ex1 - ex0) * rdz - (ez_xp - ez) * rdx);
            nhz = hz - hdt * ((ey_xp - ey0) * rdx - (ex_yp - ex0) * rdy);
            nhz_xm = hz_xm - hdt * ((ey0 - ey_xm) * rdx - (exm_yp - exm) * rdy);
            nhy_xm = hy_xm - hdt * ((exm1 - exm) * rdz - (ez - ez_xm) * rdx);
            nhz_ym = hz_ym - hdt * ((eym_xp - eym) * rdx - (ex0 - ex_ym) * rdy);
            nhx_ym = hx_ym - hdt * ((ez - ez_ym) * rdy - (eym1 - eym) * rdz);
        } else {  // the fused sweep's CPML arithmetic; the lane's own new variables are kept (a*)
            T dyEz = (ez_yp - ez) * rdy, dzEy = (ey1 - ey0) * rdz;              // Hx
            T dzEx = (ex1 - ex0) * rdz, dxEz = (ez_xp - ez) * rdx;              // Hy
            T dxEy = (ey_xp - ey0) * rdx, dyEx = (ex_yp - ex0) * rdy;           // Hz
            T dxEy_xm = (ey0 - ey_xm) * rdx, dyEx_xm = (exm_yp - exm) * rdy;    // Hz at x-1
            T dzEx_xm = (exm1 - exm) * rdz, dxEz_xm = (ez - ez_xm) * rdx;       // Hy at x-1
            T dxEy_ym = (eym_xp - eym) * rdx, dyEx_ym = (ex0 - ex_ym) * rdy;    // Hz at y-1
            T dyEz_ym = (ez - ez_ym) * rdy, dzEy_ym = (eym1 - eym) * rdz;       // Hx at y-1
            const long long rx = ((long long)kc * ny + jw) * px.P, rxm = ((long long)kc * ny + jmw) * px.P;
            if (sx >= 0) {
                const T bh = xcf[0][lane], ch = xcf[1][lane], kh = xcf[2][lane];
                T pv;
                dxEz = stretch_v(dxEz, XPRE ? ps.qh0 : ldo(px.psiH[0] + rx, osx), bh, ch, kh, ax0);
                dxEy = stretch_v(dxEy, XPRE ? ps.qh1 : ldo(px.psiH[1] + rx, osx), bh, ch, kh, ax1);
                dxEy_ym = stretch_v(dxEy_ym, XPRE ? ps.qh1ym : ldo(px.psiH[1] + rxm, osx), bh, ch, kh, pv);
            }
            if (sxm >= 0) {
                const T bh = xcf[6][lane], ch = xcf[7][lane], kh = xcf[8][lane];
                T pv;
                dxEy_xm = stretch_v(dxEy_xm, XPRE ? ps.qm1 : ldo(px.psiH[1] + rx, osxm), bh, ch, kh, pv);
                dxEz_xm = stretch_v(dxEz_xm, XPRE ? ps.qm0 : ldo(px.psiH[0] + rx, osxm), bh, ch, kh, pv);
            }
            if (sy >= 0) {
                const long long r = ((long long)kc * py.P + sy) * nx;
                const T bh = ycf[0][row], ch = ycf[1][row], kh = ycf[2][row];
                dyEx = stretch_v(dyEx, ldo(py.psiH[0] + r, oi), bh, ch, kh, ay0);
                dyEz = stretch_v(dyEz, ldo(py.psiH[1] + r, oi), bh, ch, kh, ay1);
                dyEx_xm = stretch_virtual_o(dyEx_xm, py.psiH[0] + r, oim, bh, ch, kh);
            }
            if (sym >= 0) {
                const long long r = ((long long)kc * py.P + sym) * nx;
                const T bh = ycf[6][row], ch = ycf[7][row], kh = ycf[8][row];
                dyEx_ym = stretch_virtual_o(dyEx_ym, py.psiH[0] + r, oi, bh, ch, kh);
                dyEz_ym = stretch_virtual_o(dyEz_ym, py.psiH[1] + r, oi, bh, ch, kh);
            }
            if (szc >= 0) {
                const T bh = zcf[0][it + 1], ch = zcf[1][it + 1], kh = zcf[2][it + 1];
                T pv;
                dzEy = stretch_v(dzEy, ps.zh0, bh, ch, kh, az0);
                dzEx = stretch_v(dzEx, ps.zh1, bh, ch, kh, az1);
                dzEx_xm = stretch_v(dzEx_xm, ps.zh1xm, bh, ch, kh, pv);
                dzEy_ym = stretch_v(dzEy_ym, ps.zh0ym, bh, ch, kh, pv);
            }
            nhx = hx - hdt * (dyEz - dzEy);
            nhy = hy - hdt * (dzEx - dxEz);
            nhz = hz - hdt * (dxEy - dyEx);
            nhz_xm = hz_xm - hdt * (dxEy_xm - dyEx_xm);
            nhy_xm = hy_xm - hdt * (dzEx_xm - dxEz_xm);
            nhz_ym = hz_ym - hdt * (dxEy_ym - dyEx_ym);
            nhx_ym = hx_ym - hdt * (dyEz_ym - dzEy_ym);
        }
        T ex_n, ey_n, ez_n;  // E^{n+1} at plane kc
        {
            T dyHz = (nhz - nhz_ym) * rdy, dzHy = (nhy - hy_km) * rdz;
            T dzHx = (nhx - hx_km) * rdz, dxHz = (nhz - nhz_xm) * rdx;
            T dxHy = (nhy - nhy_xm) * rdx, dyHx = (nhx - nhx_ym) * rdy;
            if constexpr (PML) {  // E-side variables of the lane's own cell (new values kept: b*)
                if (sx >= 0) {
                    const long long r = ((long long)kc * ny + jw) * px.P;
                    const T bn = xcf[3][lane], cn = xcf[4][lane], kn = xcf[5][lane];
                    dxHz = stretch_v(dxHz, XPRE ? ps.qe0 : ldo(px.psiE[0] + r, osx), bn, cn, kn, bx0);  // Ey
                    dxHy = stretch_v(dxHy, XPRE ? ps.qe1 : ldo(px.psiE[1] + r, osx), bn, cn, kn, bx1);  // Ez
                }
                if (sy >= 0) {
                    const long long r = ((long long)kc * py.P + sy) * nx;
                    const T bn = ycf[3][row], cn = ycf[4][row], kn = ycf[5][row];
                    dyHx = stretch_v(dyHx, ldo(py.psiE[0] + r, oi), bn, cn, kn, by0);  // Ez
                    dyHz = stretch_v(dyHz, ldo(py.psiE[1] + r, oi), bn, cn, kn, by1);  // Ex
                }
                if (szc >= 0) {
                    const T bn = zcf[3][it + 1], cn = zcf[4][it + 1], kn = zcf[5][it + 1];
                    dzHy = stretch_v(dzHy, ps.ze0, bn, cn, kn, bz0);  // Ex
                    dzHx = stretch_v(dzHx, ps.ze1, bn, cn, kn, bz1);  // Ey
                }
            }
            jx = qx.cj > T(0) ? jx + qx.cj * ex0 : T(0);
            jy = qy.cj > T(0) ? jy + qy.cj * ey0 : T(0);
            jz = qz.cj > T(0) ? jz + qz.cj * ez : T(0);
            ex_n = qx.ca * ex0 + qx.cb * ((dyHz - dzHy) - jx);
            ey_n = qy.ca * ey0 + qy.cb * ((dzHx - dxHz) - jy);
            ez_n = qz.ca * ez + qz.cb * ((dxHy - dyHx) - jz);
            if constexpr (PML) {  // tangential E on the PEC walls
                const bool wall_z = pz.on && kc == 0;
                ex_n = (wall_y || wall_z) ? T(0) : ex_n;
                ey_n = (wall_z || wall_x) ? T(0) : ey_n;
                ez_n = (wall_x || wall_y) ? T(0) : ez_n;
            }
            if (SIDE && (uint32_t)side != 0) {  // the first step's sources, on every lane (the halo lanes' copies too)
                ex_n = add_sources(a.side, a.side.sg, side, 0, i, j, kc, ex_n);
                ey_n = add_sources(a.side, a.side.sg, side, 1, i, j, kc, ey_n);
                ez_n = add_sources(a.side, a.side.sg, side, 2, i, j, kc, ez_n);
            }
        }
        const int buf = it & 1;
        sh.e1[buf][0][row][lane] = ex_n;
        sh.e1[buf][1][row][lane] = ey_n;
        sh.e1[buf][2][row][lane] = ez_n;
        // this wavefront's tile loads of the previous plane have landed (the barrier makes every
        // wavefront's visible): vector memory operations complete in issue order, and only the six
        // loads of the next plane's Js and classes came after them.  Then the next tile loads: E^n
        // plane kc+3, H^{n-1/2} plane kc+2, into the slots of plane kc-1, whose stage A every
        // wavefront finished before the last barrier
        __builtin_amdgcn_s_waitcnt(kWaitVm6);
        if (it + 3 <= nit) load_e(wrap_index(p0 + it + 3, nz), (it + 3) & 3);
        if (it + 2 < nit) load_h(wrap_index(p0 + it + 2, nz), (it + 2) % 3);
        lds_barrier();

        // ---- stage C: H^{n+3/2} at plane kc - 1 (the fused sweep's H arithmetic on E^{n+1})
        T h2x = T(0), h2y = T(0), h2z = T(0);
        const int kw = (kc == 0) ? nz - 1 : kc - 1;
        [[maybe_unused]] const int szw = zslot(kw);
        [[maybe_unused]] T cx0 = T(0), cx1 = T(0), cy0 = T(0), cy1 = T(0), cz0 = T(0), cz1 = T(0);
        if (it >= 1) {
            const int pb = buf ^ 1;
            const T ez1_yp = sh.e1[pb][2][ryp][lane], ex1_yp = sh.e1[pb][0][ryp][lane];
            const T ey1_xp = sh.e1[pb][1][row][lxp], ez1_xp = sh.e1[pb][2][row][lxp];
            if constexpr (!PML) {
                h2x = phx - hdt * ((ez1_yp - pez) * rdy - (ey_n - pey) * rdz);
                h2y = phy - hdt * ((ex_n - pex) * rdz - (ez1_xp - pez) * rdx);
                h2z = phz - hdt * ((ey1_xp - pey) * rdx - (ex1_yp - pex) * rdy);
            } else {  // stretched with the first step's new variables (c*: the second step's)
                T dyEz = (ez1_yp - pez) * rdy, dzEy = (ey_n - pey) * rdz;  // Hx
                T dzEx = (ex_n - pex) * rdz, dxEz = (ez1_xp - pez) * rdx;  // Hy
                T dxEy = (ey1_xp - pey) * rdx, dyEx = (ex1_yp - pex) * rdy;  // Hz
                if (sx >= 0) {
                    const T bh = xcf[0][lane], ch = xcf[1][lane], kh = xcf[2][lane];
                    dxEz = stretch_v(dxEz, pax0, bh, ch, kh, cx0);
                    dxEy = stretch_v(dxEy, pax1, bh, ch, kh, cx1);
                }
                if (sy >= 0) {
                    const T bh = ycf[0][row], ch = ycf[1][row], kh = ycf[2][row];
                    dyEx = stretch_v(dyEx, pay0, bh, ch, kh, cy0);
                    dyEz = stretch_v(dyEz, pay1, bh, ch, kh, cy1);
                }
                if (szw >= 0) {
                    const T bh = zcf[0][it], ch = zcf[1][it], kh = zcf[2][it];
                    dzEy = stretch_v(dzEy, paz0, bh, ch, kh, cz0);
                    dzEx = stretch_v(dzEx, paz1, bh, ch, kh, cz1);
                }
                h2x = phx - hdt * (dyEz - dzEy);
                h2y = phy - hdt * (dzEx - dxEz);
                h2z = phz - hdt * (dxEy - dyEx);
            }
            sh.h2[0][row][lane] = h2x;
            sh.h2[1][row][lane] = h2y;
            sh.h2[2][row][lane] = h2z;
        }
        lds_barrier();

        // ---- stage D: Js^{n+3/2} and E^{n+2} at plane kc - 1, stored for the footprint's interior
        if (it >= 2) {
            const T h2z_xm = sh.h2[2][row][lxm], h2y_xm = sh.h2[1][row][lxm];
            const T h2z_ym = sh.h2[2][rym][lane], h2x_ym = sh.h2[0][rym][lane];
            T dyHz = (h2z - h2z_ym) * rdy, dzHy = (h2y - qhy_km) * rdz;
            T dzHx = (h2x - qhx_km) * rdz, dxHz = (h2z - h2z_xm) * rdx;
            T dxHy = (h2y - h2y_xm) * rdx, dyHx = (h2x - h2x_ym) * rdy;
            [[maybe_unused]] T dx0 = T(0), dx1 = T(0), dy0 = T(0), dy1 = T(0), dz0 = T(0), dz1 = T(0);
            if constexpr (PML) {  // the second step's E-side variables (d*)
                if (sx >= 0) {
                    const T bn = xcf[3][lane], cn = xcf[4][lane], kn = xcf[5][lane];
                    dxHz = stretch_v(dxHz, pbx0, bn, cn, kn, dx0);
                    dxHy = stretch_v(dxHy, pbx1, bn, cn, kn, dx1);
                }
                if (sy >= 0) {
                    const T bn = ycf[3][row], cn = ycf[4][row], kn = ycf[5][row];
                    dyHx = stretch_v(dyHx, pby0, bn, cn, kn, dy0);
                    dyHz = stretch_v(dyHz, pby1, bn, cn, kn, dy1);
                }
                if (szw >= 0) {
                    const T bn = zcf[3][it], cn = zcf[4][it], kn = zcf[5][it];
                    dzHy = stretch_v(dzHy, pbz0, bn, cn, kn, dz0);
                    dzHx = stretch_v(dzHx, pbz1, bn, cn, kn, dz1);
                }
            }
            T j2x = pjx, j2y = pjy, j2z = pjz;
            if (px_.cj > T(0)) j2x = j2x + px_.cj * pex;
            if (py_.cj > T(0)) j2y = j2y + py_.cj * pey;
            if (pz_.cj > T(0)) j2z = j2z + pz_.cj * pez;
            T e2x = px_.ca * pex + px_.cb * ((dyHz - dzHy) - j2x);
            T e2y = py_.ca * pey + py_.cb * ((dzHx - dxHz) - j2y);
            T e2z = pz_.ca * pez + pz_.cb * ((dxHy - dyHx) - j2z);
            if constexpr (PML) {  // tangential E on the PEC walls
                const bool wall_z = pz.on && kw == 0;
                e2x = (wall_y || wall_z) ? T(0) : e2x;
                e2y = (wall_z || wall_x) ? T(0) : e2y;
                e2z = (wall_x || wall_y) ? T(0) : e2z;
            }
            if (SIDE && (uint32_t)side != 0) {  // the second step's sources
                e2x = add_sources(a.side, a.side.sg2, side, 0, i, j, kw, e2x);
                e2y = add_sources(a.side, a.side.sg2, side, 1, i, j, kw, e2y);
                e2z = add_sources(a.side, a.side.sg2, side, 2, i, j, kw, e2z);
            }
            if (out) {
                const long long bw = opaque_offset((long long)kw * sxy);
                stp_hint<NT>(a.Hout[0] + bw, o00, h2x);
                stp_hint<NT>(a.Hout[1] + bw, o00, h2y);
                stp_hint<NT>(a.Hout[2] + bw, o00, h2z);
                stp_hint<NT>(a.Eout[0] + bw, o00, e2x);
                stp_hint<NT>(a.Eout[1] + bw, o00, e2y);
                stp_hint<NT>(a.Eout[2] + bw, o00, e2z);
                if (px_.cj > T(0)) stp(a.Jout[0] + bw, o00, j2x);
                if (py_.cj > T(0)) stp(a.Jout[1] + bw, o00, j2y);
                if (pz_.cj > T(0)) stp(a.Jout[2] + bw, o00, j2z);
                if constexpr (PML) {  // the second step's auxiliary variables, to the other set
                    if (sx >= 0) {
                        const long long r = ((long long)kw * ny + jw) * px.P;
                        sto(px.psiHo[0] + r, osx, cx0);
                        sto(px.psiHo[1] + r, osx, cx1);
                        sto(px.psiEo[0] + r, osx, dx0);
                        sto(px.psiEo[1] + r, osx, dx1);
                    }
                    if (sy >= 0) {
                        const long long r = ((long long)kw * py.P + sy) * nx;
                        sto(py.psiHo[0] + r, oi, cy0);
                        sto(py.psiHo[1] + r, oi, cy1);
                        sto(py.psiEo[0] + r, oi, dy0);
                        sto(py.psiEo[1] + r, oi, dy1);
                    }
                    if (szw >= 0) {
                        const long long r = ((long long)szw * ny + jw) * nx;
                        sto(pz.psiHo[0] + r, oi, cz0);
                        sto(pz.psiHo[1] + r, oi, cz1);
                        sto(pz.psiEo[0] + r, oi, dz0);
                        sto(pz.psiEo[1] + r, oi, dz1);
                    }
                }
                if (SIDE && (side >> 32) != 0) {  // both steps' probe copies: E^{n+1} and E^{n+2}
                    probe_copy(a.side, a.side.pcopy, side, 0, i, j, kw, pex);
                    probe_copy(a.side, a.side.pcopy, side, 1, i, j, kw, pey);
                    probe_copy(a.side, a.side.pcopy, side, 2, i, j, kw, pez);
                    probe_copy(a.side, a.side.pcopy2, side, 0, i, j, kw, e2x);
                    probe_copy(a.side, a.side.pcopy2, side, 1, i, j, kw, e2y);
                    probe_copy(a.side, a.side.pcopy2, side, 2, i, j, kw, e2z);
                }
            }
        }
        // carry to the next plane
        qhx_km = h2x;
        qhy_km = h2y;
        phx = nhx;
        phy = nhy;
        phz = nhz;
        pex = ex_n;
        pey = ey_n;
        pez = ez_n;
        pjx = jx;
        pjy = jy;
        pjz = jz;
        px_ = qx;
        py_ = qy;
        pz_ = qz;
        hx_km = nhx;
        hy_km = nhy;
        if constexpr (PML) {
            pax0 = ax0; pax1 = ax1; pay0 = ay0; pay1 = ay1; paz0 = az0; paz1 = az1;
            pbx0 = bx0; pbx1 = bx1; pby0 = by0; pby1 = by1; pbz0 = bz0; pbz1 = bz1;
        }
        coefs(mn);
    }
}

// ---------------------------------------------------------------------------
// Probes on their own launch (the sample at the start of a run, probes beyond the sweeps' fold)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kProbeThreads) void probe_kernel(const ProbeArgs<T> a)
{
    const ProbeDesc &p = a.p[a.first + blockIdx.x];
    const int wx = p.i1 - p.i0, wy = p.j1 - p.j0, wz = p.k1 - p.k0;
    const long long cnt = (long long)wx * wy * wz;
    double s;
    if (blockIdx.x < kFoldProbes && a.copy[blockIdx.x] != nullptr) {
        const T *c = a.copy[blockIdx.x];
        s = probe_sum(cnt, [c](long long idx) { return (double)c[idx]; });
    } else {
        const T *E = a.E[p.comp];
        const long long ny = a.g.ny, nx = a.g.nx;
        s = probe_sum(cnt, [&](long long idx) {
            const int i = p.i0 + (int)(idx % wx);
            const long long r = idx / wx;
            const int j = p.j0 + (int)(r % wy);
            const int k = p.k0 + (int)(r / wy);
            return (double)E[((long long)k * ny + j) * nx + i];
        });
    }
    probe_record(p, s, a.n, a.dt);
}

// ---------------------------------------------------------------------------
// Integer-time half kick (Algorithm 1 steps 1 and 2 as half steps)
// ---------------------------------------------------------------------------
template <typename T>
struct CellMaps {
    T e[3][4], s[3][4], l[3][4];
};

// Gather the four cells of each of the three edges of cell index (i,j,k), in
// the q order used by the E pass.
template <typename T>
__device__ __forceinline__ void gather_edge_cells(const StepArgs<T> &a, int i, int j, int k, T em[3], T sm[3],
                                                  T lm[3])
{
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const int im = (i == 0) ? nx - 1 : i - 1;
    const int jm = (j == 0) ? ny - 1 : j - 1;
    const int km = (k == 0) ? nz - 1 : k - 1;
    auto id = [&](int ii, int jj, int kk) { return ((long long)kk * ny + jj) * nx + ii; };
    const long long c00 = id(i, j, k), c10 = id(im, j, k), c01 = id(i, jm, k), c11 = id(im, jm, k);
    const long long p00 = id(i, j, km), p10 = id(im, j, km), p01 = id(i, jm, km);
    const long long ex[4] = {c00, p00, c01, p01};
    const long long ey[4] = {c00, c10, p00, p10};
    const long long ez[4] = {c00, c01, c10, c11};
    const long long *cells[3] = {ex, ey, ez};
    for (int comp = 0; comp < 3; ++comp) {
        T e[4], s[4], l[4];
        for (int q = 0; q < 4; ++q) {
            e[q] = a.eps[cells[comp][q]];
            s[q] = a.sig[cells[comp][q]];
            l[q] = a.ell[cells[comp][q]];
        }
        edge_material(e, s, l, em[comp], sm[comp], lm[comp]);
    }
}

template <typename T>
__global__ void half_kick_kernel(const StepArgs<T> a, T sgn, T *Hx_o, T *Hy_o, T *Hz_o, T *Jx_o, T *Jy_o, T *Jz_o)
{
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const long long N = a.g.sxy * nz;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx);
        const long long r = c / nx;
        const int j = (int)(r % ny);
        const int k = (int)(r / ny);
        const int ip = (i + 1 == nx) ? 0 : i + 1;
        const int jp = (j + 1 == ny) ? 0 : j + 1;
        const int kp = (k + 1 == nz) ? 0 : k + 1;
        auto id = [&](int ii, int jj, int kk) { return ((long long)kk * ny + jj) * nx + ii; };
        const T *Ex = a.E[0], *Ey = a.E[1], *Ez = a.E[2];
        T dyEz = (Ez[id(i, jp, k)] - Ez[c]) * a.rd[1], dzEy = (Ey[id(i, j, kp)] - Ey[c]) * a.rd[2];
        T dzEx = (Ex[id(i, j, kp)] - Ex[c]) * a.rd[2], dxEz = (Ez[id(ip, j, k)] - Ez[c]) * a.rd[0];
        T dxEy = (Ey[id(ip, j, k)] - Ey[c]) * a.rd[0], dyEx = (Ex[id(i, jp, k)] - Ex[c]) * a.rd[1];
        const PmlAxis<T> &px = a.pml[0], &py = a.pml[1], &pz = a.pml[2];
        if (px.on) {
            const int sx = slab_slot(i, px.lo, px.hi, nx);
            if (sx >= 0) {
                const long long p = ((long long)k * ny + j) * px.P + sx;
                dxEz = stretch_virtual(dxEz, px.psiH[0], p, px.bh[i], px.ch[i], px.kh[i]);
                dxEy = stretch_virtual(dxEy, px.psiH[1], p, px.bh[i], px.ch[i], px.kh[i]);
            }
        }
        if (py.on) {
            const int sy = slab_slot(j, py.lo, py.hi, ny);
            if (sy >= 0) {
                const long long p = ((long long)k * py.P + sy) * nx + i;
                dyEx = stretch_virtual(dyEx, py.psiH[0], p, py.bh[j], py.ch[j], py.kh[j]);
                dyEz = stretch_virtual(dyEz, py.psiH[1], p, py.bh[j], py.ch[j], py.kh[j]);
            }
        }
        if (pz.on) {
            const int sz = slab_slot(k, pz.lo, pz.hi, nz);
            if (sz >= 0) {
                const long long p = ((long long)sz * ny + j) * nx + i;
                dzEy = stretch_virtual(dzEy, pz.psiH[0], p, pz.bh[k], pz.ch[k], pz.kh[k]);
                dzEx = stretch_virtual(dzEx, pz.psiH[1], p, pz.bh[k], pz.ch[k], pz.kh[k]);
            }
        }
        const T hh = T(0.5) * a.hdt * sgn;
        T *Ho[3] = {Hx_o, Hy_o, Hz_o};
        const T curl[3] = {dyEz - dzEy, dzEx - dxEz, dxEy - dyEx};
        if (Hx_o != nullptr)
            for (int comp = 0; comp < 3; ++comp) Ho[comp][c] = a.H[comp][c] + hh * curl[comp];
        if (Jx_o != nullptr) {
            T em[3], sm[3], lm[3];
            gather_edge_cells(a, i, j, k, em, sm, lm);
            T *Jo[3] = {Jx_o, Jy_o, Jz_o};
            for (int comp = 0; comp < 3; ++comp)
                Jo[comp][c] = (lm[comp] > T(0)) ? a.J[comp][c] - hh * lm[comp] * a.E[comp][c] : T(0);
        }
    }
}

// ---------------------------------------------------------------------------
// Energy functional and finite check (FP64 accumulation)
// ---------------------------------------------------------------------------
constexpr int kRedThreads = 256;

__device__ __forceinline__ double block_sum(double v, double *lds)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kRedThreads / 64; ++w) s += lds[w];
    return s;
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void energy_kernel(const StepArgs<T> a, double *part)
{
    __shared__ double lds[kRedThreads / 64];
    const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
    const long long N = a.g.sxy * nz;
    double we = 0.0, wh = 0.0, wj = 0.0, bad = 0.0;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N;
         c += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx);
        const long long r = c / nx;
        const int j = (int)(r % ny);
        const int k = (int)(r / ny);
        const int ip = (i + 1 == nx) ? 0 : i + 1;
        const int jp = (j + 1 == ny) ? 0 : j + 1;
        const int kp = (k + 1 == nz) ? 0 : k + 1;
        auto id = [&](int ii, int jj, int kk) { return ((long long)kk * ny + jj) * nx + ii; };
        const double E0 = (double)a.E[0][c], E1 = (double)a.E[1][c], E2 = (double)a.E[2][c];
        const double rdx = (double)a.rd[0], rdy = (double)a.rd[1], rdz = (double)a.rd[2];
        const double cx = ((double)a.E[2][id(i, jp, k)] - E2) * rdy - ((double)a.E[1][id(i, j, kp)] - E1) * rdz;
        const double cy = ((double)a.E[0][id(i, j, kp)] - E0) * rdz - ((double)a.E[2][id(ip, j, k)] - E2) * rdx;
        const double cz = ((double)a.E[1][id(ip, j, k)] - E1) * rdx - ((double)a.E[0][id(i, jp, k)] - E0) * rdy;
        const double hdt = (double)a.dt / kMu0;
        const double H[3] = {(double)a.H[0][c], (double)a.H[1][c], (double)a.H[2][c]};
        const double cu[3] = {cx, cy, cz};
        for (int comp = 0; comp < 3; ++comp) wh += 0.5 * kMu0 * H[comp] * (H[comp] - hdt * cu[comp]);
        T em[3], sm[3], lm[3];
        gather_edge_cells(a, i, j, k, em, sm, lm);
        const double Ev[3] = {E0, E1, E2};
        for (int comp = 0; comp < 3; ++comp) {
            we += 0.5 * (double)em[comp] * Ev[comp] * Ev[comp];
            if (lm[comp] > T(0)) {
                const double Jv = (double)a.J[comp][c];
                const double Jp = Jv + hdt * (double)lm[comp] * Ev[comp];
                wj += 0.5 * kMu0 * Jv * Jp / (double)lm[comp];
            }
            const double hv = H[comp], jv = (double)a.J[comp][c];
            bad += (isfinite(Ev[comp]) ? 0.0 : 1.0) + (isfinite(hv) ? 0.0 : 1.0) + (isfinite(jv) ? 0.0 : 1.0);
        }
    }
    const double dV = 1.0 / ((double)a.rd[0] * (double)a.rd[1] * (double)a.rd[2]);
    const double w = block_sum(dV * (we + wh + wj), lds);
    const double nb = block_sum(bad, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = w;
        part[2 * blockIdx.x + 1] = nb;
    }
}

// Second stage: one block folds nblocks pairs into dst[0..1] in a fixed order (dst may be part).
__global__ __launch_bounds__(kRedThreads) void fold_pairs_kernel(double *part, int nblocks, double *dst)
{
    __shared__ double lds[kRedThreads / 64];
    double a0 = 0.0, a1 = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kRedThreads) {
        a0 += part[2 * b];
        a1 += part[2 * b + 1];
    }
    const double s0 = block_sum(a0, lds);
    const double s1 = block_sum(a1, lds);
    __syncthreads();
    if (threadIdx.x == 0) {
        dst[0] = s0;
        dst[1] = s1;
    }
}

// ---------------------------------------------------------------------------
// Material map statistics (validation and the stability bound)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_min(double v, double *lds)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double s = lds[0];
    if (threadIdx.x == 0)
        for (int w = 1; w < kRedThreads / 64; ++w) s = fmin(s, lds[w]);
    return s;
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void map_stats_kernel(const T *eps, const T *sig, const T *ell, long long n,
                                                                double *part)
{
    __shared__ double lds[kRedThreads / 64];
    double me = INFINITY, ms = INFINITY, ml = INFINITY, nl = INFINITY, bad = 0.0;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const double e = (double)eps[c], s = (double)sig[c], l = (double)ell[c];
        me = fmin(me, e);
        ms = fmin(ms, s);
        ml = fmin(ml, l);
        nl = fmin(nl, -l);
        bad += (isfinite(e) && isfinite(s) && isfinite(l)) ? 0.0 : 1.0;
    }
    const double r0 = block_min(me, lds);
    const double r1 = block_min(ms, lds);
    const double r2 = block_min(ml, lds);
    const double r3 = block_min(nl, lds);
    const double r4 = block_sum(bad, lds);
    if (threadIdx.x == 0) {
        double *o = part + 5 * (size_t)blockIdx.x;
        o[0] = r0; o[1] = r1; o[2] = r2; o[3] = r3; o[4] = r4;
    }
}

__global__ __launch_bounds__(kRedThreads) void map_stats_fold_kernel(double *part, int nblocks)
{
    __shared__ double lds[kRedThreads / 64];
    double v[5] = {INFINITY, INFINITY, INFINITY, INFINITY, 0.0};
    for (int b = threadIdx.x; b < nblocks; b += kRedThreads) {
        for (int q = 0; q < 4; ++q) v[q] = fmin(v[q], part[5 * b + q]);
        v[4] += part[5 * b + 4];
    }
    double r[5];
    for (int q = 0; q < 4; ++q) r[q] = block_min(v[q], lds);
    r[4] = block_sum(v[4], lds);
    __syncthreads();
    if (threadIdx.x == 0)
        for (int q = 0; q < 5; ++q) part[q] = r[q];
}

// One entry of the class table per thread: the coefficients of the edge whose four cells hold the cell
// materials named by tuple[c] (16 bits each, in the order the sweeps pass them to edge_coef).
template <typename T>
__global__ void class_table_kernel(const StepArgs<T> a, const T *mat, const uint64_t *tuple, int ncls, T *tab)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncls) return;
    const uint64_t t = tuple[c];
    T e[4], s[4], l[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t m = uint32_t(t >> (16 * q)) & 0xffffu;
        e[q] = mat[3 * m];
        s[q] = mat[3 * m + 1];
        l[q] = mat[3 * m + 2];
    }
    const EdgeCoef<T> r = edge_coef(e, s, l, a.dt, a.theta, a.hdt);
    tab[4 * c] = r.ca;
    tab[4 * c + 1] = r.cb;
    tab[4 * c + 2] = r.cj;
    tab[4 * c + 3] = T(0);
}

// Non-finite check of the state: counts the NaN and Inf values of the nine arrays (E, H, Js);
// blocks add their counts to counter[0] and, when they found any, lower counter[1] to `step`
// (counter[1] starts at the largest value: the first step index where the check saw one).
template <typename T>
__global__ __launch_bounds__(kRedThreads) void nonfinite_kernel(const NonfiniteArgs<T> a, unsigned long long *counter,
                                                               unsigned long long step)
{
    unsigned long long bad = 0;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < a.n;
         c += (long long)gridDim.x * blockDim.x) {
#pragma unroll
        for (int q = 0; q < 9; ++q) bad += isfinite(a.f[q][c]) ? 0u : 1u;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_down(bad, off, 64);
    if ((threadIdx.x & 63) == 0 && bad != 0) {
        atomicAdd(&counter[0], bad);
        atomicMin(&counter[1], step);
    }
}

__global__ void nonfinite_reset_kernel(unsigned long long *counter)
{
    if (threadIdx.x == 0) {
        counter[0] = 0ull;
        counter[1] = ~0ull;
    }
}

__global__ void fill_zero_kernel(uint32_t *p, size_t nwords)
{
    for (size_t w = (size_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += (size_t)gridDim.x * blockDim.x)
        p[w] = 0u;
}

}  // namespace

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free entry points
// ---------------------------------------------------------------------------
// One copy per GPU, held until the process ends: the block partials (two FP64 values per block) of
// the energy reduction of tfl_energy_noalloc.  In host code `scratch` names a host-side stand-in,
// not device memory: kernels receive the device address from static_scratch() instead.
static __device__ __align__(256) double scratch[2 * kStaticScratchBlocks];

hipError_t static_scratch(double **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex lock;
    static double *ptr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(lock);
    if (!ptr[dev]) {  // first call on this device (the current one): its copy's address
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        ptr[dev] = (double *)p;
    }
    *out = ptr[dev];
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// Tile shapes of the forward sweeps per storage type: wavefronts per block, the
// longest z run, and the wavefronts a launch should at least provide (from
// sweeps of shapes on MI355X: the FP64 H pass is fastest with all its tiles
// resident in one round, the other sweeps with about two rounds of waves; the
// fused sweep varies by < 3 % over shapes).  The two passes take rows of 64,
// 32 or 16 cells (row_width); the FP32 fused sweep rows of 256 or 128 cells
// when they divide nx.
template <typename T>
struct FwdTiles;
template <>
struct FwdTiles<double> {
    static constexpr int hy = 4, hz_max = 64, ey = 8, ez_max = 64, fy = 4, fz_max = 64;
    static constexpr long long h_waves = 4096, e_waves = 8192, f_waves = 8192;
};
template <>
struct FwdTiles<float> {
    static constexpr int hy = 4, hz_max = 64, ey = 4, ez_max = 64, fy = 4, fz_max = 64;
    static constexpr long long h_waves = 8192, e_waves = 8192, f_waves = 16384;
};

template <typename T, int W>
static void launch_h_pass_w(const StepArgs<T> &a, hipStream_t s)
{
    using C = FwdTiles<T>;
    const int tz = pick_tile_z_w(a.g, C::hy, C::h_waves, C::hz_max, W);
    const dim3 blk(kTileX, C::hy), grd((unsigned)(row_tiles(a.g, C::hy, W) * ((a.g.nz + tz - 1) / tz)));
    switch (tz) {
    case 64: hipLaunchKernelGGL((h_pass_kernel<T, C::hy, 64, W>), grd, blk, 0, s, a); break;
    case 32: hipLaunchKernelGGL((h_pass_kernel<T, C::hy, 32, W>), grd, blk, 0, s, a); break;
    case 16: hipLaunchKernelGGL((h_pass_kernel<T, C::hy, 16, W>), grd, blk, 0, s, a); break;
    default: hipLaunchKernelGGL((h_pass_kernel<T, C::hy, 8, W>), grd, blk, 0, s, a); break;
    }
}

template <typename T, int W, bool CLS>
static void launch_e_pass_w(const StepArgs<T> &a, hipStream_t s)
{
    using C = FwdTiles<T>;
    const int tz = pick_tile_z_w(a.g, C::ey, C::e_waves, C::ez_max, W);
    const dim3 blk(kTileX, C::ey), grd((unsigned)(row_tiles(a.g, C::ey, W) * ((a.g.nz + tz - 1) / tz)));
    // FP32: 28 KiB of (unused) LDS per block, so that a CU takes at most 5 blocks of 4 wavefronts: at
    // 80 VGPRs the hardware would run 6 per SIMD, measured 0.261 ms at 256^3 with edge classes
    // against 0.235 ms with 5
    const size_t lds = sizeof(T) == 4 ? 28 * 1024 : 0;
    switch (tz) {
    case 64: hipLaunchKernelGGL((e_pass_kernel<T, C::ey, 64, CLS, W>), grd, blk, lds, s, a); break;
    case 32: hipLaunchKernelGGL((e_pass_kernel<T, C::ey, 32, CLS, W>), grd, blk, lds, s, a); break;
    case 16: hipLaunchKernelGGL((e_pass_kernel<T, C::ey, 16, CLS, W>), grd, blk, lds, s, a); break;
    default: hipLaunchKernelGGL((e_pass_kernel<T, C::ey, 8, CLS, W>), grd, blk, lds, s, a); break;
    }
}

template <typename T>
hipError_t launch_h_pass(const StepArgs<T> &a, hipStream_t s)
{
    switch (row_width(a.g.nx, sizeof(T))) {
    case 16: launch_h_pass_w<T, 16>(a, s); break;
    case 32: launch_h_pass_w<T, 32>(a, s); break;
    default: launch_h_pass_w<T, 64>(a, s); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_e_pass(const StepArgs<T> &a, hipStream_t s)
{
    const int w = row_width(a.g.nx, sizeof(T));
    if (a.cls[0]) {
        if (w == 16) launch_e_pass_w<T, 16, true>(a, s);
        else if (w == 32) launch_e_pass_w<T, 32, true>(a, s);
        else launch_e_pass_w<T, 64, true>(a, s);
    } else {
        if (w == 16) launch_e_pass_w<T, 16, false>(a, s);
        else if (w == 32) launch_e_pass_w<T, 32, false>(a, s);
        else launch_e_pass_w<T, 64, false>(a, s);
    }
    return hipGetLastError();
}

template <typename T, int TX, int TY, bool NT, bool CLS, bool PML>
static void launch_fused_cls(const StepArgs<T> &a, int tz, hipStream_t s)
{
    const dim3 blk(TX, TY), grd(tile_blocks(a.g, TY, tz, TX));
    switch (tz) {
    case 64: hipLaunchKernelGGL((fused_step_kernel<T, TY, 64, CLS, NT, TX, PML>), grd, blk, 0, s, a); break;
    case 32: hipLaunchKernelGGL((fused_step_kernel<T, TY, 32, CLS, NT, TX, PML>), grd, blk, 0, s, a); break;
    case 16: hipLaunchKernelGGL((fused_step_kernel<T, TY, 16, CLS, NT, TX, PML>), grd, blk, 0, s, a); break;
    default: hipLaunchKernelGGL((fused_step_kernel<T, TY, 8, CLS, NT, TX, PML>), grd, blk, 0, s, a); break;
    }
}

template <typename T, int TX, int TY, bool NT>
static void launch_fused_tx(const StepArgs<T> &a, long long waves, int max_tz, hipStream_t s)
{
    const int tz = pick_tile_z(a.g, TY, waves, max_tz, TX);
    const bool pml = a.pml[0].on || a.pml[1].on || a.pml[2].on;
    if constexpr (TX == kTileX) {  // CPML grids run rows of 64 cells (launch_fused_step)
        if (pml) {
            if (a.cls[0]) launch_fused_cls<T, TX, TY, NT, true, true>(a, tz, s);
            else launch_fused_cls<T, TX, TY, NT, false, true>(a, tz, s);
            return;
        }
    }
    if (a.cls[0]) launch_fused_cls<T, TX, TY, NT, true, false>(a, tz, s);
    else launch_fused_cls<T, TX, TY, NT, false, false>(a, tz, s);
}

template <typename T>
hipError_t launch_fused_step(const StepArgs<T> &a, hipStream_t s)
{
    using C = FwdTiles<T>;
    // bytes one step touches (E, H read and written, Js, coefficients): beyond twice the 256 MiB
    // infinity cache the new fields gain from bypassing it (256^3: 6-8 % faster); below, the next
    // step finds them there (128^3 runs 1.5x faster with ordinary stores)
    const double touched = (double)a.g.sxy * a.g.nz * (15.0 * sizeof(T) + 6.0);
    const bool nt = touched > 512.0 * 1024 * 1024;
    // FP32 on periodic grids: rows of 256 (or 128) cells per block when they tile the x extent
    // exactly (4 or 2 wavefronts per row, no x halo between them; 256^3: 282 -> 267 us).  FP64
    // gains nothing from it, and with CPML slabs rows of 64 cells were as fast or faster (512 x 256
    // x 128 CPW: 0.414 vs 0.431 ms; 256^3 with slabs 0.343 vs 0.349 ms).
    const bool pml = a.pml[0].on || a.pml[1].on || a.pml[2].on;
    if constexpr (sizeof(T) == 4) {
        const int tx = pml ? kTileX : (a.g.nx % 256 == 0) ? 256 : (a.g.nx % 128 == 0) ? 128 : kTileX;
        if (tx == 256) {
            if (nt) launch_fused_tx<T, 256, 2, true>(a, C::f_waves, C::fz_max, s);
            else launch_fused_tx<T, 256, 2, false>(a, C::f_waves, C::fz_max, s);
            return hipGetLastError();
        }
        if (tx == 128) {
            if (nt) launch_fused_tx<T, 128, 2, true>(a, C::f_waves, C::fz_max, s);
            else launch_fused_tx<T, 128, 2, false>(a, C::f_waves, C::fz_max, s);
            return hipGetLastError();
        }
    }
    if (nt) launch_fused_tx<T, kTileX, C::fy, true>(a, C::f_waves, C::fz_max, s);
    else launch_fused_tx<T, kTileX, C::fy, false>(a, C::f_waves, C::fz_max, s);
    return hipGetLastError();
}

// Two-step sweep: footprints of 64 x TY cells (the rows of a block share LDS), TZ output planes per
// block.  Measured on 256^3 (TY 4 to 16, TZ 16 to 64): FP32 is fastest with TY = 16 (126 VGPRs, 4
// wavefronts per SIMD, one block per CU) and TZ = 32, 0.196 ms per step against the fused sweep's
// 0.274; FP64 (178 VGPRs, 2 wavefronts per SIMD) with TY = 8 and TZ = 32, 0.371 against 0.553.  The
// CPML instantiations need 181-185 (FP32) and 248-256 (FP64) VGPRs: TY = 8 in both.
template <typename T>
struct TwoStepTiles;
template <>
struct TwoStepTiles<double> {
    static constexpr int ty = 8;
};
template <>
struct TwoStepTiles<float> {
    static constexpr int ty = 16;
};

template <typename T, int TY, bool NT, bool SIDE, bool PML>
static void launch_two_step_nt(const StepArgs<T> &a, hipStream_t s)
{
    constexpr int OX = kTwoStepOX, OY = TY - 2;
    const long long cols = (long long)((a.g.nx + OX - 1) / OX) * ((a.g.ny + OY - 1) / OY);
    // z runs of 32 planes (at 256^3: 16 and 64 were 3-20 % slower), shorter where the grid would then
    // give fewer than two blocks per CU (256 CUs)
    int tz = 32;
    while (tz > 8 && cols * ((a.g.nz + tz - 1) / tz) < 512) tz /= 2;
    const dim3 blk(kTileX, TY);
    const unsigned grd = (unsigned)(cols * ((a.g.nz + tz - 1) / tz));
    switch (tz) {
    case 32: hipLaunchKernelGGL((two_step_kernel<T, TY, 32, NT, SIDE, PML>), dim3(grd), blk, 0, s, a); break;
    case 16: hipLaunchKernelGGL((two_step_kernel<T, TY, 16, NT, SIDE, PML>), dim3(grd), blk, 0, s, a); break;
    default: hipLaunchKernelGGL((two_step_kernel<T, TY, 8, NT, SIDE, PML>), dim3(grd), blk, 0, s, a); break;
    }
}

template <typename T, int TY, bool PML>
static void launch_two_step_tiles(const StepArgs<T> &a, hipStream_t s)
{
    const double touched = (double)a.g.sxy * a.g.nz * (15.0 * sizeof(T) + 6.0);
    const bool nt = touched > 512.0 * 1024 * 1024;
    if (a.side.nsrc > 0 || a.side.nprobe > 0 || a.side.nred > 0) {
        if (nt) launch_two_step_nt<T, TY, true, true, PML>(a, s);
        else launch_two_step_nt<T, TY, false, true, PML>(a, s);
    } else {
        if (nt) launch_two_step_nt<T, TY, true, false, PML>(a, s);
        else launch_two_step_nt<T, TY, false, false, PML>(a, s);
    }
}

template <typename T>
hipError_t launch_two_step(const StepArgs<T> &a, hipStream_t s)
{
    // CPML grids: footprints of eight rows in both precisions (the first step's auxiliary variables
    // ride in registers, which sixteen FP32 wavefronts per block do not leave)
    if (a.pml[0].on || a.pml[1].on || a.pml[2].on) launch_two_step_tiles<T, 8, true>(a, s);
    else launch_two_step_tiles<T, TwoStepTiles<T>::ty, false>(a, s);
    return hipGetLastError();
}

template <typename T>
bool two_step_pays(const StepArgs<T> &a)
{
    if (!a.cls[0]) return false;
    // CPML grids in FP32: the first step's auxiliary variables leave room for footprints of 8 rows,
    // one block per CU (8 wavefronts instead of 16), which pays only where the fused sweep's rows of
    // 64 cells leave a fifth or more of their lanes idle; fused / two-step ms per step: 512 x 256 x
    // 128 with x and z slabs 0.316 / 0.351, the paper's CPW (nx = 146: 24 % idle) 4.58 / 4.18.  In
    // FP64 (8 wavefronts per CU either way) 0.634 / 0.572 and 8.43 / 7.62.
    if ((a.pml[0].on || a.pml[1].on || a.pml[2].on) && sizeof(T) == 4) {
        const int lanes = (a.g.nx + 63) / 64 * 64;
        if ((lanes - a.g.nx) * 5 < lanes) return false;
    }
    // The footprints' overlap costs (64/60)(TY/(TY-2)) in cells computed, repaid once the grid's
    // traffic no longer stays in the 256 MB infinity cache.  Measured, ms per step fused / two-step:
    // 128^3 FP32 0.027 / 0.031, FP64 0.050 / 0.070; 160^3 FP32 0.069 / 0.053, FP64 0.172 / 0.114;
    // 256^3 FP32 0.274 / 0.196, FP64 0.553 / 0.371; 320^3 FP32 0.512 / 0.390, FP64 1.067 / 0.711.
    return (long long)a.g.sxy * a.g.nz >= (3LL << 20) && a.g.nx >= 64 && a.g.ny >= 32 && a.g.nz >= 16;
}

template <typename T>
hipError_t launch_probes(const ProbeArgs<T> &a, int nprobe, hipStream_t s)
{
    if (nprobe <= 0) return hipSuccess;
    hipLaunchKernelGGL(probe_kernel<T>, dim3(nprobe), dim3(kProbeThreads), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_half_kick(const StepArgs<T> &a, T sgn, T *const Hout[3], T *const Jout[3], hipStream_t s)
{
    const long long N = a.g.sxy * a.g.nz;
    const long long nbl = (N + 255) / 256;
    const int nb = (int)(nbl < 65536 ? nbl : 65536);
    hipLaunchKernelGGL(half_kick_kernel<T>, dim3(nb), dim3(256), 0, s, a, sgn, Hout ? Hout[0] : nullptr,
                       Hout ? Hout[1] : nullptr, Hout ? Hout[2] : nullptr, Jout ? Jout[0] : nullptr,
                       Jout ? Jout[1] : nullptr, Jout ? Jout[2] : nullptr);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_class_table(const StepArgs<T> &a, const T *mat, const uint64_t *tuple, int ncls, T *tab,
                              hipStream_t s)
{
    if (ncls <= 0) return hipSuccess;
    hipLaunchKernelGGL(class_table_kernel<T>, dim3((ncls + 255) / 256), dim3(256), 0, s, a, mat, tuple, ncls, tab);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_energy(const StepArgs<T> &a, double *part, int nblocks, hipStream_t s, double *dst)
{
    hipLaunchKernelGGL(energy_kernel<T>, dim3(nblocks), dim3(kRedThreads), 0, s, a, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fold_pairs_kernel, dim3(1), dim3(kRedThreads), 0, s, part, nblocks, dst ? dst : part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_map_stats(const T *eps, const T *sig, const T *ell, long long n, double *scratch, int nblocks,
                            hipStream_t s)
{
    hipLaunchKernelGGL(map_stats_kernel<T>, dim3(nblocks), dim3(kRedThreads), 0, s, eps, sig, ell, n, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(map_stats_fold_kernel, dim3(1), dim3(kRedThreads), 0, s, scratch, nblocks);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_nonfinite(const NonfiniteArgs<T> &a, unsigned long long *counter, long long step, hipStream_t s)
{
    const long long nbl = (a.n + kRedThreads - 1) / kRedThreads;
    const int nb = (int)(nbl < 4096 ? nbl : 4096);
    hipLaunchKernelGGL(nonfinite_kernel<T>, dim3(nb), dim3(kRedThreads), 0, s, a, counter,
                       (unsigned long long)step);
    return hipGetLastError();
}

hipError_t launch_nonfinite_reset(unsigned long long *counter, hipStream_t s)
{
    hipLaunchKernelGGL(nonfinite_reset_kernel, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    const size_t nw = bytes / 4;
    const size_t nbl = (nw + 255) / 256;
    const int nb = (int)(nbl < 16384 ? nbl : 16384);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(nb), dim3(256), 0, s, (uint32_t *)p, nw);
    return hipGetLastError();
}

#define TFL_INSTANTIATE(T)                                                                                  \
    template hipError_t launch_h_pass<T>(const StepArgs<T> &, hipStream_t);                                 \
    template hipError_t launch_e_pass<T>(const StepArgs<T> &, hipStream_t);                                 \
    template hipError_t launch_fused_step<T>(const StepArgs<T> &, hipStream_t);                             \
    template hipError_t launch_two_step<T>(const StepArgs<T> &, hipStream_t);                               \
    template bool two_step_pays<T>(const StepArgs<T> &);                                                   \
    template hipError_t launch_class_table<T>(const StepArgs<T> &, const T *, const uint64_t *, int, T *,     \
                                              hipStream_t);                                                 \
    template hipError_t launch_probes<T>(const ProbeArgs<T> &, int, hipStream_t);                           \
    template hipError_t launch_half_kick<T>(const StepArgs<T> &, T, T *const[3], T *const[3], hipStream_t); \
    template hipError_t launch_energy<T>(const StepArgs<T> &, double *, int, hipStream_t, double *);        \
    template hipError_t launch_nonfinite<T>(const NonfiniteArgs<T> &, unsigned long long *, long long,       \
                                            hipStream_t);                                                   \
    template hipError_t launch_map_stats<T>(const T *, const T *, const T *, long long, double *, int, hipStream_t);

TFL_INSTANTIATE(double)
TFL_INSTANTIATE(float)

}  // namespace tfl
