// Internal types shared by the host driver (api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tfl.h"

namespace tfl {

constexpr double kEps0 = 8.8541878128e-12;  // F/m (CODATA 2018)
constexpr double kMu0 = 1.25663706212e-6;   // H/m (CODATA 2018)
constexpr double kTwoPi = 6.283185307179586476925286766559;

// Tiles of the 2.5-D sweeps: a block covers kTileX x TY columns of the x-y
// plane (one 64-wide wavefront per row) and marches TZ planes along z, keeping
// the z neighbour in registers.  TY and TZ are chosen per sweep at launch.
#ifndef TFL_MIN_WAVES
#define TFL_MIN_WAVES 1
#endif
constexpr int kTileX = 64;

struct GridDims {
    int nx, ny, nz;
    long long sxy;  // nx * ny
};

// One axis of the convolutional PML.  Coefficient tables are indexed by the
// node index i (integer positions, E side) or by i for the half position
// i + 1/2 (H side).  Auxiliary variables are stored only in the absorbing
// slabs; slot(i) maps a cell index to its slab column.
template <typename T>
struct PmlAxis {
    int on;     // axis is CPML
    int lo, hi; // slab cells
    int P;      // lo + hi
    int n;
    const T *bn, *cn, *kn;  // node tables
    const T *bh, *ch, *kh;  // half-node tables
    T *psiH[2];             // H-side variables (two components)
    T *psiE[2];             // E-side variables (two components)
    T *psiHo[2];            // where the fused sweep writes the new H-side variables (psiH elsewhere)
    T *psiEo[2];            // where the two-step sweep writes the new E-side variables (psiE elsewhere)
};

struct ProbeDesc;

// Work that rides along with the E update of a sweep (the fused sweep, the E pass and the two-step
// sweep), so that a step with sources and probes is still one launch:
//  - soft sources: the sweep adds sg[p] (the value source p adds at this step; sg2[p] at the second
//    step of a two-step sweep) to the new E of every edge of box p, in source order, after the PEC
//    walls are zeroed;
//  - probe copies: the new E of each edge of probe p's box goes to pcopy[p] in box order (x fastest);
//    a two-step sweep writes its first step's E there and its second step's to pcopy2[p];
//  - probe sums: blocks 0 .. nred-1 first sum the copies rcopy[b] (and then rcopy2[b]) that the
//    previous sweep wrote and record samples rn (and rn + 1) of probe b (series and DFT), with the
//    probe kernel's summation order.
constexpr int kFoldProbes = 4;
struct SideArgs {
    int nsrc;
    int nprobe;
    int nred;                      // probes whose pending samples the sweep records first (0: none)
    int nsamp;                     // pending samples per probe: 1 (rcopy) or 2 (rcopy, then rcopy2)
    int sbox[TFL_MAX_SOURCES][7];  // component, i0, i1, j0, j1, k0, k1
    double sg[TFL_MAX_SOURCES];
    double sg2[TFL_MAX_SOURCES];   // the values at the second step of a two-step sweep
    int pbox[kFoldProbes][7];
    void *pcopy[kFoldProbes];
    void *pcopy2[kFoldProbes];     // the second step's copies (two-step sweep)
    const void *rcopy[kFoldProbes];
    const void *rcopy2[kFoldProbes];
    const ProbeDesc *pdesc;        // descriptors of the probes (device memory)
    long long rn;                  // sample index of the first pending sample
    double dt;
};

template <typename T>
struct StepArgs {
    GridDims g;
    T *E[3];
    T *Eout[3];  // where the E pass writes E^{n+1} (E itself except in recomputation)
    T *H[3];
    T *Hout[3];  // where the fused sweep writes H^{n+1/2} (the two-pass H pass updates H in place)
    T *J[3];
    T *Jout[3];  // where the two-step sweep writes Js^{n+3/2} (every other sweep updates Js in place)
    const T *eps, *sig, *ell;  // per-cell maps
    const uint16_t *cls[3];    // edge classes (x, y, z edges), or null: form coefficients from the maps
    const T *ctab;             // class table: 4 values (ca, cb, cj, 0) per class
    T rd[3];                   // 1/dx, 1/dy, 1/dz
    T hdt;                     // dt / mu0
    T dt;
    T theta;
    PmlAxis<T> pml[3];
    SideArgs side;
};

struct SourceDesc {
    int comp;
    int i0, i1, j0, j1, k0, k1;
    double amp;
    int wave;
    double f, t0, tw;
};

struct ProbeDesc {
    int comp;
    int i0, i1, j0, j1, k0, k1;
    double *series;
    long long cap;
    int nfreq;
    double freq[TFL_MAX_FREQS];
    double *dft;
};

// Probe descriptors live in device memory (the bound scratch buffer); a
// launch samples probes [first, first + gridDim.x), from the fields or, where
// copy[b] is set, from the box values a sweep copied out (launch block b).
template <typename T>
struct ProbeArgs {
    GridDims g;
    const T *E[3];
    long long n;
    double dt;
    const ProbeDesc *p;
    int first;
    const T *copy[kFoldProbes];
};

// The nine state arrays (Ex, Ey, Ez, Hx, Hy, Hz, Jx, Jy, Jz) of the non-finite check.
template <typename T>
struct NonfiniteArgs {
    const T *f[9];
    long long n;
};

// Reverse-mode (adjoint) sweep arguments.  Adjoint fields are stored in the
// field precision; gradient accumulators are FP64.  lpsiH/lpsiE follow the
// compact slab layout of the forward auxiliary variables.
template <typename T>
struct AdjArgs {
    StepArgs<T> f;
    T *lE[3], *lH[3], *lJ[3], *mu[3];
    T *lpsiH[3][2], *lpsiE[3][2];
    double *gL[3], *gS[3];
    const T *En[3];  // E^m: input E of the forward step m -> m+1 (A part; ell gradient)
    int doC, doA;
    int obj;         // add og to lE[ocomp] on the objective box
    int ocomp, ob[6];
    double og;
};

// The sigma gradient of a window of up to kGradWindow reverse steps (adj_grad_sigma_kernel): per
// step w of the window, in the order the edge sweeps ran them, the mu its edge sweep stored, its
// E^{m+1} (E'_pre after the sources sg[w] are taken out of the boxes sbox) and E^m (null when theta
// is 1, where it does not enter).
constexpr int kGradWindow = 8;
template <typename T>
struct GradSigmaArgs {
    GridDims g;
    double *gS[3];
    const T *mu[kGradWindow][3];
    const T *Ep[kGradWindow][3];
    const T *En[kGradWindow][3];
    int nwin;
    double theta;
    int nsrc;
    int sbox[TFL_MAX_SOURCES][7];
    double sg[kGradWindow][TFL_MAX_SOURCES];
};

// z length of the column tiles of a z-marching sweep, chosen at launch: the
// longest of max_tz, ..., 16, 8 planes whose tiles still give at least
// target_waves wavefronts (longer runs re-read fewer halo planes; enough waves
// are needed to cover the HBM latency on small grids).
inline int pick_tile_z(const GridDims &g, int ty, long long target_waves, int max_tz, int tx = kTileX)
{
    const long long cols = (long long)((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty);
    int tz = max_tz;
    while (tz > 8 && cols * ((g.nz + tz - 1) / tz) * ty * (tx / kTileX) < target_waves) tz /= 2;
    return tz;
}

// Column tiles and z length for tiles of 64 TY / W rows of W lanes (tile_of_w).
inline long long row_tiles(const GridDims &g, int ty, int w)
{
    const int rows = kTileX * ty / w;
    return (long long)((g.nx + w - 1) / w) * ((g.ny + rows - 1) / rows);
}

inline int pick_tile_z_w(const GridDims &g, int ty, long long target_waves, int max_tz, int w)
{
    const long long cols = row_tiles(g, ty, w);
    int tz = max_tz;
    while (tz > 8 && cols * ((g.nz + tz - 1) / tz) * ty < target_waves) tz /= 2;
    return tz;
}

// Lanes per tile row of the two passes: 64 unless a narrower row (32 or 16 lanes, at least 256 bytes
// of the storage type: two cache lines) leaves clearly less of the row idle for this nx.  Measured on
// the paper's CPW (nx = 146): FP64 rows of 32 cells 4 % faster than 64; FP32 rows of 32 cells
// (128 bytes) 1 % slower.
inline int row_width(int nx, int esz)
{
    auto idle = [nx](int w) {
        const int padded = (nx + w - 1) / w * w;
        return double(padded - nx) / padded;
    };
    int best = kTileX;
    double best_idle = idle(kTileX);
    for (int w = 32; w >= 16; w /= 2) {
        if (w * esz < 256) break;
        if (idle(w) + 0.02 < best_idle) {
            best = w;
            best_idle = idle(w);
        }
    }
    return best;
}

inline int tile_blocks(const GridDims &g, int ty, int tz, int tx = kTileX)
{
    return (int)(((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty) * ((g.nz + tz - 1) / tz));
}

// Host-side launchers (kernels_fwd.hip).
template <typename T> hipError_t launch_h_pass(const StepArgs<T> &a, hipStream_t s);
template <typename T> hipError_t launch_e_pass(const StepArgs<T> &a, hipStream_t s);
// One whole step in one sweep: reads E^n (E) and H^{n-1/2} (H), writes E^{n+1} (Eout) and
// H^{n+1/2} (Hout), and on CPML axes the H-side variables from psiH to psiHo; Js and the E-side
// variables in place.  E, Eout, H, Hout and psiH, psiHo must not overlap.
template <typename T> hipError_t launch_fused_step(const StepArgs<T> &a, hipStream_t s);
// Two time steps in one sweep (edge classes bound; soft sources and folded probes ride along): reads
// E^n, H^{n-1/2}, Js^{n-1/2} from E, H, J and writes E^{n+2}, H^{n+3/2}, Js^{n+3/2} to Eout, Hout,
// Jout, and on CPML axes all four auxiliary variables from psiH, psiE to psiHo, psiEo; outputs must
// not overlap the inputs.  Results equal two fused steps bit for bit.
template <typename T> hipError_t launch_two_step(const StepArgs<T> &a, hipStream_t s);
// Whether the two-step sweep (edge classes bound) pays on this grid and storage type.
template <typename T> bool two_step_pays(const StepArgs<T> &a);
// Class table of the edge-coefficient path: entry c = coefficients of the four cells
// mat[(tuple[c] >> 16 q) & 0xffff], q = 0..3 (mat: eps_r, sigma, ell per cell material).
template <typename T>
hipError_t launch_class_table(const StepArgs<T> &a, const T *mat, const uint64_t *tuple, int ncls, T *tab,
                              hipStream_t s);
template <typename T> hipError_t launch_probes(const ProbeArgs<T> &a, int nprobe, hipStream_t s);
// Integer-time half kick: Hout = Hin + sgn dt/(2 mu0) curlE (stretched, with
// the PML variables advanced virtually), Jout = Jin - sgn dt/2 ell_e E / mu0 on
// SC edges (0 on other edges).  sgn = +1 goes back half a step, -1 forward.
template <typename T>
hipError_t launch_half_kick(const StepArgs<T> &a, T sgn, T *const Hout[3], T *const Jout[3], hipStream_t s);
// Energy partials into part (FP64, 2 nblocks values), second stage reduces to dst[0..1] (part[0..1]
// when dst is null).
template <typename T>
hipError_t launch_energy(const StepArgs<T> &a, double *part, int nblocks, hipStream_t s, double *dst = nullptr);
// Blocks of the energy reduction in the fixed device scratch of the allocation-free entry point, and
// that scratch's device address on the current device (looked up on the first call per device).
constexpr int kStaticScratchBlocks = 1024;
hipError_t static_scratch(double **out);
// Map statistics: min eps, min sigma, min ell, max ell, nonfinite count.
template <typename T>
hipError_t launch_map_stats(const T *eps, const T *sig, const T *ell, long long n, double *scratch, int nblocks,
                            hipStream_t s);
// Non-finite check: counter[0] += NaN / Inf values of the nine arrays, counter[1] = min(counter[1], step)
// when any; the reset sets counter[0] = 0 and counter[1] to the largest value (a kernel, no memset).
template <typename T>
hipError_t launch_nonfinite(const NonfiniteArgs<T> &a, unsigned long long *counter, long long step, hipStream_t s);
hipError_t launch_nonfinite_reset(unsigned long long *counter, hipStream_t s);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);

// Gram matrix of the lagged decimated series (fit.hip): for every pair
// j <= k <= P, G[j][k] = sum_{m=P}^{M-1} x_{m-j} x_{m-k}, x_m = series[start + m*decim];
// the (P+1)(P+2)/2 sums are written to out in row-major upper-triangle order.
hipError_t launch_gram(const double *series, long long start, long long count, long long decim, int order,
                       double *out, hipStream_t s);

// Residual correction of the linear predictor a (device, order P):
// out[j-1] = sum_{m=P}^{M-1} x_{m-j} (x_m - sum_k a_k x_{m-k}), j = 1..P.
hipError_t launch_lp_residual(const double *series, long long start, long long count, long long decim, int order,
                              const double *a, double *out, hipStream_t s);

// Adjoint launchers (kernels_adj.hip).
template <typename T> hipError_t launch_adj_faces(const AdjArgs<T> &a, hipStream_t s);
template <typename T> hipError_t launch_adj_edges(const AdjArgs<T> &a, hipStream_t s);
template <typename T> hipError_t launch_adj_grad_sigma(const GradSigmaArgs<T> &g, hipStream_t s);
// gL += -dt/(2 mu0) lJ E^0 on superconducting edges (dependence of Js^{-1/2} on ell).
template <typename T> hipError_t launch_adj_initial_kick(const AdjArgs<T> &a, hipStream_t s);
// Per-edge FP64 accumulators -> per-cell gradients (derivative of the edge rule).
template <typename T>
hipError_t launch_adj_edge_to_cell(const AdjArgs<T> &a, double *grad_ell, double *grad_sig, hipStream_t s);

}  // namespace tfl
