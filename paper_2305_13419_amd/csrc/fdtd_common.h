// Device helpers shared by the forward and adjoint sweeps.
#pragma once

#include "tfl_internal.h"

namespace tfl {

// Blocks are dealt to the 8 XCDs round robin; renumber them so that each XCD
// receives a contiguous range of tiles (neighbouring tiles share an L2).
static __device__ __forceinline__ int logical_block(int b, int nblocks)
{
    const int q = nblocks >> 3, r = nblocks & 7;
    const int x = b & 7, m = b >> 3;
    return x * q + min(x, r) + m;
}

// Column tile of a z-marching sweep: TX x TY columns of the x-y plane (TX / 64
// wavefronts per row) and TZ planes along z.  Tiles are numbered x fastest,
// then y, then z, and blocks are renumbered so that each XCD takes a contiguous
// range: the blocks of one XCD sweep neighbouring columns of the same planes at
// the same time.  With zmix (the fused, two-step and adjoint sweeps on grids
// whose CPML z slabs hold at least an eighth of the planes: zmix_of) z is
// numbered before y: the slab planes cost more, and with z last the XCDs would
// take one z range each, the two at the ends all the slab planes (measured on
// 32 of 128 planes: 1-7 % faster for those sweeps; 2-5 % slower for the two
// passes, which keep z last; on the paper's CPW, 32 of 1312 planes, 6 % slower,
// y halo rows being shared less within an XCD).  Returns false for lanes
// outside the grid.
template <typename P>
static __device__ __forceinline__ bool zmix_of(const P &pz, int nz)
{
    return pz.on && pz.P * 8 >= nz;
}

static __device__ __forceinline__ void tile_yz(int tr, int nty, int ntz, bool zmix, int &ty, int &tz)
{
    if (zmix) {
        tz = tr % ntz;
        ty = tr / ntz;
    } else {
        ty = tr % nty;
        tz = tr / nty;
    }
}

template <int TY, int TZ, int TX = kTileX>
static __device__ __forceinline__ bool tile_of(int nx, int ny, int nz, int &i, int &j, int &k0, int &k1,
                                               bool zmix = false)
{
    const int ntx = (nx + TX - 1) / TX, nty = (ny + TY - 1) / TY, ntz = (nz + TZ - 1) / TZ;
    const int t = logical_block(blockIdx.x, ntx * nty * ntz);
    const int tx = t % ntx;
    const int tr = t / ntx;
    int ty, tz;
    tile_yz(tr, nty, ntz, zmix, ty, tz);
    i = tx * TX + threadIdx.x;
    j = ty * TY + threadIdx.y;
    k0 = tz * TZ;
    k1 = min(k0 + TZ, nz);
    return i < nx && j < ny;
}

// The same with rows of W lanes (blockDim = (64, TY)): W = 64 is tile_of; with W = 32 or 16 a
// wavefront covers 64 / W rows of W cells and a block 64 TY / W rows, for grids whose nx would
// leave much of a 64-lane row idle.
template <int TY, int TZ, int W>
static __device__ __forceinline__ bool tile_of_w(int nx, int ny, int nz, int &i, int &j, int &k0, int &k1,
                                                 bool zmix = false)
{
    constexpr int rows = kTileX * TY / W;
    const int ntx = (nx + W - 1) / W, nty = (ny + rows - 1) / rows, ntz = (nz + TZ - 1) / TZ;
    const int t = logical_block(blockIdx.x, ntx * nty * ntz);
    const int tx = t % ntx;
    const int tr = t / ntx;
    int ty, tz;
    tile_yz(tr, nty, ntz, zmix, ty, tz);
    const int lane = threadIdx.x + kTileX * threadIdx.y;
    i = tx * W + lane % W;
    j = ty * rows + lane / W;
    k0 = tz * TZ;
    k1 = min(k0 + TZ, nz);
    return i < nx && j < ny;
}

// Access at a wave-uniform base plus a 32-bit per-lane byte offset, through a
// global (address space 1) pointer: the base stays in scalar registers and the
// access takes the "SGPR base + VGPR offset" form.
template <typename T>
static __device__ __forceinline__ T ldp(const T *base, uint32_t off)
{
    return *(const __attribute__((address_space(1))) T *)(reinterpret_cast<const char *>(base) + off);
}

template <typename T>
static __device__ __forceinline__ void stp(T *base, uint32_t off, T v)
{
    *(__attribute__((address_space(1))) T *)(reinterpret_cast<char *>(base) + off) = v;
}

// ldp / stp with the offset passed through an empty asm at the access: the
// compiler can then neither hoist its 64-bit extension out of a loop nor keep a
// 64-bit address per array and neighbour live across it (which had doubled the
// address registers of the adjoint sweeps).
template <typename T>
static __device__ __forceinline__ T ldo(const T *base, uint32_t off)
{
    asm volatile("" : "+v"(off));
    return ldp(base, off);
}

template <typename T>
static __device__ __forceinline__ void sto(T *base, uint32_t off, T v)
{
    asm volatile("" : "+v"(off));
    stp(base, off, v);
}

// stp with a nontemporal hint when NT (the line is not kept in L2 / the infinity cache)
template <bool NT, typename T>
static __device__ __forceinline__ void stp_hint(T *base, uint32_t off, T v)
{
    auto *p = (__attribute__((address_space(1))) T *)(reinterpret_cast<char *>(base) + off);
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

static __device__ __forceinline__ int slab_slot(int i, int lo, int hi, int n)
{
    if (i < lo) return i;
    if (i >= n - hi) return lo + i - (n - hi);
    return -1;
}

// 1/c for c = 1..4 without branches: 2^-(c>>1) is exact for 1, 2 and 4.
template <typename T>
static __device__ __forceinline__ T inv_count(int c)
{
    const T p2 = ldexp(T(1), -(c >> 1));
    return c == 3 ? T(1) / T(3) : p2;
}

// A wave-uniform element offset kept opaque to loop strength reduction, so that
// accesses inside z-marching loops stay "scalar base + 32-bit lane offset"
// instead of becoming per-lane 64-bit pointer induction variables.
static __device__ __forceinline__ long long opaque_offset(long long off)
{
    asm volatile("" : "+s"(off));
    return off;
}

// Per-edge material of the four cells q0..q3 sharing an edge (Sec. 3): if any
// cell is superconducting (ell > 0) the edge takes the mean over those cells,
// otherwise the mean over all four.  Summed in q order.
template <typename T>
static __device__ __forceinline__ void edge_material(const T e[4], const T s[4], const T l[4], T &eps, T &sig, T &ell)
{
    const bool anysc = (l[0] > T(0)) | (l[1] > T(0)) | (l[2] > T(0)) | (l[3] > T(0));
    T se = T(0), ss = T(0), sl = T(0);
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool use = !anysc || (l[q] > T(0));
        se += use ? e[q] : T(0);
        ss += use ? s[q] : T(0);
        sl += use ? l[q] : T(0);
        cnt += use ? 1 : 0;
    }
    const T ic = inv_count<T>(cnt);
    eps = T(kEps0) * (se * ic);
    sig = ss * ic;
    ell = sl * ic;
}

// Coefficients of one edge: E^{n+1} = ca E^n + cb (curl H - Js^{n+1/2}) and
// Js^{n+1/2} = Js^{n-1/2} + cj E^n with cj = dt ell_e / mu0 (cj = 0 off the
// superconductor, where Js stays zero and is neither read nor written).
template <typename T>
struct EdgeCoef {
    T ca, cb, cj;
};

// Coefficients of class c from the class table (4 values per entry: ca, cb, cj, 0).
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double2_t __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ EdgeCoef<T> class_coef(const T *tab, uint32_t c)
{
    if constexpr (sizeof(T) == 8) {
        const double2_t ab = ldp(reinterpret_cast<const double2_t *>(tab), c * 32u);
        return {ab.x, ab.y, ldp(tab, c * 32u + 16u)};
    } else {
        const float4_t v = ldp(reinterpret_cast<const float4_t *>(tab), c * 16u);
        return {v.x, v.y, v.z};
    }
}

// Stretched derivative: d <- kappa^-1 d + psi, psi <- b psi + c d.
template <typename T>
static __device__ __forceinline__ T stretch(T d, T *psi, long long pidx, T b, T c, T kinv)
{
    const T p = b * psi[pidx] + c * d;
    psi[pidx] = p;
    return kinv * d + p;
}

// The same with the new variable written to psio: the fused sweep reads the
// H-side variables of one set and writes the other, as it does E and H, since
// the neighbours it recomputes read their old values.
template <typename T>
static __device__ __forceinline__ T stretch_to(T d, const T *psi, T *psio, long long pidx, T b, T c, T kinv)
{
    const T p = b * psi[pidx] + c * d;
    psio[pidx] = p;
    return kinv * d + p;
}

// The stretching of d with the stored variable's value already loaded: p is
// the new variable (for the caller to store, or not).
template <typename T>
static __device__ __forceinline__ T stretch_v(T d, T psi, T b, T c, T kinv, T &p)
{
    p = b * psi + c * d;
    return kinv * d + p;
}

// stretch, stretch_to and stretch_virtual on a variable at a scalar base plus a
// lane byte offset (ldo / sto)
template <typename T>
static __device__ __forceinline__ T stretch_o(T d, T *psi, uint32_t off, T b, T c, T kinv)
{
    const T p = b * ldo(psi, off) + c * d;
    sto(psi, off, p);
    return kinv * d + p;
}

template <typename T>
static __device__ __forceinline__ T stretch_to_o(T d, const T *psi, T *psio, uint32_t off, T b, T c, T kinv)
{
    const T p = b * ldo(psi, off) + c * d;
    sto(psio, off, p);
    return kinv * d + p;
}

template <typename T>
static __device__ __forceinline__ T stretch_virtual_o(T d, const T *psi, uint32_t off, T b, T c, T kinv)
{
    const T p = b * ldo(psi, off) + c * d;
    return kinv * d + p;
}

template <typename T>
static __device__ __forceinline__ T stretch_virtual(T d, const T *psi, long long pidx, T b, T c, T kinv)
{
    const T p = b * psi[pidx] + c * d;
    return kinv * d + p;
}


}  // namespace tfl
