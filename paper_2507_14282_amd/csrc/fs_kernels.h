// fs_kernels.h -- gfx950 kernels of the faux-shock hybrid step.
//
// Data layout in HBM
//  * particles of one species: structure of arrays in fixed-capacity tile
//    bins (slots [t*cap, t*cap + count[t]) of tile t), ping-ponged between two
//    buffers every step.  Each tile is read once, contiguously, by one
//    workgroup and written back binned by destination tile, so the particle
//    state streams through HBM exactly once per step.
//  * gather grid: per field node 6 reals (E, Bbar) = the three pairs
//    (Ex, Ey), (Ez, Bbarx), (Bbary, Bbarz), staged per tile in LDS.
//  * moments: per species int64 [node][R, Gx, Gy, Gz], accumulated per tile
//    in LDS with 64-bit LDS atomics and flushed with one global atomic per
//    non-zero (node, moment).
//  * fields: FP64 planar arrays, B at cell centres, E at nodes.
#pragma once
#include "fs_device.h"

namespace fsk {

// Geometry and constants of a run, passed by value to every kernel.
struct Geo {
    int dim, nx, nyc, nzc;        // cells in x and active transverse sizes
    int nxn, ndx, g;              // field nodes in x, deposit nodes in x, deposit ghosts
    int xbc;                      // 0 box (inflow + wall), 1 periodic
    int ntx, nty, ntz, ntiles;
    int bx, by;                   // packed cell bit widths for x and y
    int b, sv;                    // fixed-point position / velocity bits
    int mclamp;                   // boundary node moment fill distance (shape order)
    double dt, dx, u_sh, u2, sigma, cr_w, dtdx, rinv;
    double c_light, ic2;          // c / v_A and 1 / c^2; both 0 without relativity
    uint64_t seed;
};

// Section pointers of one particle buffer.
template <typename R> struct PBuf {
    int32_t* cell;
    R* off[3];
    R* v[3];
    uint32_t* id;
};

// Per-species crosser list filled by the push and drained by the wall kernel.
struct XList {
    uint32_t* id;
    double* delta;                // overshoot beyond x = L (cells)
    int32_t* cy;
    int32_t* cz;
    double* oy;
    double* oz;
    double* v;                    // 3 planar arrays of cap
    int32_t* src;                 // bin slot the crosser came from (for a step's record)
    int32_t* count;
    int64_t cap;
};

// Device counters of a step.
enum {
    C_INC = 0, C_REFL, C_TRANS, C_OPEN, C_ESC, C_INJ_TH, C_INJ_CR, C_SAT, C_OOR, C_FLAGS,
    C_REM0, C_REM1, C_ADD0, C_ADD1, C_N
};
enum { F_TILE = 1, F_XLIST = 2, F_NAN = 4, F_SAT = 8 };

__device__ __forceinline__ int cell_x(int32_t c, const Geo& G) { return c & ((1 << G.bx) - 1); }
__device__ __forceinline__ int cell_y(int32_t c, const Geo& G) { return (c >> G.bx) & ((1 << G.by) - 1); }
__device__ __forceinline__ int cell_z(int32_t c, const Geo& G) { return c >> (G.bx + G.by); }
__device__ __forceinline__ int32_t pack_cell(int x, int y, int z, const Geo& G) {
    return x | (y << G.bx) | (z << (G.bx + G.by));
}

// Tile of a (wrapped, non-negative) cell.
template <int D> __device__ __forceinline__ int tile_of(int x, int y, int z, const Geo& G) {
    using T = TileShape<D>;
    unsigned r = 0;
    if constexpr (D >= 3) r = (unsigned)z / T::Z;
    if constexpr (D >= 2) r = (unsigned)y / T::Y + __umul24(G.nty, r);
    return (int)((unsigned)x / T::X + __umul24(G.ntx, r));
}

// Global deposit-grid index of node (i, j, k) (unwrapped), or -1 if it lies
// outside the deposit grid in a non-periodic x.
__device__ __forceinline__ long dep_index(int i, int j, int k, const Geo& G) {
    if (G.xbc == 1) i = wrapi(i, G.nx);
    else {
        i += G.g;
        if (i < 0 || i >= G.ndx) return -1;
    }
    j = wrapi(j, G.nyc);
    k = wrapi(k, G.nzc);
    // the layout keeps ndx and nyc*nzc below 2^24 and the grid below 2^31
    // nodes, so the index is exact in 24-bit products
    return (long)(i + (int)__umul24(G.ndx, j + (int)__umul24(G.nyc, k)));
}

// Field-node index for a gather: x clamped to the physical nodes in the box,
// wrapped when periodic; y, z wrapped.
__device__ __forceinline__ long gather_index(int i, int j, int k, const Geo& G) {
    if (G.xbc == 1) i = wrapi(i, G.nx);
    else { i = i < 0 ? 0 : i; i = i > G.nx ? G.nx : i; }
    j = wrapi(j, G.nyc);
    k = wrapi(k, G.nzc);
    return (long)(i + (int)__umul24(G.nxn, j + (int)__umul24(G.nyc, k)));
}

// Adds one particle's fixed-point moments at (unwrapped) cell (cx, cy, cz)
// with integer weights wx/wy/wz starting at the stencil offsets rx/ry/rz.
// Into LDS when the whole stencil lies in the tile's deposit box, otherwise
// straight into the global grid.
// WHICH selects the moments: 1 the density R, 2 the flux G, 3 both.
template <int D, int S, int WHICH = 3>
__device__ __forceinline__ void deposit_one(unsigned long long* lds, int bx0, int by0, int bz0,
                                            unsigned long long* mom, const Geo& G, int cx, int cy,
                                            int cz, const int* wx, const int* wy, const int* wz,
                                            int rx, int ry, int rz, const int vq[3], int& oor) {
    using X = Extent<D, S>;
    constexpr int N = Stencil<S>::N;
    constexpr int NY = D >= 2 ? N : 1, NZ = D >= 3 ? N : 1;
    int lx = cx + rx - bx0, ly = D >= 2 ? cy + ry - by0 : 0, lz = D >= 3 ? cz + rz - bz0 : 0;
    bool in_lds = lds != nullptr && lx >= 0 && lx + N <= X::DX;
    if constexpr (D >= 2) in_lds = in_lds && ly >= 0 && ly + N <= X::DY;
    if constexpr (D >= 3) in_lds = in_lds && lz >= 0 && lz + N <= X::DZ;
    if constexpr (N == 2) {
        if (in_lds) {
            // CIC: each lane walks the corners of its cell in an order set by
            // its lane bits (corner k is visited as k xor f), so two lanes in
            // the same cell update different nodes in the same instruction
            // instead of serialising on one address.
            const int lane = __lane_id();
            const int fa = lane & 1, fb = D >= 2 ? (lane >> 1) & 1 : 0, fc = D >= 3 ? (lane >> 2) & 1 : 0;
            const int ux[2] = {fa ? wx[1] : wx[0], fa ? wx[0] : wx[1]};
            const int uy[2] = {fb ? wy[1] : wy[0], fb ? wy[0] : wy[1]};
            const int uz[2] = {fc ? wz[1] : wz[0], fc ? wz[0] : wz[1]};
            const int sx = fa ? -1 : 1, sy = fb ? -X::DX : X::DX, sz = fc ? -X::DX * X::DY : X::DX * X::DY;
            const int base = ((lz + fc) * X::DY + (ly + fb)) * X::DX + (lx + fa);
#pragma unroll
            for (int c = 0; c < NZ; ++c) {
#pragma unroll
                for (int b = 0; b < NY; ++b) {
                    const int wyz = D >= 3 ? __umul24(uy[b], uz[c]) : (D >= 2 ? uy[b] : 1);
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        const int W = D >= 2 ? __umul24(ux[a], wyz) : ux[a];
                        unsigned long long* p = lds + (base + a * sx + b * sy + c * sz);
                        if constexpr (WHICH & 1) atomicAdd(p, (unsigned long long)W);
                        if constexpr (WHICH & 2) {
                            atomicAdd(p + X::DN, (unsigned long long)mul24(W, vq[0]));
                            atomicAdd(p + 2 * X::DN, (unsigned long long)mul24(W, vq[1]));
                            atomicAdd(p + 3 * X::DN, (unsigned long long)mul24(W, vq[2]));
                        }
                    }
                }
            }
            return;
        }
    }
    if constexpr (N == 3) {
        if (in_lds) {
            // TSC: the same idea with the three corners per axis visited in
            // an order rotated by the lane's base-3 digits
            const int lane = __lane_id();
            const int ra = lane % 3, rb = D >= 2 ? (lane / 3) % 3 : 0, rc = D >= 3 ? (lane / 9) % 3 : 0;
            int ux[3], uy[3] = {1, 0, 0}, uz[3] = {1, 0, 0}, ox[3], oy[3] = {0, 0, 0}, oz[3] = {0, 0, 0};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int k = a + ra >= 3 ? a + ra - 3 : a + ra;
                ux[a] = k == 0 ? wx[0] : (k == 1 ? wx[1] : wx[2]);
                ox[a] = k;
                if constexpr (D >= 2) {
                    const int kb = a + rb >= 3 ? a + rb - 3 : a + rb;
                    uy[a] = kb == 0 ? wy[0] : (kb == 1 ? wy[1] : wy[2]);
                    oy[a] = kb * X::DX;
                }
                if constexpr (D >= 3) {
                    const int kc = a + rc >= 3 ? a + rc - 3 : a + rc;
                    uz[a] = kc == 0 ? wz[0] : (kc == 1 ? wz[1] : wz[2]);
                    oz[a] = kc * X::DX * X::DY;
                }
            }
            const int base = (lz * X::DY + ly) * X::DX + lx;
#pragma unroll
            for (int c = 0; c < NZ; ++c) {
#pragma unroll
                for (int b = 0; b < NY; ++b) {
                    const int wyz = D >= 3 ? __umul24(uy[b], uz[c]) : (D >= 2 ? uy[b] : 1);
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const int W = D >= 2 ? __umul24(ux[a], wyz) : ux[a];
                        unsigned long long* p = lds + (base + ox[a] + oy[b] + oz[c]);
                        if constexpr (WHICH & 1) atomicAdd(p, (unsigned long long)W);
                        if constexpr (WHICH & 2) {
                            atomicAdd(p + X::DN, (unsigned long long)mul24(W, vq[0]));
                            atomicAdd(p + 2 * X::DN, (unsigned long long)mul24(W, vq[1]));
                            atomicAdd(p + 3 * X::DN, (unsigned long long)mul24(W, vq[2]));
                        }
                    }
                }
            }
            return;
        }
    }
#pragma unroll
    for (int c = 0; c < NZ; ++c) {
#pragma unroll
        for (int b = 0; b < NY; ++b) {
            int wyz = D >= 3 ? __umul24(wy[b], wz[c]) : (D >= 2 ? wy[b] : 1);
#pragma unroll
            for (int a = 0; a < N; ++a) {
                int W = D >= 2 ? __umul24(wx[a], wyz) : wx[a];
                unsigned long long r = (unsigned long long)W;
                unsigned long long gx = (unsigned long long)mul24(W, vq[0]);
                unsigned long long gy = (unsigned long long)mul24(W, vq[1]);
                unsigned long long gz = (unsigned long long)mul24(W, vq[2]);
                if (in_lds) {
                    // planar [moment][node]: lanes at different nodes hit different banks
                    unsigned long long* p = lds + ((lz + c) * X::DY * X::DX + (ly + b) * X::DX + (lx + a));
                    if constexpr (WHICH & 1) atomicAdd(p, r);
                    if constexpr (WHICH & 2) {
                        atomicAdd(p + X::DN, gx);
                        atomicAdd(p + 2 * X::DN, gy);
                        atomicAdd(p + 3 * X::DN, gz);
                    }
                } else {
                    long gi = dep_index(cx + rx + a, D >= 2 ? cy + ry + b : 0, D >= 3 ? cz + rz + c : 0, G);
                    if (gi < 0) { oor = 1; continue; }
                    unsigned long long* p = mom + 4 * gi;
                    if constexpr (WHICH & 1) atomicAdd(p + 0, r);
                    if constexpr (WHICH & 2) {
                        atomicAdd(p + 1, gx);
                        atomicAdd(p + 2, gy);
                        atomicAdd(p + 3, gz);
                    }
                }
            }
        }
    }
}

// Deposit of a particle whose velocity codes are already formed.
template <typename R, int D, int S, int WHICH = 3>
__device__ __forceinline__ void deposit_coded(unsigned long long* lds, int bx0, int by0, int bz0,
                                              unsigned long long* mom, const Geo& G, int cx, int cy, int cz,
                                              const R* o, const int vq[3], int& oor) {
    int wx[3], wy[3] = {1, 0, 0}, wz[3] = {1, 0, 0}, rx, ry = 0, rz = 0;
    weights_int<R, S>(o[0], G.b, rx, wx);
    if constexpr (D >= 2) weights_int<R, S>(o[1], G.b, ry, wy);
    if constexpr (D >= 3) weights_int<R, S>(o[2], G.b, rz, wz);
    deposit_one<D, S, WHICH>(lds, bx0, by0, bz0, mom, G, cx, cy, cz, wx, wy, wz, rx, ry, rz, vq, oor);
}

// Integer weights + velocity codes of a particle and its deposit.  MODE 0:
// non-relativistic (v is the velocity), 1: relativistic (v is u), 2: the
// run's 1/c^2 decides at run time (the kernels off the hot path).
template <typename R, int D, int S, int MODE = 2>
__device__ __forceinline__ int deposit_particle(unsigned long long* lds, int bx0, int by0, int bz0,
                                                unsigned long long* mom, const Geo& G, int cx, int cy,
                                                int cz, const R* o, const R* v, int& oor) {
    int status = 0, vq[3];
    if constexpr (MODE == 2) {
        if (G.ic2 != 0.0) velocity_codes<R, true>(v, G.ic2, G.sv, status, vq);
        else velocity_codes<R, false>(v, 0.0, G.sv, status, vq);
    } else {
        velocity_codes<R, MODE == 1>(v, G.ic2, G.sv, status, vq);
    }
    deposit_coded<R, D, S>(lds, bx0, by0, bz0, mom, G, cx, cy, cz, o, vq, oor);
    return status;
}

// Flush of a tile's LDS accumulators (planar [moment][node]): one global
// 64-bit atomic per non-zero (node, moment), issued node-major so that a
// wave's atomics cover consecutive addresses.  Integer addition makes the
// result independent of order.
template <int D, int S>
__device__ __forceinline__ void flush_tile(const unsigned long long* lds, unsigned long long* mom,
                                           const Geo& G, int bx0, int by0, int bz0, int& oor) {
    using X = Extent<D, S>;
    for (int l = threadIdx.x; l < X::DN * 4; l += blockDim.x) {
        int node = l >> 2, m = l & 3;
        unsigned long long val = lds[m * X::DN + node];
        if (val == 0ull) continue;
        int lx = node % X::DX, ly = (node / X::DX) % X::DY, lz = node / (X::DX * X::DY);
        long gi = dep_index(bx0 + lx, D >= 2 ? by0 + ly : 0, D >= 3 ? bz0 + lz : 0, G);
        if (gi < 0) { oor = 1; continue; }
        atomicAdd(mom + 4 * gi + m, val);
    }
}

// ---------------------------------------------------------------------------
// Continuous deposit (the differentiable variant of the step): real shape
// weights in FP64, R = sum W and G = sum W v per node, FP64 atomics.  The
// moment grids then hold doubles.  As in deposit_one, the LDS-or-global test
// is taken once per particle, and in LDS the CIC corners are visited in an
// order set by the lane bits.
// ---------------------------------------------------------------------------
template <typename R, int D, int S>
__device__ __forceinline__ void deposit_particle_c(double* lds, int bx0, int by0, int bz0, double* mom, const Geo& G,
                                                   int cx, int cy, int cz, const R* o, const R* v, int& oor) {
    using X = Extent<D, S>;
    constexpr int N = Stencil<S>::N;
    constexpr int NY = D >= 2 ? N : 1, NZ = D >= 3 ? N : 1;
    double wx[3], wy[3] = {1, 0, 0}, wz[3] = {1, 0, 0};
    int rx, ry = 0, rz = 0;
    weights_real<double, S>((double)o[0], rx, wx);
    if constexpr (D >= 2) weights_real<double, S>((double)o[1], ry, wy);
    if constexpr (D >= 3) weights_real<double, S>((double)o[2], rz, wz);
    double vd[3] = {(double)v[0], (double)v[1], (double)v[2]};
    if (G.ic2 != 0.0) {   // relativistic mode: v holds u, the flux needs u / gamma
        const double g = sqrt(1.0 + (vd[0] * vd[0] + vd[1] * vd[1] + vd[2] * vd[2]) * G.ic2);
#pragma unroll
        for (int d = 0; d < 3; ++d) vd[d] /= g;
    }
    int lx = cx + rx - bx0, ly = D >= 2 ? cy + ry - by0 : 0, lz = D >= 3 ? cz + rz - bz0 : 0;
    bool in_lds = lds != nullptr && lx >= 0 && lx + N <= X::DX;
    if constexpr (D >= 2) in_lds = in_lds && ly >= 0 && ly + N <= X::DY;
    if constexpr (D >= 3) in_lds = in_lds && lz >= 0 && lz + N <= X::DZ;
    if (in_lds) {
        int f[3] = {0, 0, 0};
        if constexpr (N == 2) {
            const int lane = __lane_id();
            f[0] = lane & 1;
            if constexpr (D >= 2) f[1] = (lane >> 1) & 1;
            if constexpr (D >= 3) f[2] = (lane >> 2) & 1;
            if (f[0]) { const double t = wx[0]; wx[0] = wx[1]; wx[1] = t; }
            if (f[1]) { const double t = wy[0]; wy[0] = wy[1]; wy[1] = t; }
            if (f[2]) { const double t = wz[0]; wz[0] = wz[1]; wz[1] = t; }
        }
        const int sx = f[0] ? -1 : 1, sy = f[1] ? -X::DX : X::DX, sz = f[2] ? -X::DX * X::DY : X::DX * X::DY;
        double* base = lds + (((lz + f[2]) * X::DY + (ly + f[1])) * X::DX + (lx + f[0]));
#pragma unroll
        for (int c = 0; c < NZ; ++c)
#pragma unroll
            for (int b = 0; b < NY; ++b)
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    const double W = wx[a] * wy[b] * wz[c];
                    double* p = base + (a * sx + b * sy + c * sz);
                    atomicAdd(p, W);
                    atomicAdd(p + X::DN, W * vd[0]);
                    atomicAdd(p + 2 * X::DN, W * vd[1]);
                    atomicAdd(p + 3 * X::DN, W * vd[2]);
                }
        return;
    }
#pragma unroll
    for (int c = 0; c < NZ; ++c)
#pragma unroll
        for (int b = 0; b < NY; ++b)
#pragma unroll
            for (int a = 0; a < N; ++a) {
                const double W = wx[a] * wy[b] * wz[c];
                long gi = dep_index(cx + rx + a, D >= 2 ? cy + ry + b : 0, D >= 3 ? cz + rz + c : 0, G);
                if (gi < 0) { oor = 1; continue; }
                double* p = mom + 4 * gi;
                unsafeAtomicAdd(p, W);
                unsafeAtomicAdd(p + 1, W * vd[0]);
                unsafeAtomicAdd(p + 2, W * vd[1]);
                unsafeAtomicAdd(p + 3, W * vd[2]);
            }
}

// Flush of a tile's FP64 accumulators of the continuous deposit, laid out
// and issued as in flush_tile.
template <int D, int S>
__device__ __forceinline__ void flush_tile_c(const double* lds, double* mom, const Geo& G, int bx0, int by0, int bz0,
                                             int& oor) {
    using X = Extent<D, S>;
    for (int l = threadIdx.x; l < X::DN * 4; l += blockDim.x) {
        int node = l >> 2, m = l & 3;
        double val = lds[m * X::DN + node];
        if (val == 0.0) continue;
        int lx = node % X::DX, ly = (node / X::DX) % X::DY, lz = node / (X::DX * X::DY);
        long gi = dep_index(bx0 + lx, D >= 2 ? by0 + ly : 0, D >= 3 ? bz0 + lz : 0, G);
        if (gi < 0) { oor = 1; continue; }
        unsafeAtomicAdd(mom + 4 * gi + m, val);
    }
}

// Wave-aggregated add of a per-lane count to a device counter.
__device__ __forceinline__ void wave_add(unsigned long long* ctr, int v) {
    unsigned long long m = __ballot(v != 0);
    if (m == 0ull) return;
    int s = v;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (__lane_id() == (int)(__ffsll((long long)m) - 1)) atomicAdd(ctr, (unsigned long long)s);
}

// ---------------------------------------------------------------------------
// Split tile bins.  The live ions of tile t in a buffer occupy
// [t*cap, t*cap + lo) (written bottom-up by the tile's own workgroup, which
// counts its stayers in LDS) and [t*cap + cap - hi, t*cap + cap) (filled
// top-down through a global counter by everyone else: ions arriving from a
// neighbour tile, reflected at the wall or injected).  counts[t] = lo,
// counts[ntiles + t] = hi.  lo + hi > cap is an overflow.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long bin_slot(int tile, int64_t cap, int lo, int i) {
    return (long)tile * cap + (i < lo ? i : (long)cap - 1 - (i - lo));
}

// Reserves a top-down slot of tile `dest`; returns -1 when the bin is full.
__device__ __forceinline__ long bin_push_top(int32_t* counts, int ntiles, int dest, int64_t cap) {
    int k = atomicAdd(counts + ntiles + dest, 1);
    return k < cap ? (long)dest * cap + (cap - 1 - k) : -1;
}

template <typename R> struct alignas(2 * sizeof(R)) Pair { R x, y; };

// LDS plan of the fused kernel: the gather stencil as three planar arrays
// of component pairs (Ex,Ey) (Ez,Bx) (By,Bz), then the planar int64 moment
// accumulators of the tile's deposit box, then one stayer counter.
template <typename R, int D, int S> struct PushLds {
    using X = Extent<D, S>;
    static constexpr size_t a16(size_t x) { return (x + 15) / 16 * 16; }
    static constexpr size_t gather = a16(3 * sizeof(Pair<R>) * X::GN);
    static constexpr size_t dep = a16(32 * X::DN);
    static constexpr size_t off_dep = gather, off_misc = gather + dep;
    static constexpr size_t bytes(bool d) { return gather + (d ? dep : 0) + 16; }
    static_assert(off_dep % 16 == 0 && off_misc % 16 == 0, "LDS regions must be aligned");
};

template <typename R, int D> struct Ion {
    int32_t cell;
    R o[3];
    R v[3];
    uint32_t id;
};

template <typename R, int D>
__device__ __forceinline__ void load_ion(const PBuf<R>& in, long src, Ion<R, D>& p) {
    p.cell = in.cell[src];
#pragma unroll
    for (int d = 0; d < 3; ++d) p.o[d] = d < D ? in.off[d][src] : (R)0;
#pragma unroll
    for (int c = 0; c < 3; ++c) p.v[c] = in.v[c][src];
    p.id = in.id[src];
}

template <typename R, int D>
__device__ __forceinline__ void store_ion(const PBuf<R>& out, long dst, const Ion<R, D>& p) {
    out.cell[dst] = p.cell;
#pragma unroll
    for (int d = 0; d < D; ++d) out.off[d][dst] = p.o[d];
#pragma unroll
    for (int c = 0; c < 3; ++c) out.v[c][dst] = p.v[c];
    out.id[dst] = p.id;
}

// ---------------------------------------------------------------------------
// REL selects the relativistic push at compile time: a run-time switch would
// cost the non-relativistic kernel registers (and occupancy) it never uses.
// The fused hot kernel: per tile, gather E/Bbar from LDS, Boris, move, apply
// the open / periodic boundaries, list wall crossers, deposit the moments
// (LDS int64 atomics into the tile's deposit box, one cell of halo; ions
// that moved further go straight to the global grid) and write each ion to
// the bin of its destination tile.
// ---------------------------------------------------------------------------
// Minimum waves per SIMD the push is compiled for (measured): 8 for the FP32
// 1D kernels (their SGPRs would otherwise cap them at 7, i.e. 6 with 8-wave
// workgroups) and the FP32 2D CIC ones (71 VGPRs otherwise), but for the
// recorded one with the continuous deposit, which would spill 28 B there
// and runs 5% faster at the 6 waves its 75 VGPRs give; 6 for the
// relativistic 3D CIC FP32 one (82 VGPRs and 5 waves otherwise) and the 3D
// CIC FP32 ones with the continuous deposit (89-94 VGPRs otherwise: at 6
// they spill 12 B, 44 B recorded, and still run 5% faster than at 4).  The
// others take what their registers give (the non-relativistic 3D CIC ones
// sit at 79-80 VGPRs, where one more register costs a wave per SIMD and 15%
// of the time).
template <typename R, int D, int S, bool REL, bool CONT, bool REC> struct PushWaves {
    static constexpr int value =
        sizeof(R) != 4 ? 1
        : (D == 1 || (D == 2 && S == 1 && !(CONT && REC))) ? 8
        : (D == 3 && S == 1 && (REL || CONT)) ? 6
                                              : 1;
};

// TC: the time-centred coupling, density deposited at the new position and
// flux at the midpoint of the move.  CONT (with DEP, non-relativistic): the
// continuous deposit, FP64 weights into an FP64 box and grid, instead of the
// fixed-point one.  REC: a recorded step (reverse mode),
// which writes where each ion went into rec_dst, keeps each crosser's
// source slot in the crosser list for the wall and, with pk_n > 0, copies
// each input ion as it is read to its packed index pk_toff[tile] + rank
// (the tape's packing of the input state, ions past pk_n dropped).
template <typename R, int D, int S, bool DEP, bool REL, bool TC = false, bool REC = false, bool CONT = false>
__global__ __launch_bounds__(PUSH_THREADS, (PushWaves<R, D, S, REL, CONT, REC>::value)) void k_push(Geo G, PBuf<R> in, PBuf<R> out, const int32_t* __restrict__ cnt_in,
                                              int32_t* __restrict__ cnt_out, int64_t cap,
                                              const R* __restrict__ gather, unsigned long long* __restrict__ mom,
                                              XList xl, unsigned long long* __restrict__ ctr, int policy,
                                              int species, int32_t* __restrict__ rec_dst, PBuf<R> pk,
                                              const int32_t* __restrict__ pk_toff, int64_t pk_n) {
    using X = Extent<D, S>;
    using T = TileShape<D>;
    using L = PushLds<R, D, S>;
    constexpr int LO = Stencil<S>::LO;
    constexpr int N = Stencil<S>::N;
    extern __shared__ __align__(16) unsigned char smem[];
    Pair<R>* sg = reinterpret_cast<Pair<R>*>(smem);
    unsigned long long* sd = reinterpret_cast<unsigned long long*>(smem + L::off_dep);
    static_assert(!CONT || (DEP && !REL && !TC), "the continuous deposit is fused only into the plain push");
    int* s_stay = reinterpret_cast<int*>(smem + (DEP ? L::off_misc : L::off_dep));

    const int tile = xcd_tile(blockIdx.x, G.ntiles);
    const int tx = tile % G.ntx;
    const int ty = D >= 2 ? (tile / G.ntx) % G.nty : 0;
    const int tz = D >= 3 ? tile / (G.ntx * G.nty) : 0;
    const int x0 = tx * T::X, y0 = ty * T::Y, z0 = tz * T::Z;
    const int gx0 = x0 - LO, gy0 = D >= 2 ? y0 - LO : 0, gz0 = D >= 3 ? z0 - LO : 0;
    const int dx0 = x0 - X::HX - LO, dy0 = D >= 2 ? y0 - X::HY - LO : 0, dz0 = D >= 3 ? z0 - X::HZ - LO : 0;

    for (int l = threadIdx.x; l < X::GN; l += blockDim.x) {
        int lx = l % X::GX, ly = (l / X::GX) % X::GY, lz = l / (X::GX * X::GY);
        long gi = gather_index(gx0 + lx, gy0 + ly, gz0 + lz, G);
        const Pair<R>* src = reinterpret_cast<const Pair<R>*>(gather + 6 * gi);
        sg[l] = src[0];
        sg[X::GN + l] = src[1];
        sg[2 * X::GN + l] = src[2];
    }
    if constexpr (DEP)
        for (int l = threadIdx.x; l < X::DN * 4; l += blockDim.x) sd[l] = 0ull;
    if (threadIdx.x == 0) *s_stay = 0;
    __syncthreads();

    const int lo_in = cnt_in[tile], hi_in = cnt_in[G.ntiles + tile];
    int status = (lo_in + hi_in > cap) ? F_TILE : 0;
    const int n = min(lo_in + hi_in, (int)cap);
    const R h = (R)(0.5 * G.dt);
    const R dtdx = (R)G.dtdx;
    const R ic2 = REL ? (R)G.ic2 : (R)0;
    int oor = 0, nesc = 0, nopen = 0;
    const int lane = __lane_id();

    long pk_base = 0;
    if constexpr (REC) pk_base = pk_n > 0 ? (long)pk_toff[tile] : 0;

    Ion<R, D> cur;
    if (n > 0) load_ion<R, D>(in, bin_slot(tile, cap, lo_in, min((int)threadIdx.x, n - 1)), cur);
    for (int i0 = 0; i0 < n; i0 += blockDim.x) {
        const int i = i0 + threadIdx.x;
        const bool valid = i < n;
        if constexpr (REC)
            if (valid && pk_base + i < pk_n) store_ion<R, D>(pk, pk_base + i, cur);
        // prefetch the next ion of this lane while the current one is pushed
        Ion<R, D> nxt;
        const int inext = i + blockDim.x;
        if (i0 + (int)blockDim.x < n) load_ion<R, D>(in, bin_slot(tile, cap, lo_in, min(inext, n - 1)), nxt);

        int cx = cell_x(cur.cell, G), cy = D >= 2 ? cell_y(cur.cell, G) : 0, cz = D >= 3 ? cell_z(cur.cell, G) : 0;
        R o[3] = {cur.o[0], cur.o[1], cur.o[2]};
        R v[3] = {cur.v[0], cur.v[1], cur.v[2]};

        // gather E^n, Bbar^n from the staged stencil; a binned ion always
        // lies in its tile, the clamp only guards against a corrupt state
        R wx[3], wy[3] = {1, 0, 0}, wz[3] = {1, 0, 0};
        int rx, ry = 0, rz = 0;
        weights_real<R, S>(o[0], rx, wx);
        if constexpr (D >= 2) weights_real<R, S>(o[1], ry, wy);
        if constexpr (D >= 3) weights_real<R, S>(o[2], rz, wz);
        const bool inside = (unsigned)(cx - x0) < (unsigned)T::X && (D < 2 || (unsigned)(cy - y0) < (unsigned)T::Y) &&
                            (D < 3 || (unsigned)(cz - z0) < (unsigned)T::Z);
        if (valid && !inside) oor = 1;
        const int lx = min(max(cx - gx0 + rx, 0), X::GX - N);
        const int ly = D >= 2 ? min(max(cy - gy0 + ry, 0), X::GY - N) : 0;
        const int lz = D >= 3 ? min(max(cz - gz0 + rz, 0), X::GZ - N) : 0;
        R E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
        constexpr int NY = D >= 2 ? N : 1, NZ = D >= 3 ? N : 1;
#pragma unroll
        for (int c = 0; c < NZ; ++c)
#pragma unroll
            for (int b = 0; b < NY; ++b) {
                R wyz = wy[b] * wz[c];
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    R W = wx[a] * wyz;
                    const int l = ((lz + c) * X::GY + (ly + b)) * X::GX + (lx + a);
                    const Pair<R> p0 = sg[l], p1 = sg[X::GN + l], p2 = sg[2 * X::GN + l];
                    E[0] += W * p0.x; E[1] += W * p0.y; E[2] += W * p1.x;
                    B[0] += W * p1.y; B[1] += W * p2.x; B[2] += W * p2.y;
                }
            }
        boris<R, REL>(v, E, B, h, ic2);

        // move in cell units (no CFL assumption) with the velocity (u / gamma
        // in relativistic mode, 1 / gamma kept for the deposit codes)
        R vel[3] = {v[0], v[1], v[2]};
        double ig = 1.0;
        if constexpr (REL) {
            ig = inv_gamma_u<R>(v, G.ic2);
#pragma unroll
            for (int d = 0; d < 3; ++d) vel[d] = v[d] * (R)ig;
        }
        int nc[3] = {cx, cy, cz};
        // time-centred coupling: the midpoint of the move, where the flux goes
        int hc[3] = {cx, cy, cz};
        R ho[3] = {o[0], o[1], o[2]};
        if constexpr (TC) {
            const R hdtdx = (R)(0.5 * G.dtdx);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                R xh = o[d] + vel[d] * hdtdx;
                R fh = floor(xh);
                hc[d] += (int)fh;
                ho[d] = xh - fh;
                if (ho[d] >= (R)1) { ho[d] = (R)0; hc[d] += 1; }
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            R xi = o[d] + vel[d] * dtdx;
            R fl = floor(xi);
            nc[d] += (int)fl;
            o[d] = xi - fl;
            if (o[d] >= (R)1) { o[d] = (R)0; nc[d] += 1; }
        }

        // boundaries: 0 keep, 1 wall crosser, 2 escaped (x < 0), 3 open wall
        int kind = 0;
        int wxc = nc[0];
        if (G.xbc == 1) wxc = wrapi(nc[0], G.nx);
        else if (nc[0] >= G.nx) kind = policy == 0 ? 3 : 1;
        else if (nc[0] < 0) kind = 2;
        const int wyc = D >= 2 ? wrapi(nc[1], G.nyc) : 0;
        const int wzc = D >= 3 ? wrapi(nc[2], G.nzc) : 0;
        if (!valid) kind = 4;

        if (kind == 1) {
            int slot = atomicAdd(xl.count, 1);
            if (slot < xl.cap) {
                xl.id[slot] = cur.id;
                if constexpr (REC) xl.src[slot] = (int32_t)bin_slot(tile, cap, lo_in, i);
                xl.delta[slot] = (double)(nc[0] - G.nx) + (double)o[0];
                xl.cy[slot] = wyc;
                xl.cz[slot] = wzc;
                xl.oy[slot] = (double)o[1];
                xl.oz[slot] = (double)o[2];
                xl.v[slot] = (double)v[0];
                xl.v[xl.cap + slot] = (double)v[1];
                xl.v[2 * xl.cap + slot] = (double)v[2];
            } else {
                status |= F_XLIST;
            }
        }
        nesc += kind == 2;
        nopen += kind == 3;

        if constexpr (DEP) {
            if (kind == 0) {
                if constexpr (CONT) {
                    deposit_particle_c<R, D, S>(reinterpret_cast<double*>(sd), dx0, dy0, dz0,
                                                reinterpret_cast<double*>(mom), G, nc[0], nc[1], nc[2], o, v, oor);
                } else if constexpr (TC) {
                    int vq[3];
                    if constexpr (REL) velocity_codes_ig<R>(v, ig, G.sv, status, vq);
                    else velocity_codes<R, false>(v, 0.0, G.sv, status, vq);
                    deposit_coded<R, D, S, 1>(sd, dx0, dy0, dz0, mom, G, nc[0], nc[1], nc[2], o, vq, oor);
                    deposit_coded<R, D, S, 2>(sd, dx0, dy0, dz0, mom, G, hc[0], hc[1], hc[2], ho, vq, oor);
                } else if constexpr (REL) {
                    int vq[3];
                    velocity_codes_ig<R>(v, ig, G.sv, status, vq);
                    deposit_coded<R, D, S>(sd, dx0, dy0, dz0, mom, G, nc[0], nc[1], nc[2], o, vq, oor);
                } else {
                    status |= deposit_particle<R, D, S, 0>(sd, dx0, dy0, dz0, mom, G, nc[0], nc[1], nc[2], o, v, oor);
                }
            }
        }

        // write to the destination tile's bin: stayers bottom-up through one
        // LDS counter per wave, others top-down through the global counter
        const int dest = kind == 0 ? tile_of<D>(wxc, wyc, wzc, G) : -1;
        const bool stay = dest == tile;
        const unsigned long long sm = __ballot(stay);
        long dst = -1;
        if (sm) {
            int leader = (int)__ffsll((long long)sm) - 1;
            int s0 = 0;
            if (lane == leader) s0 = atomicAdd(s_stay, (int)__popcll(sm));
            s0 = __shfl(s0, leader);
            if (stay) {
                int slot = s0 + (int)__popcll(sm & ((1ull << lane) - 1ull));
                dst = slot < cap ? (long)tile * cap + slot : -1;
            }
        }
        if (kind == 0 && !stay) dst = bin_push_top(cnt_out, G.ntiles, dest, cap);
        // step record: where each ion went (the wall fills in its reflections)
        if constexpr (REC)
            if (valid) rec_dst[bin_slot(tile, cap, lo_in, i)] = (kind == 0 && dst >= 0) ? (int32_t)dst : -1;
        if (kind == 0) {
            if (dst >= 0) {
                out.cell[dst] = pack_cell(wxc, wyc, wzc, G);
#pragma unroll
                for (int d = 0; d < D; ++d) out.off[d][dst] = o[d];
#pragma unroll
                for (int c = 0; c < 3; ++c) out.v[c][dst] = v[c];
                out.id[dst] = cur.id;
            } else {
                status |= F_TILE;
            }
        }
        cur = nxt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int ns = *s_stay;
        cnt_out[tile] = min(ns, (int)cap);
        if (ns > cap) status |= F_TILE;
    }
    if constexpr (DEP && CONT)
        flush_tile_c<D, S>(reinterpret_cast<const double*>(sd), reinterpret_cast<double*>(mom), G, dx0, dy0, dz0, oor);
    else if constexpr (DEP) flush_tile<D, S>(sd, mom, G, dx0, dy0, dz0, oor);
    wave_add(ctr + C_ESC, nesc);
    wave_add(ctr + C_OPEN, nopen);
    wave_add(ctr + (species == 0 ? C_REM0 : C_REM1), nesc + nopen);
    wave_add(ctr + C_SAT, (status & F_SAT) ? 1 : 0);
    wave_add(ctr + C_OOR, oor);
    if (status) atomicOr(reinterpret_cast<unsigned int*>(ctr + C_FLAGS), (unsigned int)status);
}

// Overflow check of every bin after all writers of a step.
__global__ void k_check_bins(const int32_t* counts, int ntiles, int64_t cap, unsigned long long* ctr) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntiles && (long)counts[t] + counts[ntiles + t] > cap)
        atomicOr(reinterpret_cast<unsigned int*>(ctr + C_FLAGS), (unsigned int)F_TILE);
}

// ---------------------------------------------------------------------------
// Faux-shock wall on the crosser list of one species (or SPECULAR mirror),
// with eq. (1) or, when wm.on, the prescribed wall.
// Reflected ions are binned into their new tile and deposited directly
// (CONT: the continuous deposit into an FP64 grid).
// ---------------------------------------------------------------------------
template <typename R, int D, int S, bool DEP, bool CONT = false>
__global__ __launch_bounds__(256) void k_wall(Geo G, XList xl, PBuf<R> out, int32_t* cnt_out, int64_t cap,
                                              unsigned long long* mom, unsigned long long* ctr,
                                              int policy, int species, uint64_t step, int32_t* rec_dst,
                                              WallModel wm) {
    int ncross = *xl.count;
    if (ncross > xl.cap) ncross = (int)xl.cap;
    int status = 0, oor = 0;
    int n_inc = 0, n_trans = 0, n_refl = 0, n_esc = 0;   // summed per wave at the end
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncross; i += gridDim.x * blockDim.x) {
        uint32_t pid = xl.id[i];
        double v[3] = {xl.v[i], xl.v[xl.cap + i], xl.v[2 * xl.cap + i]};
        double vout[3], back = 0.0;
        int refl;
        if (policy == 1) {
            refl = wm.on ? faux_shock_event_prescribed(wm, G.seed, step, pid, G.c_light, xl.delta[i], v, vout, back)
                         : faux_shock_event(G.seed, step, pid, G.u2, G.c_light, xl.delta[i], v, vout, back);
        } else {
            vout[0] = -v[0]; vout[1] = v[1]; vout[2] = v[2];
            back = xl.delta[i];
            refl = 1;
        }
        ++n_inc;
        if (!refl) {
            ++n_trans;
            continue;
        }
        ++n_refl;
        double xi = (double)G.nx - back;
        double fl = floor(xi);
        int cx = (int)fl;
        double ox = xi - fl;
        if (cx >= G.nx) { cx = G.nx - 1; ox = 1.0; }
        if (cx < 0) {
            ++n_esc;
            continue;
        }
        R o[3] = {to_offset<R>(ox), (R)xl.oy[i], (R)xl.oz[i]};
        R vr[3] = {(R)vout[0], (R)vout[1], (R)vout[2]};
        int cy = xl.cy[i], cz = xl.cz[i];
        int dest = tile_of<D>(cx, cy, cz, G);
        long dst = bin_push_top(cnt_out, G.ntiles, dest, cap);
        if (dst < 0) { status |= F_TILE; continue; }
        out.cell[dst] = pack_cell(cx, cy, cz, G);
#pragma unroll
        for (int d = 0; d < D; ++d) out.off[d][dst] = o[d];
#pragma unroll
        for (int c = 0; c < 3; ++c) out.v[c][dst] = vr[c];
        out.id[dst] = pid;
        if (rec_dst != nullptr) rec_dst[xl.src[i]] = (int32_t)(-2 - dst);   // step record: reflected into dst
        if constexpr (DEP && CONT)
            deposit_particle_c<R, D, S>(nullptr, 0, 0, 0, reinterpret_cast<double*>(mom), G, cx, cy, cz, o, vr, oor);
        else if constexpr (DEP) status |= deposit_particle<R, D, S>(nullptr, 0, 0, 0, mom, G, cx, cy, cz, o, vr, oor);
    }
    wave_add(ctr + C_INC, n_inc);
    wave_add(ctr + C_TRANS, n_trans);
    wave_add(ctr + C_REFL, n_refl);
    wave_add(ctr + C_ESC, n_esc);
    wave_add(ctr + (species == 0 ? C_REM0 : C_REM1), n_trans + n_esc);
    if (status & F_SAT) atomicAdd(ctr + C_SAT, 1ull);
    if (oor) atomicAdd(ctr + C_OOR, 1ull);
    if (status) atomicOr(reinterpret_cast<unsigned int*>(ctr + C_FLAGS), (unsigned int)status);
}

// ---------------------------------------------------------------------------
// Injection: thermal ions at x = 0 (drifting Maxwellian) and CRs at x = L
// (isotropic in the downstream frame, flux weighted), with deterministic
// counts and ids handed out by the host (CONT: deposited continuously).
// ---------------------------------------------------------------------------
template <typename R, int D, int S, bool DEP, bool CONT = false>
__global__ __launch_bounds__(256) void k_inject(Geo G, PBuf<R> out0, int32_t* cnt0, int64_t cap0, unsigned long long* mom0,
                                                PBuf<R> out1, int32_t* cnt1, int64_t cap1, unsigned long long* mom1,
                                                unsigned long long* ctr, uint64_t step, int64_t id0,
                                                int64_t cnt_th, int64_t cnt_cr, int64_t ntr) {
    const int64_t nth = cnt_th * ntr, ncr = cnt_cr * ntr;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // per-wave totals of the step counters (one atomic per wave, not per ion)
    const int is_th = g < nth, is_cr = g >= nth && g < nth + ncr;
    wave_add(ctr + C_ADD0, is_th);
    wave_add(ctr + C_INJ_TH, is_th);
    wave_add(ctr + C_ADD1, is_cr);
    wave_add(ctr + C_INJ_CR, is_cr);
    if (g >= nth + ncr) return;
    int status = 0, oor = 0;
    const bool cr = g >= nth;
    const int64_t k = cr ? g - nth : g;
    const int64_t per = cr ? cnt_cr : cnt_th;
    const int64_t t = k / per;
    const uint64_t id = (uint64_t)(id0 + g);
    double U[4], V[4], vv[3], xi;
    if (!cr) {
        draw4(G.seed, kStreamInjectTh, step, id, 0, U);
        draw4(G.seed, kStreamInjectTh, step, id, 1, V);
        double n1, n2, n3, n4;
        box_muller(V[0], V[1], n1, n2);
        box_muller(V[2], V[3], n3, n4);
        vv[0] = fabs(G.u_sh + G.sigma * n1);
        vv[1] = G.sigma * n2;
        vv[2] = G.sigma * n3;
        xi = vv[0] * U[0] * G.dt / G.dx;
        if (G.c_light > 0.0) {   // relativistic mode: store the four-velocity
            const double cc = G.c_light * G.c_light;
            const double g = 1.0 / sqrt(1.0 - (vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]) / cc);
#pragma unroll
            for (int c = 0; c < 3; ++c) vv[c] *= g;
        }
    } else {
        draw4(G.seed, kStreamInjectCr, step, id, 0, U);
        draw4(G.seed, kStreamInjectCr, step, id, 1, V);
        double a = G.u2 / G.cr_w;
        double mu = a + (1.0 - a) * sqrt(U[2]);
        double st = sqrt(fmax(0.0, 1.0 - mu * mu));
        double phi = kTwoPi * U[3];
        vv[0] = G.u2 - G.cr_w * mu;
        vv[1] = G.cr_w * st * cos(phi);
        vv[2] = G.cr_w * st * sin(phi);
        double vx = vv[0];
        if (G.c_light > 0.0) {
            // relativistic mode: four-velocity of speed cr_w in the downstream
            // frame, boosted to the lab along x
            const double cc = G.c_light * G.c_light;
            const double g2 = 1.0 / sqrt(1.0 - (G.u2 * G.u2) / cc);
            const double Gw = 1.0 / sqrt(1.0 - (G.cr_w * G.cr_w) / cc);
            const double Wabs = Gw * G.cr_w, Wx = -Wabs * mu;
            vv[0] = g2 * (Wx + G.u2 * Gw);
            vv[1] = Wabs * st * cos(phi);
            vv[2] = Wabs * st * sin(phi);
            vx = vv[0] / (g2 * (Gw + G.u2 * Wx / cc));
        }
        xi = (double)G.nx - fabs(vx) * U[0] * G.dt / G.dx;
    }
    double fl = floor(xi);
    int cx = (int)fl;
    double ox = xi - fl;
    if (cx >= G.nx) { cx = G.nx - 1; ox = 1.0; }
    if (cx < 0) { cx = 0; ox = 0.0; }
    int cy = D >= 2 ? (int)(t % G.nyc) : 0;
    int cz = D >= 3 ? (int)(t / G.nyc) : 0;
    R o[3] = {to_offset<R>(ox), D >= 2 ? to_offset<R>(U[1]) : (R)0,
              D >= 3 ? to_offset<R>(cr ? V[0] : U[2]) : (R)0};
    R vr[3] = {(R)vv[0], (R)vv[1], (R)vv[2]};
    PBuf<R> out = cr ? out1 : out0;
    int32_t* cnt = cr ? cnt1 : cnt0;
    int64_t cap = cr ? cap1 : cap0;
    unsigned long long* mom = cr ? mom1 : mom0;
    int dest = tile_of<D>(cx, cy, cz, G);
    long dst = bin_push_top(cnt, G.ntiles, dest, cap);
    if (dst < 0) {
        atomicOr(reinterpret_cast<unsigned int*>(ctr + C_FLAGS), (unsigned int)F_TILE);
        return;
    }
    out.cell[dst] = pack_cell(cx, cy, cz, G);
#pragma unroll
    for (int d = 0; d < D; ++d) out.off[d][dst] = o[d];
#pragma unroll
    for (int c = 0; c < 3; ++c) out.v[c][dst] = vr[c];
    out.id[dst] = (uint32_t)id;
    if constexpr (DEP && CONT)
        deposit_particle_c<R, D, S>(nullptr, 0, 0, 0, reinterpret_cast<double*>(mom), G, cx, cy, cz, o, vr, oor);
    else if constexpr (DEP) status |= deposit_particle<R, D, S>(nullptr, 0, 0, 0, mom, G, cx, cy, cz, o, vr, oor);
    if (status & F_SAT) atomicAdd(ctr + C_SAT, 1ull);
    if (oor) atomicAdd(ctr + C_OOR, 1ull);
    if (status) atomicOr(reinterpret_cast<unsigned int*>(ctr + C_FLAGS), (unsigned int)status);
}

template <typename R, int D, int S>
__global__ __launch_bounds__(256) void k_deposit_c(Geo G, PBuf<R> in, const int32_t* __restrict__ cnt, int64_t cap,
                                                   double* __restrict__ mom, unsigned long long* __restrict__ ctr,
                                                   int split) {
    using X = Extent<D, S>;
    using T = TileShape<D>;
    constexpr int LO = Stencil<S>::LO;
    extern __shared__ __align__(16) unsigned char smem[];
    double* sd = reinterpret_cast<double*>(smem);
    // a tile's ions may be spread over `split` consecutive workgroups
    const int tile = blockIdx.x / split, part = blockIdx.x % split;
    const int tx = tile % G.ntx;
    const int ty = D >= 2 ? (tile / G.ntx) % G.nty : 0;
    const int tz = D >= 3 ? tile / (G.ntx * G.nty) : 0;
    const int dx0 = tx * T::X - X::HX - LO, dy0 = D >= 2 ? ty * T::Y - X::HY - LO : 0, dz0 = D >= 3 ? tz * T::Z - X::HZ - LO : 0;
    for (int l = threadIdx.x; l < X::DN * 4; l += blockDim.x) sd[l] = 0.0;
    __syncthreads();
    const int lo = cnt[tile];
    const int n = min(lo + cnt[G.ntiles + tile], (int)cap);
    const int chunk = (n + split - 1) / split, i0 = min(n, part * chunk), i1 = min(n, i0 + chunk);
    int oor = 0;
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        long src = bin_slot(tile, cap, lo, i);
        int32_t pc = in.cell[src];
        R o[3] = {0, 0, 0}, v[3];
#pragma unroll
        for (int d = 0; d < D; ++d) o[d] = in.off[d][src];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = in.v[c][src];
        deposit_particle_c<R, D, S>(sd, dx0, dy0, dz0, mom, G, cell_x(pc, G), D >= 2 ? cell_y(pc, G) : 0,
                                    D >= 3 ? cell_z(pc, G) : 0, o, v, oor);
    }
    __syncthreads();
    flush_tile_c<D, S>(sd, mom, G, dx0, dy0, dz0, oor);
    if (oor) atomicAdd(ctr + C_OOR, 1ull);
}

// Standalone deposit of the live particles of every tile.
template <typename R, int D, int S>
__global__ __launch_bounds__(256) void k_deposit(Geo G, PBuf<R> in, const int32_t* __restrict__ cnt, int64_t cap,
                                                 unsigned long long* __restrict__ mom,
                                                 unsigned long long* __restrict__ ctr) {
    using X = Extent<D, S>;
    using T = TileShape<D>;
    constexpr int LO = Stencil<S>::LO;
    extern __shared__ __align__(16) unsigned char smem[];
    unsigned long long* sd = reinterpret_cast<unsigned long long*>(smem);
    const int tile = xcd_tile(blockIdx.x, G.ntiles);
    const int tx = tile % G.ntx;
    const int ty = D >= 2 ? (tile / G.ntx) % G.nty : 0;
    const int tz = D >= 3 ? tile / (G.ntx * G.nty) : 0;
    const int dx0 = tx * T::X - X::HX - LO, dy0 = D >= 2 ? ty * T::Y - X::HY - LO : 0, dz0 = D >= 3 ? tz * T::Z - X::HZ - LO : 0;
    for (int l = threadIdx.x; l < X::DN * 4; l += blockDim.x) sd[l] = 0ull;
    __syncthreads();
    const int lo = cnt[tile];
    const int n = min(lo + cnt[G.ntiles + tile], (int)cap);
    int status = 0, oor = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        long src = bin_slot(tile, cap, lo, i);
        int32_t pc = in.cell[src];
        R o[3] = {0, 0, 0}, v[3];
#pragma unroll
        for (int d = 0; d < D; ++d) o[d] = in.off[d][src];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = in.v[c][src];
        status |= deposit_particle<R, D, S>(sd, dx0, dy0, dz0, mom, G, cell_x(pc, G),
                                            D >= 2 ? cell_y(pc, G) : 0, D >= 3 ? cell_z(pc, G) : 0, o, v, oor);
    }
    __syncthreads();
    flush_tile<D, S>(sd, mom, G, dx0, dy0, dz0, oor);
    if (status & F_SAT) atomicAdd(ctr + C_SAT, 1ull);
    if (oor) atomicAdd(ctr + C_OOR, 1ull);
    if (status) atomicOr(reinterpret_cast<unsigned int*>(ctr + C_FLAGS), (unsigned int)status);
}

}  // namespace fsk
