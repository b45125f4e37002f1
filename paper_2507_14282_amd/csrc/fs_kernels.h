// fs_kernels.h -- gfx950 kernels of the faux-shock hybrid step.
//
// Data layout in HBM
//  * particles of one species: structure of arrays in fixed-capacity tile
//    bins (slots [t*cap, t*cap + count[t]) of tile t), ping-ponged between two
//    buffers every step.  Each tile is read once, contiguously, by one
//    workgroup and written back binned by destination tile, so the particle
//    state streams through HBM exactly once per step.
//  * gather grid: per field node 8 reals (E, 0, Bbar, 0) = two 16-byte (FP32)
//    vectors, staged per tile in LDS.
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
    double dt, dx, u_sh, u2, sigma, cr_w, dtdx;
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

template <int D> __device__ __forceinline__ int tile_of(int x, int y, int z, const Geo& G) {
    using T = TileShape<D>;
    int t = x / T::X;
    if constexpr (D >= 2) t += G.ntx * (y / T::Y);
    if constexpr (D >= 3) t += G.ntx * G.nty * (z / T::Z);
    return t;
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
    return (long)i + (long)G.ndx * ((long)j + (long)G.nyc * k);
}

// Field-node index for a gather: x clamped to the physical nodes in the box,
// wrapped when periodic; y, z wrapped.
__device__ __forceinline__ long gather_index(int i, int j, int k, const Geo& G) {
    if (G.xbc == 1) i = wrapi(i, G.nx);
    else { i = i < 0 ? 0 : i; i = i > G.nx ? G.nx : i; }
    j = wrapi(j, G.nyc);
    k = wrapi(k, G.nzc);
    return (long)i + (long)G.nxn * ((long)j + (long)G.nyc * k);
}

// Adds one particle's fixed-point moments at (unwrapped) cell (cx, cy, cz)
// with integer weights wx/wy/wz starting at the stencil offsets rx/ry/rz.
// Into LDS when the whole stencil lies in the tile's deposit box, otherwise
// straight into the global grid.
template <int D, int S>
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
                    unsigned long long* p = lds + 4 * ((lz + c) * X::DY * X::DX + (ly + b) * X::DX + (lx + a));
                    atomicAdd(p + 0, r);
                    atomicAdd(p + 1, gx);
                    atomicAdd(p + 2, gy);
                    atomicAdd(p + 3, gz);
                } else {
                    long gi = dep_index(cx + rx + a, D >= 2 ? cy + ry + b : 0, D >= 3 ? cz + rz + c : 0, G);
                    if (gi < 0) { oor = 1; continue; }
                    unsigned long long* p = mom + 4 * gi;
                    atomicAdd(p + 0, r);
                    atomicAdd(p + 1, gx);
                    atomicAdd(p + 2, gy);
                    atomicAdd(p + 3, gz);
                }
            }
        }
    }
}

// Integer weights + velocity codes of a particle and its deposit.
template <typename R, int D, int S>
__device__ __forceinline__ int deposit_particle(unsigned long long* lds, int bx0, int by0, int bz0,
                                                unsigned long long* mom, const Geo& G, int cx, int cy,
                                                int cz, const R* o, const R* v, int& oor) {
    int wx[3], wy[3] = {1, 0, 0}, wz[3] = {1, 0, 0}, rx, ry = 0, rz = 0;
    weights_int<R, S>(o[0], G.b, rx, wx);
    if constexpr (D >= 2) weights_int<R, S>(o[1], G.b, ry, wy);
    if constexpr (D >= 3) weights_int<R, S>(o[2], G.b, rz, wz);
    int status = 0, vq[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) vq[d] = vcode<R>(v[d], G.sv, status);
    deposit_one<D, S>(lds, bx0, by0, bz0, mom, G, cx, cy, cz, wx, wy, wz, rx, ry, rz, vq, oor);
    return status;
}

// Flush of a tile's LDS accumulators: one global 64-bit atomic per non-zero
// (node, moment).  Integer addition makes the result independent of order.
template <int D, int S>
__device__ __forceinline__ void flush_tile(const unsigned long long* lds, unsigned long long* mom,
                                           const Geo& G, int bx0, int by0, int bz0, int& oor) {
    using X = Extent<D, S>;
    for (int l = threadIdx.x; l < X::DN * 4; l += blockDim.x) {
        unsigned long long val = lds[l];
        if (val == 0ull) continue;
        int node = l >> 2, m = l & 3;
        int lx = node % X::DX, ly = (node / X::DX) % X::DY, lz = node / (X::DX * X::DY);
        long gi = dep_index(bx0 + lx, D >= 2 ? by0 + ly : 0, D >= 3 ? bz0 + lz : 0, G);
        if (gi < 0) { oor = 1; continue; }
        atomicAdd(mom + 4 * gi + m, val);
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
// The fused hot kernel: per tile, gather E/Bbar from LDS, Boris, move, apply
// the open / periodic boundaries, list wall crossers, deposit the moments in
// LDS and write each ion to the bin of its destination tile.
// ---------------------------------------------------------------------------
template <typename R, int D, int S, bool DEP>
__global__ __launch_bounds__(256) void k_push(Geo G, PBuf<R> in, PBuf<R> out, const int32_t* __restrict__ cnt_in,
                                              int32_t* __restrict__ cnt_out, int64_t cap,
                                              const R* __restrict__ gather, unsigned long long* __restrict__ mom,
                                              XList xl, unsigned long long* __restrict__ ctr, int policy,
                                              int species) {
    using X = Extent<D, S>;
    using T = TileShape<D>;
    constexpr int LO = Stencil<S>::LO;
    constexpr int N = Stencil<S>::N;
    extern __shared__ __align__(16) unsigned char smem[];
    R* sg = reinterpret_cast<R*>(smem);
    unsigned long long* sd = reinterpret_cast<unsigned long long*>(smem + sizeof(R) * 8 * X::GN);

    const int tile = xcd_tile(blockIdx.x, G.ntiles);
    const int tx = tile % G.ntx;
    const int ty = D >= 2 ? (tile / G.ntx) % G.nty : 0;
    const int tz = D >= 3 ? tile / (G.ntx * G.nty) : 0;
    const int x0 = tx * T::X, y0 = ty * T::Y, z0 = tz * T::Z;
    const int gx0 = x0 - LO, gy0 = D >= 2 ? y0 - LO : 0, gz0 = D >= 3 ? z0 - LO : 0;
    const int dx0 = x0 - 1 - LO, dy0 = D >= 2 ? y0 - 1 - LO : 0, dz0 = D >= 3 ? z0 - 1 - LO : 0;

    // stage the gather stencil of the tile
    for (int l = threadIdx.x; l < X::GN; l += blockDim.x) {
        int lx = l % X::GX, ly = (l / X::GX) % X::GY, lz = l / (X::GX * X::GY);
        long gi = gather_index(gx0 + lx, gy0 + ly, gz0 + lz, G);
        const R* src = gather + 8 * gi;
        R* dst = sg + 8 * l;
#pragma unroll
        for (int q = 0; q < 8; ++q) dst[q] = src[q];
    }
    if constexpr (DEP)
        for (int l = threadIdx.x; l < X::DN * 4; l += blockDim.x) sd[l] = 0ull;
    __syncthreads();

    const int n = min(cnt_in[tile], (int)cap);
    const long base = (long)tile * cap;
    const R h = (R)(0.5 * G.dt);
    const R dtdx = (R)G.dtdx;
    int oor = 0, status = 0;
    const int lane = __lane_id();

    for (int i0 = 0; i0 < n; i0 += blockDim.x) {
        const int i = i0 + threadIdx.x;
        const bool valid = i < n;
        const long src = base + (valid ? i : 0);
        int32_t pc = in.cell[src];
        R o[3] = {0, 0, 0}, v[3];
#pragma unroll
        for (int d = 0; d < D; ++d) o[d] = in.off[d][src];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = in.v[c][src];
        uint32_t pid = in.id[src];
        int cx = cell_x(pc, G), cy = D >= 2 ? cell_y(pc, G) : 0, cz = D >= 3 ? cell_z(pc, G) : 0;

        // gather E^n, Bbar^n from the staged stencil
        R wx[3], wy[3] = {1, 0, 0}, wz[3] = {1, 0, 0};
        int rx, ry = 0, rz = 0;
        weights_real<R, S>(o[0], rx, wx);
        if constexpr (D >= 2) weights_real<R, S>(o[1], ry, wy);
        if constexpr (D >= 3) weights_real<R, S>(o[2], rz, wz);
        // a binned ion always lies in its tile; clamp so that a corrupt state
        // can never index outside the staged stencil
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
                    const R* s = sg + 8 * (((lz + c) * X::GY + (ly + b)) * X::GX + (lx + a));
                    E[0] += W * s[0]; E[1] += W * s[1]; E[2] += W * s[2];
                    B[0] += W * s[4]; B[1] += W * s[5]; B[2] += W * s[6];
                }
            }
        boris<R>(v, E, B, h);

        // move in cell units (no CFL assumption)
        int nc[3] = {cx, cy, cz};
#pragma unroll
        for (int d = 0; d < D; ++d) {
            R xi = o[d] + v[d] * dtdx;
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
        int wyc = D >= 2 ? wrapi(nc[1], G.nyc) : 0;
        int wzc = D >= 3 ? wrapi(nc[2], G.nzc) : 0;
        if (!valid) kind = 4;

        if (kind == 1) {
            int slot = atomicAdd(xl.count, 1);
            if (slot < xl.cap) {
                xl.id[slot] = pid;
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
        wave_add(ctr + C_ESC, kind == 2);
        wave_add(ctr + C_OPEN, kind == 3);
        wave_add(ctr + (species == 0 ? C_REM0 : C_REM1), kind == 2 || kind == 3);

        if constexpr (DEP) {
            if (kind == 0)
                status |= deposit_particle<R, D, S>(sd, dx0, dy0, dz0, mom, G, nc[0], nc[1], nc[2], o, v, oor);
        }

        // write to the destination tile's bin; ions staying in this tile get
        // one wave-aggregated slot reservation
        const int dest = kind == 0 ? tile_of<D>(wxc, wyc, wzc, G) : -1;
        const bool stay = dest == tile;
        const unsigned long long sm = __ballot(stay);
        int slot = -1;
        if (sm) {
            int leader = (int)__ffsll((long long)sm) - 1;
            int s0 = 0;
            if (lane == leader) s0 = atomicAdd(cnt_out + tile, (int)__popcll(sm));
            s0 = __shfl(s0, leader);
            if (stay) slot = s0 + (int)__popcll(sm & ((1ull << lane) - 1ull));
        }
        if (kind == 0 && !stay) slot = atomicAdd(cnt_out + dest, 1);
        if (kind == 0) {
            if (slot < cap) {
                long dst = (long)dest * cap + slot;
                out.cell[dst] = pack_cell(wxc, wyc, wzc, G);
#pragma unroll
                for (int d = 0; d < D; ++d) out.off[d][dst] = o[d];
#pragma unroll
                for (int c = 0; c < 3; ++c) out.v[c][dst] = v[c];
                out.id[dst] = pid;
            } else {
                status |= F_TILE;
            }
        }
    }
    if constexpr (DEP) {
        __syncthreads();
        flush_tile<D, S>(sd, mom, G, dx0, dy0, dz0, oor);
    }
    wave_add(ctr + C_SAT, (status & F_SAT) ? 1 : 0);
    wave_add(ctr + C_OOR, oor);
    if (status) atomicOr(reinterpret_cast<unsigned int*>(ctr + C_FLAGS), (unsigned int)status);
}

// ---------------------------------------------------------------------------
// Faux-shock wall on the crosser list of one species (or SPECULAR mirror).
// Reflected ions are binned into their new tile and deposited directly.
// ---------------------------------------------------------------------------
template <typename R, int D, int S, bool DEP>
__global__ __launch_bounds__(256) void k_wall(Geo G, XList xl, PBuf<R> out, int32_t* cnt_out, int64_t cap,
                                              unsigned long long* mom, unsigned long long* ctr,
                                              int policy, int species, uint64_t step) {
    int ncross = *xl.count;
    if (ncross > xl.cap) ncross = (int)xl.cap;
    int status = 0, oor = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ncross; i += gridDim.x * blockDim.x) {
        uint32_t pid = xl.id[i];
        double v[3] = {xl.v[i], xl.v[xl.cap + i], xl.v[2 * xl.cap + i]};
        double vout[3], back = 0.0;
        int refl;
        if (policy == 1) {
            refl = faux_shock_event(G.seed, step, pid, G.u2, xl.delta[i], v, vout, back);
        } else {
            vout[0] = -v[0]; vout[1] = v[1]; vout[2] = v[2];
            back = xl.delta[i];
            refl = 1;
        }
        atomicAdd(ctr + C_INC, 1ull);
        if (!refl) {
            atomicAdd(ctr + C_TRANS, 1ull);
            atomicAdd(ctr + (species == 0 ? C_REM0 : C_REM1), 1ull);
            continue;
        }
        atomicAdd(ctr + C_REFL, 1ull);
        double xi = (double)G.nx - back;
        double fl = floor(xi);
        int cx = (int)fl;
        double ox = xi - fl;
        if (cx >= G.nx) { cx = G.nx - 1; ox = 1.0; }
        if (cx < 0) {
            atomicAdd(ctr + C_ESC, 1ull);
            atomicAdd(ctr + (species == 0 ? C_REM0 : C_REM1), 1ull);
            continue;
        }
        R o[3] = {to_offset<R>(ox), (R)xl.oy[i], (R)xl.oz[i]};
        R vr[3] = {(R)vout[0], (R)vout[1], (R)vout[2]};
        int cy = xl.cy[i], cz = xl.cz[i];
        int dest = tile_of<D>(cx, cy, cz, G);
        int slot = atomicAdd(cnt_out + dest, 1);
        if (slot >= cap) { status |= F_TILE; continue; }
        long dst = (long)dest * cap + slot;
        out.cell[dst] = pack_cell(cx, cy, cz, G);
#pragma unroll
        for (int d = 0; d < D; ++d) out.off[d][dst] = o[d];
#pragma unroll
        for (int c = 0; c < 3; ++c) out.v[c][dst] = vr[c];
        out.id[dst] = pid;
        if constexpr (DEP) status |= deposit_particle<R, D, S>(nullptr, 0, 0, 0, mom, G, cx, cy, cz, o, vr, oor);
    }
    if (status & F_SAT) atomicAdd(ctr + C_SAT, 1ull);
    if (oor) atomicAdd(ctr + C_OOR, 1ull);
    if (status) atomicOr(reinterpret_cast<unsigned int*>(ctr + C_FLAGS), (unsigned int)status);
}

// ---------------------------------------------------------------------------
// Injection: thermal ions at x = 0 (drifting Maxwellian) and CRs at x = L
// (isotropic in the downstream frame, flux weighted), with deterministic
// counts and ids handed out by the host.
// ---------------------------------------------------------------------------
template <typename R, int D, int S, bool DEP>
__global__ __launch_bounds__(256) void k_inject(Geo G, PBuf<R> out0, int32_t* cnt0, int64_t cap0, unsigned long long* mom0,
                                                PBuf<R> out1, int32_t* cnt1, int64_t cap1, unsigned long long* mom1,
                                                unsigned long long* ctr, uint64_t step, int64_t id0,
                                                int64_t cnt_th, int64_t cnt_cr, int64_t ntr) {
    const int64_t nth = cnt_th * ntr, ncr = cnt_cr * ntr;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
        xi = (double)G.nx - fabs(vv[0]) * U[0] * G.dt / G.dx;
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
    int slot = atomicAdd(cnt + dest, 1);
    atomicAdd(ctr + (cr ? C_ADD1 : C_ADD0), 1ull);
    atomicAdd(ctr + (cr ? C_INJ_CR : C_INJ_TH), 1ull);
    if (slot >= cap) {
        atomicOr(reinterpret_cast<unsigned int*>(ctr + C_FLAGS), (unsigned int)F_TILE);
        return;
    }
    long dst = (long)dest * cap + slot;
    out.cell[dst] = pack_cell(cx, cy, cz, G);
#pragma unroll
    for (int d = 0; d < D; ++d) out.off[d][dst] = o[d];
#pragma unroll
    for (int c = 0; c < 3; ++c) out.v[c][dst] = vr[c];
    out.id[dst] = (uint32_t)id;
    if constexpr (DEP) status |= deposit_particle<R, D, S>(nullptr, 0, 0, 0, mom, G, cx, cy, cz, o, vr, oor);
    if (status & F_SAT) atomicAdd(ctr + C_SAT, 1ull);
    if (oor) atomicAdd(ctr + C_OOR, 1ull);
    if (status) atomicOr(reinterpret_cast<unsigned int*>(ctr + C_FLAGS), (unsigned int)status);
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
    const int dx0 = tx * T::X - 1 - LO, dy0 = D >= 2 ? ty * T::Y - 1 - LO : 0, dz0 = D >= 3 ? tz * T::Z - 1 - LO : 0;
    for (int l = threadIdx.x; l < X::DN * 4; l += blockDim.x) sd[l] = 0ull;
    __syncthreads();
    const int n = min(cnt[tile], (int)cap);
    const long base = (long)tile * cap;
    int status = 0, oor = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        long src = base + i;
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
