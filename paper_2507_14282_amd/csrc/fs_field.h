// fs_field.h -- FP64 field update of the hybrid model and the init / utility
// kernels.
//
// Grid: nodes x_i = i dx hold E and the ion moments, cell centres hold B.
// Centre->node and node->centre derivatives are one-cell differences
// averaged over the transverse cell pairs, so the discrete div B of the
// Faraday update vanishes identically (the averaging and difference
// operators commute).  Boundaries of the box in x: the inflow ghost centre
// holds B0, the wall ghost centre copies the last cell; moments within
// `shape` nodes of either x boundary are copied from the nearest node that
// both sides' particles cover; y and z are periodic.
#pragma once
#include "fs_kernels.h"

namespace fsk {

struct FieldGeo {
    int dim, nx, nyc, nzc, nxn, ndx, g, xbc, mclamp;
    double dx, B0[3];
    double n_floor, beta_e, gamma_e, eta, j_ext;
    double wth, wcr, scR, scG;    // species weights and fixed-point scales
    int has_cr;
};

// B component c at centre (i, j, k), ghost rules in x, periodic in y/z.
__device__ __forceinline__ double centre_B(const double* __restrict__ B, const FieldGeo& F, long nc,
                                           int i, int j, int k, int c) {
    j = wrapi(j, F.nyc);
    k = wrapi(k, F.nzc);
    if (F.xbc == 1) i = wrapi(i, F.nx);
    else if (i < 0) return F.B0[c];
    else if (i >= F.nx) i = F.nx - 1;
    return B[(long)c * nc + i + (long)F.nx * (j + (long)F.nyc * k)];
}

// Launch shape of the field kernels: 64 x 4 threads over (x, y), one z per
// block layer, so every thread knows its (i, j, k) without any division.
constexpr int kFX = 64, kFY = 4;

// Ion density / flux at the field nodes from both species' integer moments,
// boundary-filled, floored, plus the rigid external current, and the
// electron pressure p_e = (beta_e / 2) n_e^gamma_e.
__global__ __launch_bounds__(256) void k_fluid(FieldGeo F, const long long* __restrict__ m0,
                                               const long long* __restrict__ m1, double* __restrict__ fl,
                                               long nnode) {
    int i = blockIdx.x * kFX + threadIdx.x;
    const int j = blockIdx.y * kFY + threadIdx.y, k = blockIdx.z;
    if (i >= F.nxn || j >= F.nyc) return;
    const long n = i + (long)F.nxn * (j + (long)F.nyc * k);
    if (F.xbc == 0) {
        if (i < F.mclamp) i = F.mclamp;
        if (i > F.nx - F.mclamp) i = F.nx - F.mclamp;
    }
    const long dn = (long)(i + F.g) + (long)F.ndx * (j + (long)F.nyc * k);
    double dens = F.wth * ((double)m0[4 * dn] * F.scR);
    double G[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) G[c] = F.wth * ((double)m0[4 * dn + 1 + c] * F.scG);
    if (F.has_cr) {
        dens += F.wcr * ((double)m1[4 * dn] * F.scR);
#pragma unroll
        for (int c = 0; c < 3; ++c) G[c] += F.wcr * ((double)m1[4 * dn + 1 + c] * F.scG);
    }
    double ne = fmax(dens, F.n_floor);
    fl[n] = ne;
    fl[nnode + n] = 0.5 * F.beta_e * pow(ne, F.gamma_e);
    fl[2 * nnode + n] = G[0] + F.j_ext;
    fl[3 * nnode + n] = G[1];
    fl[4 * nnode + n] = G[2];
}

__device__ __forceinline__ long fnode(const FieldGeo& F, int i, int j, int k) {
    if (F.xbc == 1) i = wrapi(i, F.nx);
    else { i = i < 0 ? 0 : i; i = i > F.nx ? F.nx : i; }
    j = wrapi(j, F.nyc);
    k = wrapi(k, F.nzc);
    return (long)i + (long)F.nxn * (j + (long)F.nyc * k);
}

// Ohm's law at every node: E = (-Gamma x Bbar + J x Bbar - grad p_e)/n_e + eta J
// with Bbar the mean of the 2^D centres around the node and J = curl B from
// their differences.  With `gather` set it also writes E and Bbar in the
// particle precision for the push.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_ohm(FieldGeo F, const double* __restrict__ B, const double* __restrict__ fl,
                                             double* __restrict__ E, R* __restrict__ gather, long nnode, long ncent) {
    const int i = blockIdx.x * kFX + threadIdx.x;
    const int j = blockIdx.y * kFY + threadIdx.y, k = blockIdx.z;
    if (i >= F.nxn || j >= F.nyc) return;
    const long n = i + (long)F.nxn * (j + (long)F.nyc * k);
    constexpr int NB = D >= 2 ? 2 : 1, NC = D >= 3 ? 2 : 1;
    // C[a][b][c] = B at centre (i-1+a, j-1+b, k-1+c)
    double C[2][NB][NC][3];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    C[a][b][c][d] = centre_B(B, F, ncent, i - 1 + a, D >= 2 ? j - 1 + b : 0, D >= 3 ? k - 1 + c : 0, d);
    double bb[3] = {0, 0, 0}, dBx[3] = {0, 0, 0}, dBy[3] = {0, 0, 0}, dBz[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) bb[d] += C[a][b][c][d];
#pragma unroll
    for (int d = 0; d < 3; ++d) bb[d] *= 1.0 / (double)(2 * NB * NC);
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) dBx[d] += C[1][b][c][d] - C[0][b][c][d];
#pragma unroll
    for (int d = 0; d < 3; ++d) dBx[d] = dBx[d] / (double)(NB * NC) / F.dx;
    if constexpr (D >= 2) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) dBy[d] += C[a][1][c][d] - C[a][0][c][d];
#pragma unroll
        for (int d = 0; d < 3; ++d) dBy[d] = dBy[d] / (double)(2 * NC) / F.dx;
    }
    if constexpr (D >= 3) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int d = 0; d < 3; ++d) dBz[d] += C[a][b][1][d] - C[a][b][0][d];
#pragma unroll
        for (int d = 0; d < 3; ++d) dBz[d] = dBz[d] / 4.0 / F.dx;
    }
    const double J[3] = {dBy[2] - dBz[1], dBz[0] - dBx[2], dBx[1] - dBy[0]};
    const double* pe = fl + nnode;
    double gp[3] = {0, 0, 0};
    gp[0] = (pe[fnode(F, i + 1, j, k)] - pe[fnode(F, i - 1, j, k)]) / (2.0 * F.dx);
    if constexpr (D >= 2) gp[1] = (pe[fnode(F, i, j + 1, k)] - pe[fnode(F, i, j - 1, k)]) / (2.0 * F.dx);
    if constexpr (D >= 3) gp[2] = (pe[fnode(F, i, j, k + 1)] - pe[fnode(F, i, j, k - 1)]) / (2.0 * F.dx);
    const double ne = fl[n];
    const double G[3] = {fl[2 * nnode + n], fl[3 * nnode + n], fl[4 * nnode + n]};
    double num[3];
    num[0] = -(G[1] * bb[2] - G[2] * bb[1]) + (J[1] * bb[2] - J[2] * bb[1]) - gp[0];
    num[1] = -(G[2] * bb[0] - G[0] * bb[2]) + (J[2] * bb[0] - J[0] * bb[2]) - gp[1];
    num[2] = -(G[0] * bb[1] - G[1] * bb[0]) + (J[0] * bb[1] - J[1] * bb[0]) - gp[2];
    double e[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        e[d] = num[d] / ne + F.eta * J[d];
        E[(long)d * nnode + n] = e[d];
    }
    if (gather) {
        R* gp8 = gather + 8 * n;
        gp8[0] = (R)e[0]; gp8[1] = (R)e[1]; gp8[2] = (R)e[2]; gp8[3] = (R)0;
        gp8[4] = (R)bb[0]; gp8[5] = (R)bb[1]; gp8[6] = (R)bb[2]; gp8[7] = (R)0;
    }
}

// One SSP-RK3 stage at every centre: Bout = c0 Bn + c1 (Bin - h curl E),
// with curl E from the 2^D nodes around the centre.
template <int D>
__global__ __launch_bounds__(256) void k_faraday(FieldGeo F, const double* __restrict__ E, const double* __restrict__ Bn,
                                                 const double* __restrict__ Bin, double* __restrict__ Bout,
                                                 double c0, double c1, double h, long nnode, long ncent) {
    const int i = blockIdx.x * kFX + threadIdx.x;
    const int j = blockIdx.y * kFY + threadIdx.y, k = blockIdx.z;
    if (i >= F.nx || j >= F.nyc) return;
    const long n = i + (long)F.nx * (j + (long)F.nyc * k);
    constexpr int NB = D >= 2 ? 2 : 1, NC = D >= 3 ? 2 : 1;
    double P[2][NB][NC][3];   // E at node (i+a, j+b, k+c)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                long q = fnode(F, i + a, j + b, k + c);
#pragma unroll
                for (int d = 0; d < 3; ++d) P[a][b][c][d] = E[(long)d * nnode + q];
            }
    double dEx[3] = {0, 0, 0}, dEy[3] = {0, 0, 0}, dEz[3] = {0, 0, 0};
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) dEx[d] += P[1][b][c][d] - P[0][b][c][d];
#pragma unroll
    for (int d = 0; d < 3; ++d) dEx[d] = dEx[d] / (double)(NB * NC) / F.dx;
    if constexpr (D >= 2) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) dEy[d] += P[a][1][c][d] - P[a][0][c][d];
#pragma unroll
        for (int d = 0; d < 3; ++d) dEy[d] = dEy[d] / (double)(2 * NC) / F.dx;
    }
    if constexpr (D >= 3) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int d = 0; d < 3; ++d) dEz[d] += P[a][b][1][d] - P[a][b][0][d];
#pragma unroll
        for (int d = 0; d < 3; ++d) dEz[d] = dEz[d] / 4.0 / F.dx;
    }
    const double rhs[3] = {-(dEy[2] - dEz[1]), -(dEz[0] - dEx[2]), -(dEx[1] - dEy[0])};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        long q = (long)d * ncent + n;
        double s = Bin[q] + h * rhs[d];
        Bout[q] = c0 == 0.0 ? c1 * s : c0 * Bn[q] + c1 * s;
    }
}

// ---------------------------------------------------------------------------
// initial load
// ---------------------------------------------------------------------------
__global__ void k_phases(uint64_t seed, int n_modes, double* phase) {
    int m = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (m > n_modes) return;
    double U[4];
    draw4(seed, kStreamFourier, (uint64_t)m, 0, 0, U);
    phase[m] = kTwoPi * U[0];
}

// B0 plus the seeded circularly polarised modes dBy = A cos(k x + phi),
// dBz = A sin(k x + phi), k_m = 2 pi m / L.
__global__ void k_init_B(FieldGeo F, int n_modes, const double* __restrict__ amps, double mode_amp,
                         const double* __restrict__ phase, double L, double* __restrict__ B, long ncent) {
    long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= ncent) return;
    int i = (int)(n % F.nx);
    double x = ((double)i + 0.5) * F.dx;
    double by = F.B0[1], bz = F.B0[2];
    for (int m = 1; m <= n_modes; ++m) {
        double A = amps ? amps[m - 1] : mode_amp;
        double ph = kTwoPi * (double)m * x / L + phase[m];
        by += A * cos(ph);
        bz += A * sin(ph);
    }
    B[n] = F.B0[0];
    B[ncent + n] = by;
    B[2 * ncent + n] = bz;
}

// ppc thermal ions per cell, ids cell-major; each lands in a fixed slot of
// its tile (local cell index * ppc + q), so no atomics are needed.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_init_particles(Geo G, PBuf<R> out, int64_t cap, int ppc, long np) {
    using T = TileShape<D>;
    long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= np) return;
    long cell = id / ppc;
    int q = (int)(id % ppc);
    int cx = (int)(cell % G.nx);
    int cy = (int)((cell / G.nx) % G.nyc);
    int cz = (int)(cell / ((long)G.nx * G.nyc));
    double U[4], V[4], n1, n2, n3, n4;
    draw4(G.seed, kStreamInit, 0, (uint64_t)id, 0, U);
    draw4(G.seed, kStreamInit, 0, (uint64_t)id, 1, V);
    box_muller(V[0], V[1], n1, n2);
    box_muller(V[2], V[3], n3, n4);
    int tile = tile_of<D>(cx, cy, cz, G);
    int tx = tile % G.ntx, ty = (tile / G.ntx) % G.nty, tz = tile / (G.ntx * G.nty);
    int ex = min(T::X, G.nx - tx * T::X), ey = min(T::Y, G.nyc - ty * T::Y);
    int lc = (cx - tx * T::X) + ex * ((cy - ty * T::Y) + ey * (cz - tz * T::Z));
    long dst = (long)tile * cap + (long)lc * ppc + q;
    out.cell[dst] = pack_cell(cx, cy, cz, G);
    out.off[0][dst] = to_offset<R>(U[0]);
    if constexpr (D >= 2) out.off[1][dst] = to_offset<R>(U[1]);
    if constexpr (D >= 3) out.off[2][dst] = to_offset<R>(U[2]);
    out.v[0][dst] = (R)(G.u_sh + G.sigma * n1);
    out.v[1][dst] = (R)(G.sigma * n2);
    out.v[2][dst] = (R)(G.sigma * n3);
    out.id[dst] = (uint32_t)id;
}

template <int D>
__global__ void k_init_counts(Geo G, int32_t* cnt, int ppc) {
    using T = TileShape<D>;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= G.ntiles) return;
    cnt[G.ntiles + t] = 0;
    int tx = t % G.ntx, ty = (t / G.ntx) % G.nty, tz = t / (G.ntx * G.nty);
    int ex = min(T::X, G.nx - tx * T::X);
    int ey = D >= 2 ? min(T::Y, G.nyc - ty * T::Y) : 1;
    int ez = D >= 3 ? min(T::Z, G.nzc - tz * T::Z) : 1;
    cnt[t] = ex * ey * ez * ppc;
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t* p, int32_t v, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

// Live-particle totals after a step: count += injected - removed.
__global__ void k_count_update(int64_t* c0, int64_t* c1, const unsigned long long* ctr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (c0) *c0 += (int64_t)ctr[C_ADD0] - (int64_t)ctr[C_REM0];
        if (c1) *c1 += (int64_t)ctr[C_ADD1] - (int64_t)ctr[C_REM1];
    }
}

__global__ void k_set_i64(int64_t* p, int64_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Copy the live particles of every tile to flat arrays (host offsets).
template <typename R, int D>
__global__ void k_compact(Geo G, PBuf<R> in, const int32_t* cnt, const int64_t* offs, int64_t cap,
                          int64_t* cell3, double* off3, double* v3, uint64_t* id) {
    int tile = blockIdx.x;
    int lo = cnt[tile];
    int n = min(lo + cnt[G.ntiles + tile], (int)cap);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        long src = bin_slot(tile, cap, lo, i);
        long dst = offs[tile] + i;
        int32_t pc = in.cell[src];
        cell3[3 * dst] = cell_x(pc, G);
        cell3[3 * dst + 1] = D >= 2 ? cell_y(pc, G) : 0;
        cell3[3 * dst + 2] = D >= 3 ? cell_z(pc, G) : 0;
        for (int d = 0; d < 3; ++d) off3[3 * dst + d] = d < D ? (double)in.off[d][src] : 0.0;
        for (int d = 0; d < 3; ++d) v3[3 * dst + d] = (double)in.v[d][src];
        id[dst] = in.id[src];
    }
}

// ---------------------------------------------------------------------------
// diagnostics: deterministic FP64 block partial sums, reduced in fixed order
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double x, double* sh) {
    int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Field sums per block: |B|^2, By^2 + Bz^2, loss region, max |div B|.
__global__ __launch_bounds__(256) void k_diag_field(FieldGeo F, const double* __restrict__ B, long ncent,
                                                    double* __restrict__ part) {
    __shared__ double sh[256];
    long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double b2 = 0, bp = 0, loss = 0, dv = 0;
    if (n < ncent) {
        double bx = B[n], by = B[ncent + n], bz = B[2 * ncent + n];
        b2 = bx * bx + by * by + bz * bz;
        bp = by * by + bz * bz;
        int i = (int)(n % F.nx);
        if (i >= F.nx / 2) loss = bp;
        // div B at the node (i, j, k) = lower corner of this centre, interior nodes
        int j = (int)((n / F.nx) % F.nyc), k = (int)(n / ((long)F.nx * F.nyc));
        if (F.xbc == 1 || i >= 1) {
            const int D = F.dim, nb = D >= 2 ? 2 : 1, nc = D >= 3 ? 2 : 1;
            double dx = 0, dy = 0, dz = 0;
            for (int b = 0; b < nb; ++b)
                for (int c = 0; c < nc; ++c)
                    dx += centre_B(B, F, ncent, i, j - 1 + b, k - 1 + c, 0) - centre_B(B, F, ncent, i - 1, j - 1 + b, k - 1 + c, 0);
            dx = dx / (double)(nb * nc) / F.dx;
            if (D >= 2) {
                for (int a = 0; a < 2; ++a)
                    for (int c = 0; c < nc; ++c)
                        dy += centre_B(B, F, ncent, i - 1 + a, j, k - 1 + c, 1) - centre_B(B, F, ncent, i - 1 + a, j - 1, k - 1 + c, 1);
                dy = dy / (double)(2 * nc) / F.dx;
            }
            if (D >= 3) {
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        dz += centre_B(B, F, ncent, i - 1 + a, j - 1 + b, k, 2) - centre_B(B, F, ncent, i - 1 + a, j - 1 + b, k - 1, 2);
                dz = dz / 4.0 / F.dx;
            }
            dv = fabs(dx + dy + dz);
        }
    }
    double s0 = block_sum(b2, sh), s1 = block_sum(bp, sh), s2 = block_sum(loss, sh);
    sh[threadIdx.x] = dv;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x] = s0;
        part[4 * blockIdx.x + 1] = s1;
        part[4 * blockIdx.x + 2] = s2;
        part[4 * blockIdx.x + 3] = sh[0];
    }
}

// Per-tile kinetic energy sums (sum of |v|^2) in FP64.
template <typename R>
__global__ __launch_bounds__(256) void k_diag_kin(PBuf<R> in, const int32_t* cnt, int ntiles, int64_t cap, double* part) {
    __shared__ double sh[256];
    int tile = blockIdx.x;
    int lo = cnt[tile];
    int n = min(lo + cnt[ntiles + tile], (int)cap);
    double s = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        long src = bin_slot(tile, cap, lo, i);
        double a = in.v[0][src], b = in.v[1][src], c = in.v[2][src];
        s += a * a + b * b + c * c;
    }
    double t = block_sum(s, sh);
    if (threadIdx.x == 0) part[tile] = t;
}

__global__ void k_profile(FieldGeo F, const double* __restrict__ B, long ncent, double* prof) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= F.nx) return;
    double s = 0;
    for (long jk = 0; jk < (long)F.nyc * F.nzc; ++jk) {
        long n = i + (long)F.nx * jk;
        double by = B[ncent + n], bz = B[2 * ncent + n];
        s += by * by + bz * bz;
    }
    prof[i] = s;
}

}  // namespace fsk
