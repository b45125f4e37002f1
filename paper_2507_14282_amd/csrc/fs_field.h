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
    double dx, rdx, B0[3];
    double n_floor, beta_e, gamma_e, eta, j_ext, u_sh;
    double wth, wcr, scR, scG;    // species weights and fixed-point scales
    int has_cr;
    int cont;                     // moments hold FP64 sums (continuous deposit)
    int smooth;                   // binomial passes on the fluid moments (0: none)
    int conduct;                  // conducting wall at x = L: E_y = E_z = 0 there
};

// The inflow node x = 0 of the box carries the motional field of the
// unperturbed upstream plasma, E = -u_sh x_hat x B0, in place of Ohm's law
// evaluated against the fixed ghost centre (which lets 2D perturbations grow
// at the boundary).
__device__ __forceinline__ bool inflow_node(const FieldGeo& F, int i) { return F.xbc == 0 && i == 0; }
// A conducting wall at x = L (box only): the tangential E vanishes at its node.
__device__ __forceinline__ void wall_E(const FieldGeo& F, int i, double e[3]) {
    if (F.conduct && i == F.nx) { e[1] = 0.0; e[2] = 0.0; }
}
__device__ __forceinline__ void inflow_E(const FieldGeo& F, double e[3]) {
    e[0] = 0.0;
    e[1] = F.u_sh * F.B0[2];
    e[2] = -F.u_sh * F.B0[1];
}

// Linear index i + sx (j + sy k) of a wrapped grid point.  The layout keeps
// sx and sy * nzc below 2^24 and every grid below 2^31 points, so 24-bit
// products are exact.
__device__ __forceinline__ long lin(int i, int j, int k, int sx, int sy) {
    return (long)(i + (int)__umul24(sx, j + (int)__umul24(sy, k)));
}

// B component c at centre (i, j, k), ghost rules in x, periodic in y/z.
__device__ __forceinline__ double centre_B(const double* __restrict__ B, const FieldGeo& F, long nc,
                                           int i, int j, int k, int c) {
    j = wrapi(j, F.nyc);
    k = wrapi(k, F.nzc);
    if (F.xbc == 1) i = wrapi(i, F.nx);
    else if (i < 0) return F.B0[c];
    else if (i >= F.nx) i = F.nx - 1;
    return B[(long)c * nc + lin(i, j, k, F.nx, F.nyc)];
}

// Launch shape of the field kernels: 64 x 4 threads over (x, y), one z per
// block layer, so every thread knows its (i, j, k) without any division.
constexpr int kFX = 64, kFY = 4;

// One node's fluid record: n_e = max(n, n_floor), p_e = (beta_e / 2)
// n_e^gamma_e and the flux plus the rigid external current (added after the
// filter when smoothing).
__device__ __forceinline__ void store_fluid(const FieldGeo& F, double* __restrict__ fl, long nnode, long n,
                                            double dens, const double G[3]) {
    const double ne = fmax(dens, F.n_floor);
    fl[n] = ne;
    fl[nnode + n] = 0.5 * F.beta_e * pow(ne, F.gamma_e);
    fl[2 * nnode + n] = F.smooth ? G[0] : G[0] + F.j_ext;
    fl[3 * nnode + n] = G[1];
    fl[4 * nnode + n] = G[2];
}

// Ion density / flux at the field nodes from both species' integer moments,
// boundary-filled, floored, plus the rigid external current, and the
// electron pressure p_e = (beta_e / 2) n_e^gamma_e.  tc selects the
// time-centred coupling: 0 off; 1 also keep the density and flux as the
// previous step's (nprev, gprev: a load or a refresh); 2 a step's field
// update: fl gets the moments at t_{n+1/2} (the mean of the previous and new
// densities, the flux as deposited at the moves' midpoints), fl2 those of the
// final Ohm's law at t_{n+1} (the new density, the flux extrapolated,
// (3 Gamma^{n+1/2} - Gamma^{n-1/2}) / 2), and nprev / gprev move on.
__global__ __launch_bounds__(256) void k_fluid(FieldGeo F, const long long* __restrict__ m0,
                                               const long long* __restrict__ m1, double* __restrict__ fl,
                                               long nnode, double* __restrict__ fl2, double* __restrict__ nprev,
                                               double* __restrict__ gprev, int tc) {
    int i = blockIdx.x * kFX + threadIdx.x;
    const int j = blockIdx.y * kFY + threadIdx.y, k = blockIdx.z;
    if (i >= F.nxn || j >= F.nyc) return;
    const long n = lin(i, j, k, F.nxn, F.nyc);
    if (F.xbc == 0) {
        if (i < F.mclamp) i = F.mclamp;
        if (i > F.nx - F.mclamp) i = F.nx - F.mclamp;
    }
    const long dn = lin(i + F.g, j, k, F.ndx, F.nyc);
    // one node's four moments are 32 contiguous bytes: two 16-byte loads
    double dens, G[3];
    if (F.cont) {
        const double2* d0 = reinterpret_cast<const double2*>(m0) + 2 * dn;
        const double2 a = d0[0], b = d0[1];
        dens = F.wth * a.x;
        G[0] = F.wth * a.y; G[1] = F.wth * b.x; G[2] = F.wth * b.y;
        if (F.has_cr) {
            const double2* d1 = reinterpret_cast<const double2*>(m1) + 2 * dn;
            const double2 c = d1[0], d = d1[1];
            dens += F.wcr * c.x;
            G[0] += F.wcr * c.y; G[1] += F.wcr * d.x; G[2] += F.wcr * d.y;
        }
    } else {
        const longlong2* q0 = reinterpret_cast<const longlong2*>(m0) + 2 * dn;
        const longlong2 a = q0[0], b = q0[1];
        dens = F.wth * ((double)a.x * F.scR);
        G[0] = F.wth * ((double)a.y * F.scG); G[1] = F.wth * ((double)b.x * F.scG); G[2] = F.wth * ((double)b.y * F.scG);
        if (F.has_cr) {
            const longlong2* q1 = reinterpret_cast<const longlong2*>(m1) + 2 * dn;
            const longlong2 c = q1[0], d = q1[1];
            dens += F.wcr * ((double)c.x * F.scR);
            G[0] += F.wcr * ((double)c.y * F.scG); G[1] += F.wcr * ((double)d.x * F.scG);
            G[2] += F.wcr * ((double)d.y * F.scG);
        }
    }
    if (tc == 2) {
#pragma clang fp contract(off)
        const double dh = 0.5 * (nprev[n] + dens);
        store_fluid(F, fl, nnode, n, dh, G);
        double Ge[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) Ge[c] = 1.5 * G[c] - 0.5 * gprev[c * nnode + n];
        store_fluid(F, fl2, nnode, n, dens, Ge);
    } else {
        store_fluid(F, fl, nnode, n, dens, G);
    }
    if (tc) {
        nprev[n] = dens;
#pragma unroll
        for (int c = 0; c < 3; ++c) gprev[c * nnode + n] = G[c];
    }
}

// One pass of the 1-2-1 binomial filter along one axis over the fluid
// planes 0 (n_e, floored) and 2-4 (Gamma without J_ext):
// f_i <- (f_{i-1} + 2 f_i + f_{i+1}) / 4 in this operation order.  In the box
// the x end nodes keep their values; y, z and periodic x wrap.  Plane 1 is
// left alone (p_e follows from the filtered n_e at the end).
__global__ __launch_bounds__(256) void k_smooth_axis(FieldGeo F, const double* __restrict__ in,
                                                     double* __restrict__ out, int axis, long nnode) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * kFX + threadIdx.x;
    const int j = blockIdx.y * kFY + threadIdx.y, k = blockIdx.z;
    if (i >= F.nxn || j >= F.nyc) return;
    const long n = lin(i, j, k, F.nxn, F.nyc);
    long m = n, p = n;
    bool keep = false;
    if (axis == 0) {
        if (F.xbc == 1) {
            m = lin(wrapi(i - 1, F.nx), j, k, F.nxn, F.nyc);
            p = lin(wrapi(i + 1, F.nx), j, k, F.nxn, F.nyc);
        } else if (i == 0 || i == F.nx) {
            keep = true;
        } else {
            m = n - 1;
            p = n + 1;
        }
    } else if (axis == 1) {
        m = lin(i, wrapi(j - 1, F.nyc), k, F.nxn, F.nyc);
        p = lin(i, wrapi(j + 1, F.nyc), k, F.nxn, F.nyc);
    } else {
        m = lin(i, j, wrapi(k - 1, F.nzc), F.nxn, F.nyc);
        p = lin(i, j, wrapi(k + 1, F.nzc), F.nxn, F.nyc);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        if (q == 1) continue;
        const double* x = in + q * nnode;
        out[q * nnode + n] = keep ? x[n] : 0.25 * ((x[m] + 2.0 * x[n]) + x[p]);
    }
}

// After the passes: the boundary fill again (box nodes within `shape` of an
// x end copy the nearest covered node), the floor, p_e and J_ext.  Reads
// `src`, writes `fl` (distinct buffers).
__global__ __launch_bounds__(256) void k_smooth_finish(FieldGeo F, const double* __restrict__ src,
                                                       double* __restrict__ fl, long nnode) {
    const int i = blockIdx.x * kFX + threadIdx.x;
    const int j = blockIdx.y * kFY + threadIdx.y, k = blockIdx.z;
    if (i >= F.nxn || j >= F.nyc) return;
    const long n = lin(i, j, k, F.nxn, F.nyc);
    int ic = i;
    if (F.xbc == 0) {
        if (ic < F.mclamp) ic = F.mclamp;
        if (ic > F.nx - F.mclamp) ic = F.nx - F.mclamp;
    }
    const long c = lin(ic, j, k, F.nxn, F.nyc);
    const double ne = fmax(src[c], F.n_floor);
    fl[n] = ne;
    fl[nnode + n] = 0.5 * F.beta_e * pow(ne, F.gamma_e);
    fl[2 * nnode + n] = src[2 * nnode + c] + F.j_ext;
    fl[3 * nnode + n] = src[3 * nnode + c];
    fl[4 * nnode + n] = src[4 * nnode + c];
}

__device__ __forceinline__ long fnode(const FieldGeo& F, int i, int j, int k) {
    if (F.xbc == 1) i = wrapi(i, F.nx);
    else { i = i < 0 ? 0 : i; i = i > F.nx ? F.nx : i; }
    j = wrapi(j, F.nyc);
    k = wrapi(k, F.nzc);
    return lin(i, j, k, F.nxn, F.nyc);
}

// Block shape (cells) of the tiled field kernels, and the LDS tiles one
// block stages: B at centres x0-1 .. x0+X (and likewise in y, z where the
// dimension exists), E at nodes x0 .. x0+X, p_e at nodes x0-1 .. x0+X+1.
template <int D> struct FieldBlock;
template <> struct FieldBlock<1> { static constexpr int X = 256, Y = 1, Z = 1; };
template <> struct FieldBlock<2> { static constexpr int X = 32, Y = 8, Z = 1; };
template <> struct FieldBlock<3> { static constexpr int X = 16, Y = 4, Z = 4; };

template <int D> struct FieldTile {
    using FB = FieldBlock<D>;
    static constexpr int OY = D >= 2 ? 1 : 0, OZ = D >= 3 ? 1 : 0;
    static constexpr int CX = FB::X + 2, CY = FB::Y + 2 * OY, CZ = FB::Z + 2 * OZ;
    static constexpr int NX = FB::X + 1, NY = FB::Y + OY, NZ = FB::Z + OZ;
    static constexpr int PX = FB::X + 3, PY = FB::Y + 3 * OY, PZ = FB::Z + 3 * OZ;
    static constexpr int CN = CX * CY * CZ, NN = NX * NY * NZ, PN = PX * PY * PZ;
    static_assert(FB::X * FB::Y * FB::Z == 256, "one centre per thread");
};

// Stage the block's B (centres, ghost rules in x) and p_e (nodes, clamped in
// x for the box) into LDS.  Every load of the block is issued before the
// first LDS store, so each thread keeps a dozen HBM requests in flight.
template <int D>
__device__ __forceinline__ void stage_tiles(const FieldGeo& F, const double* __restrict__ B,
                                            const double* __restrict__ pe, long ncent, int x0, int y0, int z0,
                                            double (*sB)[FieldTile<D>::CN], double* sP) {
    using T = FieldTile<D>;
    constexpr int IC = (T::CN + 255) / 256, IP = (T::PN + 255) / 256;
    double vb[IC][3], vp[IP];
#pragma unroll
    for (int it = 0; it < IC; ++it) {
        const int l = threadIdx.x + 256 * it;
        vb[it][0] = vb[it][1] = vb[it][2] = 0.0;
        if (it + 1 < IC || l < T::CN) {
            const int lx = l % T::CX, r = l / T::CX, ly = r % T::CY, lz = r / T::CY;
            int i = x0 - 1 + lx;
            const int j = D >= 2 ? wrapi(y0 - 1 + ly, F.nyc) : 0, k = D >= 3 ? wrapi(z0 - 1 + lz, F.nzc) : 0;
            if (F.xbc == 1) i = wrapi(i, F.nx);
            else if (i >= F.nx) i = F.nx - 1;
            if (i < 0) {
                vb[it][0] = F.B0[0]; vb[it][1] = F.B0[1]; vb[it][2] = F.B0[2];
            } else {
                const long q = lin(i, j, k, F.nx, F.nyc);
                vb[it][0] = B[q]; vb[it][1] = B[ncent + q]; vb[it][2] = B[2 * ncent + q];
            }
        }
    }
#pragma unroll
    for (int it = 0; it < IP; ++it) {
        const int l = threadIdx.x + 256 * it;
        vp[it] = 0.0;
        if (it + 1 < IP || l < T::PN) {
            const int lx = l % T::PX, r = l / T::PX, ly = r % T::PY, lz = r / T::PY;
            int i = x0 - 1 + lx;
            const int j = D >= 2 ? wrapi(y0 - 1 + ly, F.nyc) : 0, k = D >= 3 ? wrapi(z0 - 1 + lz, F.nzc) : 0;
            if (F.xbc == 1) i = wrapi(i, F.nx);
            else i = i < 0 ? 0 : (i > F.nx ? F.nx : i);
            vp[it] = pe[lin(i, j, k, F.nxn, F.nyc)];
        }
    }
#pragma unroll
    for (int it = 0; it < IC; ++it) {
        const int l = threadIdx.x + 256 * it;
        if (it + 1 < IC || l < T::CN) { sB[0][l] = vb[it][0]; sB[1][l] = vb[it][1]; sB[2][l] = vb[it][2]; }
    }
#pragma unroll
    for (int it = 0; it < IP; ++it) {
        const int l = threadIdx.x + 256 * it;
        if (it + 1 < IP || l < T::PN) sP[l] = vp[it];
    }
}

// Block -> tile of the field grid, XCD-aware: the blocks one XCD receives
// (round robin over 8) cover a contiguous run of tiles, x fastest, so the
// halos they share stay in that XCD's L2.
__device__ __forceinline__ void field_block(int gx, int gy, int& bx, int& by, int& bz) {
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    bx = t % gx;
    const int r = t / gx;
    by = r % gy;
    bz = r / gy;
}

// Ohm's law at one node: E = (-Gamma x Bbar + J x Bbar - grad p_e)/n_e
// + eta J, with Bbar the mean of the 2^D surrounding centres
// (C[a][b][c] = B at centre (x-1+a, y-1+b, z-1+c)), J = curl B from their
// transverse-averaged differences, and dp the central p_e differences across
// the node (zero along absent dimensions).
template <int D>
__device__ __forceinline__ void ohm_core(const FieldGeo& F, const double (&C)[2][D >= 2 ? 2 : 1][D >= 3 ? 2 : 1][3],
                                         const double dp[3], double ne, const double G[3], double e[3],
                                         double bb[3]) {
    constexpr int NB = D >= 2 ? 2 : 1, NC = D >= 3 ? 2 : 1;
    double dBx[3] = {0, 0, 0}, dBy[3] = {0, 0, 0}, dBz[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) bb[d] = 0.0;
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
    for (int d = 0; d < 3; ++d) dBx[d] = dBx[d] * (1.0 / (double)(NB * NC)) * F.rdx;
    if constexpr (D >= 2) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) dBy[d] += C[a][1][c][d] - C[a][0][c][d];
#pragma unroll
        for (int d = 0; d < 3; ++d) dBy[d] = dBy[d] * (1.0 / (double)(2 * NC)) * F.rdx;
    }
    if constexpr (D >= 3) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int d = 0; d < 3; ++d) dBz[d] += C[a][b][1][d] - C[a][b][0][d];
#pragma unroll
        for (int d = 0; d < 3; ++d) dBz[d] = dBz[d] * 0.25 * F.rdx;
    }
    const double J[3] = {dBy[2] - dBz[1], dBz[0] - dBx[2], dBx[1] - dBy[0]};
    const double h2 = 0.5 * F.rdx;
    const double gp[3] = {dp[0] * h2, dp[1] * h2, dp[2] * h2};
    const double rne = 1.0 / ne;
    double num[3];
    num[0] = -(G[1] * bb[2] - G[2] * bb[1]) + (J[1] * bb[2] - J[2] * bb[1]) - gp[0];
    num[1] = -(G[2] * bb[0] - G[0] * bb[2]) + (J[2] * bb[0] - J[0] * bb[2]) - gp[1];
    num[2] = -(G[0] * bb[1] - G[1] * bb[0]) + (J[0] * bb[1] - J[1] * bb[0]) - gp[2];
#pragma unroll
    for (int d = 0; d < 3; ++d) e[d] = num[d] * rne + F.eta * J[d];
}

// Ohm's law at the node of local tile position (lx, ly, lz), global node
// index n, from the block's LDS tiles.
template <int D>
__device__ __forceinline__ void ohm_tile(const FieldGeo& F, const double (*sB)[FieldTile<D>::CN],
                                         const double* sP, const double* __restrict__ fl, long nnode, long n,
                                         int lx, int ly, int lz, double e[3], double bb[3]) {
    using T = FieldTile<D>;
    constexpr int NB = D >= 2 ? 2 : 1, NC = D >= 3 ? 2 : 1;
    double C[2][NB][NC][3];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int l = (lx + a) + T::CX * ((ly + b) + T::CY * (lz + c));
#pragma unroll
                for (int d = 0; d < 3; ++d) C[a][b][c][d] = sB[d][l];
            }
    auto P = [&](int ex, int ey, int ez) {
        return sP[(lx + 1 + ex) + T::PX * ((ly + T::OY + ey) + T::PY * (lz + T::OZ + ez))];
    };
    double dp[3] = {P(1, 0, 0) - P(-1, 0, 0), 0.0, 0.0};
    if constexpr (D >= 2) dp[1] = P(0, 1, 0) - P(0, -1, 0);
    if constexpr (D >= 3) dp[2] = P(0, 0, 1) - P(0, 0, -1);
    const double G[3] = {fl[2 * nnode + n], fl[3 * nnode + n], fl[4 * nnode + n]};
    ohm_core<D>(F, C, dp, fl[n], G, e, bb);
}

// One node of the gather grid (Ex Ey Ez Bbarx Bbary Bbarz) in the particle
// precision, as three 2-vector stores: the pairs (Ex, Ey), (Ez, Bbarx),
// (Bbary, Bbarz) that the push stages.
template <typename R> struct Vec2;
template <> struct Vec2<float> { using T = float2; };
template <> struct Vec2<double> { using T = double2; };
template <typename R> __device__ __forceinline__ void store_gather(R* g6, const double e[3], const double bb[3]) {
    using V = typename Vec2<R>::T;
    V* v = reinterpret_cast<V*>(g6);
    v[0] = V{(R)e[0], (R)e[1]};
    v[1] = V{(R)e[2], (R)bb[0]};
    v[2] = V{(R)bb[1], (R)bb[2]};
}

// Ohm's law at every node of the block, writing E (FP64) and E, Bbar in the
// particle precision into the gather grid.  Grid: nodes in x, centres in y/z.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_ohm(FieldGeo F, const double* __restrict__ B, const double* __restrict__ fl,
                                             double* __restrict__ E, R* __restrict__ gather, long nnode, long ncent,
                                             int gx, int gy) {
    using T = FieldTile<D>;
    using FB = FieldBlock<D>;
    __shared__ double sB[3][T::CN];
    __shared__ double sP[T::PN];
    int bx, by, bz;
    field_block(gx, gy, bx, by, bz);
    const int x0 = bx * FB::X, y0 = by * FB::Y, z0 = bz * FB::Z;
    stage_tiles<D>(F, B, fl + nnode, ncent, x0, y0, z0, sB, sP);
    __syncthreads();
    const int t = threadIdx.x;
    const int tx = t % FB::X, ty = (t / FB::X) % FB::Y, tz = t / (FB::X * FB::Y);
    const int i = x0 + tx, j = y0 + ty, k = z0 + tz;
    if (i >= F.nxn || j >= F.nyc || k >= F.nzc) return;
    const long n = lin(i, j, k, F.nxn, F.nyc);
    double e[3], bb[3];
    ohm_tile<D>(F, sB, sP, fl, nnode, n, tx, ty, tz, e, bb);
    if (inflow_node(F, i)) inflow_E(F, e);
    wall_E(F, i, e);
#pragma unroll
    for (int d = 0; d < 3; ++d) E[(long)d * nnode + n] = e[d];
    store_gather(gather + 6 * n, e, bb);
}

// One SSP-RK3 stage, fused: E = Ohm(Bin) at the block's nodes (its centres
// plus one node of halo) into LDS, then Bout = c0 Bn + c1 (Bin - h curl E)
// at the block's centres.  Neither E nor a second copy of Bin goes through
// HBM.  With c0 == 0, Bn is not read.
template <int D>
__global__ __launch_bounds__(256) void k_stage(FieldGeo F, const double* __restrict__ Bin, const double* __restrict__ Bn,
                                               double* __restrict__ Bout, const double* __restrict__ fl, double c0,
                                               double c1, double h, long nnode, long ncent, int gx, int gy) {
    using T = FieldTile<D>;
    using FB = FieldBlock<D>;
    __shared__ double sB[3][T::CN];
    __shared__ double sP[T::PN];
    __shared__ double sE[3][T::NN];
    int bx, by, bz;
    field_block(gx, gy, bx, by, bz);
    const int x0 = bx * FB::X, y0 = by * FB::Y, z0 = bz * FB::Z;
    stage_tiles<D>(F, Bin, fl + nnode, ncent, x0, y0, z0, sB, sP);
    __syncthreads();
    for (int l = threadIdx.x; l < T::NN; l += 256) {
        const int lx = l % T::NX, r = l / T::NX, ly = r % T::NY, lz = r / T::NY;
        int i = x0 + lx;
        const int j = D >= 2 ? wrapi(y0 + ly, F.nyc) : 0, k = D >= 3 ? wrapi(z0 + lz, F.nzc) : 0;
        double e[3] = {0, 0, 0}, bb[3];
        // nodes past the box are read only by centres that do not exist
        if (F.xbc == 1 || i <= F.nx) {
            if (F.xbc == 1) i = wrapi(i, F.nx);
            const long n = lin(i, j, k, F.nxn, F.nyc);
            ohm_tile<D>(F, sB, sP, fl, nnode, n, lx, ly, lz, e, bb);
            if (inflow_node(F, i)) inflow_E(F, e);
            wall_E(F, i, e);
        }
        sE[0][l] = e[0]; sE[1][l] = e[1]; sE[2][l] = e[2];
    }
    __syncthreads();
    const int t = threadIdx.x;
    const int tx = t % FB::X, ty = (t / FB::X) % FB::Y, tz = t / (FB::X * FB::Y);
    const int i = x0 + tx, j = y0 + ty, k = z0 + tz;
    if (i >= F.nx || j >= F.nyc || k >= F.nzc) return;
    constexpr int NB = D >= 2 ? 2 : 1, NC = D >= 3 ? 2 : 1;
    double dEx[3] = {0, 0, 0}, dEy[3] = {0, 0, 0}, dEz[3] = {0, 0, 0};
    auto at = [&](int a, int b, int c) { return (tx + a) + T::NX * ((ty + b) + T::NY * (tz + c)); };
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) dEx[d] += sE[d][at(1, b, c)] - sE[d][at(0, b, c)];
#pragma unroll
    for (int d = 0; d < 3; ++d) dEx[d] = dEx[d] * (1.0 / (double)(NB * NC)) * F.rdx;
    if constexpr (D >= 2) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) dEy[d] += sE[d][at(a, 1, c)] - sE[d][at(a, 0, c)];
#pragma unroll
        for (int d = 0; d < 3; ++d) dEy[d] = dEy[d] * (1.0 / (double)(2 * NC)) * F.rdx;
    }
    if constexpr (D >= 3) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int d = 0; d < 3; ++d) dEz[d] += sE[d][at(a, b, 1)] - sE[d][at(a, b, 0)];
#pragma unroll
        for (int d = 0; d < 3; ++d) dEz[d] = dEz[d] * 0.25 * F.rdx;
    }
    const double rhs[3] = {-(dEy[2] - dEz[1]), -(dEz[0] - dEx[2]), -(dEx[1] - dEy[0])};
    const long n = lin(i, j, k, F.nx, F.nyc);
    const int lc = (tx + 1) + T::CX * ((ty + T::OY) + T::CY * (tz + T::OZ));
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const long q = (long)d * ncent + n;
        const double sv = sB[d][lc] + h * rhs[d];
        Bout[q] = c0 == 0.0 ? c1 * sv : c0 * Bn[q] + c1 * sv;
    }
}

// ---------------------------------------------------------------------------
// 3D field kernels that march through z.  A 32 x 8 block in (x, y) walks a
// run of z planes and keeps rings of B centre planes (3), p_e node planes
// (3) and E node planes (2) in LDS, so each value comes from HBM about once
// per column (halo 1.3x in x/y, none in z) instead of once per face of a
// small 3D tile.
// ---------------------------------------------------------------------------
struct ZMarch {
    static constexpr int X = 32, Y = 8;
    static constexpr int CX = X + 2, CY = Y + 2, CN = CX * CY;   // centres x0-1 .. x0+X
    static constexpr int PX = X + 3, PY = Y + 3, PN = PX * PY;   // p_e at nodes x0-1 .. x0+X+1
    static constexpr int NX = X + 1, NY = Y + 1, NN = NX * NY;   // nodes x0 .. x0+X
    static constexpr int IC = (CN + 255) / 256, IP = (PN + 255) / 256, IN = (NN + 255) / 256;
};

// Block -> (x0, y0, z range), XCD-aware over (x, y, z-run) with x fastest.
__device__ __forceinline__ void zm_block(int gx, int gy, int zc, int nzc, int& x0, int& y0, int& zs, int& ze) {
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    x0 = (t % gx) * ZMarch::X;
    const int r = t / gx;
    y0 = (r % gy) * ZMarch::Y;
    zs = (r / gy) * zc;
    ze = min(zs + zc, nzc);
}

// Registers of one thread's share of a B centre plane / p_e node plane.
struct ZPlane {
    double b[ZMarch::IC][3];
    double p[ZMarch::IP];
};

__device__ __forceinline__ void zm_fetch_B(const FieldGeo& F, const double* __restrict__ B, long ncent, int x0, int y0,
                                           int k, ZPlane& r) {
    using Z = ZMarch;
    k = wrapi(k, F.nzc);
#pragma unroll
    for (int it = 0; it < Z::IC; ++it) {
        const int l = threadIdx.x + 256 * it;
        r.b[it][0] = r.b[it][1] = r.b[it][2] = 0.0;
        if (it + 1 < Z::IC || l < Z::CN) {
            int i = x0 - 1 + l % Z::CX;
            const int j = wrapi(y0 - 1 + l / Z::CX, F.nyc);
            if (F.xbc == 1) i = wrapi(i, F.nx);
            else if (i >= F.nx) i = F.nx - 1;
            if (i < 0) {
                r.b[it][0] = F.B0[0]; r.b[it][1] = F.B0[1]; r.b[it][2] = F.B0[2];
            } else {
                const long q = lin(i, j, k, F.nx, F.nyc);
                r.b[it][0] = B[q]; r.b[it][1] = B[ncent + q]; r.b[it][2] = B[2 * ncent + q];
            }
        }
    }
}

__device__ __forceinline__ void zm_fetch_P(const FieldGeo& F, const double* __restrict__ pe, int x0, int y0, int k,
                                           ZPlane& r) {
    using Z = ZMarch;
    k = wrapi(k, F.nzc);
#pragma unroll
    for (int it = 0; it < Z::IP; ++it) {
        const int l = threadIdx.x + 256 * it;
        r.p[it] = 0.0;
        if (it + 1 < Z::IP || l < Z::PN) {
            int i = x0 - 1 + l % Z::PX;
            const int j = wrapi(y0 - 1 + l / Z::PX, F.nyc);
            if (F.xbc == 1) i = wrapi(i, F.nx);
            else i = i < 0 ? 0 : (i > F.nx ? F.nx : i);
            r.p[it] = pe[lin(i, j, k, F.nxn, F.nyc)];
        }
    }
}

__device__ __forceinline__ void zm_store_B(const ZPlane& r, double (*sB)[ZMarch::CN]) {
#pragma unroll
    for (int it = 0; it < ZMarch::IC; ++it) {
        const int l = threadIdx.x + 256 * it;
        if (it + 1 < ZMarch::IC || l < ZMarch::CN) { sB[0][l] = r.b[it][0]; sB[1][l] = r.b[it][1]; sB[2][l] = r.b[it][2]; }
    }
}

__device__ __forceinline__ void zm_store_P(const ZPlane& r, double* sP) {
#pragma unroll
    for (int it = 0; it < ZMarch::IP; ++it) {
        const int l = threadIdx.x + 256 * it;
        if (it + 1 < ZMarch::IP || l < ZMarch::PN) sP[l] = r.p[it];
    }
}

// n_e and Gamma at one node, fetched ahead of the LDS phase that uses them.
struct ZFluid {
    double ne, G[3];
    long n;
    bool ok;
};

// Node (x0 + lx, y0 + ly, k); nodes past the box are never read, flagged !ok.
__device__ __forceinline__ void zm_fetch_fluid(const FieldGeo& F, const double* __restrict__ fl, long nnode, int x0,
                                               int y0, int k, int lx, int ly, ZFluid& f) {
    int i = x0 + lx;
    f.ok = F.xbc == 1 || i <= F.nx;
    f.ne = 1.0; f.G[0] = f.G[1] = f.G[2] = 0.0; f.n = 0;
    if (!f.ok) return;
    if (F.xbc == 1) i = wrapi(i, F.nx);
    f.n = lin(i, wrapi(y0 + ly, F.nyc), wrapi(k, F.nzc), F.nxn, F.nyc);
    f.ne = fl[f.n];
    f.G[0] = fl[2 * nnode + f.n]; f.G[1] = fl[3 * nnode + f.n]; f.G[2] = fl[4 * nnode + f.n];
}

// Ohm's law at local node (lx, ly) of the plane whose centre planes below /
// above sit in sB0 / sB1 and whose p_e planes below / at / above in
// sP0 / sP1 / sP2.
__device__ __forceinline__ void zm_ohm(const FieldGeo& F, const double (*sB0)[ZMarch::CN],
                                       const double (*sB1)[ZMarch::CN], const double* sP0, const double* sP1,
                                       const double* sP2, const ZFluid& f, int lx, int ly, double e[3], double bb[3]) {
    using Z = ZMarch;
    double C[2][2][2][3];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int l = (lx + a) + Z::CX * (ly + b);
#pragma unroll
            for (int d = 0; d < 3; ++d) { C[a][b][0][d] = sB0[d][l]; C[a][b][1][d] = sB1[d][l]; }
        }
    const int pc = (lx + 1) + Z::PX * (ly + 1);
    const double dp[3] = {sP1[pc + 1] - sP1[pc - 1], sP1[pc + Z::PX] - sP1[pc - Z::PX], sP2[pc] - sP0[pc]};
    ohm_core<3>(F, C, dp, f.ne, f.G, e, bb);
}

// One SSP-RK3 stage in 3D (see k_stage), marching through z.
__global__ __launch_bounds__(256) void k_stage3(FieldGeo F, const double* __restrict__ Bin,
                                                const double* __restrict__ Bn, double* __restrict__ Bout,
                                                const double* __restrict__ fl, double c0, double c1, double h,
                                                long nnode, long ncent, int gx, int gy, int zc) {
    using Z = ZMarch;
    __shared__ double sB[2][3][Z::CN];
    __shared__ double sP[3][Z::PN];
    __shared__ double sE[2][3][Z::NN];
    int x0, y0, zs, ze;
    zm_block(gx, gy, zc, F.nzc, x0, y0, zs, ze);
    const double* pe = fl + nnode;
    const int t = threadIdx.x, tx = t % Z::X, ty = t / Z::X;
    const int ci = x0 + tx, cj = y0 + ty;
    const bool own = ci < F.nx && cj < F.nyc;
    ZPlane pl;
    ZFluid fn[Z::IN];

    // E at node plane k into sE[slot], ring positions of its B / p_e planes given
    auto node_plane = [&](int slot, int b0, int b1, int p0, int p1, int p2) {
#pragma unroll
        for (int it = 0; it < Z::IN; ++it) {
            const int l = t + 256 * it;
            if (it + 1 < Z::IN || l < Z::NN) {
                // nodes flagged !ok keep the motional field: the inflow node
                // needs exactly that, nodes past the box are never read (this
                // costs fewer registers than overwriting the inflow node after
                // Ohm's law)
                double e[3], bb[3];
                inflow_E(F, e);
                if (fn[it].ok) zm_ohm(F, sB[b0], sB[b1], sP[p0], sP[p1], sP[p2], fn[it], l % Z::NX, l / Z::NX, e, bb);
                wall_E(F, x0 + l % Z::NX, e);
                sE[slot][0][l] = e[0]; sE[slot][1][l] = e[1]; sE[slot][2][l] = e[2];
            }
        }
    };
    auto fetch_fluid = [&](int k) {
#pragma unroll
        for (int it = 0; it < Z::IN; ++it) {
            const int l = t + 256 * it;
            fn[it].ok = false;
            if (it + 1 < Z::IN || l < Z::NN) zm_fetch_fluid(F, fl, nnode, x0, y0, k, l % Z::NX, l / Z::NX, fn[it]);
            if (inflow_node(F, x0 + l % Z::NX)) fn[it].ok = false;   // motional field, not Ohm's law
        }
    };

    // prologue: B planes zs-1, zs; p_e planes zs-1 .. zs+1; E at node plane zs
    zm_fetch_B(F, Bin, ncent, x0, y0, zs - 1, pl);
    zm_fetch_P(F, pe, x0, y0, zs - 1, pl);
    zm_store_B(pl, sB[0]);
    zm_store_P(pl, sP[0]);
    zm_fetch_B(F, Bin, ncent, x0, y0, zs, pl);
    zm_fetch_P(F, pe, x0, y0, zs, pl);
    zm_store_B(pl, sB[1]);
    zm_store_P(pl, sP[1]);
    zm_fetch_P(F, pe, x0, y0, zs + 1, pl);
    fetch_fluid(zs);
    zm_store_P(pl, sP[2]);
    __syncthreads();
    node_plane(0, 0, 1, 0, 1, 2);
    const int lc = (tx + 1) + Z::CX * (ty + 1);
    // this thread's own centre of plane k, read from the ring before its slot is reused
    double bk[3] = {sB[1][0][lc], sB[1][1][lc], sB[1][2][lc]};
    __syncthreads();

    for (int k = zs; k < ze; ++k) {
        const int r = k - zs;
        // global loads of the next planes, then into their ring slots: B plane
        // k+1 replaces k-1, p_e plane k+2 replaces k-1
        zm_fetch_B(F, Bin, ncent, x0, y0, k + 1, pl);
        zm_fetch_P(F, pe, x0, y0, k + 2, pl);
        fetch_fluid(k + 1);
        zm_store_B(pl, sB[r & 1]);
        zm_store_P(pl, sP[r % 3]);
        __syncthreads();
        node_plane((r + 1) & 1, (r + 1) & 1, r & 1, (r + 1) % 3, (r + 2) % 3, r % 3);
        const double bk1[3] = {sB[r & 1][0][lc], sB[r & 1][1][lc], sB[r & 1][2][lc]};
        __syncthreads();
        if (own) {
            // Bn is read here rather than ahead of the node plane: held across
            // Ohm's law its registers cost the kernel a wave per SIMD
            double bn[3] = {0, 0, 0};
            const long q = lin(ci, cj, k, F.nx, F.nyc);
            if (c0 != 0.0) { bn[0] = Bn[q]; bn[1] = Bn[ncent + q]; bn[2] = Bn[2 * ncent + q]; }
            const double(*E0)[Z::NN] = sE[r & 1];
            const double(*E1)[Z::NN] = sE[(r + 1) & 1];
            double dEx[3] = {0, 0, 0}, dEy[3] = {0, 0, 0}, dEz[3] = {0, 0, 0};
            auto at = [&](int a, int b) { return (tx + a) + Z::NX * (ty + b); };
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    dEx[d] += (E0[d][at(1, b)] - E0[d][at(0, b)]) + (E1[d][at(1, b)] - E1[d][at(0, b)]);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    dEy[d] += (E0[d][at(a, 1)] - E0[d][at(a, 0)]) + (E1[d][at(a, 1)] - E1[d][at(a, 0)]);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int d = 0; d < 3; ++d) dEz[d] += E1[d][at(a, b)] - E0[d][at(a, b)];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                dEx[d] = dEx[d] * 0.25 * F.rdx;
                dEy[d] = dEy[d] * 0.25 * F.rdx;
                dEz[d] = dEz[d] * 0.25 * F.rdx;
            }
            const double rhs[3] = {-(dEy[2] - dEz[1]), -(dEz[0] - dEx[2]), -(dEx[1] - dEy[0])};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double sv = bk[d] + h * rhs[d];
                Bout[(long)d * ncent + q] = c0 == 0.0 ? c1 * sv : c0 * bn[d] + c1 * sv;
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) bk[d] = bk1[d];
    }
}

// Final Ohm's law in 3D (see k_ohm), marching through node planes.
template <typename R>
__global__ __launch_bounds__(256) void k_ohm3(FieldGeo F, const double* __restrict__ B, const double* __restrict__ fl,
                                              double* __restrict__ E, R* __restrict__ gather, long nnode, long ncent,
                                              int gx, int gy, int zc) {
    using Z = ZMarch;
    __shared__ double sB[2][3][Z::CN];
    __shared__ double sP[3][Z::PN];
    int x0, y0, zs, ze;
    zm_block(gx, gy, zc, F.nzc, x0, y0, zs, ze);
    const double* pe = fl + nnode;
    const int t = threadIdx.x, tx = t % Z::X, ty = t / Z::X;
    const bool own = x0 + tx < F.nxn && y0 + ty < F.nyc;
    ZPlane pl;
    zm_fetch_B(F, B, ncent, x0, y0, zs - 1, pl);
    zm_fetch_P(F, pe, x0, y0, zs - 1, pl);
    zm_store_B(pl, sB[0]);
    zm_store_P(pl, sP[0]);
    zm_fetch_P(F, pe, x0, y0, zs, pl);
    zm_store_P(pl, sP[1]);
    for (int k = zs; k < ze; ++k) {
        const int r = k - zs;
        zm_fetch_B(F, B, ncent, x0, y0, k, pl);
        zm_fetch_P(F, pe, x0, y0, k + 1, pl);
        ZFluid f;
        f.ok = false;
        if (own) zm_fetch_fluid(F, fl, nnode, x0, y0, k, tx, ty, f);
        zm_store_B(pl, sB[(r + 1) & 1]);
        zm_store_P(pl, sP[(r + 2) % 3]);
        __syncthreads();
        if (own) {
            double e[3], bb[3];
            zm_ohm(F, sB[r & 1], sB[(r + 1) & 1], sP[r % 3], sP[(r + 1) % 3], sP[(r + 2) % 3], f, tx, ty, e, bb);
            if (inflow_node(F, x0 + tx)) inflow_E(F, e);
            wall_E(F, x0 + tx, e);
#pragma unroll
            for (int d = 0; d < 3; ++d) E[(long)d * nnode + f.n] = e[d];
            store_gather(gather + 6 * f.n, e, bb);
        }
        __syncthreads();
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
__device__ __forceinline__ long gcd_l(long a, long b) {
    while (b != 0) { long t = a % b; a = b; b = t; }
    return a;
}

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
    // Slot within the tile bin: a stride permutation of (cell, q) order.  The
    // order of ions in a bin is arbitrary; a scattered one keeps the lanes of
    // a wave in different cells, as the ion order becomes after a few hundred
    // steps of flow anyway, so that they rarely hit one LDS address together.
    const int ez = D >= 3 ? min(T::Z, G.nzc - tz * T::Z) : 1;
    const long nt = (long)ex * (D >= 2 ? ey : 1) * ez * ppc;
    long m = ((long)(0.6180339887 * (double)nt)) | 1;
    while (gcd_l(m, nt) != 1) m += 2;
    long dst = (long)tile * cap + ((long)(lc * ppc + q) * m) % nt;
    out.cell[dst] = pack_cell(cx, cy, cz, G);
    out.off[0][dst] = to_offset<R>(U[0]);
    if constexpr (D >= 2) out.off[1][dst] = to_offset<R>(U[1]);
    if constexpr (D >= 3) out.off[2][dst] = to_offset<R>(U[2]);
    double v[3] = {G.u_sh + G.sigma * n1, G.sigma * n2, G.sigma * n3};
    if (G.c_light > 0.0) {   // relativistic mode: store the four-velocity
        const double g = 1.0 / sqrt(1.0 - (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / (G.c_light * G.c_light));
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] *= g;
    }
    out.v[0][dst] = (R)v[0];
    out.v[1][dst] = (R)v[1];
    out.v[2][dst] = (R)v[2];
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
__global__ void k_fill_u8(uint8_t* p, uint8_t v, long n) {
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

// Checkpoint: the live ions of each tile, packed tile after tile at the
// offsets toff, in the particle buffers' own section layout.
template <typename R, int D>
__global__ void k_ckpt_pack(Geo G, PBuf<R> in, const int32_t* __restrict__ cnt, const int64_t* __restrict__ toff,
                            int64_t cap, PBuf<R> out) {
    const int tile = blockIdx.x;
    const int lo = cnt[tile];
    const int n = min(lo + cnt[G.ntiles + tile], (int)cap);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const long src = bin_slot(tile, cap, lo, i), dst = toff[tile] + i;
        out.cell[dst] = in.cell[src];
#pragma unroll
        for (int d = 0; d < D; ++d) out.off[d][dst] = in.off[d][src];
#pragma unroll
        for (int c = 0; c < 3; ++c) out.v[c][dst] = in.v[c][src];
        out.id[dst] = in.id[src];
    }
}

// Restore: tile t's packed ions back into the bottom of its bin (counts lo =
// n_t, hi = 0).  toff has been checked on the host: ascending, n_t <= cap.
template <typename R, int D>
__global__ void k_ckpt_unpack(Geo G, PBuf<R> in, const int64_t* __restrict__ toff, int64_t cap, PBuf<R> out,
                              int32_t* cnt) {
    const int tile = blockIdx.x;
    const long b = toff[tile];
    const int n = (int)(toff[tile + 1] - b);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const long src = b + i, dst = (long)tile * cap + i;
        out.cell[dst] = in.cell[src];
#pragma unroll
        for (int d = 0; d < D; ++d) out.off[d][dst] = in.off[d][src];
#pragma unroll
        for (int c = 0; c < 3; ++c) out.v[c][dst] = in.v[c][src];
        out.id[dst] = in.id[src];
    }
    if (threadIdx.x == 0) {
        cnt[tile] = n;
        cnt[G.ntiles + tile] = 0;
    }
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

// Precursor loss of the reverse-mode workload, L = sum over the cell
// centres with x index i >= nx/2 of B_y^2 + B_z^2.  k_loss_part: workgroup b
// of a fixed grid sums a fixed strided share of the precursor half-rows into
// part[b]; k_loss_final adds the partials in a fixed order, so the value
// does not depend on scheduling.
constexpr int kLossParts = 1024;   // largest grid of k_loss_part (partials)

__global__ __launch_bounds__(256) void k_loss_part(FieldGeo F, const double* __restrict__ B, long ncent,
                                                   double* __restrict__ part) {
    __shared__ double sh[256];
    const long h0 = F.nx / 2, nh = F.nx - h0;
    const long total = nh * (ncent / F.nx);
    double acc = 0.0;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
        const long n = (h0 + t % nh) + (long)F.nx * (t / nh);
        const double by = B[ncent + n], bz = B[2 * ncent + n];
        acc += by * by + bz * bz;
    }
    const double sum = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = sum;
}

__global__ __launch_bounds__(256) void k_loss_final(const double* __restrict__ part, int nparts,
                                                    double* __restrict__ out) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += part[i];
    const double sum = block_sum(acc, sh);
    if (threadIdx.x == 0) *out = sum;
}

// Seed of the reverse sweep: lB = dL/dB of the precursor loss,
// (0, 2 B_y, 2 B_z) at centres with i >= nx/2 and 0 elsewhere.
__global__ __launch_bounds__(256) void k_loss_seed(FieldGeo F, const double* __restrict__ B, long ncent,
                                                   double* __restrict__ lB) {
    const long n = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= ncent) return;
    const bool pre = (int)(n % F.nx) >= F.nx / 2;
    lB[n] = 0.0;
    lB[ncent + n] = pre ? 2.0 * B[ncent + n] : 0.0;
    lB[2 * ncent + n] = pre ? 2.0 * B[2 * ncent + n] : 0.0;
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
// Kinetic energy per unit mass summed over a tile: |v|^2 / 2, or in
// relativistic mode (gamma - 1) c^2 = |u|^2 / (gamma + 1).
__global__ __launch_bounds__(256) void k_diag_kin(PBuf<R> in, const int32_t* cnt, int ntiles, int64_t cap, double ic2,
                                                  double* part) {
    __shared__ double sh[256];
    int tile = blockIdx.x;
    int lo = cnt[tile];
    int n = min(lo + cnt[ntiles + tile], (int)cap);
    double s = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        long src = bin_slot(tile, cap, lo, i);
        double a = in.v[0][src], b = in.v[1][src], c = in.v[2][src];
        const double uu = a * a + b * b + c * c;
        s += ic2 != 0.0 ? uu / (sqrt(1.0 + uu * ic2) + 1.0) : 0.5 * uu;
    }
    double t = block_sum(s, sh);
    if (threadIdx.x == 0) part[tile] = t;
}

// Momentum phase space (the paper's phase-space and spectrum figures): one
// count per ion into (x bin, momentum bin).  The binned quantity is |p|^2 =
// (p_x p_x + p_y p_y) + p_z p_z against the squared edges (comp < 0) or the
// component p_comp against the edges, all FP64 without contraction, so the
// counts are an exact function of the stored state; p is the stored velocity
// variable (the four-velocity in relativistic mode).  Ions outside the edges
// are not counted.
template <typename R>
__global__ __launch_bounds__(256) void k_phase_space(Geo G, PBuf<R> in, const int32_t* cnt, int ntiles, int64_t cap,
                                                     int comp, int xpb, int nxb, int nb,
                                                     const double* __restrict__ edges,
                                                     unsigned long long* __restrict__ counts) {
#pragma clang fp contract(off)
    const int tile = blockIdx.x;
    const int lo = cnt[tile];
    const int n = min(lo + cnt[ntiles + tile], (int)cap);
    auto edge = [&](int j) {
        const double e = edges[j];
        return comp < 0 ? e * e : e;
    };
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const long src = bin_slot(tile, cap, lo, i);
        double q;
        if (comp < 0) {
            const double a = in.v[0][src], b = in.v[1][src], c = in.v[2][src];
            q = a * a + b * b + c * c;
        } else {
            q = (double)in.v[comp][src];
        }
        if (!(edge(0) <= q) || !(q < edge(nb))) continue;
        int a = 0, b = nb;   // edge(a) <= q < edge(b)
        while (b - a > 1) {
            const int mid = (a + b) >> 1;
            if (edge(mid) <= q) a = mid;
            else b = mid;
        }
        // a cell outside the box (only a corrupt state has one) is not counted
        const int xb = cell_x(in.cell[src], G) / xpb;
        if ((unsigned)xb >= (unsigned)nxb) continue;
        atomicAdd(counts + (long)xb * nb + a, 1ull);
    }
}

// Twiddles of the x transform: (cos, sin)(2 pi m / nx), m = 0 .. nx-1.
__global__ void k_twiddles(int nx, double* tw) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nx) return;
    double s, c;
    sincospi(2.0 * (double)m / (double)nx, &s, &c);
    tw[2 * m] = c;
    tw[2 * m + 1] = s;
}

// Perpendicular power spectrum along x, partial sum over one group of (y, z)
// lines: thread k accumulates |sum_x By(x) e^{-2 pi i k x / nx}|^2 plus the
// same for Bz over the group's lines.  The phase index k x mod nx advances by
// k per cell, so the twiddle table replaces every transcendental; the groups
// are summed in a fixed order afterwards (deterministic result).
__global__ __launch_bounds__(256) void k_bperp_dft(FieldGeo F, const double* __restrict__ B, long ncent,
                                                   const double* __restrict__ tw, int nk, int ngroups,
                                                   double* __restrict__ part) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (k >= nk) return;
    const long nlines = (long)F.nyc * F.nzc;
    const long l0 = nlines * g / ngroups, l1 = nlines * (g + 1) / ngroups;
    double acc = 0.0;
    for (long l = l0; l < l1; ++l) {
        const double* by = B + ncent + (long)F.nx * l;
        const double* bz = B + 2 * ncent + (long)F.nx * l;
        double yr = 0.0, yi = 0.0, zr = 0.0, zi = 0.0;
        int m = 0;
        for (int x = 0; x < F.nx; ++x) {
            const double c = tw[2 * m], s = tw[2 * m + 1], a = by[x], b = bz[x];
            yr += a * c; yi -= a * s;
            zr += b * c; zi -= b * s;
            m += k;
            if (m >= F.nx) m -= F.nx;
        }
        acc += yr * yr + yi * yi + zr * zr + zi * zi;
    }
    part[(long)g * nk + k] = acc;
}

// Sum of the groups in order, normalised to the mean over lines of
// |B^_y(k)|^2 + |B^_z(k)|^2 with B^(k) = (1/nx) sum_x B(x) e^{-2 pi i k x / nx}.
__global__ void k_bperp_reduce(int nk, int ngroups, double norm, const double* __restrict__ part, double* out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nk) return;
    double s = 0.0;
    for (int g = 0; g < ngroups; ++g) s += part[(long)g * nk + k];
    out[k] = s * norm;
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
