// fs_adjoint.h -- reverse-mode (adjoint) kernels of the faux-shock hybrid step.
//
// The derivative is that of the continuous-deposit step (real shape weights,
// FP64 moments) with every discrete decision of the forward run held fixed:
// the cell of each ion, FS reflections (the eq. 1 decision), removals,
// injection counts and the density floor.  The FS kick that follows a
// reflection is differentiated, including its dependence on u2 = u_sh / r;
// the reflecting wall's mirror (x' = 2L - x, v_x' = -v_x) is its own
// transpose on the x components.
//
// One reverse step n+1 -> n, given the adjoints lam(B^{n+1}), lam(E^{n+1}),
// lam(Bbar^{n+1}) and the particle adjoints lam(x^{n+1}), lam(v^{n+1/2}):
//   final Ohm^T -> SSP-RK3^T (the stages kept by the recorded step, or
//   recomputed) -> fluid^T -> injection^T of the injected ions -> for every
//   other ion deposit^T at n+1 -> (FS kick^T) -> move^T -> Boris^T ->
//   gather^T, in one pass.
// The reverse pass reads its particle states from a tape packed to the live
// ions (tile t's ions at [toff[t], toff[t + 1]) in bin order), each with the
// record of the step that leaves it in packed indices of the next state.
// Particle adjoints are stored in the particle precision and indexed like
// the packed states, in two buffers: a reverse step reads the adjoints after
// the step at the packed index the record gives for each ion and writes
// those before it at the ion's own packed index, so every particle pass
// streams its arrays in the same order as the packed state (an ion removed
// by the step gets zero).  Grid adjoints are FP64.  The push pass
// accumulates per tile in LDS (FP64 atomics) and flushes once per node.
#pragma once
#include "fs_field.h"

namespace fsk {

// Planar particle adjoints of one species in one buffer, one entry per
// packed index of that species' tape states: x[d] (d < D, per cell of
// position) and v[3].
template <typename R> struct PLam {
    R* x[3];
    R* v[3];
};

// a[i] for a loop index the compiler keeps rolled (an unrolled select, so
// that a stays in registers).
template <typename T> __device__ __forceinline__ T pick3(const T a[3], int i) {
    return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]);
}

// Real shape weights in FP64 and their derivatives d/d(offset).
template <int S> __device__ __forceinline__ void weights_dw(double o, int& rel, double w[3], double dw[3]) {
    if constexpr (S == 1) {
        rel = 0; w[0] = 1.0 - o; w[1] = o; w[2] = 0.0;
        dw[0] = -1.0; dw[1] = 1.0; dw[2] = 0.0;
    } else {
        double xi = o;
        rel = -1;
        if (o >= 0.5) { xi = o - 1.0; rel = 0; }
        w[0] = 0.5 * (0.5 - xi) * (0.5 - xi);
        w[1] = 0.75 - xi * xi;
        w[2] = 0.5 * (0.5 + xi) * (0.5 + xi);
        dw[0] = -(0.5 - xi); dw[1] = -2.0 * xi; dw[2] = 0.5 + xi;
    }
}

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// Transpose of the Boris map v^{n-1/2} -> v^{n+1/2} (half-step h = dt/2):
// lo = lam(v^{n+1/2}) -> lam(v^{n-1/2}), lam(E), lam(B).
__device__ __forceinline__ void boris_vjp(const double v[3], const double E[3], const double B[3], double h,
                                          const double lo[3], double lv[3], double lE[3], double lB[3]) {
    double vm[3], t[3], s[3], vp[3], c1[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) { vm[d] = v[d] + h * E[d]; t[d] = h * B[d]; }
    const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    const double den = 1.0 + tt;
#pragma unroll
    for (int d = 0; d < 3; ++d) s[d] = 2.0 * t[d] / den;
    cross3(vm, t, c1);
#pragma unroll
    for (int d = 0; d < 3; ++d) vp[d] = vm[d] + c1[d];
    double lvp[3], ls[3], lt[3], tmp[3];
    cross3(s, lo, lvp);
    cross3(lo, vp, ls);
    cross3(t, lvp, tmp);
    double lvm[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) lvm[d] = lo[d] + lvp[d] + tmp[d];
    cross3(lvp, vm, lt);
    const double ts = t[0] * ls[0] + t[1] * ls[1] + t[2] * ls[2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lt[d] += 2.0 * ls[d] / den - 4.0 * t[d] * ts / (den * den);
        lB[d] = h * lt[d];
        lv[d] = lvm[d];
        lE[d] = h * lo[d] + h * lvm[d];
    }
}

// Transpose of the FS kick of a reflected ion (reading of the kick in the
// paper's Sec. 2: |w| kept, mu' = a + (1 - a) sqrt(U3), azimuth 2 pi U4,
// re-entry at x' = nx + delta v'_x / v_x).  Inputs: pre-wall velocity v,
// overshoot delta (cells), lam(x'), lam(v').  Outputs lam(delta) (= lam of
// the pre-wall x), lam(v) and the u2 adjoint.
__device__ __forceinline__ void kick_vjp(uint64_t seed, uint64_t step, uint32_t id, double u2, double nx,
                                         const double v[3], double delta, double lx, const double lvo[3],
                                         double& lxpre, double lv[3], double& lu2) {
    const double wv[3] = {v[0] - u2, v[1], v[2]};
    const double wabs = sqrt(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
    double U[4];
    draw4(seed, kStreamWall, step, (uint64_t)id, 0, U);
    const double a = u2 / wabs, su = sqrt(U[2]);
    const double mu = a + (1.0 - a) * su;
    const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    const double phi = kTwoPi * U[3], cp = cos(phi), sp = sin(phi);
    const double vox = u2 - wabs * mu;
    double lvox = lvo[0];
    double ldelta = 0.0, lvx_direct = 0.0;
    const double xnew = nx - (v[0] > 0.0 ? delta * (-vox) / v[0] : 0.0);
    if (v[0] > 0.0 && xnew < nx) {
        ldelta = lx * vox / v[0];
        lvox += lx * delta / v[0];
        lvx_direct = -lx * delta * vox / (v[0] * v[0]);
    }
    lxpre = ldelta;
    double lu = lvox;
    double lwabs = -mu * lvox + st * (cp * lvo[1] + sp * lvo[2]);
    double lmu = -wabs * lvox;
    const double lst = wabs * (cp * lvo[1] + sp * lvo[2]);
    if (st > 0.0) lmu += -mu / st * lst;
    const double la = lmu * (1.0 - su);
    lu += la / wabs;
    lwabs += -la * u2 / (wabs * wabs);
#pragma unroll
    for (int d = 0; d < 3; ++d) lv[d] = lwabs * wv[d] / wabs;
    lu += -lv[0];
    lv[0] += lvx_direct;
    lu2 = lu;
}

// Sum of a per-thread double over the block, added to *out by one lane.
__device__ __forceinline__ void block_add(double v, double* out) {
    __shared__ double red[32];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if (__lane_id() == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < nw; ++i) s += red[i];
        if (s != 0.0) unsafeAtomicAdd(out, s);
    }
}

// ---------------------------------------------------------------------------
// Particle passes.  A tile's ions may be spread over `split` workgroups
// (consecutive blocks), each taking a contiguous share of the bin, so that
// few large tiles still fill the chip.
// ---------------------------------------------------------------------------
// The share of a packed tile's ions one workgroup takes: tiles with many
// ions are split over `split` workgroups (blockIdx.x = tile * split + part).
struct PackShare {
    int tile;
    long begin, end;
};
__device__ __forceinline__ PackShare pack_share(const int32_t* toff, int64_t n, int split) {
    PackShare r;
    r.tile = blockIdx.x / split;
    const int part = blockIdx.x % split;
    const long b = min((long)toff[r.tile], (long)n), e = min((long)toff[r.tile + 1], (long)n);
    const long len = e > b ? e - b : 0;
    const long chunk = (len + split - 1) / split;
    r.begin = b + min(len, part * chunk);
    r.end = min(e, r.begin + chunk);
    return r;
}

// ---------------------------------------------------------------------------
// The tape: particle states packed to their live ions
// ---------------------------------------------------------------------------

// Tile offsets of a packed state, toff[t] = ions of the tiles before t, in
// two launches over chunks of kScanChunk tiles, one workgroup of 1024
// threads a chunk, four adjacent tiles a thread (neighbouring threads read
// neighbouring counts): k_tape_chunks sums each chunk's live counts into
// part[c]; k_tape_offsets then scans its chunk (a wave scan and a scan of
// the 16 wave totals) from the sum of the chunks before it.  The last
// chunk's workgroup writes toff[ntiles] and sets *status when the total
// exceeds n.
constexpr int kScanChunk = 4096;

__device__ __forceinline__ long long live_count(const int32_t* __restrict__ cnt, int ntiles, int64_t cap, int i) {
    return i < ntiles ? min((long long)cnt[i] + cnt[ntiles + i], (long long)cap) : 0;
}

__global__ __launch_bounds__(1024) void k_tape_chunks(const int32_t* __restrict__ cnt, int ntiles, int64_t cap,
                                                      long long* __restrict__ part) {
    __shared__ long long wsum[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int base = blockIdx.x * kScanChunk;
    long long x = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) x += live_count(cnt, ntiles, cap, base + 4 * t + u);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if (lane == 0) wsum[w] = x;
    __syncthreads();
    if (t == 0) {
        long long tot = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) tot += wsum[q];
        part[blockIdx.x] = tot;
    }
}

__global__ __launch_bounds__(1024) void k_tape_offsets(const int32_t* __restrict__ cnt, int ntiles, int64_t cap,
                                                       const long long* __restrict__ part,
                                                       int32_t* __restrict__ toff, int64_t n,
                                                       int32_t* __restrict__ status) {
    __shared__ long long wsum[16];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int chunk = blockIdx.x, base = chunk * kScanChunk;
    long long carry = 0;
    for (int c = 0; c < chunk; ++c) carry += part[c];
    long long c4[4], loc = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        c4[u] = live_count(cnt, ntiles, cap, base + 4 * t + u);
        loc += c4[u];
    }
    long long x = loc;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const long long y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    long long before = 0, total = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const long long v = wsum[q];
        before += q < w ? v : 0;
        total += v;
    }
    long long run = carry + before + x - loc;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = base + 4 * t + u;
        if (i < ntiles) toff[i] = (int32_t)run;
        run += c4[u];
    }
    if (t == 0 && chunk == (int)gridDim.x - 1) {
        toff[ntiles] = (int32_t)(carry + total);
        if (carry + total > n) *status = 1;
    }
}

// The ranks [begin, end) of a tile's m live ions that workgroup `part` of
// the tile's `split` takes.
struct RankShare {
    int tile, begin, end;
};
__device__ __forceinline__ RankShare rank_share(const int32_t* cnt, int ntiles, int64_t cap, int split, int& lo) {
    RankShare r;
    r.tile = blockIdx.x / split;
    const int part = blockIdx.x % split;
    lo = cnt[r.tile];
    const int m = min(lo + cnt[ntiles + r.tile], (int)cap);
    const int chunk = (m + split - 1) / split;
    r.begin = min(m, part * chunk);
    r.end = min(m, r.begin + chunk);
    return r;
}

// Copy of every tile's live ions, in bin order, to its packed range (ions
// past n are dropped; k_tape_offsets flagged them); `split` workgroups a
// tile.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_tape_pack(Geo G, PBuf<R> in, const int32_t* __restrict__ cnt, int64_t cap,
                                                   const int32_t* __restrict__ toff, int64_t n, PBuf<R> out,
                                                   int split) {
    int lo;
    const RankShare rs = rank_share(cnt, G.ntiles, cap, split, lo);
    const int tile = rs.tile;
    const long base = toff[tile];
    for (int i = rs.begin + threadIdx.x; i < rs.end; i += blockDim.x) {
        const long dst = base + i;
        if (dst >= n) break;
        const long src = bin_slot(tile, cap, lo, i);
        out.cell[dst] = in.cell[src];
#pragma unroll
        for (int d = 0; d < D; ++d) out.off[d][dst] = in.off[d][src];
#pragma unroll
        for (int c = 0; c < 3; ++c) out.v[c][dst] = in.v[c][src];
        out.id[dst] = in.id[src];
    }
}

// A packed state back into bins: tile t's ions [toff[t], toff[t + 1]) to
// the bottom run of its bin (slots t cap .. t cap + m - 1, counts (m, 0)),
// in packed order; `split` workgroups a tile.  Workgroup 0 sets the total
// count.  A tile with more than cap ions sets *status (those beyond are
// dropped).
template <typename R, int D>
__global__ __launch_bounds__(256) void k_tape_unpack(Geo G, PBuf<R> in, const int32_t* __restrict__ toff, int64_t n,
                                                     PBuf<R> out, int32_t* __restrict__ cnt, int64_t cap,
                                                     long long* __restrict__ count, int split,
                                                     int32_t* __restrict__ status) {
    const int tile = blockIdx.x / split, part = blockIdx.x % split;
    const long b = min((long)toff[tile], (long)n), e = min((long)toff[tile + 1], (long)n);
    const long m = e > b ? e - b : 0;
    const long kept = min(m, (long)cap);
    if (part == 0 && threadIdx.x == 0) {
        cnt[tile] = (int32_t)kept;
        cnt[G.ntiles + tile] = 0;
        if (m > cap) *status = 1;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = min((long)toff[G.ntiles], (long)n);
    const long chunk = (kept + split - 1) / split;
    const long r0 = min(kept, (long)part * chunk), r1 = min(kept, r0 + chunk);
    for (long i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
        const long src = b + i, dst = (long)tile * cap + i;
        out.cell[dst] = in.cell[src];
#pragma unroll
        for (int d = 0; d < D; ++d) out.off[d][dst] = in.off[d][src];
#pragma unroll
        for (int c = 0; c < 3; ++c) out.v[c][dst] = in.v[c][src];
        out.id[dst] = in.id[src];
    }
}

// A step's record from bin slots to packed indices: for each ion of the
// input state (tile t, rank i in its bin, packed at toff_in[t] + i), the
// output bin slot it went to, turned into the packed index of the output
// state (the slot's tile, its rank in that bin); `split` workgroups a tile.
__global__ __launch_bounds__(256) void k_tape_record(Geo G, const int32_t* __restrict__ cnt_in, int64_t cap,
                                                     const int32_t* __restrict__ toff_in, int64_t n_in,
                                                     const int32_t* __restrict__ dst_bin,
                                                     const int32_t* __restrict__ cnt_out,
                                                     const int32_t* __restrict__ toff_out, int64_t n_out,
                                                     int32_t* __restrict__ dst, int32_t* __restrict__ status, int split) {
    int lo;
    const RankShare rs = rank_share(cnt_in, G.ntiles, cap, split, lo);
    const int tile = rs.tile;
    const long base = toff_in[tile];
    // most ions stay in their tile: its output count and offset, read once
    const int lo_own = cnt_out[tile];
    const long toff_own = toff_out[tile];
    for (int i = rs.begin + threadIdx.x; i < rs.end; i += blockDim.x) {
        const long p = base + i;
        if (p >= n_in) break;
        const int32_t d = dst_bin[bin_slot(tile, cap, lo, i)];
        int32_t r = -1;
        if (d != -1) {
            // slots fit int32 (the record's encoding)
            const unsigned slot = d >= 0 ? (unsigned)d : (unsigned)(-2 - d), ucap = (unsigned)cap;
            const unsigned own0 = (unsigned)tile * ucap;
            const bool stay = slot - own0 < ucap;
            const int t2 = stay ? tile : (int)(slot / ucap);
            const int j = (int)(slot - (unsigned)t2 * ucap);
            const int lo2 = stay ? lo_own : cnt_out[t2];
            const long q = (stay ? toff_own : (long)toff_out[t2]) + (j < lo2 ? j : lo2 + (int)(cap - 1 - j));
            if (q < n_out) r = d >= 0 ? (int32_t)q : (int32_t)(-2 - q);
            else *status = 1;
        }
        dst[p] = r;
    }
}

// u_sh adjoint of one ion injected during the step (reading of the
// injection: thermal v_x = |u_sh + sigma n1| entering at x = v_x U0 dt/dx;
// CRs with |w| = cr_w, mu = a + (1 - a) sqrt(U2), a = u2 / |w|, entering at
// x = nx - |v_x| U0 dt/dx), from its adjoints lx (x) and lv after the step.
__device__ __forceinline__ double inject_vjp(const Geo& G, uint64_t step, uint64_t id, bool cr, double lx,
                                             const double lv[3]) {
    const double dtdx = G.dt / G.dx;
    double U[4];
    if (!cr) {
        double V[4], n1, n2;
        draw4(G.seed, kStreamInjectTh, step, id, 0, U);
        draw4(G.seed, kStreamInjectTh, step, id, 1, V);
        box_muller(V[0], V[1], n1, n2);
        const double vx = G.u_sh + G.sigma * n1;
        const double sg = vx >= 0.0 ? 1.0 : -1.0;
        const double xi = fabs(vx) * U[0] * dtdx;
        return lv[0] * sg + (xi < (double)G.nx ? lx * sg * U[0] * dtdx : 0.0);
    }
    draw4(G.seed, kStreamInjectCr, step, id, 0, U);
    const double a = G.u2 / G.cr_w, su = sqrt(U[2]);
    const double mu = a + (1.0 - a) * su;
    const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    const double phi = kTwoPi * U[3];
    const double vx = G.u2 - G.cr_w * mu;
    const double dmu = (1.0 - su) / G.cr_w;
    const double dvx = 1.0 - G.cr_w * dmu;
    const double dst = st > 0.0 ? -mu / st * dmu : 0.0;
    const double sg = vx >= 0.0 ? 1.0 : -1.0;
    const double xi = (double)G.nx - fabs(vx) * U[0] * dtdx;
    const double dxi = xi < (double)G.nx ? -sg * dvx * U[0] * dtdx : 0.0;
    return (lv[0] * dvx + lv[1] * G.cr_w * cos(phi) * dst + lv[2] * G.cr_w * sin(phi) * dst + lx * dxi) * G.rinv;
}

// Staging of the moment adjoints of a tile's stencil nodes into LDS,
// [node][R, Gx, Gy, Gz] (nodes outside the deposit grid hold zero).
template <int D, int S>
__device__ __forceinline__ void stage_moment_adj(const Geo& G, const double* __restrict__ lM, int gx0, int gy0, int gz0,
                                                 double* sm) {
    using X = Extent<D, S>;
    for (int l = threadIdx.x; l < X::GN; l += blockDim.x) {
        const int lx = l % X::GX, ly = (l / X::GX) % X::GY, lz = l / (X::GX * X::GY);
        const long gi = dep_index(gx0 + lx, gy0 + ly, gz0 + lz, G);
#pragma unroll
        for (int q = 0; q < 4; ++q) sm[4 * l + q] = gi < 0 ? 0.0 : lM[4 * gi + q];
    }
}

// Deposit transpose of one ion (cell pc, offsets o, velocity v):
// gx[d] = sum_nodes dW/dx_d (lam_R + lam_G . v) (per cell of position),
// gv = sum_nodes W lam_G.  The moment adjoints come from sm, staged for the
// nodes [gx0, gx0 + GX) x [gy0, ..) x [gz0, ..), when the ion's stencil lies
// there, else from lM in global memory.
template <typename R, int D, int S>
__device__ __forceinline__ void deposit_vjp(const Geo& G, const double* sm, const double* __restrict__ lM, int gx0,
                                            int gy0, int gz0, int32_t pc, const R* o, const R* vr, double gx[3],
                                            double gv[3]) {
    using X = Extent<D, S>;
    constexpr int N = Stencil<S>::N;
    constexpr int NY = D >= 2 ? N : 1, NZ = D >= 3 ? N : 1;
    const int cx = cell_x(pc, G), cy = D >= 2 ? cell_y(pc, G) : 0, cz = D >= 3 ? cell_z(pc, G) : 0;
    double w[3][3], dw[3][3];
    int rel[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        w[d][0] = 1.0; w[d][1] = w[d][2] = 0.0;
        dw[d][0] = dw[d][1] = dw[d][2] = 0.0;
    }
#pragma unroll
    for (int d = 0; d < D; ++d) weights_dw<S>((double)o[d], rel[d], w[d], dw[d]);
    const double v[3] = {(double)vr[0], (double)vr[1], (double)vr[2]};
    const int ax = cx + rel[0], ay = cy + rel[1], az = cz + rel[2];
    const int lx0 = ax - gx0, ly0 = D >= 2 ? ay - gy0 : 0, lz0 = D >= 3 ? az - gz0 : 0;
    const bool inside = lx0 >= 0 && lx0 <= X::GX - N && ly0 >= 0 && ly0 <= X::GY - NY && lz0 >= 0 &&
                        lz0 <= X::GZ - NZ;
#pragma unroll
    for (int d = 0; d < 3; ++d) gx[d] = gv[d] = 0.0;
    // the z planes of a 3D stencil one at a time (registers)
#pragma unroll 1
    for (int c = 0; c < NZ; ++c) {
        const double wz = pick3(w[2], c), dwz = pick3(dw[2], c);
#pragma unroll
        for (int b = 0; b < NY; ++b)
#pragma unroll
            for (int a = 0; a < N; ++a) {
                double m[4];
                if (inside) {
                    const double* ms = sm + 4 * (((lz0 + c) * X::GY + (ly0 + b)) * X::GX + (lx0 + a));
#pragma unroll
                    for (int q = 0; q < 4; ++q) m[q] = ms[q];
                } else {
                    const long gi = dep_index(ax + a, D >= 2 ? ay + b : 0, D >= 3 ? az + c : 0, G);
#pragma unroll
                    for (int q = 0; q < 4; ++q) m[q] = gi < 0 ? 0.0 : lM[4 * gi + q];
                }
                const double lm = m[0] + m[1] * v[0] + m[2] * v[1] + m[3] * v[2];
                const double W = w[0][a] * w[1][b] * wz;
                gx[0] += dw[0][a] * w[1][b] * wz * lm;
                if (D >= 2) gx[1] += w[0][a] * dw[1][b] * wz * lm;
                if (D >= 3) gx[2] += w[0][a] * w[1][b] * dwz * lm;
#pragma unroll
                for (int d = 0; d < 3; ++d) gv[d] += W * m[1 + d];
            }
    }
}

// An origin no stencil lies beyond: deposit_vjp then reads every node from
// global memory.
constexpr int kNoRegion = -(1 << 29);

// Tile origin of the staged stencil region of `tile`.
template <int D, int S>
__device__ __forceinline__ void tile_origin(const Geo& G, int tile, int& gx0, int& gy0, int& gz0) {
    using T = TileShape<D>;
    constexpr int LO = Stencil<S>::LO;
    const int tx = tile % G.ntx;
    const int ty = D >= 2 ? (tile / G.ntx) % G.nty : 0;
    const int tz = D >= 3 ? tile / (G.ntx * G.nty) : 0;
    gx0 = tx * T::X - LO;
    gy0 = D >= 2 ? ty * T::Y - LO : 0;
    gz0 = D >= 3 ? tz * T::Z - LO : 0;
}

// Deposit transpose over the ions of a packed state (the initial load):
// lam(x) += sum_nodes dW/dx (lam_R + lam_G . v), lam(v) += sum W lam_G, added
// to the adjoints at the ions' packed indices.
template <typename R, int D, int S>
__global__ __launch_bounds__(256) void k_deposit_adj(Geo G, PBuf<R> in, const int32_t* __restrict__ toff, int64_t n,
                                                     const double* __restrict__ lM, PLam<R> lam, int split) {
    using X = Extent<D, S>;
    __shared__ double sm[4 * X::GN];
    const PackShare ts = pack_share(toff, n, split);
    int gx0, gy0, gz0;
    tile_origin<D, S>(G, ts.tile, gx0, gy0, gz0);
    stage_moment_adj<D, S>(G, lM, gx0, gy0, gz0, sm);
    __syncthreads();
    for (long src = ts.begin + threadIdx.x; src < ts.end; src += blockDim.x) {
        R o[3] = {0, 0, 0}, v[3];
#pragma unroll
        for (int d = 0; d < D; ++d) o[d] = in.off[d][src];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = in.v[c][src];
        double gx[3], gv[3];
        deposit_vjp<R, D, S>(G, sm, lM, gx0, gy0, gz0, in.cell[src], o, v, gx, gv);
#pragma unroll
        for (int d = 0; d < D; ++d) lam.x[d][src] = (R)((double)lam.x[d][src] + gx[d]);
#pragma unroll
        for (int d = 0; d < 3; ++d) lam.v[d][src] = (R)((double)lam.v[d][src] + gv[d]);
    }
}

// The ions a step injected (ids id0 .. id0 + ninj - 1, thermal first, nth
// of them), found in the packed state after the step: their adjoint there
// (post plus the deposit transpose at that state) goes into dL/du_sh
// through their injection.  Injection places an ion within a bounded depth
// of its boundary, so only the tile columns [cx0, cx0 + ncols) are read,
// one workgroup per tile of them; few ions: the moment adjoints are read
// from global memory.  The workgroups count the injected ions they find
// and the last one to finish compares the total with `expect`, sets
// *status = 2 on a mismatch (an ion outside the columns) and resets ctr
// (two counters, zero between launches).
template <typename R, int D, int S>
__global__ __launch_bounds__(256) void k_inject_adj(Geo G, PBuf<R> in, const int32_t* __restrict__ toff, int64_t n,
                                                    const double* __restrict__ lM, PLam<R> post, uint64_t step,
                                                    int64_t id0, int64_t nth, int64_t ninj, int cx0, int ncols,
                                                    unsigned long long* ctr, int64_t expect, int32_t* status,
                                                    double* grads) {
    const int tile = (cx0 + (int)(blockIdx.x % ncols)) + G.ntx * (int)(blockIdx.x / ncols);
    const long b = min((long)toff[tile], (long)n), e = min((long)toff[tile + 1], (long)n);
    double acc = 0.0;
    int found = 0;
    for (long q = b + threadIdx.x; q < e; q += blockDim.x) {
        const int64_t g = (int64_t)in.id[q] - id0;
        if (g < 0 || g >= ninj) continue;
        ++found;
        R o[3] = {0, 0, 0}, v[3];
#pragma unroll
        for (int d = 0; d < D; ++d) o[d] = in.off[d][q];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = in.v[c][q];
        double gx[3], gv[3];
        // no staged region: every stencil node is read from lM
        deposit_vjp<R, D, S>(G, nullptr, lM, kNoRegion, kNoRegion, kNoRegion, in.cell[q], o, v, gx, gv);
        const double lx0 = (double)post.x[0][q] + gx[0];
        const double lv[3] = {(double)post.v[0][q] + gv[0], (double)post.v[1][q] + gv[1],
                              (double)post.v[2][q] + gv[2]};
        acc += inject_vjp(G, step, (uint64_t)(id0 + g), g >= nth, lx0, lv);
    }
    block_add(acc, grads);
    __shared__ int cnt[16];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) found += __shfl_xor(found, o);
    if (__lane_id() == 0) cnt[threadIdx.x >> 6] = found;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long tot = 0;
        for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) tot += cnt[w];
        atomicAdd(&ctr[0], (unsigned long long)tot);
        __threadfence();
        if (atomicAdd(&ctr[1], 1ull) == gridDim.x - 1) {
            const unsigned long long all = atomicAdd(&ctr[0], 0ull);
            if ((int64_t)all != expect) *status = 2;
            ctr[0] = 0;
            ctr[1] = 0;
        }
    }
}

// Particle adjoints between two packings of the same ions, matched by id
// through an id-indexed scratch (the D + 3 components of id q at
// [q (D + 3), (q + 1)(D + 3)), so a scattered ion touches one run of
// memory): k_lam_park writes the adjoints of every ion of `from` at its id,
// k_lam_unpark reads them back at the ions of `to`.  The scratch is zeroed
// first, so an id `from` lacks reads zero; ids >= nid are skipped.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_lam_park(const uint32_t* __restrict__ id, const int32_t* __restrict__ toff,
                                                  int ntiles, int64_t n, PLam<R> lam, R* __restrict__ scratch,
                                                  int64_t nid) {
    const long m = min((long)toff[ntiles], (long)n);
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (long)gridDim.x * blockDim.x) {
        const int64_t q = id[p];
        if (q >= nid) continue;
        R* o = scratch + q * (D + 3);
#pragma unroll
        for (int d = 0; d < D; ++d) o[d] = lam.x[d][p];
#pragma unroll
        for (int c = 0; c < 3; ++c) o[D + c] = lam.v[c][p];
    }
}

template <typename R, int D>
__global__ __launch_bounds__(256) void k_lam_unpark(const uint32_t* __restrict__ id, const int32_t* __restrict__ toff,
                                                    int ntiles, int64_t n, PLam<R> lam, const R* __restrict__ scratch,
                                                    int64_t nid) {
    const long m = min((long)toff[ntiles], (long)n);
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (long)gridDim.x * blockDim.x) {
        const int64_t q = id[p];
        const bool ok = q < nid;
        const R* o = scratch + (ok ? q : 0) * (D + 3);
#pragma unroll
        for (int d = 0; d < D; ++d) lam.x[d][p] = ok ? o[d] : (R)0;
#pragma unroll
        for (int c = 0; c < 3; ++c) lam.v[c][p] = ok ? o[D + c] : (R)0;
    }
}

// u_sh adjoint of the initial load (v_x = u_sh + sigma n1 for every thermal
// ion), over the packed initial state.
template <typename R>
__global__ __launch_bounds__(256) void k_init_adj(const int32_t* __restrict__ toff, int ntiles, int64_t n, PLam<R> lam,
                                                  double* grads) {
    const long m = min((long)toff[ntiles], (long)n);
    double acc = 0.0;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (long)gridDim.x * blockDim.x)
        acc += (double)lam.v[0][p];
    block_add(acc, grads);
}

// Push transpose over the ions of the packed state at n, with the deposit
// transpose of the state after the step fused in: each ion finds itself
// after the step at the packed index the step's record gives (dst >= 0
// kept, -2 - i reflected, -1 removed), takes its adjoint there from post
// plus the deposit transpose at its position and velocity there (moment
// adjoints lM; the ions the step injected are k_inject_adj's), then
// recomputes the gather, Boris and move as the forward step did, undoes
// the FS kick for the ions the step reflected, the move, Boris and the
// gather, and writes its adjoint before the step into pre at its own index,
// zero for an ion the step removed.  in1 / n1: the packed state after the
// step.  lam(E^n), lam(Bbar^n) (6 planar FP64 arrays of nnode) accumulate
// per tile in LDS.
// Workgroup size and minimum waves per SIMD the push transpose is compiled
// for.  In 3D its LDS (the FP64 lam(E, Bbar) sums, the gather grid and the
// moment adjoints of the tile's stencil: 80 KB in FP32) allows two
// workgroups per CU, so 512-thread workgroups held to 128 VGPRs run four
// waves per SIMD where 256-thread ones at their natural 166 VGPRs ran two
// (the z planes of the stencil are walked in a loop to fit, without
// spills).  The FP32 2D CIC kernel sits at 97 VGPRs, one above five waves
// (the TSC one would spill there).
template <typename R, int D, int S> struct AdjPush {
    static constexpr int threads = D == 3 ? 512 : 256;
    static constexpr int waves = sizeof(R) != 4 ? 1 : (D == 3 ? 4 : ((D == 2 && S == 1) ? 5 : 1));
};

template <typename R, int D, int S>
__global__ __launch_bounds__((AdjPush<R, D, S>::threads), (AdjPush<R, D, S>::waves)) void k_push_adj(Geo G, PBuf<R> in, const int32_t* __restrict__ toff, int64_t n,
                                                  PBuf<R> in1, const double* __restrict__ lM,
                                                  const R* __restrict__ gather, const int32_t* __restrict__ dst_of,
                                                  PLam<R> post, PLam<R> pre, double* __restrict__ lEB, long nnode,
                                                  uint64_t step, double* grads, int split, int mirror) {
    using X = Extent<D, S>;
    constexpr int N = Stencil<S>::N;
    constexpr int NY = D >= 2 ? N : 1, NZ = D >= 3 ? N : 1;
    __shared__ double sl[6 * X::GN];
    // the gather grid of the tile's stencil, as the forward push stages it
    __shared__ Pair<R> sg[3 * X::GN];
    // the moment adjoints of the same nodes (most ions stay in their tile),
    // where LDS holds them beside the rest (not the FP64 3D TSC stencil)
    constexpr bool SM = (6 * sizeof(double) + 3 * sizeof(Pair<R>) + 4 * sizeof(double)) * X::GN <= 163840;
    __shared__ double sm[SM ? 4 * X::GN : 1];
    const PackShare ts = pack_share(toff, n, split);
    int gx0, gy0, gz0;
    tile_origin<D, S>(G, ts.tile, gx0, gy0, gz0);
    if constexpr (SM) stage_moment_adj<D, S>(G, lM, gx0, gy0, gz0, sm);
    const int mx0 = SM ? gx0 : kNoRegion, my0 = SM ? gy0 : kNoRegion, mz0 = SM ? gz0 : kNoRegion;
    for (int l = threadIdx.x; l < 6 * X::GN; l += blockDim.x) sl[l] = 0.0;
    for (int l = threadIdx.x; l < X::GN; l += blockDim.x) {
        const int lx = l % X::GX, ly = (l / X::GX) % X::GY, lz = l / (X::GX * X::GY);
        const Pair<R>* g6 = reinterpret_cast<const Pair<R>*>(gather + 6 * gather_index(gx0 + lx, gy0 + ly, gz0 + lz, G));
        sg[l] = g6[0];
        sg[X::GN + l] = g6[1];
        sg[2 * X::GN + l] = g6[2];
    }
    __syncthreads();
    const R hR = (R)(0.5 * G.dt);
    const R dtdxR = (R)G.dtdx;
    const double hD = 0.5 * G.dt, dtdx = G.dtdx;
    double acc = 0.0;
    for (long src = ts.begin + threadIdx.x; src < ts.end; src += blockDim.x) {
        // the ion before the step, read in order, issued ahead of the
        // dependent reads through its record entry (its id only where the
        // wall reflected it)
        const int32_t pc = in.cell[src];
        R o[3] = {0, 0, 0}, v[3];
#pragma unroll
        for (int d = 0; d < D; ++d) o[d] = in.off[d][src];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = in.v[c][src];
        // adjoint of the ion after the step, where the step put it
        const int32_t dr = dst_of[src];
        const bool refl = dr <= -2;
        const long slot = refl ? (long)(-2 - dr) : (long)dr;
        double lx[3] = {0, 0, 0}, lv[3] = {0, 0, 0};
        bool any = false;
        if (dr != -1) {
            R o1[3] = {0, 0, 0}, v1[3];
#pragma unroll
            for (int d = 0; d < D; ++d) o1[d] = in1.off[d][slot];
#pragma unroll
            for (int c = 0; c < 3; ++c) v1[c] = in1.v[c][slot];
            double gx[3], gv[3];
            deposit_vjp<R, D, S>(G, sm, lM, mx0, my0, mz0, in1.cell[slot], o1, v1, gx, gv);
#pragma unroll
            for (int d = 0; d < D; ++d) { lx[d] = (double)post.x[d][slot] + gx[d]; any |= lx[d] != 0.0; }
#pragma unroll
            for (int d = 0; d < 3; ++d) { lv[d] = (double)post.v[d][slot] + gv[d]; any |= lv[d] != 0.0; }
        }
        if (!any) {   // removed by the step (or no influence): zero before it too
#pragma unroll
            for (int d = 0; d < D; ++d) pre.x[d][src] = (R)0;
#pragma unroll
            for (int d = 0; d < 3; ++d) pre.v[d][src] = (R)0;
            continue;
        }
        const int cx = cell_x(pc, G), cy = D >= 2 ? cell_y(pc, G) : 0, cz = D >= 3 ? cell_z(pc, G) : 0;
        // the forward gather and Boris, in the particle precision
        R wx[3], wy[3] = {1, 0, 0}, wz[3] = {1, 0, 0};
        int rx, ry = 0, rz = 0;
        weights_real<R, S>(o[0], rx, wx);
        if constexpr (D >= 2) weights_real<R, S>(o[1], ry, wy);
        if constexpr (D >= 3) weights_real<R, S>(o[2], rz, wz);
        R E[3] = {0, 0, 0}, B[3] = {0, 0, 0};
        // a binned ion lies in its tile; the clamps only guard a corrupt state
        const int lx0 = min(max(cx - gx0 + rx, 0), X::GX - N);
        const int ly0 = D >= 2 ? min(max(cy - gy0 + ry, 0), X::GY - N) : 0;
        const int lz0 = D >= 3 ? min(max(cz - gz0 + rz, 0), X::GZ - N) : 0;
#pragma unroll 1
        for (int c = 0; c < NZ; ++c)
#pragma unroll
            for (int b = 0; b < NY; ++b) {
                const R wyz = wy[b] * pick3(wz, c);
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    const R W = wx[a] * wyz;
                    const int l = ((lz0 + c) * X::GY + (ly0 + b)) * X::GX + (lx0 + a);
                    const Pair<R> p0 = sg[l], p1 = sg[X::GN + l], p2 = sg[2 * X::GN + l];
                    E[0] += W * p0.x; E[1] += W * p0.y; E[2] += W * p1.x;
                    B[0] += W * p1.y; B[1] += W * p2.x; B[2] += W * p2.y;
                }
            }
        R v1[3] = {v[0], v[1], v[2]};
        boris<R, false>(v1, E, B, hR, (R)0);   // the adjoint covers the non-relativistic push
        if (refl && mirror) {
            // the reflecting wall: x' = 2 L - x and v_x' = -v_x
            lx[0] = -lx[0];
            lv[0] = -lv[0];
        } else if (refl) {
            // overshoot as the forward move computed it
            R xi = o[0] + v1[0] * dtdxR;
            R fl = floor(xi);
            int ncx = cx + (int)fl;
            R ox = xi - fl;
            if (ox >= (R)1) { ox = (R)0; ncx += 1; }
            const double delta = (double)(ncx - G.nx) + (double)ox;
            const double vp[3] = {(double)v1[0], (double)v1[1], (double)v1[2]};
            double lxpre, lvpre[3], lu2;
            kick_vjp(G.seed, step, in.id[src], G.u2, (double)G.nx, vp, delta, lx[0], lv, lxpre, lvpre, lu2);
            acc += lu2 * G.rinv;
            lx[0] = lxpre;
#pragma unroll
            for (int d = 0; d < 3; ++d) lv[d] = lvpre[d];
        }
        // move: x^{n+1} = x^n + v^{n+1/2} dt/dx
#pragma unroll
        for (int d = 0; d < D; ++d) lv[d] += lx[d] * dtdx;
        const double vd[3] = {(double)v[0], (double)v[1], (double)v[2]};
        const double Ed[3] = {(double)E[0], (double)E[1], (double)E[2]};
        const double Bd[3] = {(double)B[0], (double)B[1], (double)B[2]};
        double lv0[3], lE[3], lB[3];
        boris_vjp(vd, Ed, Bd, hD, lv, lv0, lE, lB);
        // gather transpose
        double w[3][3], dw[3][3];
        int rel[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            w[d][0] = 1.0; w[d][1] = w[d][2] = 0.0;
            dw[d][0] = dw[d][1] = dw[d][2] = 0.0;
        }
#pragma unroll
        for (int d = 0; d < D; ++d) weights_dw<S>((double)o[d], rel[d], w[d], dw[d]);
#pragma unroll 1
        for (int c = 0; c < NZ; ++c) {
            const double wz2 = pick3(w[2], c), dwz2 = pick3(dw[2], c);
#pragma unroll
            for (int b = 0; b < NY; ++b)
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    const int l = ((lz0 + c) * X::GY + (ly0 + b)) * X::GX + (lx0 + a);
                    const Pair<R> p0 = sg[l], p1 = sg[X::GN + l], p2 = sg[2 * X::GN + l];
                    const double dot = (double)p0.x * lE[0] + (double)p0.y * lE[1] + (double)p1.x * lE[2] +
                                       (double)p1.y * lB[0] + (double)p2.x * lB[1] + (double)p2.y * lB[2];
                    const double W = w[0][a] * w[1][b] * wz2;
                    lx[0] += dw[0][a] * w[1][b] * wz2 * dot;
                    if (D >= 2) lx[1] += w[0][a] * dw[1][b] * wz2 * dot;
                    if (D >= 3) lx[2] += w[0][a] * w[1][b] * dwz2 * dot;
                    atomicAdd(&sl[l], W * lE[0]);
                    atomicAdd(&sl[X::GN + l], W * lE[1]);
                    atomicAdd(&sl[2 * X::GN + l], W * lE[2]);
                    atomicAdd(&sl[3 * X::GN + l], W * lB[0]);
                    atomicAdd(&sl[4 * X::GN + l], W * lB[1]);
                    atomicAdd(&sl[5 * X::GN + l], W * lB[2]);
                }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) pre.x[d][src] = (R)lx[d];
#pragma unroll
        for (int d = 0; d < 3; ++d) pre.v[d][src] = (R)lv0[d];
    }
    __syncthreads();
    for (int l = threadIdx.x; l < X::GN; l += blockDim.x) {
        const int lx = l % X::GX, ly = (l / X::GX) % X::GY, lz = l / (X::GX * X::GY);
        const long gi = gather_index(gx0 + lx, gy0 + ly, gz0 + lz, G);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double val = sl[k * X::GN + l];
            if (val != 0.0) unsafeAtomicAdd(lEB + (long)k * nnode + gi, val);
        }
    }
    block_add(acc, grads);
}

// ---------------------------------------------------------------------------
// Field passes (FP64, one thread per node or centre)
// ---------------------------------------------------------------------------

// Storage index of centre (i, j, k) under the ghost rules, -1 for the
// inflow ghost that holds B0.
__device__ __forceinline__ long centre_index(const FieldGeo& F, int i, int j, int k) {
    j = wrapi(j, F.nyc);
    k = wrapi(k, F.nzc);
    if (F.xbc == 1) i = wrapi(i, F.nx);
    else if (i < 0) return -1;
    else if (i >= F.nx) i = F.nx - 1;
    return i + (long)F.nx * (j + (long)F.nyc * k);
}

// Transpose of F(B) = -curl E (nodes -> centres) at node (i, j, k): lam_E
// there, gathered from lam_F of the centres that use the node.
template <int D>
__device__ __forceinline__ void faraday_adj_at(const FieldGeo& F, const double* __restrict__ lF, int i, int j, int k,
                                               long ncent, double out[3]) {
    constexpr int NB = D >= 2 ? 2 : 1, NC = D >= 3 ? 2 : 1;
    out[0] = out[1] = out[2] = 0.0;
    // node (i, j, k) = centre (ci + a, cj + b, ck + c) for a, b, c in {0, 1}
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                int ci = i - a;
                const int cj = D >= 2 ? wrapi(j - b, F.nyc) : 0, ck = D >= 3 ? wrapi(k - c, F.nzc) : 0;
                if (F.xbc == 1) ci = wrapi(ci, F.nx);
                else if (ci < 0 || ci >= F.nx) continue;
                const long q = ci + (long)F.nx * (cj + (long)F.nyc * ck);
                const double l0 = lF[q], l1 = lF[ncent + q], l2 = lF[2 * ncent + q];
                const double ldEx[3] = {0.0, -l2, l1}, ldEy[3] = {l2, 0.0, -l0}, ldEz[3] = {-l1, l0, 0.0};
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    double s = (a == 1 ? 1.0 : -1.0) * ldEx[d] * (1.0 / (double)(NB * NC)) * F.rdx;
                    if (D >= 2) s += (b == 1 ? 1.0 : -1.0) * ldEy[d] * (1.0 / (double)(2 * NC)) * F.rdx;
                    if (D >= 3) s += (c == 1 ? 1.0 : -1.0) * ldEz[d] * 0.25 * F.rdx;
                    out[d] += s;
                }
            }
}

// Transpose of Ohm's law at one node, E = (-Gamma x Bbar + J x Bbar -
// grad p_e) / n_e + eta J, from lam_E (lEn) and lam_Bbar (lBbn) to the
// adjoints of Bbar (lbb) and J (lJ), of n_e (lne) and Gamma (lG), and
// lnum = lam_E / n_e, which carries the p_e adjoint to the neighbours.  At
// the inflow node E is the motional field of the inflow (its adjoint goes
// to u_sh, not through Ohm's law); at a conducting wall E_y = E_z = 0.
__device__ __forceinline__ void ohm_adj_at(const FieldGeo& F, const double bb[3], const double J[3],
                                           const double gp[3], double ne, const double Gm[3], const double lEn[3],
                                           const double lBbn[3], bool inflow, bool conduct, double lbb[3],
                                           double lJ[3], double lnum[3], double& lne, double lG[3]) {
    double c1[3], c2[3], num[3], tmp[3];
    cross3(Gm, bb, c1);
    cross3(J, bb, c2);
#pragma unroll
    for (int d = 0; d < 3; ++d) num[d] = -c1[d] + c2[d] - gp[d];
    lne = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double le = (inflow || (conduct && d > 0)) ? 0.0 : lEn[d];
        lnum[d] = le / ne;
        lne -= num[d] * le / (ne * ne);
        lJ[d] = F.eta * le;
        lbb[d] = lBbn[d];
    }
    cross3(bb, lnum, tmp);
#pragma unroll
    for (int d = 0; d < 3; ++d) { lG[d] = -tmp[d]; lJ[d] += tmp[d]; }
    const double dv[3] = {J[0] - Gm[0], J[1] - Gm[1], J[2] - Gm[2]};
    cross3(lnum, dv, tmp);
#pragma unroll
    for (int d = 0; d < 3; ++d) lbb[d] += tmp[d];
}

// Transpose of Ohm's law, first pass, one thread per node: (lam_E,
// lam_Bbar) at the node -> the adjoints of its fluid state (n_e and Gamma of
// the node, added; p_e of its neighbours, added atomically, several nodes
// share one near a box end), of u_sh through the inflow node, and
// ob = (lam_Bbar, lam_J) of the node (6 planar arrays of nnode) for the
// centre pass.  fl is the forward fluid state the E was computed from.
// With CURL, lam_E is not read from lE but gathered from lam_F of an RK
// stage (lE then points at lam_F, 3 planar arrays of ncent): the Faraday
// transpose fused into the node pass.
template <int D, bool CURL>
__global__ __launch_bounds__(256) void k_ohm_adj_node(FieldGeo F, const double* __restrict__ B,
                                                      const double* __restrict__ fl, const double* __restrict__ lE,
                                                      const double* __restrict__ lBb, double* __restrict__ ob,
                                                      double* __restrict__ lfl, double* grads, long nnode, long ncent) {
    const int n = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (n >= nnode) return;
    const int i = n % F.nxn;
    const int rest = n / F.nxn;
    const int j = rest % F.nyc, k = rest / F.nyc;
    constexpr int NB = D >= 2 ? 2 : 1, NC = D >= 3 ? 2 : 1;
    double lEn[3];
    if constexpr (CURL) {
        faraday_adj_at<D>(F, lE, i, j, k, ncent, lEn);
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) lEn[d] = lE[(long)d * nnode + n];
    }
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
    for (int d = 0; d < 3; ++d) dBx[d] *= (1.0 / (double)(NB * NC)) * F.rdx;
    if constexpr (D >= 2) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) dBy[d] += C[a][1][c][d] - C[a][0][c][d];
#pragma unroll
        for (int d = 0; d < 3; ++d) dBy[d] *= (1.0 / (double)(2 * NC)) * F.rdx;
    }
    if constexpr (D >= 3) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int d = 0; d < 3; ++d) dBz[d] += C[a][b][1][d] - C[a][b][0][d];
#pragma unroll
        for (int d = 0; d < 3; ++d) dBz[d] *= 0.25 * F.rdx;
    }
    const double J[3] = {dBy[2] - dBz[1], dBz[0] - dBx[2], dBx[1] - dBy[0]};
    const double* pe = fl + nnode;
    const long nxp = fnode(F, i + 1, j, k), nxm = fnode(F, i - 1, j, k);
    double gp[3] = {(pe[nxp] - pe[nxm]) * 0.5 * F.rdx, 0.0, 0.0};
    long nyp = 0, nym = 0, nzp = 0, nzm = 0;
    if constexpr (D >= 2) {
        nyp = fnode(F, i, j + 1, k); nym = fnode(F, i, j - 1, k);
        gp[1] = (pe[nyp] - pe[nym]) * 0.5 * F.rdx;
    }
    if constexpr (D >= 3) {
        nzp = fnode(F, i, j, k + 1); nzm = fnode(F, i, j, k - 1);
        gp[2] = (pe[nzp] - pe[nzm]) * 0.5 * F.rdx;
    }
    const double ne = fl[n];
    const double Gm[3] = {fl[2 * nnode + n], fl[3 * nnode + n], fl[4 * nnode + n]};
    const bool inflow = inflow_node(F, i);
    const bool conduct = F.conduct && i == F.nx;
    if (inflow) unsafeAtomicAdd(grads, lEn[1] * F.B0[2] - lEn[2] * F.B0[1]);
    double lBbn[3] = {0.0, 0.0, 0.0};
    if (lBb)
#pragma unroll
        for (int d = 0; d < 3; ++d) lBbn[d] = lBb[(long)d * nnode + n];
    double lnum[3], lJ[3], lbb[3], lG[3], lne;
    ohm_adj_at(F, bb, J, gp, ne, Gm, lEn, lBbn, inflow, conduct, lbb, lJ, lnum, lne, lG);
    // fluid adjoints: n_e and Gamma belong to this node only (stored by the
    // first transpose of a step, the one without the curl, added by the
    // others), p_e to the neighbours
    if constexpr (CURL) {
        lfl[n] += lne;
#pragma unroll
        for (int d = 0; d < 3; ++d) lfl[(long)(2 + d) * nnode + n] += lG[d];
    } else {
        lfl[n] = lne;
#pragma unroll
        for (int d = 0; d < 3; ++d) lfl[(long)(2 + d) * nnode + n] = lG[d];
    }
    double* lpe = lfl + nnode;
    const double h2 = 0.5 * F.rdx;
    unsafeAtomicAdd(lpe + nxp, -lnum[0] * h2);
    unsafeAtomicAdd(lpe + nxm, lnum[0] * h2);
    if constexpr (D >= 2) {
        unsafeAtomicAdd(lpe + nyp, -lnum[1] * h2);
        unsafeAtomicAdd(lpe + nym, lnum[1] * h2);
    }
    if constexpr (D >= 3) {
        unsafeAtomicAdd(lpe + nzp, -lnum[2] * h2);
        unsafeAtomicAdd(lpe + nzm, lnum[2] * h2);
    }
    // lam(Bbar) and lam(J) for the centres around the node
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        ob[(long)d * nnode + n] = lbb[d];
        ob[(long)(3 + d) * nnode + n] = lJ[d];
    }
}

// Where the centre pass puts v = base + (its gather), per centre and
// component: the vector updates of the SSP-RK3 transpose (Shu-Osher form
// B1 = B0 + h F(B0), B2 = 3/4 B0 + 1/4 (B1 + h F(B1)),
// B3 = 1/3 B0 + 2/3 (B2 + h F(B2))) fused into the pass that completes
// the adjoint they start from.  The part of v that the next stage starts
// from (lam of B2 gets 2 v/3 from B3, lam of B1 gets v/4 from B2) is the
// lam_F the pass stores divided by h, and the next pass reads that lam_F
// anyway: the passes that emit kEmitStage2 and kEmitStage1 take their base
// as lam_F(in) / h, and no copy of it is stored.
enum RkEmit {
    kEmitOut = 0,     // out = v (out may be base)
    kEmitStage1 = 1,  // l0 += v, lF = h v          (v: lam of B1; base = lam_F(in) / h)
    kEmitStage2 = 2,  // l0 += 3/4 v, lF = h v/4    (v: lam of B2; base = lam_F(in) / h)
    kEmitStage3 = 3   // l0 = v/3, lF = 2 h v/3     (v: lam of B3)
};
struct RkOut {
    const double* base;   // kEmitOut, kEmitStage3
    double *l0, *lF, *out;
    const double* lFin;   // lam_F(in), for the base of kEmitStage1 and kEmitStage2
    double h;
};
template <int EMIT> constexpr bool kBaseFromLamF = EMIT == kEmitStage1 || EMIT == kEmitStage2;

// Transpose of Ohm's law, second pass, one thread per centre: v = base +
// the Bbar average and J differences of the 2^D nodes around the centre,
// transposed, from their (lam_Bbar, lam_J) in ob, stored as EMIT says.  In
// the box the centre next to the wall also takes the wall ghost's share of
// node nx (the ghost holds a copy of it); the inflow ghost (a constant B0)
// takes none.  base may alias l0 (each thread reads its centre before
// writing it).
template <int D, int EMIT>
__global__ __launch_bounds__(256) void k_ohm_adj_centre(FieldGeo F, const double* __restrict__ ob, RkOut o, long nnode,
                                                        long ncent) {
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= ncent) return;
    constexpr int NB = D >= 2 ? 2 : 1, NC = D >= 3 ? 2 : 1;
    const int I = q % F.nx, rest = q / F.nx;
    const int J = rest % F.nyc, K = rest / F.nyc;
    const double wbb = 1.0 / (double)(2 * NB * NC);
    const double wx = (1.0 / (double)(NB * NC)) * F.rdx, wy = (1.0 / (double)(2 * NC)) * F.rdx, wz = 0.25 * F.rdx;
    double acc[3] = {0.0, 0.0, 0.0};
    // the node whose centre (i-1+a, j-1+b, k-1+c) this is: (I+1-a, J+1-b, K+1-c)
    auto add = [&](int ni, int a, int b, int c) {
        const int nj = D >= 2 ? wrapi(J + 1 - b, F.nyc) : 0, nk = D >= 3 ? wrapi(K + 1 - c, F.nzc) : 0;
        if (F.xbc == 1) ni = wrapi(ni, F.nx);
        const long n = lin(ni, nj, nk, F.nxn, F.nyc);
        double lbb[3], lJ[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lbb[d] = ob[(long)d * nnode + n];
            lJ[d] = ob[(long)(3 + d) * nnode + n];
        }
        // J = (dBy_z - dBz_y, dBz_x - dBx_z, dBx_y - dBy_x)
        const double ldBx[3] = {0.0, lJ[2], -lJ[1]};
        const double ldBy[3] = {-lJ[2], 0.0, lJ[0]};
        const double ldBz[3] = {lJ[1], -lJ[0], 0.0};
        const double sa = a == 1 ? 1.0 : -1.0, sb = b == 1 ? 1.0 : -1.0, sc = c == 1 ? 1.0 : -1.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double v = lbb[d] * wbb;
            v += sa * ldBx[d] * wx;
            if (D >= 2) v += sb * ldBy[d] * wy;
            if (D >= 3) v += sc * ldBz[d] * wz;
            acc[d] += v;
        }
    };
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                add(I + 1 - a, a, b, c);
                if (F.xbc == 0 && I == F.nx - 1 && a == 0) add(F.nx, 1, b, c);   // the wall ghost at nx
            }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const long e = (long)d * ncent + q;
        const double v = (kBaseFromLamF<EMIT> ? o.lFin[e] / o.h : o.base[e]) + acc[d];
        if constexpr (EMIT == kEmitStage1) {
            o.l0[e] += v;
            o.lF[e] = o.h * v;
        } else if constexpr (EMIT == kEmitStage2) {
            o.l0[e] += 0.75 * v;
            o.lF[e] = 0.25 * o.h * v;
        } else if constexpr (EMIT == kEmitStage3) {
            o.l0[e] = v * (1.0 / 3.0);
            o.lF[e] = v * (2.0 / 3.0) * o.h;
        } else {
            o.out[e] = v;
        }
    }
}

// Transpose of the fluid moments (continuous deposit): lam of (n_e, p_e,
// Gamma) at the nodes -> lam of the per-species moment sums (R, Gx, Gy, Gz)
// at the deposit nodes (the boundary fill maps several nodes onto one), and
// the alpha_cr adjoint (the CR weight is alpha_cr n_cr / ppc_cr).
__global__ __launch_bounds__(256) void k_fluid_adj(FieldGeo F, const double* __restrict__ m0, const double* __restrict__ m1,
                                                   const double* __restrict__ lfl, double* __restrict__ lM0,
                                                   double* __restrict__ lM1, long nnode, double dwcr, double* grads) {
    const int n = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    double acc = 0.0;
    if (n < nnode) {
        const int i0 = n % F.nxn, rest = n / F.nxn;
        int i = i0;
        // nodes near a box end share the deposit entry of the nearest fully
        // covered node; only those entries take more than one contribution
        bool shared = false;
        if (F.xbc == 0) {
            shared = i0 <= F.mclamp || i0 >= F.nx - F.mclamp;
            if (i < F.mclamp) i = F.mclamp;
            if (i > F.nx - F.mclamp) i = F.nx - F.mclamp;
        }
        const long dn = (long)(i + F.g) + (long)F.ndx * rest;
        double dens = F.wth * m0[4 * dn];
        if (F.has_cr) dens += F.wcr * m1[4 * dn];
        double ld = 0.0;
        if (dens > F.n_floor)
            ld = lfl[n] + lfl[nnode + n] * 0.5 * F.beta_e * F.gamma_e * pow(dens, F.gamma_e - 1.0);
        const double lg[3] = {lfl[2 * nnode + n], lfl[3 * nnode + n], lfl[4 * nnode + n]};
        auto put = [&](double* a, double v) {
            if (shared) unsafeAtomicAdd(a, v);
            else *a = v;
        };
        put(lM0 + 4 * dn, F.wth * ld);
#pragma unroll
        for (int d = 0; d < 3; ++d) put(lM0 + 4 * dn + 1 + d, F.wth * lg[d]);
        if (F.has_cr) {
            put(lM1 + 4 * dn, F.wcr * ld);
#pragma unroll
            for (int d = 0; d < 3; ++d) put(lM1 + 4 * dn + 1 + d, F.wcr * lg[d]);
            acc = dwcr * (m1[4 * dn] * ld + m1[4 * dn + 1] * lg[0] + m1[4 * dn + 2] * lg[1] + m1[4 * dn + 3] * lg[2]);
        }
    }
    block_add(acc, grads);
}

// Zeroes, in every row of a species' moment adjoints (4 doubles per deposit
// entry), the x entries e <= lo and e >= hi of a box: the guard entries that
// k_fluid_adj never writes and the two clamped entries it adds into.  The
// entries between are each stored by exactly one node.
__global__ __launch_bounds__(256) void k_zero_dep_ends(double* __restrict__ a, int ndx, long rows, int lo, int hi) {
    const int nl = lo + 1, nc = nl + (ndx - hi);
    const long n = rows * nc * 4;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const long q = t >> 2;
        const int c = (int)(q % nc);
        const int e = c < nl ? c : hi + (c - nl);
        a[4 * ((q / nc) * ndx + e) + (t & 3)] = 0.0;
    }
}

// A centre plane of lam_F into LDS, for the z-marching transpose below:
// centres x0-1 .. x0+X, y0-1 .. y0+Y of plane k, under the Faraday
// transpose's rules (y and z wrap, x wraps when periodic; in the box a
// centre past either end of x contributes nothing).
__device__ __forceinline__ void zm_load_F(const FieldGeo& F, const double* __restrict__ lF, long ncent, int x0, int y0,
                                          int k, double (*s)[ZMarch::CN]) {
    using Z = ZMarch;
    k = wrapi(k, F.nzc);
    for (int l = threadIdx.x; l < Z::CN; l += blockDim.x) {
        int i = x0 - 1 + l % Z::CX;
        const int j = wrapi(y0 - 1 + l / Z::CX, F.nyc);
        bool ok = true;
        if (F.xbc == 1) i = wrapi(i, F.nx);
        else ok = i >= 0 && i < F.nx;
        double v[3] = {0.0, 0.0, 0.0};
        if (ok) {
            const long q = lin(i, j, k, F.nx, F.nyc);
            v[0] = lF[q]; v[1] = lF[ncent + q]; v[2] = lF[2 * ncent + q];
        }
        s[0][l] = v[0]; s[1][l] = v[1]; s[2][l] = v[2];
    }
}

// The 3D transpose of Ohm's law at every node and of its Bbar average and
// curl at every centre in one pass, marching through z like the forward
// stage kernels (k_stage3): a workgroup takes the 32 x 8 centres of a block
// column and a run of z planes.  At node plane k it stages B (and, with
// CURL, lam_F) at the centre planes k-1 and k and p_e at node plane k,
// computes the nodes x0 .. x0+32, y0 .. y0+8 of the plane (the node pass:
// lam_E from lE or, with CURL, the Faraday transpose of lam_F; Ohm's
// transpose; the fluid adjoints of the nodes it owns) into LDS, and adds
// each node's (lam_Bbar, lam_J) to the centre planes k-1 and k of the
// thread that owns the centre column; the centre of plane k-1 is then
// complete and goes out as EMIT says (the centre pass of k_ohm_adj_centre,
// the wall ghost's share included).  Node plane ze, the next run's first,
// is computed for its centres only.
template <bool CURL, int EMIT>
__global__ __launch_bounds__(256, 3) void k_ohm_adj3(FieldGeo F, const double* __restrict__ B,
                                                  const double* __restrict__ fl, const double* __restrict__ lEF,
                                                  const double* __restrict__ lBb, double* __restrict__ lfl, RkOut o,
                                                  double* grads, long nnode, long ncent, int gx, int gy, int zc) {
    using Z = ZMarch;
    __shared__ double sB[2][3][Z::CN];
    __shared__ double sF[CURL ? 2 : 1][3][CURL ? Z::CN : 1];
    __shared__ double sP[Z::PN];
    __shared__ double sO[6][Z::NN];
    int x0, y0, zs, ze;
    zm_block(gx, gy, zc, F.nzc, x0, y0, zs, ze);
    const double* pe = fl + nnode;
    double* lpe = lfl + nnode;
    const int t = threadIdx.x, tx = t % Z::X, ty = t / Z::X;
    const int I = x0 + tx, Jc = y0 + ty;
    const bool own_c = I < F.nx && Jc < F.nyc;
    const double h2 = 0.5 * F.rdx;
    const double wbb = 0.125, wd = 0.25 * F.rdx;
    const int nxo = F.xbc == 1 ? F.nx : F.nx + 1;   // nodes along x
    double accK1[3] = {0.0, 0.0, 0.0}, accK[3] = {0.0, 0.0, 0.0};
    ZPlane pl;
    {
        const int kp = zs - 1, slot = kp & 1;
        zm_fetch_B(F, B, ncent, x0, y0, kp, pl);
        zm_store_B(pl, sB[slot]);
        if constexpr (CURL) zm_load_F(F, lEF, ncent, x0, y0, kp, sF[slot]);
    }
    for (int k = zs; k <= ze; ++k) {
        const int cur = k & 1, prv = cur ^ 1;
        zm_fetch_B(F, B, ncent, x0, y0, k, pl);
        zm_fetch_P(F, pe, x0, y0, k, pl);
        zm_store_B(pl, sB[cur]);
        zm_store_P(pl, sP);
        if constexpr (CURL) zm_load_F(F, lEF, ncent, x0, y0, k, sF[cur]);
        __syncthreads();
        // node plane k
#pragma unroll 1
        for (int l = t; l < Z::NN; l += 256) {
            const int lx = l % Z::NX, ly = l / Z::NX;
            const int i = x0 + lx, jg = y0 + ly;
            double lbb[3] = {0.0, 0.0, 0.0}, lJ[3] = {0.0, 0.0, 0.0};
            if (F.xbc == 1 || i <= F.nx) {
                const int iw = F.xbc == 1 ? wrapi(i, F.nx) : i;
                const long n = lin(iw, wrapi(jg, F.nyc), wrapi(k, F.nzc), F.nxn, F.nyc);
                // Bbar and the B differences from the 8 centres around the node
                double bb[3] = {0, 0, 0}, dBx[3] = {0, 0, 0}, dBy[3] = {0, 0, 0}, dBz[3] = {0, 0, 0};
#pragma unroll
                for (int c = 0; c < 2; ++c)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int a = 0; a < 2; ++a)
#pragma unroll
                            for (int d = 0; d < 3; ++d) {
                                const double v = sB[c == 1 ? cur : prv][d][(lx + a) + Z::CX * (ly + b)];
                                bb[d] += v;
                                dBx[d] += a == 1 ? v : -v;
                                dBy[d] += b == 1 ? v : -v;
                                dBz[d] += c == 1 ? v : -v;
                            }
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    bb[d] *= 0.125;
                    dBx[d] *= 0.25 * F.rdx;
                    dBy[d] *= 0.25 * F.rdx;
                    dBz[d] *= 0.25 * F.rdx;
                }
                const double J[3] = {dBy[2] - dBz[1], dBz[0] - dBx[2], dBx[1] - dBy[0]};
                const int pc = (lx + 1) + Z::PX * (ly + 1);
                const long nzp = fnode(F, i, jg, k + 1), nzm = fnode(F, i, jg, k - 1);
                const double gp[3] = {(sP[pc + 1] - sP[pc - 1]) * h2, (sP[pc + Z::PX] - sP[pc - Z::PX]) * h2,
                                      (pe[nzp] - pe[nzm]) * h2};
                double lEn[3] = {0.0, 0.0, 0.0}, lBbn[3] = {0.0, 0.0, 0.0};
                if constexpr (CURL) {
                    // node (i, j, k) = centre (i - a, j - b, k - c) + (a, b, c)
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int b = 0; b < 2; ++b)
#pragma unroll
                            for (int a = 0; a < 2; ++a) {
                                const int cl = (lx + 1 - a) + Z::CX * (ly + 1 - b);
                                const int sl = c == 0 ? cur : prv;
                                const double l0 = sF[sl][0][cl], l1 = sF[sl][1][cl], l2 = sF[sl][2][cl];
                                const double ldEx[3] = {0.0, -l2, l1}, ldEy[3] = {l2, 0.0, -l0},
                                             ldEz[3] = {-l1, l0, 0.0};
#pragma unroll
                                for (int d = 0; d < 3; ++d)
                                    lEn[d] += ((a == 1 ? 1.0 : -1.0) * ldEx[d] + (b == 1 ? 1.0 : -1.0) * ldEy[d] +
                                               (c == 1 ? 1.0 : -1.0) * ldEz[d]) * wd;
                            }
                } else {
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        lEn[d] = lEF[(long)d * nnode + n];
                        if (lBb) lBbn[d] = lBb[(long)d * nnode + n];
                    }
                }
                const double ne = fl[n];
                const double Gm[3] = {fl[2 * nnode + n], fl[3 * nnode + n], fl[4 * nnode + n]};
                const bool inflow = inflow_node(F, i);
                const bool conduct = F.conduct && i == F.nx;
                double lnum[3], lG[3], lne;
                ohm_adj_at(F, bb, J, gp, ne, Gm, lEn, lBbn, inflow, conduct, lbb, lJ, lnum, lne, lG);
                // the node's own fluid adjoints, by the workgroup that owns it
                const bool own_n = ((lx < Z::X && i < nxo) || (F.xbc == 0 && i == F.nx)) && ly < Z::Y &&
                                   jg < F.nyc && k < ze;
                if (own_n) {
                    if (inflow) unsafeAtomicAdd(grads, lEn[1] * F.B0[2] - lEn[2] * F.B0[1]);
                    // stored by the first transpose of a step (no curl), added by the others
                    if constexpr (CURL) {
                        lfl[n] += lne;
#pragma unroll
                        for (int d = 0; d < 3; ++d) lfl[(long)(2 + d) * nnode + n] += lG[d];
                    } else {
                        lfl[n] = lne;
#pragma unroll
                        for (int d = 0; d < 3; ++d) lfl[(long)(2 + d) * nnode + n] = lG[d];
                    }
                    unsafeAtomicAdd(lpe + fnode(F, i + 1, jg, k), -lnum[0] * h2);
                    unsafeAtomicAdd(lpe + fnode(F, i - 1, jg, k), lnum[0] * h2);
                    unsafeAtomicAdd(lpe + fnode(F, i, jg + 1, k), -lnum[1] * h2);
                    unsafeAtomicAdd(lpe + fnode(F, i, jg - 1, k), lnum[1] * h2);
                    unsafeAtomicAdd(lpe + nzp, -lnum[2] * h2);
                    unsafeAtomicAdd(lpe + nzm, lnum[2] * h2);
                }
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                sO[d][l] = lbb[d];
                sO[3 + d][l] = lJ[d];
            }
        }
        // lam_F(in) of this thread's centre of plane k-1, the base of a
        // kEmitStage2 / kEmitStage1 emit, read before the next plane's load
        // may overwrite its slot
        double bF[3] = {0.0, 0.0, 0.0};
        if constexpr (CURL && kBaseFromLamF<EMIT>)
#pragma unroll
            for (int d = 0; d < 3; ++d) bF[d] = sF[prv][d][(tx + 1) + Z::CX * (ty + 1)];
        __syncthreads();
        // the node plane into the centre planes k-1 (as their upper plane)
        // and k (lower) of this thread's column
        if (own_c) {
            auto add = [&](int lxn, int a, int b) {
                const int l = lxn + Z::NX * (ty + 1 - b);
                const double lJ0 = sO[3][l], lJ1 = sO[4][l], lJ2 = sO[5][l];
                const double ldBx[3] = {0.0, lJ2, -lJ1}, ldBy[3] = {-lJ2, 0.0, lJ0}, ldBz[3] = {lJ1, -lJ0, 0.0};
                const double sa = a == 1 ? 1.0 : -1.0, sb = b == 1 ? 1.0 : -1.0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double v = sO[d][l] * wbb + (sa * ldBx[d] + sb * ldBy[d]) * wd;
                    accK1[d] += v - ldBz[d] * wd;   // c = 0: the node is the upper corner of centre k-1
                    accK[d] += v + ldBz[d] * wd;    // c = 1: the lower corner of centre k
                }
            };
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    add(tx + 1 - a, a, b);
                    if (F.xbc == 0 && I == F.nx - 1 && a == 0) add(tx + 1, 1, b);   // the wall ghost at nx
                }
            if (k > zs) {
                const long q = lin(I, Jc, k - 1, F.nx, F.nyc);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const long e = (long)d * ncent + q;
                    const double v = (kBaseFromLamF<EMIT> ? bF[d] / o.h : o.base[e]) + accK1[d];
                    if constexpr (EMIT == kEmitStage1) {
                        o.l0[e] += v;
                        o.lF[e] = o.h * v;
                    } else if constexpr (EMIT == kEmitStage2) {
                        o.l0[e] += 0.75 * v;
                        o.lF[e] = 0.25 * o.h * v;
                    } else if constexpr (EMIT == kEmitStage3) {
                        o.l0[e] = v * (1.0 / 3.0);
                        o.lF[e] = v * (2.0 / 3.0) * o.h;
                    } else {
                        o.out[e] = v;
                    }
                }
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            accK1[d] = accK[d];
            accK[d] = 0.0;
        }
    }
}

// The 2D form of k_ohm_adj3: a block of 256 threads takes RX = 255 centre
// columns x0 .. x0+254 (so its 256 node columns x0 .. x0+255 are one per
// thread) and marches through a run of y rows.  Per row j it stages the B
// and lam_F centre rows j-1 and j and the p_e node row j in LDS, computes
// node row j (lam_E from lE or, with CURL, the Faraday transpose of lam_F;
// Ohm's transpose; the fluid adjoints of the nodes it owns) into LDS, and
// adds each node's (lam_Bbar, lam_J) to the centre rows j-1 and j of the
// thread owning the column; centre row j-1 is then complete and goes out as
// EMIT says.  Node row ye, the next run's first, is computed for its
// centres only.
struct YMarch {
    static constexpr int RX = 255;            // centre columns per block
    static constexpr int CX = RX + 2;         // centres x0-1 .. x0+RX
    static constexpr int NX = RX + 1;         // nodes x0 .. x0+RX, one per thread
    static constexpr int PX = RX + 3;         // p_e at nodes x0-1 .. x0+RX+1
};

// A centre row of B (the box's x ghosts: B0 at the inflow, the last
// centre at the wall) or of lam_F (nothing past either end of a box) into LDS.
template <bool LAMF>
__device__ __forceinline__ void ym_load_row(const FieldGeo& F, const double* __restrict__ a, long ncent, int x0, int j,
                                            double (*s)[YMarch::CX]) {
    j = wrapi(j, F.nyc);
    for (int l = threadIdx.x; l < YMarch::CX; l += blockDim.x) {
        int i = x0 - 1 + l;
        double v[3] = {0.0, 0.0, 0.0};
        if (F.xbc == 1) i = wrapi(i, F.nx);
        if (LAMF) {
            if (F.xbc == 1 || (i >= 0 && i < F.nx)) {
                const long q = lin(i, j, 0, F.nx, F.nyc);
                v[0] = a[q]; v[1] = a[ncent + q]; v[2] = a[2 * ncent + q];
            }
        } else {
            if (i >= F.nx) i = F.nx - 1;
            if (i < 0) {
                v[0] = F.B0[0]; v[1] = F.B0[1]; v[2] = F.B0[2];
            } else {
                const long q = lin(i, j, 0, F.nx, F.nyc);
                v[0] = a[q]; v[1] = a[ncent + q]; v[2] = a[2 * ncent + q];
            }
        }
        s[0][l] = v[0]; s[1][l] = v[1]; s[2][l] = v[2];
    }
}

template <bool CURL, int EMIT>
__global__ __launch_bounds__(256) void k_ohm_adj2(FieldGeo F, const double* __restrict__ B,
                                                  const double* __restrict__ fl, const double* __restrict__ lEF,
                                                  const double* __restrict__ lBb, double* __restrict__ lfl, RkOut o,
                                                  double* grads, long nnode, long ncent, int gx, int yc) {
    using Y = YMarch;
    __shared__ double sB[2][3][Y::CX];
    __shared__ double sF[CURL ? 2 : 1][3][CURL ? Y::CX : 1];
    __shared__ double sP[Y::PX];
    __shared__ double sO[6][Y::NX];
    const int b = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int x0 = (b % gx) * Y::RX, ys = (b / gx) * yc, ye = min(ys + yc, (int)F.nyc);
    const double* pe = fl + nnode;
    double* lpe = lfl + nnode;
    const int t = threadIdx.x;
    const int I = x0 + t;
    const bool own_c = t < Y::RX && I < F.nx;
    const double h2 = 0.5 * F.rdx;
    const double wbb = 0.25, wd = 0.5 * F.rdx;
    const int nxo = F.xbc == 1 ? F.nx : F.nx + 1;   // nodes along x
    double accJ1[3] = {0.0, 0.0, 0.0}, accJ[3] = {0.0, 0.0, 0.0};
    ym_load_row<false>(F, B, ncent, x0, ys - 1, sB[(ys - 1) & 1]);
    if constexpr (CURL) ym_load_row<true>(F, lEF, ncent, x0, ys - 1, sF[(ys - 1) & 1]);
    for (int j = ys; j <= ye; ++j) {
        const int cur = j & 1, prv = cur ^ 1;
        ym_load_row<false>(F, B, ncent, x0, j, sB[cur]);
        if constexpr (CURL) ym_load_row<true>(F, lEF, ncent, x0, j, sF[cur]);
        {
            const int jw = wrapi(j, F.nyc);
            for (int l = t; l < Y::PX; l += blockDim.x) {
                int i = x0 - 1 + l;
                if (F.xbc == 1) i = wrapi(i, F.nx);
                else i = i < 0 ? 0 : (i > F.nx ? F.nx : i);
                sP[l] = pe[lin(i, jw, 0, F.nxn, F.nyc)];
            }
        }
        __syncthreads();
        // node row j: node (x0 + t, j)
        {
            const int lx = t, i = x0 + lx;
            double lbb[3] = {0.0, 0.0, 0.0}, lJ[3] = {0.0, 0.0, 0.0};
            if (F.xbc == 1 || i <= F.nx) {
                const int iw = F.xbc == 1 ? wrapi(i, F.nx) : i;
                const long n = lin(iw, wrapi(j, F.nyc), 0, F.nxn, F.nyc);
                // Bbar and the B differences from the 4 centres around the node
                double bb[3] = {0, 0, 0}, dBx[3] = {0, 0, 0}, dBy[3] = {0, 0, 0};
#pragma unroll
                for (int bq = 0; bq < 2; ++bq)
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int d = 0; d < 3; ++d) {
                            const double v = sB[bq == 1 ? cur : prv][d][lx + a];
                            bb[d] += v;
                            dBx[d] += a == 1 ? v : -v;
                            dBy[d] += bq == 1 ? v : -v;
                        }
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    bb[d] *= 0.25;
                    dBx[d] *= 0.5 * F.rdx;
                    dBy[d] *= 0.5 * F.rdx;
                }
                const double J[3] = {dBy[2], -dBx[2], dBx[1] - dBy[0]};
                const long nyp = fnode(F, i, j + 1, 0), nym = fnode(F, i, j - 1, 0);
                const double gp[3] = {(sP[lx + 2] - sP[lx]) * h2, (pe[nyp] - pe[nym]) * h2, 0.0};
                double lEn[3] = {0.0, 0.0, 0.0}, lBbn[3] = {0.0, 0.0, 0.0};
                if constexpr (CURL) {
                    // node (i, j) = centre (i - a, j - bq) + (a, bq)
#pragma unroll
                    for (int bq = 0; bq < 2; ++bq)
#pragma unroll
                        for (int a = 0; a < 2; ++a) {
                            const int cl = lx + 1 - a;
                            const int sl = bq == 0 ? cur : prv;
                            const double l0 = sF[sl][0][cl], l1 = sF[sl][1][cl], l2 = sF[sl][2][cl];
                            const double ldEx[3] = {0.0, -l2, l1}, ldEy[3] = {l2, 0.0, -l0};
#pragma unroll
                            for (int d = 0; d < 3; ++d)
                                lEn[d] += ((a == 1 ? 1.0 : -1.0) * ldEx[d] + (bq == 1 ? 1.0 : -1.0) * ldEy[d]) * wd;
                        }
                } else {
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        lEn[d] = lEF[(long)d * nnode + n];
                        if (lBb) lBbn[d] = lBb[(long)d * nnode + n];
                    }
                }
                const double ne = fl[n];
                const double Gm[3] = {fl[2 * nnode + n], fl[3 * nnode + n], fl[4 * nnode + n]};
                const bool inflow = inflow_node(F, i);
                const bool conduct = F.conduct && i == F.nx;
                double lnum[3], lG[3], lne;
                ohm_adj_at(F, bb, J, gp, ne, Gm, lEn, lBbn, inflow, conduct, lbb, lJ, lnum, lne, lG);
                // the node's own fluid adjoints, by the block that owns it
                const bool own_n = ((lx < Y::RX && i < nxo) || (F.xbc == 0 && i == F.nx)) && j < ye;
                if (own_n) {
                    if (inflow) unsafeAtomicAdd(grads, lEn[1] * F.B0[2] - lEn[2] * F.B0[1]);
                    // stored by the first transpose of a step (no curl), added by the others
                    if constexpr (CURL) {
                        lfl[n] += lne;
#pragma unroll
                        for (int d = 0; d < 3; ++d) lfl[(long)(2 + d) * nnode + n] += lG[d];
                    } else {
                        lfl[n] = lne;
#pragma unroll
                        for (int d = 0; d < 3; ++d) lfl[(long)(2 + d) * nnode + n] = lG[d];
                    }
                    unsafeAtomicAdd(lpe + fnode(F, i + 1, j, 0), -lnum[0] * h2);
                    unsafeAtomicAdd(lpe + fnode(F, i - 1, j, 0), lnum[0] * h2);
                    unsafeAtomicAdd(lpe + nyp, -lnum[1] * h2);
                    unsafeAtomicAdd(lpe + nym, lnum[1] * h2);
                }
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                sO[d][lx] = lbb[d];
                sO[3 + d][lx] = lJ[d];
            }
        }
        // lam_F(in) of this thread's centre of row j-1, the base of a
        // kEmitStage2 / kEmitStage1 emit, read before the next row's load may
        // overwrite its slot
        double bF[3] = {0.0, 0.0, 0.0};
        if constexpr (CURL && kBaseFromLamF<EMIT>)
#pragma unroll
            for (int d = 0; d < 3; ++d) bF[d] = sF[prv][d][t + 1];
        __syncthreads();
        // the node row into the centre rows j-1 (as their upper row) and j
        // (lower) of this thread's column
        if (own_c) {
            auto add = [&](int lxn, int a) {
                const double lJ0 = sO[3][lxn], lJ1 = sO[4][lxn], lJ2 = sO[5][lxn];
                const double ldBx[3] = {0.0, lJ2, -lJ1}, ldBy[3] = {-lJ2, 0.0, lJ0};
                const double sa = a == 1 ? 1.0 : -1.0;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double v = sO[d][lxn] * wbb + sa * ldBx[d] * wd;
                    accJ1[d] += v - ldBy[d] * wd;   // bq = 0: the node is an upper corner of centre j-1
                    accJ[d] += v + ldBy[d] * wd;    // bq = 1: a lower corner of centre j
                }
            };
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                add(t + 1 - a, a);
                if (F.xbc == 0 && I == F.nx - 1 && a == 0) add(t + 1, 1);   // the wall ghost at nx
            }
            if (j > ys) {
                const long q = lin(I, wrapi(j - 1, F.nyc), 0, F.nx, F.nyc);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const long e = (long)d * ncent + q;
                    const double v = (kBaseFromLamF<EMIT> ? bF[d] / o.h : o.base[e]) + accJ1[d];
                    if constexpr (EMIT == kEmitStage1) {
                        o.l0[e] += v;
                        o.lF[e] = o.h * v;
                    } else if constexpr (EMIT == kEmitStage2) {
                        o.l0[e] += 0.75 * v;
                        o.lF[e] = 0.25 * o.h * v;
                    } else if constexpr (EMIT == kEmitStage3) {
                        o.l0[e] = v * (1.0 / 3.0);
                        o.lF[e] = v * (2.0 / 3.0) * o.h;
                    } else {
                        o.out[e] = v;
                    }
                }
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            accJ1[d] = accJ[d];
            accJ[d] = 0.0;
        }
    }
}

// Amplitude adjoints of the initial modes: dB_y = A cos(k_m x + phi_m),
// dB_z = A sin(k_m x + phi_m) at every centre; blockIdx.y is the mode, the
// blocks along x share its centres.
__global__ __launch_bounds__(256) void k_amps_adj(FieldGeo F, const double* __restrict__ lB, const double* __restrict__ phase,
                                                  double Lx, long ncent, double* grads) {
    const int m = blockIdx.y + 1;
    double acc = 0.0;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < ncent; q += (long)gridDim.x * blockDim.x) {
        const int i = (int)(q % F.nx);
        const double x = ((double)i + 0.5) * F.dx;
        const double ph = kTwoPi * (double)m * x / Lx + phase[m];
        acc += lB[ncent + q] * cos(ph) + lB[2 * ncent + q] * sin(ph);
    }
    block_add(acc, grads + 1 + m);
}

}  // namespace fsk
