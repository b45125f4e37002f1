// fs_device.h -- device-side building blocks of the faux-shock hybrid step
// for gfx950: counter-based random numbers, shape functions, the fixed-point
// deposit format, the Boris rotation and the faux-shock wall event.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#ifndef DEP_HALO
#define DEP_HALO 1
#endif
#ifndef DEP_HALO_T
#define DEP_HALO_T 0
#endif
#ifndef PUSH_THREADS
#define PUSH_THREADS 512
#endif

namespace fsk {

// Random-number streams: the key of every Philox draw is (seed, stream).
constexpr uint64_t kStreamInit = 1, kStreamInjectTh = 2, kStreamInjectCr = 3,
                   kStreamWall = 4, kStreamFourier = 5;
constexpr int kVsat = 8388607;            // 2^23 - 1: largest velocity code
constexpr double kTwoPi = 6.283185307179586;

// Compile-time tile shapes (cells per tile) per dimensionality.  A tile is
// the unit of work of one workgroup: its particles, its gather stencil and
// its deposit accumulators all live in LDS.
template <int D> struct TileShape;
template <> struct TileShape<1> { static constexpr int X = 32, Y = 1, Z = 1; };
template <> struct TileShape<2> { static constexpr int X = 16, Y = 8, Z = 1; };
template <> struct TileShape<3> { static constexpr int X = 16, Y = 8, Z = 4; };

// Shape-function stencil relative to the particle's cell c: CIC touches
// nodes c, c+1; TSC touches the nearest node and its neighbours, i.e. some
// three of c-1 .. c+2.
template <int S> struct Stencil;
template <> struct Stencil<1> { static constexpr int LO = 0, HI = 1, N = 2; };
template <> struct Stencil<2> { static constexpr int LO = 1, HI = 2, N = 3; };

// LDS extents of one tile: GX.. for the gather grid (the tile's cells plus
// the stencil), DX.. for the deposit accumulators (HX, HY, HZ extra cells of
// halo on each side, so ions that left the tile by that much still deposit in
// LDS; the rest deposit straight into the global grid).  The flow is along x,
// so in 3D only x gets a halo: transverse crossers are rare, and the smaller
// box leaves room in LDS for three 512-thread workgroups per CU.
template <int D, int S> struct Extent {
    static constexpr int TX = TileShape<D>::X, TY = TileShape<D>::Y, TZ = TileShape<D>::Z;
    static constexpr int W = Stencil<S>::LO + Stencil<S>::HI;
    static constexpr int HX = DEP_HALO;
    static constexpr int HY = D >= 3 ? DEP_HALO_T : (D >= 2 ? DEP_HALO : 0);
    static constexpr int HZ = D >= 3 ? DEP_HALO_T : 0;
    static constexpr int GX = TX + W, GY = D >= 2 ? TY + W : 1, GZ = D >= 3 ? TZ + W : 1;
    static constexpr int DX = TX + 2 * HX + W, DY = D >= 2 ? TY + 2 * HY + W : 1, DZ = D >= 3 ? TZ + 2 * HZ + W : 1;
    static constexpr int GN = GX * GY * GZ, DN = DX * DY * DZ;
};

// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 64x64->128-bit products, key advanced by the Weyl constants each round.
__device__ __forceinline__ void philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                       uint64_t k0, uint64_t k1, uint64_t out[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = 0xD2E7470EE14C6C93ull, m1 = 0xCA5A826395121157ull;
        uint64_t lo0 = m0 * c0, hi0 = __umul64hi(m0, c0);
        uint64_t lo1 = m1 * c2, hi1 = __umul64hi(m1, c2);
        uint64_t y0 = hi1 ^ c1 ^ k0, y2 = hi0 ^ c3 ^ k1;
        c0 = y0; c1 = lo1; c2 = y2; c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Top 53 bits to a double in the open interval (0, 1), exactly.
__device__ __forceinline__ double unit(uint64_t r) {
    return ((double)(r >> 11) + 0.5) * 0x1.0p-53;
}

__device__ __forceinline__ void draw4(uint64_t seed, uint64_t stream, uint64_t c0, uint64_t c1,
                                      uint64_t c2, double u[4]) {
    uint64_t r[4];
    philox(c0, c1, c2, 0, seed, stream, r);
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = unit(r[i]);
}

// Box-Muller pair.
__device__ __forceinline__ void box_muller(double a, double b, double& n1, double& n2) {
    double rad = sqrt(-2.0 * log(a));
    n1 = rad * cos(kTwoPi * b);
    n2 = rad * sin(kTwoPi * b);
}

template <typename R> __device__ __forceinline__ R below_one();
template <> __device__ __forceinline__ float below_one<float>() { return 0x1.fffffep-1f; }
template <> __device__ __forceinline__ double below_one<double>() { return 0x1.fffffffffffffp-1; }

// Offset stored in the particle's precision, kept strictly below 1.
template <typename R> __device__ __forceinline__ R to_offset(double o) {
    R r = (R)o;
    return r >= (R)1 ? below_one<R>() : r;
}

// Real-valued 1D shape weights for the gather.  `rel` is the first node
// relative to the cell index.
template <typename R, int S> __device__ __forceinline__ void weights_real(R o, int& rel, R w[3]) {
    if constexpr (S == 1) {
        rel = 0; w[0] = (R)1 - o; w[1] = o; w[2] = (R)0;
    } else {
        R xi = o;
        rel = -1;
        if (o >= (R)0.5) { xi = o - (R)1; rel = 0; }
        R a = (R)0.5 - xi, b = (R)0.5 + xi;
        w[0] = (R)0.5 * a * a;
        w[1] = (R)0.75 - xi * xi;
        w[2] = (R)0.5 * b * b;
    }
}

// Integer 1D weights of the fixed-point deposit: the offset is quantised to
// q = floor(o 2^b + 1/2) (exact in the storage precision), and the weights
// of the CIC / TSC stencil are integers summing exactly to 2^b (CIC) or
// 2^(2b+1) (TSC).
template <typename R, int S> __device__ __forceinline__ void weights_int(R o, int b, int& rel, int w[3]) {
    int one = 1 << b;
    int q = (int)floor(o * (R)one + (R)0.5);
    if constexpr (S == 1) {
        rel = 0; w[0] = one - q; w[1] = q; w[2] = 0;
    } else {
        int half = one >> 1, d = q;
        rel = -1;
        if (q > half) { d = q - one; rel = 0; }
        w[0] = (half - d) * (half - d);
        w[2] = (half + d) * (half + d);
        w[1] = (1 << (2 * b + 1)) - w[0] - w[2];
    }
}

// Velocity code rint(v 2^sv), saturated to the 24-bit signed range so that
// weight x code is a single 24x24 -> 48-bit product.  Returns the saturation
// / NaN status in bits (8 = saturated, 4 = NaN).
template <typename R> __device__ __forceinline__ int vcode(R v, int sv, int& status) {
    if (v != v) { status |= 4; return 0; }
    R t = rint(ldexp(v, sv));
    if (t > (R)kVsat) { status |= 8; return kVsat; }
    if (t < -(R)kVsat) { status |= 8; return -kVsat; }
    return (int)t;
}

// 1 / gamma = 1 / sqrt(1 + x) with x = |u|^2 / c^2, IEEE square root and
// division (the hardware reciprocal square root, about 1 ulp, moved enough
// FP32 deposit codes to matter against the FP64 oracle).
template <typename R> __device__ __forceinline__ R inv_gamma(R x) { return (R)1 / sqrt((R)1 + x); }

// 1 / gamma of a stored four-velocity u, in FP64 whatever the particle
// precision and in a fixed order without contraction:
// 1 / sqrt(1 + ((u_x u_x + u_y u_y) + u_z u_z) / c^2).  The relativistic push
// moves with u * (1/gamma) and codes the deposit velocity from the same
// FP64 product, so that each code is that of the stored u (an FP32 quotient
// would move codes by one).
template <typename R> __device__ __forceinline__ double inv_gamma_u(const R u[3], double ic2) {
#pragma clang fp contract(off)
    const double a = (double)u[0], b = (double)u[1], c = (double)u[2];
    return 1.0 / sqrt(1.0 + (a * a + b * b + c * c) * ic2);
}

// Deposit velocity codes of a relativistic ion from u and its 1 / gamma.
template <typename R>
__device__ __forceinline__ void velocity_codes_ig(const R u[3], double ig, int sv, int& status, int vq[3]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int d = 0; d < 3; ++d) vq[d] = vcode<double>((double)u[d] * ig, sv, status);
}

// Velocity codes of the deposit from the stored velocity variable: of
// u / gamma in relativistic mode (REL), of the velocity itself otherwise.
template <typename R, bool REL>
__device__ __forceinline__ void velocity_codes(const R u[3], double ic2, int sv, int& status, int vq[3]) {
    if constexpr (REL) {
        velocity_codes_ig<R>(u, inv_gamma_u<R>(u, ic2), sv, status, vq);
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) vq[d] = vcode<R>(u[d], sv, status);
    }
}

// Exact weight x velocity-code product via the 24-bit multiplier pair.
__device__ __forceinline__ long long mul24(int w, int q) {
    w = (w << 8) >> 8;
    q = (q << 8) >> 8;
    return (long long)w * (long long)q;
}

// Boris rotation with half electric kicks (q/m = 1): v^{n-1/2} -> v^{n+1/2}.
// Relativistic mode (REL, ic2 = 1/c^2): v is the four-velocity u and the
// rotation vector is divided by the Lorentz factor sqrt(1 + |u^-|^2 / c^2)
// after the first half kick.  REL is a compile-time choice: the hot kernel
// is instantiated per mode, so neither pays for the other's registers.
template <typename R, bool REL> __device__ __forceinline__ void boris(R v[3], const R E[3], const R B[3], R h, R ic2) {
    R vm[3], t[3], s[3], vp[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) vm[d] = v[d] + h * E[d];
    R hb = h;
    if constexpr (REL) hb = h * inv_gamma((vm[0] * vm[0] + vm[1] * vm[1] + vm[2] * vm[2]) * ic2);
#pragma unroll
    for (int d = 0; d < 3; ++d) t[d] = hb * B[d];
    R tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    R f = (R)2 / ((R)1 + tt);
#pragma unroll
    for (int d = 0; d < 3; ++d) s[d] = f * t[d];
    vp[0] = vm[0] + (vm[1] * t[2] - vm[2] * t[1]);
    vp[1] = vm[1] + (vm[2] * t[0] - vm[0] * t[2]);
    vp[2] = vm[2] + (vm[0] * t[1] - vm[1] * t[0]);
    v[0] = vm[0] + (vp[1] * s[2] - vp[2] * s[1]) + h * E[0];
    v[1] = vm[1] + (vp[2] * s[0] - vp[0] * s[2]) + h * E[1];
    v[2] = vm[2] + (vp[0] * s[1] - vp[1] * s[0]) + h * E[2];
}

// Faux-shock event (eq. 1 of the paper with the speed measured in the
// downstream frame).  The reflect/transmit decision is sqrt-free FP64 with a
// fixed operation order and no contraction, so any two IEEE implementations
// agree bit for bit: with m = max(U1, U2), reflect iff
// |w|^2 > (u2 (1 + m) / (1 - m))^2, which happens with probability
// ((1 - u2/|w|) / (1 + u2/|w|))^2.  A reflected ion keeps |w| and leaves
// with direction cosine mu' = a + (1 - a) sqrt(U3), a = u2/|w|, azimuth
// 2 pi U4 (the flux of an isotropic downstream population that outruns the
// flow).  Returns 1 on reflection, with the new velocity and the distance
// (cells) the ion travels back from x = L during the rest of the step.
//
// Relativistic mode (c_light > 0): v and vout are four-velocities and the
// event happens in the downstream rest frame, reached by the exact Lorentz
// boost along x with speed u2 (factor g2).  There the four-velocity is W,
// the Lorentz factor Gam and the speed |w| = |W| / Gam, which enters the
// same decision; the kick keeps |W| (so Gam and |w|) and the inverse boost
// returns to the lab.  The decision arithmetic follows a fixed order (with
// IEEE square roots), so two implementations agree bit for bit.
__device__ __noinline__ int faux_shock_event(uint64_t seed, uint64_t step, uint32_t id, double u2, double c_light,
                                             double delta, const double v[3], double vout[3],
                                             double& back) {
#pragma clang fp contract(off)
    if (c_light > 0.0) {
        const double cc = c_light * c_light;
        const double gam = sqrt(1.0 + (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / cc);
        const double g2 = 1.0 / sqrt(1.0 - (u2 * u2) / cc);
        const double Gam = g2 * (gam - u2 * v[0] / cc);
        const double Wx = g2 * (v[0] - u2 * gam), Wy = v[1], Wz = v[2];
        const double W2 = Wx * Wx + Wy * Wy + Wz * Wz;
        const double w2 = W2 / (Gam * Gam);
        double U[4];
        draw4(seed, kStreamWall, step, (uint64_t)id, 0, U);
        const double m = U[0] > U[1] ? U[0] : U[1];
        const double T = u2 * (1.0 + m) / (1.0 - m);
        if (!(w2 > T * T)) return 0;
        const double Wabs = sqrt(W2);
        const double a = u2 / (Wabs / Gam);
        const double mu = a + (1.0 - a) * sqrt(U[2]);
        const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
        const double phi = kTwoPi * U[3];
        const double Wxn = -Wabs * mu;
        vout[0] = g2 * (Wxn + u2 * Gam);
        vout[1] = Wabs * st * cos(phi);
        vout[2] = Wabs * st * sin(phi);
        const double gn = g2 * (Gam + u2 * Wxn / cc);
        const double vx = v[0] / gam, vxn = vout[0] / gn;
        back = vx > 0.0 ? delta * (-vxn) / vx : 0.0;
        return 1;
    }
    double wx = v[0] - u2, wy = v[1], wz = v[2];
    double w2 = wx * wx + wy * wy + wz * wz;
    double U[4];
    draw4(seed, kStreamWall, step, (uint64_t)id, 0, U);
    double m = U[0] > U[1] ? U[0] : U[1];
    double T = u2 * (1.0 + m) / (1.0 - m);
    if (!(w2 > T * T)) return 0;
    double wabs = sqrt(w2);
    double a = u2 / wabs;
    double mu = a + (1.0 - a) * sqrt(U[2]);
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double phi = kTwoPi * U[3];
    vout[0] = u2 - wabs * mu;
    vout[1] = wabs * st * cos(phi);
    vout[2] = wabs * st * sin(phi);
    back = v[0] > 0.0 ? delta * (-vout[0]) / v[0] : 0.0;
    return 1;
}

// Prescribed faux-shock wall: the calibration the paper leaves open (Sec. 1:
// return rate, anisotropy and energy gain fitted to RW runs; Sec. 4: a wall
// that changes in time).  u2 is that of the step, u_sh / max(1, r + r_dot t),
// set on the host.  A crosser of downstream-frame speed |w| > u2 returns
// with probability min(1, f rho^2), rho = (|w| - u2) / (|w| + u2) (eq. 1 is
// rho^2) and f = f0 (|w| / w_ref)^alpha, decided by U1; it leaves with speed
// (relativistic: four-velocity magnitude) times gain, direction cosine mu'
// of pdf ~ (mu' - a)^(1 + kappa) on (a, 1], a = u2 / new speed, drawn by
// inversion from U3, and azimuth 2 pi U4.  A return that cannot outrun u2 is
// a transmission.  With kappa = 0 the direction is drawn with the IEEE square
// root, so a return the eq. (1) event also makes gets its kick bit for bit
// (non-relativistic mode).  pow() may differ from another implementation's
// in the last bit: a decision within one ulp of f rho^2 could then differ.
// Loss cone (lc_dep > 0): downstream CRs gyrate about the compressed field
// b2; a return direction whose motion along b2 alone outruns the receding
// shock is in the loss cone and returns as above, any other return becomes
// a transmission with probability lc_dep (uniform U2), which the paper
// expects at oblique shocks (Sec. 3.2).  cos(phi) of another libm may differ
// in the last bit: a direction within one ulp of the cone's edge could then
// be placed differently.
struct WallModel {
    int on;
    double u2, f0, alpha, wref, gain, kappa;
    double lc_dep, lc_cx, lc_sy;   // loss-cone depletion, |b2_x| and the y part of the upstream field direction
};

__device__ __noinline__ int faux_shock_event_prescribed(const WallModel& M, uint64_t seed, uint64_t step, uint32_t id,
                                                        double c_light, double delta, const double v[3],
                                                        double vout[3], double& back) {
#pragma clang fp contract(off)
    const bool rel = c_light > 0.0;
    const double u2 = M.u2;
    const double cc = rel ? c_light * c_light : 1.0;
    double gam = 1.0, g2 = 1.0, Gam = 1.0, Wx;
    if (rel) {
        gam = sqrt(1.0 + (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / cc);
        g2 = 1.0 / sqrt(1.0 - (u2 * u2) / cc);
        Gam = g2 * (gam - u2 * v[0] / cc);
        Wx = g2 * (v[0] - u2 * gam);
    } else {
        Wx = v[0] - u2;
    }
    const double Wabs = sqrt(Wx * Wx + v[1] * v[1] + v[2] * v[2]);
    const double w = Wabs / Gam;
    if (!(w > u2)) return 0;
    const double rho = (w - u2) / (w + u2);
    double f = M.f0;
    if (M.alpha != 0.0) f = f * pow(w / M.wref, M.alpha);
    double P = f * (rho * rho);
    if (P > 1.0) P = 1.0;
    double U[4];
    draw4(seed, kStreamWall, step, (uint64_t)id, 0, U);
    if (!(U[0] < P)) return 0;
    const double Wn = M.gain * Wabs;
    const double Gn = rel ? sqrt(1.0 + (Wn * Wn) / cc) : 1.0;
    const double wn = Wn / Gn;
    if (!(wn > u2)) return 0;
    const double a = u2 / wn;
    const double q = M.kappa == 0.0 ? sqrt(U[2]) : pow(U[2], 1.0 / (2.0 + M.kappa));
    const double mu = a + (1.0 - a) * q;
    const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    const double phi = kTwoPi * U[3];
    if (M.lc_dep > 0.0) {
        // loss cone: the direction n = (-mu, st cos phi, st sin phi) against
        // the upstream field direction s = (-lc_cx, -lc_sy, 0); outside the
        // cone a return is removed with probability lc_dep, decided by U2
        const double ns = mu * M.lc_cx - (st * cos(phi)) * M.lc_sy;
        if (!(ns * M.lc_cx > a) && U[1] < M.lc_dep) return 0;
    }
    const double Wxn = -Wn * mu;
    vout[1] = Wn * st * cos(phi);
    vout[2] = Wn * st * sin(phi);
    if (rel) {
        vout[0] = g2 * (Wxn + u2 * Gn);
        const double gl = g2 * (Gn + u2 * Wxn / cc);
        const double vx = v[0] / gam, vxn = vout[0] / gl;
        back = vx > 0.0 ? delta * (-vxn) / vx : 0.0;
    } else {
        vout[0] = u2 + Wxn;
        back = v[0] > 0.0 ? delta * (-vout[0]) / v[0] : 0.0;
    }
    return 1;
}

// Workgroup index -> tile, so that the workgroups the hardware hands to one
// XCD (round robin over 8) get a contiguous run of tiles and share its L2.
__device__ __forceinline__ int xcd_tile(int bid, int n) {
    int per = n >> 3, rem = n & 7, x = bid & 7, l = bid >> 3;
    return x * per + (x < rem ? x : rem) + l;
}

__device__ __forceinline__ int wrapi(int i, int n) {
    if (i < 0) { i += n; if (i < 0) i = ((i % n) + n) % n; }
    else if (i >= n) { i -= n; if (i >= n) i %= n; }
    return i;
}

}  // namespace fsk
