/*
 * fsoracle_adj.c -- TEST INFRASTRUCTURE ONLY (never part of the product path).
 *
 * Plain FP64 reverse-mode derivative (discrete adjoint) of the oracle's
 * continuous-deposit step, for small boxes.  It gives the gradient of the
 * precursor magnetic energy
 *
 *     L = sum over centres with i >= nx/2 of (B_y^2 + B_z^2), after N steps,
 *
 * with respect to the upstream flow speed u_sh, the CR current multiplier
 * alpha_cr and the amplitudes A_m of the seeded Fourier modes.
 *
 * What is differentiated.  The forward map is the oracle's step with the
 * deposit in real-valued weights (deposit_mode 1; the fixed-point deposit
 * has no derivative).  Every discrete decision is held at the value it took
 * on the forward trajectory (the pathwise derivative with common random
 * numbers): which cell a particle is in, which particles reflect at the FS
 * wall, escape or are removed, how many are injected, and whether n falls
 * under the density floor.  The FS decision (eq. 1) is such a decision; the
 * kick that follows a reflection (reading R7) is differentiated, including
 * its dependence on u2 = u_sh / r.
 *
 * How.  The forward trajectory is run by the oracle itself (ora_step) and
 * recorded through its public interface, one full snapshot per step.  The
 * reverse sweep then walks the step backwards:
 *
 *   final Ohm -> SSP-RK3 Faraday (stages recomputed) -> fluid moments ->
 *   deposit -> injection -> FS wall kick -> move -> Boris -> gather,
 *
 * each written out here as the transpose of the forward formula.  Particle
 * adjoints are indexed by particle id.  The index rules of the grid (ghost
 * centres, moment fill, gather clamp, deposit ghosts) are the readings R3 and
 * R9 listed in fsoracle.c, written again here.
 *
 * Pins: tests/test_oracle_adjoint.py checks every piece and the whole
 * gradient against central finite differences of the forward oracle.
 */
#include "fsoracle.h"
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ADJ_TWO_PI 6.283185307179586

typedef struct {
    ora_cfg c;
    int D;
    int64_t nx, nyc, nzc, nxn, ndx, g, ncent, nnode, ndep;
    int mclamp;
    double B0[3], u2, h2dx;
    double* lu_inflow;   /* where dL/du_sh of the inflow-node field is added, or NULL */
} geo;

typedef struct {
    int64_t n;
    int64_t* c;
    double *o, *v;
    uint64_t* id;
} psnap;

typedef struct {
    psnap sp[2];
    double *B, *E, *Bb, *fn, *fg, *Mc[2];
    int64_t next_id;
} snap;

static int64_t wrap(int64_t i, int64_t n) { int64_t r = i % n; return r < 0 ? r + n : r; }

static void geo_init(geo* G, const ora_cfg* c)
{
    G->c = *c;
    G->D = c->dim;
    G->nx = c->nx;
    G->nyc = c->dim >= 2 ? c->ny : 1;
    G->nzc = c->dim >= 3 ? c->nz : 1;
    G->nxn = c->xbc == ORA_XBC_PERIODIC ? c->nx : c->nx + 1;
    G->g = (c->xbc == ORA_XBC_BOX && c->shape == 2) ? 1 : 0;
    G->ndx = G->nxn + 2 * G->g;
    G->ncent = G->nx * G->nyc * G->nzc;
    G->nnode = G->nxn * G->nyc * G->nzc;
    G->ndep = G->ndx * G->nyc * G->nzc;
    G->mclamp = c->shape;
    double th = c->theta_deg * (ADJ_TWO_PI / 360.0);
    G->B0[0] = cos(th); G->B0[1] = sin(th); G->B0[2] = 0.0;
    G->u2 = c->u_sh / c->r;
    G->h2dx = 1.0 / (2.0 * c->dx);
    G->lu_inflow = NULL;
}

/* The inflow node x = 0 of the box (reading R10). */
static int inflow_node(const geo* G, int64_t i) { return G->c.xbc != ORA_XBC_PERIODIC && i == 0; }
/* The conducting wall node x = L (reading R14): E_y = E_z = 0 there. */
static int conduct_node(const geo* G, int64_t i)
{
    return G->c.xbc != ORA_XBC_PERIODIC && G->c.wall_field == 1 && i == G->c.nx;
}

/* ---------------------------------------------------------------------- */
/* index rules (readings R3, R9)                                          */
/* ---------------------------------------------------------------------- */
/* Centre (i,j,k) -> storage index, or -1 for the inflow ghost (holds B0). */
static int64_t cent_at(const geo* G, int64_t i, int64_t j, int64_t k)
{
    j = wrap(j, G->nyc); k = wrap(k, G->nzc);
    if (G->c.xbc == ORA_XBC_PERIODIC) i = wrap(i, G->nx);
    else if (i < 0) return -1;
    else if (i >= G->nx) i = G->nx - 1;
    return i + G->nx * (j + G->nyc * k);
}
static double B_at(const geo* G, const double* B, int64_t i, int64_t j, int64_t k, int d)
{
    int64_t q = cent_at(G, i, j, k);
    return q < 0 ? G->B0[d] : B[3 * q + d];
}
static int64_t node_at(const geo* G, int64_t i, int64_t j, int64_t k)
{
    j = wrap(j, G->nyc); k = wrap(k, G->nzc);
    if (G->c.xbc == ORA_XBC_PERIODIC) i = wrap(i, G->nx);
    return i + G->nxn * (j + G->nyc * k);
}
static int64_t fluid_at(const geo* G, int64_t i, int64_t j, int64_t k)
{
    j = wrap(j, G->nyc); k = wrap(k, G->nzc);
    if (G->c.xbc == ORA_XBC_PERIODIC) i = wrap(i, G->nx);
    else {
        if (i < G->mclamp) i = G->mclamp;
        if (i > G->nx - G->mclamp) i = G->nx - G->mclamp;
    }
    return i + G->nxn * (j + G->nyc * k);
}
static int64_t gather_at(const geo* G, int64_t i, int64_t j, int64_t k)
{
    j = wrap(j, G->nyc); k = wrap(k, G->nzc);
    if (G->c.xbc == ORA_XBC_PERIODIC) i = wrap(i, G->nx);
    else { if (i < 0) i = 0; if (i > G->nx) i = G->nx; }
    return i + G->nxn * (j + G->nyc * k);
}
static int64_t dep_at(const geo* G, int64_t i, int64_t j, int64_t k)
{
    j = wrap(j, G->nyc); k = wrap(k, G->nzc);
    if (G->c.xbc == ORA_XBC_PERIODIC) i = wrap(i, G->nx);
    else { i += G->g; if (i < 0 || i >= G->ndx) return -1; }
    return i + G->ndx * (j + G->nyc * k);
}

/* Real shape weights of offset o in cell c and their derivatives d/do. */
static int shape_wd(int shape, int64_t c, double o, int64_t* first, double w[3], double dw[3])
{
    if (shape == 1) {
        *first = c; w[0] = 1.0 - o; w[1] = o; w[2] = 0.0;
        dw[0] = -1.0; dw[1] = 1.0; dw[2] = 0.0;
        return 2;
    }
    int64_t ic = c; double xi = o;
    if (o >= 0.5) { ic = c + 1; xi = o - 1.0; }
    *first = ic - 1;
    w[0] = 0.5 * (0.5 - xi) * (0.5 - xi);
    w[1] = 0.75 - xi * xi;
    w[2] = 0.5 * (0.5 + xi) * (0.5 + xi);
    dw[0] = -(0.5 - xi);
    dw[1] = -2.0 * xi;
    dw[2] = 0.5 + xi;
    return 3;
}

/* Stencil of one particle: node offsets, weights W and dW/dx_d. */
typedef struct {
    int np[3];
    int64_t first[3];
    double w[3][3], dw[3][3];
} stencil;

static void stencil_of(const geo* G, const int64_t c[3], const double o[3], stencil* S)
{
    for (int d = 0; d < 3; ++d) {
        S->np[d] = 1; S->first[d] = 0;
        S->w[d][0] = 1.0; S->w[d][1] = S->w[d][2] = 0.0;
        S->dw[d][0] = S->dw[d][1] = S->dw[d][2] = 0.0;
    }
    for (int d = 0; d < G->D; ++d) S->np[d] = shape_wd(G->c.shape, c[d], o[d], &S->first[d], S->w[d], S->dw[d]);
}

/* W and its gradient for stencil entry (a, b, cc). */
static double stencil_w(const stencil* S, int a, int b, int cc, double gW[3])
{
    double wx = S->w[0][a], wy = S->w[1][b], wz = S->w[2][cc];
    gW[0] = S->dw[0][a] * wy * wz;
    gW[1] = wx * S->dw[1][b] * wz;
    gW[2] = wx * wy * S->dw[2][cc];
    return wx * wy * wz;
}

/* ---------------------------------------------------------------------- */
/* random numbers (reading R6/R8 counter layout; Philox from the oracle)   */
/* ---------------------------------------------------------------------- */
static void draw4(const ora_cfg* c, uint64_t stream, int64_t c0, uint64_t c1, uint64_t c2, double u[4])
{
    uint64_t ctr[4] = {(uint64_t)c0, c1, c2, 0}, r[4];
    ora_philox(ctr, c->seed, stream, r);
    for (int i = 0; i < 4; ++i) u[i] = ((double)(r[i] >> 11) + 0.5) * 0x1.0p-53;
}

/* ---------------------------------------------------------------------- */
/* forward pieces recomputed in the reverse sweep                          */
/* ---------------------------------------------------------------------- */
static void gather_fw(const geo* G, const snap* S, const int64_t c[3], const double o[3], double E[3], double B[3])
{
    stencil st;
    stencil_of(G, c, o, &st);
    for (int d = 0; d < 3; ++d) E[d] = B[d] = 0.0;
    for (int a = 0; a < st.np[0]; ++a)
        for (int b = 0; b < st.np[1]; ++b)
            for (int cc = 0; cc < st.np[2]; ++cc) {
                double gW[3], W = stencil_w(&st, a, b, cc, gW);
                int64_t n = gather_at(G, st.first[0] + a, st.first[1] + b, st.first[2] + cc);
                for (int d = 0; d < 3; ++d) { E[d] += W * S->E[3 * n + d]; B[d] += W * S->Bb[3 * n + d]; }
            }
}

static void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Boris (q/m = 1): returns v^{n+1/2} for v^{n-1/2}. */
static void boris_fw(const double v[3], const double E[3], const double B[3], double dt, double out[3])
{
    double h = 0.5 * dt, vm[3], t[3], s[3], vp[3], c1[3], c2[3];
    for (int d = 0; d < 3; ++d) { vm[d] = v[d] + h * E[d]; t[d] = h * B[d]; }
    double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int d = 0; d < 3; ++d) s[d] = 2.0 * t[d] / (1.0 + tt);
    cross(vm, t, c1);
    for (int d = 0; d < 3; ++d) vp[d] = vm[d] + c1[d];
    cross(vp, s, c2);
    for (int d = 0; d < 3; ++d) out[d] = vm[d] + c2[d] + h * E[d];
}

/* Transpose of the Boris Jacobian: lam_out -> lam_v, lam_E, lam_B. */
static void boris_vjp(const double v[3], const double E[3], const double B[3], double dt, const double lo[3],
                      double lv[3], double lE[3], double lB[3])
{
    double h = 0.5 * dt, vm[3], t[3], s[3], vp[3], c1[3];
    for (int d = 0; d < 3; ++d) { vm[d] = v[d] + h * E[d]; t[d] = h * B[d]; }
    double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int d = 0; d < 3; ++d) s[d] = 2.0 * t[d] / (1.0 + tt);
    cross(vm, t, c1);
    for (int d = 0; d < 3; ++d) vp[d] = vm[d] + c1[d];
    /* out = vm + vp x s + h E */
    double lvm[3], lvp[3], ls[3], lt[3], tmp[3];
    for (int d = 0; d < 3; ++d) { lvm[d] = lo[d]; lE[d] = h * lo[d]; }
    cross(s, lo, lvp);                        /* d(vp x s).lo / d vp = s x lo */
    cross(lo, vp, ls);                        /* d(vp x s).lo / d s  = lo x vp */
    /* vp = vm + vm x t */
    cross(t, lvp, tmp);
    for (int d = 0; d < 3; ++d) lvm[d] += lvp[d] + tmp[d];
    cross(lvp, vm, lt);
    /* s = 2 t / (1 + tt) */
    double ts = t[0] * ls[0] + t[1] * ls[1] + t[2] * ls[2];
    double den = 1.0 + tt;
    for (int d = 0; d < 3; ++d) lt[d] += 2.0 * ls[d] / den - 4.0 * t[d] * ts / (den * den);
    /* t = h B, vm = v + h E */
    for (int d = 0; d < 3; ++d) { lB[d] = h * lt[d]; lv[d] = lvm[d]; lE[d] += h * lvm[d]; }
}

/* FS kick (reading R7) for a reflected particle: pre-wall velocity v and
 * overshoot delta (cells) -> new velocity and x (cells); returns 0 if the
 * re-entry was clamped (x has no derivative then). */
static int kick_fw(const geo* G, int64_t step, uint64_t id, const double v[3], double delta, double u2,
                   double vout[3], double* xnew)
{
    double wx = v[0] - u2, wy = v[1], wz = v[2];
    double wabs = sqrt(wx * wx + wy * wy + wz * wz);
    double U[4];
    draw4(&G->c, ORA_STREAM_WALL, step, id, 0, U);
    double a = u2 / wabs;
    double mu = a + (1.0 - a) * sqrt(U[2]);
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double phi = ADJ_TWO_PI * U[3];
    vout[0] = u2 - wabs * mu;
    vout[1] = wabs * st * cos(phi);
    vout[2] = wabs * st * sin(phi);
    double back = v[0] > 0.0 ? delta * (-vout[0]) / v[0] : 0.0;
    *xnew = (double)G->nx - back;
    return *xnew < (double)G->nx && v[0] > 0.0;
}

/* Transpose of the kick: (lam_x', lam_v') -> (lam_xpre, lam_vpre), and the
 * u2 adjoint added to *lu2. */
static void kick_vjp(const geo* G, int64_t step, uint64_t id, const double v[3], double delta, double u2,
                     double lx, const double lvo[3], double* lxpre, double lv[3], double* lu2)
{
    double wv[3] = {v[0] - u2, v[1], v[2]};
    double wabs = sqrt(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
    double U[4];
    draw4(&G->c, ORA_STREAM_WALL, step, id, 0, U);
    double a = u2 / wabs, su = sqrt(U[2]);
    double mu = a + (1.0 - a) * su;
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double phi = ADJ_TWO_PI * U[3], cp = cos(phi), sp = sin(phi);
    double vox = u2 - wabs * mu;
    double vo[3];
    double xnew;
    int live = kick_fw(G, step, id, v, delta, u2, vo, &xnew);
    double lvox = lvo[0], lvoy = lvo[1], lvoz = lvo[2];
    double ldelta = 0.0, lvx_direct = 0.0;
    if (live) {
        /* x' = nx + delta vox / vx */
        ldelta = lx * vox / v[0];
        lvox += lx * delta / v[0];
        lvx_direct = -lx * delta * vox / (v[0] * v[0]);
    }
    *lxpre = ldelta;
    double lu = lvox;
    double lwabs = -mu * lvox + st * (cp * lvoy + sp * lvoz);
    double lmu = -wabs * lvox;
    double lst = wabs * (cp * lvoy + sp * lvoz);
    if (st > 0.0) lmu += -mu / st * lst;
    double la = lmu * (1.0 - su);
    lu += la / wabs;
    lwabs += -la * u2 / (wabs * wabs);
    for (int d = 0; d < 3; ++d) lv[d] = lwabs * wv[d] / wabs;
    lu += -lv[0];
    lv[0] += lvx_direct;
    *lu2 += lu;
}

/* ---------------------------------------------------------------------- */
/* Ohm's law (reading R5) and its transpose                                */
/* ---------------------------------------------------------------------- */
static double pres(const geo* G, double n)
{
    double ne = fmax(n, G->c.n_floor);
    return 0.5 * G->c.beta_e * pow(ne, G->c.gamma_e);
}
static double dpres(const geo* G, double n)
{
    if (!(n > G->c.n_floor)) return 0.0;
    return 0.5 * G->c.beta_e * G->c.gamma_e * pow(n, G->c.gamma_e - 1.0);
}

/* Intermediates of Ohm's law at node (i,j,k). */
typedef struct {
    double bb[3], J[3], gp[3], Gm[3], num[3], ne;
    int64_t f;
} ohm_parts;

static void ohm_eval(const geo* G, const double* B, const double* fn, const double* fg, int64_t i, int64_t j,
                     int64_t k, ohm_parts* P)
{
    int D = G->D, nb = D >= 2 ? 2 : 1, nc = D >= 3 ? 2 : 1;
    double dx = G->c.dx, dBx[3] = {0, 0, 0}, dBy[3] = {0, 0, 0}, dBz[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) P->bb[d] = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < nb; ++b)
            for (int c = 0; c < nc; ++c)
                for (int d = 0; d < 3; ++d) P->bb[d] += B_at(G, B, i - 1 + a, j - 1 + b, k - 1 + c, d);
    for (int d = 0; d < 3; ++d) P->bb[d] /= (double)(2 * nb * nc);
    for (int b = 0; b < nb; ++b)
        for (int c = 0; c < nc; ++c)
            for (int d = 0; d < 3; ++d)
                dBx[d] += B_at(G, B, i, j - 1 + b, k - 1 + c, d) - B_at(G, B, i - 1, j - 1 + b, k - 1 + c, d);
    for (int d = 0; d < 3; ++d) dBx[d] = dBx[d] / (double)(nb * nc) / dx;
    if (D >= 2) {
        for (int a = 0; a < 2; ++a)
            for (int c = 0; c < nc; ++c)
                for (int d = 0; d < 3; ++d)
                    dBy[d] += B_at(G, B, i - 1 + a, j, k - 1 + c, d) - B_at(G, B, i - 1 + a, j - 1, k - 1 + c, d);
        for (int d = 0; d < 3; ++d) dBy[d] = dBy[d] / (double)(2 * nc) / dx;
    }
    if (D >= 3) {
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int d = 0; d < 3; ++d)
                    dBz[d] += B_at(G, B, i - 1 + a, j - 1 + b, k, d) - B_at(G, B, i - 1 + a, j - 1 + b, k - 1, d);
        for (int d = 0; d < 3; ++d) dBz[d] = dBz[d] / 4.0 / dx;
    }
    P->J[0] = dBy[2] - dBz[1];
    P->J[1] = dBz[0] - dBx[2];
    P->J[2] = dBx[1] - dBy[0];
    P->gp[0] = P->gp[1] = P->gp[2] = 0.0;
    P->gp[0] = (pres(G, fn[fluid_at(G, i + 1, j, k)]) - pres(G, fn[fluid_at(G, i - 1, j, k)])) * G->h2dx;
    if (D >= 2) P->gp[1] = (pres(G, fn[fluid_at(G, i, j + 1, k)]) - pres(G, fn[fluid_at(G, i, j - 1, k)])) * G->h2dx;
    if (D >= 3) P->gp[2] = (pres(G, fn[fluid_at(G, i, j, k + 1)]) - pres(G, fn[fluid_at(G, i, j, k - 1)])) * G->h2dx;
    P->f = fluid_at(G, i, j, k);
    P->ne = fmax(fn[P->f], G->c.n_floor);
    P->Gm[0] = fg[3 * P->f] + G->c.j_ext;
    P->Gm[1] = fg[3 * P->f + 1];
    P->Gm[2] = fg[3 * P->f + 2];
    double c1[3], c2[3];
    cross(P->Gm, P->bb, c1);
    cross(P->J, P->bb, c2);
    for (int d = 0; d < 3; ++d) P->num[d] = -c1[d] + c2[d] - P->gp[d];
}

/* Forward Ohm at node (i,j,k): E and Bbar. */
static void ohm_fw(const geo* G, const double* B, const double* fn, const double* fg, int64_t i, int64_t j,
                   int64_t k, double E[3], double bb[3])
{
    ohm_parts P;
    ohm_eval(G, B, fn, fg, i, j, k, &P);
    for (int d = 0; d < 3; ++d) { E[d] = P.num[d] / P.ne + G->c.eta * P.J[d]; bb[d] = P.bb[d]; }
    if (inflow_node(G, i)) {
        /* E = -u_sh x_hat x B0 */
        E[0] = 0.0;
        E[1] = G->c.u_sh * G->B0[2];
        E[2] = -G->c.u_sh * G->B0[1];
    }
    if (conduct_node(G, i)) { E[1] = 0.0; E[2] = 0.0; }
}

/* Transpose of Ohm at one node: (lam_E, lam_Bbar) -> lam_B (centres),
 * lam_fn, lam_fg (nodes). */
static void ohm_vjp_node(const geo* G, const double* B, const double* fn, const double* fg, int64_t i, int64_t j,
                         int64_t k, const double lE[3], const double lbbo[3], double* lB, double* lfn, double* lfg)
{
    int D = G->D, nb = D >= 2 ? 2 : 1, nc = D >= 3 ? 2 : 1;
    double dx = G->c.dx;
    ohm_parts P;
    ohm_eval(G, B, fn, fg, i, j, k, &P);
    double ne = P.ne;
    /* at the inflow node E depends on u_sh only: lam_E goes there and
     * nowhere else (lam_Bbar still reaches the centres) */
    static const double lE0[3] = {0, 0, 0};
    if (inflow_node(G, i)) {
        if (G->lu_inflow) *G->lu_inflow += lE[1] * G->B0[2] - lE[2] * G->B0[1];
        lE = lE0;
    }
    /* at the conducting wall node E_y, E_z are constants: only lam_E_x passes */
    double lEc[3];
    if (conduct_node(G, i)) {
        lEc[0] = lE[0]; lEc[1] = 0.0; lEc[2] = 0.0;
        lE = lEc;
    }
    /* E = num / ne + eta J */
    double lnum[3], lJ[3], lbb[3], lG[3], lgp[3], tmp[3];
    double lne = 0.0;
    for (int d = 0; d < 3; ++d) {
        lnum[d] = lE[d] / ne;
        lne += -P.num[d] * lE[d] / (ne * ne);
        lJ[d] = G->c.eta * lE[d];
        lbb[d] = lbbo[d];
    }
    /* num = -(G x bb) + (J x bb) - gp */
    cross(P.bb, lnum, tmp);                    /* d(a x bb).l / da = bb x l */
    for (int d = 0; d < 3; ++d) { lG[d] = -tmp[d]; lJ[d] += tmp[d]; }
    double diffv[3] = {P.J[0] - P.Gm[0], P.J[1] - P.Gm[1], P.J[2] - P.Gm[2]};
    cross(lnum, diffv, tmp);                   /* d(a x bb).l / dbb = l x a */
    for (int d = 0; d < 3; ++d) { lbb[d] += tmp[d]; lgp[d] = -lnum[d]; }
    /* fluid */
    int64_t f = P.f;
    if (fn[f] > G->c.n_floor) lfn[f] += lne;
    for (int d = 0; d < 3; ++d) lfg[3 * f + d] += lG[d];
    {
        int64_t fp = fluid_at(G, i + 1, j, k), fm = fluid_at(G, i - 1, j, k);
        lfn[fp] += lgp[0] * G->h2dx * dpres(G, fn[fp]);
        lfn[fm] -= lgp[0] * G->h2dx * dpres(G, fn[fm]);
    }
    if (D >= 2) {
        int64_t fp = fluid_at(G, i, j + 1, k), fm = fluid_at(G, i, j - 1, k);
        lfn[fp] += lgp[1] * G->h2dx * dpres(G, fn[fp]);
        lfn[fm] -= lgp[1] * G->h2dx * dpres(G, fn[fm]);
    }
    if (D >= 3) {
        int64_t fp = fluid_at(G, i, j, k + 1), fm = fluid_at(G, i, j, k - 1);
        lfn[fp] += lgp[2] * G->h2dx * dpres(G, fn[fp]);
        lfn[fm] -= lgp[2] * G->h2dx * dpres(G, fn[fm]);
    }
    /* J = (dBy_z - dBz_y, dBz_x - dBx_z, dBx_y - dBy_x) */
    double ldBx[3] = {0, 0, 0}, ldBy[3] = {0, 0, 0}, ldBz[3] = {0, 0, 0};
    ldBy[2] += lJ[0]; ldBz[1] -= lJ[0];
    ldBz[0] += lJ[1]; ldBx[2] -= lJ[1];
    ldBx[1] += lJ[2]; ldBy[0] -= lJ[2];
    /* bb and the differences back to the centres */
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < nb; ++b)
            for (int c = 0; c < nc; ++c) {
                int64_t q = cent_at(G, i - 1 + a, j - 1 + b, k - 1 + c);
                if (q < 0) continue;
                for (int d = 0; d < 3; ++d) {
                    double acc = lbb[d] / (double)(2 * nb * nc);
                    acc += (a == 1 ? 1.0 : -1.0) * ldBx[d] / (double)(nb * nc) / dx;
                    if (D >= 2) acc += (b == 1 ? 1.0 : -1.0) * ldBy[d] / (double)(2 * nc) / dx;
                    if (D >= 3) acc += (c == 1 ? 1.0 : -1.0) * ldBz[d] / 4.0 / dx;
                    lB[3 * q + d] += acc;
                }
            }
}

static void ohm_vjp_all(const geo* G, const double* B, const double* fn, const double* fg, const double* lE,
                        const double* lbb, double* lB, double* lfn, double* lfg)
{
    static const double zero[3] = {0, 0, 0};
    for (int64_t k = 0; k < G->nzc; ++k)
        for (int64_t j = 0; j < G->nyc; ++j)
            for (int64_t i = 0; i < G->nxn; ++i) {
                int64_t n = i + G->nxn * (j + G->nyc * k);
                ohm_vjp_node(G, B, fn, fg, i, j, k, &lE[3 * n], lbb ? &lbb[3 * n] : zero, lB, lfn, lfg);
            }
}

static void ohm_all_fw(const geo* G, const double* B, const double* fn, const double* fg, double* E)
{
    for (int64_t k = 0; k < G->nzc; ++k)
        for (int64_t j = 0; j < G->nyc; ++j)
            for (int64_t i = 0; i < G->nxn; ++i) {
                double e[3], b[3];
                ohm_fw(G, B, fn, fg, i, j, k, e, b);
                int64_t n = i + G->nxn * (j + G->nyc * k);
                for (int d = 0; d < 3; ++d) E[3 * n + d] = e[d];
            }
}

/* -curl E at the centres (node -> centre differences). */
static void faraday_fw(const geo* G, const double* E, double* F)
{
    int D = G->D, nb = D >= 2 ? 2 : 1, nc = D >= 3 ? 2 : 1;
    double dx = G->c.dx;
    for (int64_t k = 0; k < G->nzc; ++k)
        for (int64_t j = 0; j < G->nyc; ++j)
            for (int64_t i = 0; i < G->nx; ++i) {
                double dEx[3] = {0, 0, 0}, dEy[3] = {0, 0, 0}, dEz[3] = {0, 0, 0};
                for (int b = 0; b < nb; ++b)
                    for (int c = 0; c < nc; ++c)
                        for (int d = 0; d < 3; ++d)
                            dEx[d] += E[3 * node_at(G, i + 1, j + b, k + c) + d] - E[3 * node_at(G, i, j + b, k + c) + d];
                for (int d = 0; d < 3; ++d) dEx[d] = dEx[d] / (double)(nb * nc) / dx;
                if (D >= 2) {
                    for (int a = 0; a < 2; ++a)
                        for (int c = 0; c < nc; ++c)
                            for (int d = 0; d < 3; ++d)
                                dEy[d] += E[3 * node_at(G, i + a, j + 1, k + c) + d] - E[3 * node_at(G, i + a, j, k + c) + d];
                    for (int d = 0; d < 3; ++d) dEy[d] = dEy[d] / (double)(2 * nc) / dx;
                }
                if (D >= 3) {
                    for (int a = 0; a < 2; ++a)
                        for (int b = 0; b < 2; ++b)
                            for (int d = 0; d < 3; ++d)
                                dEz[d] += E[3 * node_at(G, i + a, j + b, k + 1) + d] - E[3 * node_at(G, i + a, j + b, k) + d];
                    for (int d = 0; d < 3; ++d) dEz[d] = dEz[d] / 4.0 / dx;
                }
                int64_t n = i + G->nx * (j + G->nyc * k);
                F[3 * n + 0] = -(dEy[2] - dEz[1]);
                F[3 * n + 1] = -(dEz[0] - dEx[2]);
                F[3 * n + 2] = -(dEx[1] - dEy[0]);
            }
}

/* Transpose of faraday_fw: lam_F (centres) -> lam_E (nodes, added). */
static void faraday_vjp(const geo* G, const double* lF, double* lE)
{
    int D = G->D, nb = D >= 2 ? 2 : 1, nc = D >= 3 ? 2 : 1;
    double dx = G->c.dx;
    for (int64_t k = 0; k < G->nzc; ++k)
        for (int64_t j = 0; j < G->nyc; ++j)
            for (int64_t i = 0; i < G->nx; ++i) {
                int64_t n = i + G->nx * (j + G->nyc * k);
                double l0 = lF[3 * n], l1 = lF[3 * n + 1], l2 = lF[3 * n + 2];
                double ldEx[3] = {0, -l2, l1}, ldEy[3] = {l2, 0, -l0}, ldEz[3] = {-l1, l0, 0};
                for (int b = 0; b < nb; ++b)
                    for (int c = 0; c < nc; ++c)
                        for (int d = 0; d < 3; ++d) {
                            double s = ldEx[d] / (double)(nb * nc) / dx;
                            lE[3 * node_at(G, i + 1, j + b, k + c) + d] += s;
                            lE[3 * node_at(G, i, j + b, k + c) + d] -= s;
                        }
                if (D >= 2)
                    for (int a = 0; a < 2; ++a)
                        for (int c = 0; c < nc; ++c)
                            for (int d = 0; d < 3; ++d) {
                                double s = ldEy[d] / (double)(2 * nc) / dx;
                                lE[3 * node_at(G, i + a, j + 1, k + c) + d] += s;
                                lE[3 * node_at(G, i + a, j, k + c) + d] -= s;
                            }
                if (D >= 3)
                    for (int a = 0; a < 2; ++a)
                        for (int b = 0; b < 2; ++b)
                            for (int d = 0; d < 3; ++d) {
                                double s = ldEz[d] / 4.0 / dx;
                                lE[3 * node_at(G, i + a, j + b, k + 1) + d] += s;
                                lE[3 * node_at(G, i + a, j + b, k) + d] -= s;
                            }
            }
}

/* F(B) = -curl Ohm(B) and the transpose of its Jacobian applied to lam_F. */
static void rhs_fw(const geo* G, const double* B, const double* fn, const double* fg, double* E, double* F)
{
    ohm_all_fw(G, B, fn, fg, E);
    faraday_fw(G, E, F);
}
static void rhs_vjp(const geo* G, const double* B, const double* fn, const double* fg, const double* lF, double* lB,
                    double* lfn, double* lfg)
{
    double* lE = (double*)calloc((size_t)(3 * G->nnode), sizeof(double));
    faraday_vjp(G, lF, lE);
    ohm_vjp_all(G, B, fn, fg, lE, NULL, lB, lfn, lfg);
    free(lE);
}

/* SSP-RK3 over dt in n_sub substeps (reading R4), transposed: lam_B holds
 * lam(B^{n+1}) on entry and lam(B^n) on exit; lam_fn, lam_fg are added to. */
static void rk3_vjp(const geo* G, const double* Bn, const double* fn, const double* fg, double* lB, double* lfn,
                    double* lfg)
{
    int ns = G->c.n_sub;
    int64_t N = 3 * G->ncent;
    size_t nb = (size_t)N * sizeof(double);
    double h = G->c.dt / (double)ns;
    double* Bs = (double*)malloc(nb * (size_t)ns);   /* B at the start of each substep */
    double *B1 = (double*)malloc(nb), *B2 = (double*)malloc(nb), *F = (double*)malloc(nb);
    double* E = (double*)malloc((size_t)(3 * G->nnode) * sizeof(double));
    memcpy(Bs, Bn, nb);
    for (int s = 0; s < ns; ++s) {
        double* B0 = Bs + (size_t)s * N;
        rhs_fw(G, B0, fn, fg, E, F);
        for (int64_t q = 0; q < N; ++q) B1[q] = B0[q] + h * F[q];
        rhs_fw(G, B1, fn, fg, E, F);
        for (int64_t q = 0; q < N; ++q) B2[q] = 0.75 * B0[q] + 0.25 * (B1[q] + h * F[q]);
        rhs_fw(G, B2, fn, fg, E, F);
        if (s + 1 < ns)
            for (int64_t q = 0; q < N; ++q) Bs[(size_t)(s + 1) * N + q] = (1.0 / 3.0) * B0[q] + (2.0 / 3.0) * (B2[q] + h * F[q]);
    }
    double *l0 = (double*)malloc(nb), *l1 = (double*)malloc(nb), *l2 = (double*)malloc(nb), *lF = (double*)malloc(nb);
    for (int s = ns - 1; s >= 0; --s) {
        double* B0 = Bs + (size_t)s * N;
        rhs_fw(G, B0, fn, fg, E, F);
        for (int64_t q = 0; q < N; ++q) B1[q] = B0[q] + h * F[q];
        rhs_fw(G, B1, fn, fg, E, F);
        for (int64_t q = 0; q < N; ++q) B2[q] = 0.75 * B0[q] + 0.25 * (B1[q] + h * F[q]);
        /* B3 = 1/3 B0 + 2/3 (B2 + h F(B2)) */
        for (int64_t q = 0; q < N; ++q) {
            l0[q] = (1.0 / 3.0) * lB[q];
            l2[q] = (2.0 / 3.0) * lB[q];
            lF[q] = (2.0 / 3.0) * h * lB[q];
        }
        rhs_vjp(G, B2, fn, fg, lF, l2, lfn, lfg);
        /* B2 = 3/4 B0 + 1/4 (B1 + h F(B1)) */
        for (int64_t q = 0; q < N; ++q) {
            l0[q] += 0.75 * l2[q];
            l1[q] = 0.25 * l2[q];
            lF[q] = 0.25 * h * l2[q];
        }
        rhs_vjp(G, B1, fn, fg, lF, l1, lfn, lfg);
        /* B1 = B0 + h F(B0) */
        for (int64_t q = 0; q < N; ++q) {
            l0[q] += l1[q];
            lF[q] = h * l1[q];
        }
        rhs_vjp(G, B0, fn, fg, lF, l0, lfn, lfg);
        memcpy(lB, l0, nb);
    }
    free(Bs); free(B1); free(B2); free(F); free(E); free(l0); free(l1); free(l2); free(lF);
}

/* ---------------------------------------------------------------------- */
/* tape                                                                    */
/* ---------------------------------------------------------------------- */
static void snap_take(const geo* G, ora_sim* s, snap* S)
{
    for (int k = 0; k < 2; ++k) {
        int64_t n = ora_count(s, k);
        psnap* p = &S->sp[k];
        p->n = n;
        p->c = (int64_t*)malloc((size_t)(3 * n + 3) * sizeof(int64_t));
        p->o = (double*)malloc((size_t)(3 * n + 3) * sizeof(double));
        p->v = (double*)malloc((size_t)(3 * n + 3) * sizeof(double));
        p->id = (uint64_t*)malloc((size_t)(n + 1) * sizeof(uint64_t));
        ora_get_particles(s, k, p->c, p->o, p->v, p->id);
    }
    S->B = (double*)malloc((size_t)(3 * G->ncent) * sizeof(double));
    S->E = (double*)malloc((size_t)(3 * G->nnode) * sizeof(double));
    S->Bb = (double*)malloc((size_t)(3 * G->nnode) * sizeof(double));
    S->fn = (double*)malloc((size_t)G->nnode * sizeof(double));
    S->fg = (double*)malloc((size_t)(3 * G->nnode) * sizeof(double));
    ora_get_B(s, S->B);
    ora_get_E(s, S->E);
    ora_get_Bbar(s, S->Bb);
    ora_get_fluid(s, S->fn, S->fg);
    for (int k = 0; k < 2; ++k) {
        S->Mc[k] = (double*)malloc((size_t)(4 * G->ndep) * sizeof(double));
        ora_get_cmoments(s, k, S->Mc[k]);
    }
    S->next_id = ora_next_id(s);
}

static void snap_free(snap* S)
{
    for (int k = 0; k < 2; ++k) {
        free(S->sp[k].c); free(S->sp[k].o); free(S->sp[k].v); free(S->sp[k].id);
        free(S->Mc[k]);
    }
    free(S->B); free(S->E); free(S->Bb); free(S->fn); free(S->fg);
}

static double species_w(const geo* G, int k)
{
    /* a species with no ions per cell contributes no moments: weight 0 */
    return k == 0 ? (G->c.ppc > 0 ? 1.0 / (double)G->c.ppc : 0.0) : G->c.alpha_cr * G->c.n_cr / (double)G->c.ppc_cr;
}

/* Transpose of fluid_from_moments: lam_fn, lam_fg -> lam_Mc per species;
 * returns the alpha_cr adjoint. */
static double fluid_vjp(const geo* G, const snap* S, const double* lfn, const double* lfg, double* lM[2])
{
    double la = 0.0;
    int has_cr = G->c.n_cr > 0.0;
    for (int k = 0; k < 2; ++k) memset(lM[k], 0, (size_t)(4 * G->ndep) * sizeof(double));
    for (int64_t n = 0; n < G->nnode; ++n) {
        int64_t i = n % G->nxn, rest = n / G->nxn;
        int64_t dn = (i + G->g) + G->ndx * rest;
        for (int k = 0; k < (has_cr ? 2 : 1); ++k) {
            double w = species_w(G, k);
            lM[k][4 * dn] += w * lfn[n];
            for (int d = 0; d < 3; ++d) lM[k][4 * dn + 1 + d] += w * lfg[3 * n + d];
        }
        if (has_cr) {
            double dw = G->c.n_cr / (double)G->c.ppc_cr;
            la += dw * S->Mc[1][4 * dn] * lfn[n];
            for (int d = 0; d < 3; ++d) la += dw * S->Mc[1][4 * dn + 1 + d] * lfg[3 * n + d];
        }
    }
    return la;
}

/* Transpose of the real-weight deposit of the particles of one snapshot. */
static void deposit_vjp(const geo* G, const snap* S, double* lM[2], double* lx, double* lv)
{
    for (int k = 0; k < 2; ++k) {
        const psnap* p = &S->sp[k];
        for (int64_t q = 0; q < p->n; ++q) {
            stencil st;
            stencil_of(G, &p->c[3 * q], &p->o[3 * q], &st);
            const double* v = &p->v[3 * q];
            uint64_t id = p->id[q];
            for (int a = 0; a < st.np[0]; ++a)
                for (int b = 0; b < st.np[1]; ++b)
                    for (int cc = 0; cc < st.np[2]; ++cc) {
                        int64_t n = dep_at(G, st.first[0] + a, st.first[1] + b, st.first[2] + cc);
                        if (n < 0) continue;
                        double gW[3], W = stencil_w(&st, a, b, cc, gW);
                        double lm = lM[k][4 * n] + lM[k][4 * n + 1] * v[0] + lM[k][4 * n + 2] * v[1] + lM[k][4 * n + 3] * v[2];
                        for (int d = 0; d < G->D; ++d) lx[3 * id + d] += gW[d] * lm;
                        for (int d = 0; d < 3; ++d) lv[3 * id + d] += W * lM[k][4 * n + 1 + d];
                    }
        }
    }
}

/* u_sh adjoint of one particle injected at `step` (reading R8). */
static double inject_vjp(const geo* G, int k, int64_t step, uint64_t id, const double* lx, const double* lv)
{
    const ora_cfg* c = &G->c;
    double dtdx = c->dt / c->dx;
    if (k == 0) {
        double U[4], V[4];
        draw4(c, ORA_STREAM_INJECT_TH, step, id, 0, U);
        draw4(c, ORA_STREAM_INJECT_TH, step, id, 1, V);
        double n1 = sqrt(-2.0 * log(V[0])) * cos(ADJ_TWO_PI * V[1]);
        double sig = sqrt(0.5 * c->beta_i);
        double vx = c->u_sh + sig * n1;
        double sgn = vx >= 0.0 ? 1.0 : -1.0;
        double xi = fabs(vx) * U[0] * dtdx;
        double dx_du = xi < (double)c->nx ? sgn * U[0] * dtdx : 0.0;
        return lv[0] * sgn + lx[0] * dx_du;
    }
    double U[4];
    draw4(c, ORA_STREAM_INJECT_CR, step, id, 0, U);
    double wabs = c->cr_w, u2 = G->u2, a = u2 / wabs, su = sqrt(U[2]);
    double mu = a + (1.0 - a) * su;
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double phi = ADJ_TWO_PI * U[3];
    double vx = u2 - wabs * mu;
    double dmu = (1.0 - su) / wabs;
    double dvx = 1.0 - wabs * dmu;
    double dst = st > 0.0 ? -mu / st * dmu : 0.0;
    double dvy = wabs * cos(phi) * dst, dvz = wabs * sin(phi) * dst;
    double sgn = vx >= 0.0 ? 1.0 : -1.0;
    double xi = (double)c->nx - fabs(vx) * U[0] * dtdx;
    double dxi = xi < (double)c->nx ? -sgn * dvx * U[0] * dtdx : 0.0;
    return (lv[0] * dvx + lv[1] * dvy + lv[2] * dvz + lx[0] * dxi) / c->r;
}

/* ---------------------------------------------------------------------- */
/* the whole reverse sweep                                                 */
/* ---------------------------------------------------------------------- */
int ora_adjoint(const ora_cfg* cfg, const double* amps, int64_t nsteps, double* loss, double* grad)
{
    /* the reverse sweep covers the non-relativistic push only */
    if (cfg->c_light != 0.0) return -1;
    ora_cfg c = *cfg;
    c.deposit_mode = 1;
    if (c.n_sub < 1) c.n_sub = 1;
    geo G;
    geo_init(&G, &c);
    ora_sim* s = ora_new(&c);
    if (!s) return -1;
    ora_init(s, amps);
    snap* T = (snap*)calloc((size_t)(nsteps + 1), sizeof(snap));
    snap_take(&G, s, &T[0]);
    for (int64_t n = 0; n < nsteps; ++n) {
        ora_stats st;
        ora_step(s, ORA_ALL, &st);
        snap_take(&G, s, &T[n + 1]);
    }
    ora_free(s);

    int64_t nid = T[nsteps].next_id + 1;
    double* lx = (double*)calloc((size_t)(3 * nid), sizeof(double));
    double* lv = (double*)calloc((size_t)(3 * nid), sizeof(double));
    double* lB = (double*)calloc((size_t)(3 * G.ncent), sizeof(double));
    double* lE = (double*)calloc((size_t)(3 * G.nnode), sizeof(double));
    double* lbb = (double*)calloc((size_t)(3 * G.nnode), sizeof(double));
    double* lfn = (double*)calloc((size_t)G.nnode, sizeof(double));
    double* lfg = (double*)calloc((size_t)(3 * G.nnode), sizeof(double));
    double* lM[2];
    for (int k = 0; k < 2; ++k) lM[k] = (double*)calloc((size_t)(4 * G.ndep), sizeof(double));
    char* alive = (char*)calloc((size_t)nid, 1);
    double lu = 0.0, la = 0.0;
    G.lu_inflow = &lu;

    /* loss and its seed */
    double L = 0.0;
    for (int64_t k = 0; k < G.nzc; ++k)
        for (int64_t j = 0; j < G.nyc; ++j)
            for (int64_t i = G.nx / 2; i < G.nx; ++i) {
                int64_t q = i + G.nx * (j + G.nyc * k);
                double by = T[nsteps].B[3 * q + 1], bz = T[nsteps].B[3 * q + 2];
                L += by * by + bz * bz;
                lB[3 * q + 1] = 2.0 * by;
                lB[3 * q + 2] = 2.0 * bz;
            }
    *loss = L;

    double dtdx = c.dt / c.dx;
    for (int64_t n = nsteps - 1; n >= 0; --n) {
        const snap* S0 = &T[n];
        const snap* S1 = &T[n + 1];
        memset(lfn, 0, (size_t)G.nnode * sizeof(double));
        memset(lfg, 0, (size_t)(3 * G.nnode) * sizeof(double));
        /* final Ohm of step n, then the RK3 update with the moments frozen */
        ohm_vjp_all(&G, S1->B, S1->fn, S1->fg, lE, lbb, lB, lfn, lfg);
        rk3_vjp(&G, S0->B, S1->fn, S1->fg, lB, lfn, lfg);
        /* fluid moments and the deposit at x^{n+1} */
        la += fluid_vjp(&G, S1, lfn, lfg, lM);
        deposit_vjp(&G, S1, lM, lx, lv);
        /* particles injected during step n exist from n+1 on */
        memset(alive, 0, (size_t)nid);
        for (int k = 0; k < 2; ++k)
            for (int64_t q = 0; q < S1->sp[k].n; ++q) {
                uint64_t id = S1->sp[k].id[q];
                alive[id] = 1;
                if ((int64_t)id >= S0->next_id) {
                    lu += inject_vjp(&G, k, n, id, &lx[3 * id], &lv[3 * id]);
                    for (int d = 0; d < 3; ++d) lx[3 * id + d] = lv[3 * id + d] = 0.0;
                }
            }
        /* push, wall, gather of the particles that lived at step n */
        memset(lE, 0, (size_t)(3 * G.nnode) * sizeof(double));
        memset(lbb, 0, (size_t)(3 * G.nnode) * sizeof(double));
        for (int k = 0; k < 2; ++k) {
            const psnap* p = &S0->sp[k];
            int policy = k == 0 ? c.wall_th : c.wall_cr;
            for (int64_t q = 0; q < p->n; ++q) {
                uint64_t id = p->id[q];
                if (!alive[id]) continue;   /* removed during step n: no adjoint */
                const int64_t* cc = &p->c[3 * q];
                const double* o = &p->o[3 * q];
                const double* v0 = &p->v[3 * q];
                double Ep[3], Bp[3], v1[3];
                gather_fw(&G, S0, cc, o, Ep, Bp);
                boris_fw(v0, Ep, Bp, c.dt, v1);
                /* the move in x exactly as the forward step takes it */
                double xi = o[0] + v1[0] * dtdx, fl = floor(xi);
                int64_t cnew = cc[0] + (int64_t)fl;
                double onew = xi - fl;
                if (onew >= 1.0) { onew = 0.0; cnew += 1; }
                double lxp[3], lvp[3];
                for (int d = 0; d < 3; ++d) { lxp[d] = lx[3 * id + d]; lvp[d] = lv[3 * id + d]; }
                if (c.xbc == ORA_XBC_BOX && cnew >= G.nx && policy != ORA_OPEN) {
                    /* reflected at the wall during step n (it survived) */
                    double delta = (double)(cnew - G.nx) + onew;
                    double lxpre, lvpre[3], lu2 = 0.0;
                    if (policy == ORA_FAUX_SHOCK) {
                        kick_vjp(&G, n, id, v1, delta, G.u2, lxp[0], lvp, &lxpre, lvpre, &lu2);
                    } else {
                        lxpre = -lxp[0];
                        lvpre[0] = -lvp[0]; lvpre[1] = lvp[1]; lvpre[2] = lvp[2];
                    }
                    lu += lu2 / c.r;
                    lxp[0] = lxpre;
                    for (int d = 0; d < 3; ++d) lvp[d] = lvpre[d];
                }
                /* move: x^{n+1} = x^n + v^{n+1/2} dt/dx */
                for (int d = 0; d < G.D; ++d) lvp[d] += lxp[d] * dtdx;
                double lv0[3], lEp[3], lBp[3];
                boris_vjp(v0, Ep, Bp, c.dt, lvp, lv0, lEp, lBp);
                /* gather */
                stencil st;
                stencil_of(&G, cc, o, &st);
                double lx0[3] = {lxp[0], lxp[1], lxp[2]};
                for (int a = 0; a < st.np[0]; ++a)
                    for (int b = 0; b < st.np[1]; ++b)
                        for (int c3 = 0; c3 < st.np[2]; ++c3) {
                            double gW[3], W = stencil_w(&st, a, b, c3, gW);
                            int64_t m = gather_at(&G, st.first[0] + a, st.first[1] + b, st.first[2] + c3);
                            double dot = 0.0;
                            for (int d = 0; d < 3; ++d) {
                                dot += S0->E[3 * m + d] * lEp[d] + S0->Bb[3 * m + d] * lBp[d];
                                lE[3 * m + d] += W * lEp[d];
                                lbb[3 * m + d] += W * lBp[d];
                            }
                            for (int d = 0; d < G.D; ++d) lx0[d] += gW[d] * dot;
                        }
                for (int d = 0; d < 3; ++d) { lx[3 * id + d] = lx0[d]; lv[3 * id + d] = lv0[d]; }
            }
        }
    }
    /* E^0 = Ohm(B^0, moments^0) and the initial load */
    {
        const snap* S0 = &T[0];
        memset(lfn, 0, (size_t)G.nnode * sizeof(double));
        memset(lfg, 0, (size_t)(3 * G.nnode) * sizeof(double));
        ohm_vjp_all(&G, S0->B, S0->fn, S0->fg, lE, lbb, lB, lfn, lfg);
        la += fluid_vjp(&G, S0, lfn, lfg, lM);
        deposit_vjp(&G, S0, lM, lx, lv);
        for (int64_t q = 0; q < S0->sp[0].n; ++q) lu += lv[3 * S0->sp[0].id[q]];   /* v_x = u_sh + sigma n1 */
    }
    grad[0] = lu;
    grad[1] = la;
    /* Fourier amplitudes: dB_y = A cos(k x + phi), dB_z = A sin(k x + phi) */
    double Lx = (double)G.nx * c.dx;
    for (int m = 1; m <= c.n_modes; ++m) {
        double U[4];
        draw4(&c, ORA_STREAM_FOURIER, m, 0, 0, U);
        double ph0 = ADJ_TWO_PI * U[0], g = 0.0;
        for (int64_t k = 0; k < G.nzc; ++k)
            for (int64_t j = 0; j < G.nyc; ++j)
                for (int64_t i = 0; i < G.nx; ++i) {
                    double x = ((double)i + 0.5) * c.dx;
                    double ph = ADJ_TWO_PI * (double)m * x / Lx + ph0;
                    int64_t q = i + G.nx * (j + G.nyc * k);
                    g += lB[3 * q + 1] * cos(ph) + lB[3 * q + 2] * sin(ph);
                }
        grad[1 + m] = g;
    }
    for (int64_t n = 0; n <= nsteps; ++n) snap_free(&T[n]);
    free(T); free(lx); free(lv); free(lB); free(lE); free(lbb); free(lfn); free(lfg);
    free(lM[0]); free(lM[1]); free(alive);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* single-piece transposes, exported for the finite-difference pins        */
/* ---------------------------------------------------------------------- */
void ora_adj_boris(const double v[3], const double E[3], const double B[3], double dt, const double lo[3],
                   double out[3], double lv[3], double lE[3], double lB[3])
{
    boris_fw(v, E, B, dt, out);
    boris_vjp(v, E, B, dt, lo, lv, lE, lB);
}

void ora_adj_kick(const ora_cfg* cfg, int64_t step, uint64_t id, const double v[3], double delta, double u2,
                  double lxo, const double lvo[3], double out4[4], double lin5[5])
{
    geo G;
    geo_init(&G, cfg);
    double vo[3], xn;
    kick_fw(&G, step, id, v, delta, u2, vo, &xn);
    out4[0] = xn; out4[1] = vo[0]; out4[2] = vo[1]; out4[3] = vo[2];
    double lxpre, lv[3], lu2 = 0.0;
    kick_vjp(&G, step, id, v, delta, u2, lxo, lvo, &lxpre, lv, &lu2);
    lin5[0] = lxpre; lin5[1] = lv[0]; lin5[2] = lv[1]; lin5[3] = lv[2]; lin5[4] = lu2;
}

/* Ohm at every node for given B (3 x ncent) and fluid (fn, fg), and the
 * transpose applied to lam_E: lam_B, lam_fn, lam_fg (overwritten). */
void ora_adj_ohm(const ora_cfg* cfg, const double* B, const double* fn, const double* fg, const double* lE,
                 double* E, double* lB, double* lfn, double* lfg)
{
    geo G;
    geo_init(&G, cfg);
    ohm_all_fw(&G, B, fn, fg, E);
    memset(lB, 0, (size_t)(3 * G.ncent) * sizeof(double));
    memset(lfn, 0, (size_t)G.nnode * sizeof(double));
    memset(lfg, 0, (size_t)(3 * G.nnode) * sizeof(double));
    ohm_vjp_all(&G, B, fn, fg, lE, NULL, lB, lfn, lfg);
}

/* One SSP-RK3 field update (n_sub substeps) and its transpose applied to
 * lam_out: lam_B (in place), lam_fn, lam_fg (overwritten). */
void ora_adj_rk3(const ora_cfg* cfg, const double* B, const double* fn, const double* fg, double* Bout, double* lB,
                 double* lfn, double* lfg)
{
    geo G;
    geo_init(&G, cfg);
    int64_t N = 3 * G.ncent;
    double h = cfg->dt / (double)(cfg->n_sub < 1 ? 1 : cfg->n_sub);
    double* F = (double*)malloc((size_t)N * sizeof(double));
    double* B1 = (double*)malloc((size_t)N * sizeof(double));
    double* B2 = (double*)malloc((size_t)N * sizeof(double));
    double* E = (double*)malloc((size_t)(3 * G.nnode) * sizeof(double));
    memcpy(Bout, B, (size_t)N * sizeof(double));
    for (int s = 0; s < (cfg->n_sub < 1 ? 1 : cfg->n_sub); ++s) {
        rhs_fw(&G, Bout, fn, fg, E, F);
        for (int64_t q = 0; q < N; ++q) B1[q] = Bout[q] + h * F[q];
        rhs_fw(&G, B1, fn, fg, E, F);
        for (int64_t q = 0; q < N; ++q) B2[q] = 0.75 * Bout[q] + 0.25 * (B1[q] + h * F[q]);
        rhs_fw(&G, B2, fn, fg, E, F);
        for (int64_t q = 0; q < N; ++q) Bout[q] = (1.0 / 3.0) * Bout[q] + (2.0 / 3.0) * (B2[q] + h * F[q]);
    }
    memset(lfn, 0, (size_t)G.nnode * sizeof(double));
    memset(lfg, 0, (size_t)(3 * G.nnode) * sizeof(double));
    rk3_vjp(&G, B, fn, fg, lB, lfn, lfg);
    free(F); free(B1); free(B2); free(E);
}
