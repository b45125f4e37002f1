/*
 * fsoracle.c -- TEST INFRASTRUCTURE ONLY (never part of the product path).
 *
 * Plain, slow, obviously-correct FP64 CPU implementation of one time step of
 * the faux-shock (FS) hybrid particle-in-cell method of Simon, Caprioli,
 * Haggerty & Reville (2025).  Loops over particles, nodes and cells in their
 * natural order; no sorting, no atomics, no blocking.  Only tests/, the smoke
 * check and the benchmark's CPU-baseline leg load it.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * What the paper fixes and what is read into it
 * ----------------------------------------------
 * The paper (Sec. 2) adds a boundary condition to an existing hybrid code
 * (kinetic ions, massless charge-neutralising electron fluid) and defers the
 * discretisation to earlier papers.  The FS boundary itself is specified by
 * its return probability, eq. (1), the downstream speed u2 = u_sh / r, and the
 * statement that returning particles leave as if scattered isotropically in
 * the downstream frame.  Everything else below is a reading, written out here
 * and in the design notes, and shared with the GPU library only as a
 * specification (never as code):
 *
 *  R1 units: lengths d_i, times 1/Omega_ci, speeds v_A, B in B0, n in n_g;
 *     q/m = 1 (the paper's units, Sec. 2, last paragraph before Sec. 3).
 *  R2 geometry: FS wall at x = L, upstream plasma enters at x = 0 and flows
 *     toward the wall with +u_sh (the paper puts the FS on the left and flows
 *     in -x; the mirror image is the same physics).
 *  R3 grid: nodes at x_i = i dx hold E, n, Gamma; cell centres hold B.
 *     Centre->node and node->centre derivatives are differences averaged
 *     over the transverse directions, so div B stays at round-off.
 *  R4 step n -> n+1: gather E^n and Bbar^n with shape S (CIC or TSC); Boris
 *     rotation; move in cell units; boundaries (x<0 open, y/z periodic, FS
 *     wall at x >= L); injection; fixed-point deposit at x^{n+1} with
 *     v^{n+1/2}; SSP-RK3 Faraday update with the moments frozen; final Ohm.
 *  R5 Ohm: E = (-Gamma x Bbar + J x Bbar - grad p_e)/n_e + eta J, with
 *     J = curl B, p_e = (beta_e/2) n_e^gamma_e, n_e = max(n, n_floor),
 *     Gamma += J_ext x (rigid external current for the Bell test).
 *  R6 FS decision (eq. 1 with v_cr the downstream-frame speed |w|,
 *     w = v - u2 x): draw U1..U4 from Philox4x64-10 keyed (seed, WALL) with
 *     counter (step, id, 0, 0); m = max(U1, U2); reflect iff
 *     |w|^2 > (u2 (1+m)/(1-m))^2.  Since P(max(U1,U2) < rho) = rho^2 this
 *     reflects with probability ((1-u2/|w|)/(1+u2/|w|))^2, zero if |w| <= u2.
 *  R7 FS kick: |w| kept; direction cosine into the box
 *     mu' = a + (1-a) sqrt(U3), a = u2/|w| (flux of an isotropic downstream
 *     population that can outrun the flow); azimuth 2 pi U4; v' = w' + u2 x.
 *     The particle re-enters at x = L - (overshoot) |v'_x| / v_x.
 *  R8 injection: thermal at x = 0 with floor(F(s+1)) - floor(F s) particles
 *     per transverse cell, F = ppc u_sh dt/dx; CRs at x = L with
 *     F_cr = ppc_cr (|w| - u2) dt / (2 dx), directions from the R7 sampler.
 *  R9 fixed-point deposit: per-dimension integer weights from the quantised
 *     offset q = floor(off 2^b + 1/2), an exact partition of unity; velocity
 *     codes rint(v 2^s_v) saturated at 2^23-1 with s_v = 23 - ceil(log2
 *     v_max) for the run's largest expected speed v_max; int64 sums.
 *  R10 x boundaries of the box: the ghost centre at x = -1 holds B0, the one
 *     at nx copies the last cell; the inflow node x = 0 carries the motional
 *     field of the unperturbed upstream plasma, E = -u_sh x_hat x B0 (the
 *     plasma the boundary injects), not Ohm's law against the ghost: with
 *     the latter a 2D perturbation grows without bound at the boundary.
 *  R11 relativistic mode (the dHybridR push the paper runs with, Sec. 2),
 *     switched on by c_light = c / v_A > 0.  The velocity arrays then hold
 *     the four-velocity u = gamma v (momentum per unit mass), gamma =
 *     sqrt(1 + |u|^2 / c^2).  Push: half electric kick on u, rotation with
 *     t = (dt/2) B / gamma(u^-) (the relativistic Boris rotation), half
 *     kick, move with v = u / gamma.  Deposit: the flux uses v = u / gamma.
 *     Wall: eq. (1) and the R7 kick act in the downstream rest frame,
 *     reached by an exact Lorentz boost along x with speed u2; |w| is the
 *     speed in that frame, the kick keeps it.  Thermal loading and
 *     injection sample the R8 drifting Maxwellian in velocity and convert
 *     to u; CRs get the R8 downstream-frame speed cr_w, boosted to the lab.
 *     Kinetic energy is (gamma - 1) c^2 = |u|^2 / (gamma + 1) per mass.  The
 *     field update is unchanged.  c_light = 0 is the non-relativistic R4.
 *  R12 prescribed wall (wall_model = 1): the paper leaves the return rate,
 *     the anisotropy and the energy gain of the FS open to calibration
 *     against RW runs (Sec. 1) and allows a boundary that changes in time
 *     (Sec. 4).  Read as: at step s the wall uses u2 = u_sh / max(1, r +
 *     r_dot s dt); a crosser of downstream-frame speed |w| > u2 returns with
 *     probability min(1, f rho^2), rho = (|w| - u2) / (|w| + u2) (eq. 1 is
 *     rho^2), f = ret_f0 (|w| / cr_w)^ret_alpha; it leaves with speed (or,
 *     relativistic, four-velocity magnitude) multiplied by gain, in the
 *     direction cosine mu' of pdf ~ (mu' - a)^(1 + kappa) on (a, 1], a = u2 /
 *     new speed (kappa = 0 is R7's isotropic flux), azimuth uniform.  A
 *     return slower than u2 cannot leave and counts as transmitted.
 *  R13 smoothing (smooth = N > 0): the paper's codes smooth their fields
 *     but the paper does not say how.  Read as N passes of the 1-2-1
 *     binomial filter, f_i <- (f_{i-1} + 2 f_i + f_{i+1}) / 4, along x, then
 *     y, then z, on the boundary-filled ion density n_e = max(n, n_floor)
 *     and flux Gamma (without J_ext) at the nodes, before Ohm's law.  In the
 *     box the end nodes x = 0 and x = L keep their values; y, z (and x when
 *     periodic) wrap.  The boundary fill and the floor then apply again.
 *  R15 loss cone of the prescribed wall (lc_depletion > 0): the paper
 *     expects highly oblique shocks not to fill the CR loss cone isotropically,
 *     which changes the return probability and the energy gain (Sec. 3.2),
 *     and leaves the anisotropy to calibration (Sec. 1).  Read as: downstream
 *     CRs gyrate about the downstream field b2, whose normal component is
 *     B0's and whose tangential one is compressed by the wall's ratio r(t),
 *     b2 ~ (cos th_Bn, r sin th_Bn, 0).  A return direction n (drawn as in
 *     R12) lies in the loss cone when its motion along b2 alone outruns the
 *     receding shock, (n . s) |b2_x| > a = u2 / (return speed), s the field
 *     direction pointing upstream; such returns keep R12's weight, the rest
 *     (which reach the shock only through their gyration) are removed with
 *     probability lc_depletion, decided by U[1].  A parallel shock's cone
 *     holds every return direction, so the knob acts only at oblique ones;
 *     lc_depletion = 0 is R12 itself.
 *  R16 time-centred ion-field coupling (coupling = 2): the paper's 2D runs
 *     use dHybridR (Sec. 2), whose coupling is second order in time; the
 *     paper gives no scheme.  Read as: the push as in R4; the density is
 *     deposited at x^{n+1} and the flux at the midpoint of the move,
 *     x^{n+1/2} = x^n + v^{n+1/2} dt / 2, with v^{n+1/2} (ions reflected or
 *     injected during the step deposit both at their new position); the
 *     Faraday update from B^n to B^{n+1} holds the moments frozen at
 *     t_{n+1/2}: n^{n+1/2} = (n^n + n^{n+1}) / 2 and the midpoint flux; E^{n+1}
 *     takes n^{n+1} and the flux extrapolated to t_{n+1},
 *     (3 Gamma^{n+1/2} - Gamma^{n-1/2}) / 2.  The initial load's flux stands in
 *     for Gamma^{-1/2} and its density for n^0.  Smoothing is not combined
 *     with it.
 *  R14 conducting wall (wall_field = 1): the paper does not give the field
 *     boundary of its reflecting wall.  Read as a perfect conductor at rest
 *     in the simulation frame: the tangential E vanishes at the wall node
 *     x = L, E_y = E_z = 0, and E_x keeps Ohm's law.  With 0 the wall node
 *     keeps Ohm's law against the copied ghost (R10), the open boundary the
 *     faux-shock runs need.
 */
#include "fsoracle.h"
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORA_VSAT 8388607LL /* 2^23 - 1 */
#define ORA_TWO_PI 6.283185307179586

typedef struct ora_sp {
    int64_t n, cap;
    int64_t *c;    /* 3 per particle: cell index per dimension */
    double  *o;    /* 3 per particle: offset in [0,1) per dimension */
    double  *v;    /* 3 per particle */
    uint64_t *id;
    int64_t *ch;   /* R16: cell and offset of the midpoint of the last move */
    double  *oh;
} ora_sp;

typedef struct ora_event { int64_t step; uint64_t id; int32_t kind; } ora_event;

struct ora_sim {
    ora_cfg c;
    int64_t nyc, nzc;          /* active transverse sizes (1 when absent) */
    int64_t nxn, g, ndx;       /* field nodes in x, deposit ghosts, deposit nodes in x */
    int64_t ncent, nnode, ndep;
    int b, sv, SW, mclamp;
    double B0[3];
    double *B, *E, *Bb;        /* B at centres, E and Bbar at nodes (3 per point) */
    int64_t *M[2];             /* fixed-point moments per species: R, Gx, Gy, Gz */
    double *Mc[2];             /* continuous moments */
    double *fn, *fg;           /* fluid density and ion flux at nodes */
    double *fn_prev, *fg_prev; /* R16: density n^n and flux Gamma^{n-1/2} of the previous step */
    ora_sp sp[2];
    int64_t step, next_id;
    int32_t recording;
    ora_event *ev; int64_t nev, capev;
    const struct ora_sim *replay_ref; int64_t mismatch;
};

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11), written from the */
/* published round function: two 64x64->128 multiplies per round, key   */
/* bumped by the Weyl constants after every round.                      */
/* ------------------------------------------------------------------ */
void ora_philox(const uint64_t ctr[4], uint64_t k0, uint64_t k1, uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int r = 0; r < 10; ++r) {
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * x0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ x1 ^ k0, n1 = lo1, n2 = hi0 ^ x3 ^ k1, n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 53 random bits mapped to the open interval (0,1), exactly. */
static double u01(uint64_t r) { return ((double)(r >> 11) + 0.5) * 0x1.0p-53; }

static void draw(const ora_cfg* c, uint64_t stream, int64_t c0, uint64_t c1, uint64_t c2, double u[4])
{
    uint64_t ctr[4] = {(uint64_t)c0, c1, c2, 0}, r[4];
    ora_philox(ctr, c->seed, stream, r);
    for (int i = 0; i < 4; ++i) u[i] = u01(r[i]);
}

/* Box-Muller: two standard normals from two uniforms. */
static void normals(double ua, double ub, double* n1, double* n2)
{
    double rad = sqrt(-2.0 * log(ua));
    *n1 = rad * cos(ORA_TWO_PI * ub);
    *n2 = rad * sin(ORA_TWO_PI * ub);
}

static int64_t wrapi(int64_t i, int64_t n) { int64_t r = i % n; return r < 0 ? r + n : r; }

/* ------------------------------------------------------------------ */
/* relativistic mode (reading R11)                                      */
/* ------------------------------------------------------------------ */
static int relativistic(const ora_cfg* c) { return c->c_light > 0.0; }

/* Lorentz factor of the four-velocity u (momentum per unit mass). */
static double lorentz_u(const ora_cfg* c, const double u[3])
{
    double cc = c->c_light * c->c_light;
    return sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / cc);
}

/* Velocity of a particle from its stored velocity variable: u / gamma in
 * relativistic mode, the stored velocity itself otherwise. */
static void velocity_of(const ora_cfg* c, const double u[3], double v[3])
{
    if (!relativistic(c)) { for (int d = 0; d < 3; ++d) v[d] = u[d]; return; }
    double g = lorentz_u(c, u);
    for (int d = 0; d < 3; ++d) v[d] = u[d] / g;
}

/* Four-velocity of a particle moving with velocity v, |v| < c. */
static void four_velocity(const ora_cfg* c, const double v[3], double u[3])
{
    double cc = c->c_light * c->c_light;
    double g = 1.0 / sqrt(1.0 - (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / cc);
    for (int d = 0; d < 3; ++d) u[d] = g * v[d];
}

/* ------------------------------------------------------------------ */
/* construction                                                         */
/* ------------------------------------------------------------------ */
static int default_bits(int dim, int shape)
{
    static const int cic[4] = {0, 22, 11, 7};
    static const int tsc[4] = {0, 10, 5, 3};
    return shape == 2 ? tsc[dim] : cic[dim];
}

/* Velocity code scale: the largest |v| the run expects (v_max) maps to just
 * under 2^23, so s_v = 23 - ceil(log2 v_max). */
static int sv_bits(double v_max)
{
    int e;
    double m = frexp(v_max, &e);
    if (m == 0.5) e -= 1;
    return 23 - e;
}

ora_sim* ora_new(const ora_cfg* cfg)
{
    if (cfg->dim < 1 || cfg->dim > 3 || cfg->nx < 4 || cfg->shape < 1 || cfg->shape > 2) return NULL;
    if (!(cfg->v_max > 0.0)) return NULL;
    if (cfg->coupling != 1 && cfg->coupling != 2) return NULL;
    if (cfg->coupling == 2 && cfg->smooth > 0) return NULL;
    if (cfg->c_light < 0.0 || cfg->c_light != cfg->c_light) return NULL;
    if (relativistic(cfg)) {
        /* every sampled velocity below c: a Box-Muller normal is at most
         * sqrt(2 * 54 ln 2) < 8.66 in size, three of them < 15 */
        double sig = sqrt(0.5 * cfg->beta_i);
        if (!(cfg->u_sh + 15.0 * sig < cfg->c_light)) return NULL;
        if (!(cfg->u_sh / cfg->r < cfg->c_light)) return NULL;
        if (cfg->n_cr > 0.0 && !(cfg->cr_w < cfg->c_light)) return NULL;
    }
    ora_sim* s = (ora_sim*)calloc(1, sizeof(ora_sim));
    s->c = *cfg;
    if (s->c.n_sub < 1) s->c.n_sub = 1;
    s->nyc = cfg->dim >= 2 ? cfg->ny : 1;
    s->nzc = cfg->dim >= 3 ? cfg->nz : 1;
    s->nxn = cfg->xbc == ORA_XBC_PERIODIC ? cfg->nx : cfg->nx + 1;
    s->g = (cfg->xbc == ORA_XBC_BOX && cfg->shape == 2) ? 1 : 0;
    s->ndx = s->nxn + 2 * s->g;
    s->ncent = (int64_t)cfg->nx * s->nyc * s->nzc;
    s->nnode = s->nxn * s->nyc * s->nzc;
    s->ndep = s->ndx * s->nyc * s->nzc;
    s->b = default_bits(cfg->dim, cfg->shape);
    s->sv = sv_bits(cfg->v_max);
    s->SW = cfg->shape == 2 ? cfg->dim * (2 * s->b + 1) : cfg->dim * s->b;
    s->mclamp = cfg->shape;
    double th = cfg->theta_deg * (ORA_TWO_PI / 360.0);
    s->B0[0] = cos(th); s->B0[1] = sin(th); s->B0[2] = 0.0;
    s->B = (double*)calloc((size_t)(3 * s->ncent), sizeof(double));
    s->E = (double*)calloc((size_t)(3 * s->nnode), sizeof(double));
    s->Bb = (double*)calloc((size_t)(3 * s->nnode), sizeof(double));
    s->fn = (double*)calloc((size_t)s->nnode, sizeof(double));
    s->fg = (double*)calloc((size_t)(3 * s->nnode), sizeof(double));
    s->fn_prev = (double*)calloc((size_t)s->nnode, sizeof(double));
    s->fg_prev = (double*)calloc((size_t)(3 * s->nnode), sizeof(double));
    for (int k = 0; k < 2; ++k) {
        s->M[k] = (int64_t*)calloc((size_t)(4 * s->ndep), sizeof(int64_t));
        s->Mc[k] = (double*)calloc((size_t)(4 * s->ndep), sizeof(double));
    }
    for (int64_t i = 0; i < s->ncent; ++i)
        for (int d = 0; d < 3; ++d) s->B[3 * i + d] = s->B0[d];
    return s;
}

void ora_free(ora_sim* s)
{
    if (!s) return;
    free(s->B); free(s->E); free(s->Bb); free(s->fn); free(s->fg); free(s->fn_prev); free(s->fg_prev);
    for (int k = 0; k < 2; ++k) {
        free(s->M[k]); free(s->Mc[k]);
        free(s->sp[k].c); free(s->sp[k].o); free(s->sp[k].v); free(s->sp[k].id);
        free(s->sp[k].ch); free(s->sp[k].oh);
    }
    free(s->ev);
    free(s);
}

static void sp_reserve(ora_sp* p, int64_t n)
{
    if (n <= p->cap) return;
    int64_t cap = p->cap ? p->cap : 1024;
    while (cap < n) cap *= 2;
    p->c = (int64_t*)realloc(p->c, (size_t)(3 * cap) * sizeof(int64_t));
    p->o = (double*)realloc(p->o, (size_t)(3 * cap) * sizeof(double));
    p->v = (double*)realloc(p->v, (size_t)(3 * cap) * sizeof(double));
    p->id = (uint64_t*)realloc(p->id, (size_t)cap * sizeof(uint64_t));
    p->ch = (int64_t*)realloc(p->ch, (size_t)(3 * cap) * sizeof(int64_t));
    p->oh = (double*)realloc(p->oh, (size_t)(3 * cap) * sizeof(double));
    p->cap = cap;
}

static void sp_append(ora_sp* p, const int64_t c[3], const double o[3], const double v[3], uint64_t id)
{
    sp_reserve(p, p->n + 1);
    int64_t k = p->n++;
    for (int d = 0; d < 3; ++d) {
        p->c[3 * k + d] = c[d]; p->o[3 * k + d] = o[d]; p->v[3 * k + d] = v[d];
        p->ch[3 * k + d] = c[d]; p->oh[3 * k + d] = o[d];   /* born here: no move this step */
    }
    p->id[k] = id;
}

/* ------------------------------------------------------------------ */
/* grid access                                                          */
/* ------------------------------------------------------------------ */
static int64_t cent_idx(const ora_sim* s, int64_t i, int64_t j, int64_t k)
{
    return i + s->c.nx * (j + s->nyc * k);
}
static int64_t node_idx(const ora_sim* s, int64_t i, int64_t j, int64_t k)
{
    return i + s->nxn * (j + s->nyc * k);
}

/* B at a (possibly ghost) centre: inflow ghost holds B0, wall ghost copies
 * the last interior centre, transverse directions wrap (reading R3). */
static double centre_B(const ora_sim* s, const double* B, int64_t i, int64_t j, int64_t k, int comp)
{
    j = wrapi(j, s->nyc); k = wrapi(k, s->nzc);
    if (s->c.xbc == ORA_XBC_PERIODIC) i = wrapi(i, s->c.nx);
    else if (i < 0) return s->B0[comp];
    else if (i >= s->c.nx) i = s->c.nx - 1;
    return B[3 * cent_idx(s, i, j, k) + comp];
}

/* E at a node: x nodes 0..nx in the box, wrapped when periodic. */
static double node_E(const ora_sim* s, const double* E, int64_t i, int64_t j, int64_t k, int comp)
{
    j = wrapi(j, s->nyc); k = wrapi(k, s->nzc);
    if (s->c.xbc == ORA_XBC_PERIODIC) i = wrapi(i, s->c.nx);
    return E[3 * node_idx(s, i, j, k) + comp];
}

/* Node whose moments stand in for node i: within `shape` nodes of either
 * x boundary of the box the nearest fully-covered node is used. */
static int64_t fluid_node(const ora_sim* s, int64_t i, int64_t j, int64_t k)
{
    j = wrapi(j, s->nyc); k = wrapi(k, s->nzc);
    if (s->c.xbc == ORA_XBC_PERIODIC) i = wrapi(i, s->c.nx);
    else {
        if (i < s->mclamp) i = s->mclamp;
        if (i > s->c.nx - s->mclamp) i = s->c.nx - s->mclamp;
    }
    return node_idx(s, i, j, k);
}

/* Gather node index: box x clamped to the physical nodes, wrap otherwise. */
static int64_t gather_node(const ora_sim* s, int64_t i, int64_t j, int64_t k)
{
    j = wrapi(j, s->nyc); k = wrapi(k, s->nzc);
    if (s->c.xbc == ORA_XBC_PERIODIC) i = wrapi(i, s->c.nx);
    else { if (i < 0) i = 0; if (i > s->c.nx) i = s->c.nx; }
    return node_idx(s, i, j, k);
}

/* ------------------------------------------------------------------ */
/* shape functions                                                      */
/* ------------------------------------------------------------------ */
/* Real-valued 1D weights: CIC to nodes c, c+1; TSC to the nearest node and
 * its two neighbours.  Returns the number of nodes, first node in *first. */
static int shape_real(int shape, int64_t c, double o, int64_t* first, double w[3])
{
    if (shape == 1) {
        *first = c; w[0] = 1.0 - o; w[1] = o; return 2;
    }
    int64_t ic = c; double xi = o;
    if (o >= 0.5) { ic = c + 1; xi = o - 1.0; }
    *first = ic - 1;
    w[0] = 0.5 * (0.5 - xi) * (0.5 - xi);
    w[1] = 0.75 - xi * xi;
    w[2] = 0.5 * (0.5 + xi) * (0.5 + xi);
    return 3;
}

/* Integer 1D weights of the fixed-point deposit (reading R9). */
static int shape_int(int shape, int b, int64_t c, double o, int64_t* first, int64_t w[3])
{
    int64_t one = (int64_t)1 << b;
    int64_t q = (int64_t)floor(ldexp(o, b) + 0.5);
    if (shape == 1) {
        *first = c; w[0] = one - q; w[1] = q; return 2;
    }
    int64_t half = one >> 1, ic = c, d = q;
    if (q > half) { ic = c + 1; d = q - one; }
    *first = ic - 1;
    w[0] = (half - d) * (half - d);
    w[2] = (half + d) * (half + d);
    w[1] = ((int64_t)1 << (2 * b + 1)) - w[0] - w[2];
    return 3;
}

/* ------------------------------------------------------------------ */
/* particle push (reading R4, H1-H3)                                    */
/* ------------------------------------------------------------------ */
static void gather(const ora_sim* s, const int64_t c[3], const double o[3], double E[3], double B[3])
{
    int64_t first[3] = {0, 0, 0};
    double w[3][3] = {{1, 0, 0}, {1, 0, 0}, {1, 0, 0}};
    int np[3] = {1, 1, 1};
    for (int d = 0; d < s->c.dim; ++d) np[d] = shape_real(s->c.shape, c[d], o[d], &first[d], w[d]);
    for (int d = 0; d < 3; ++d) { E[d] = 0.0; B[d] = 0.0; }
    for (int a = 0; a < np[0]; ++a)
        for (int bb = 0; bb < np[1]; ++bb)
            for (int cc = 0; cc < np[2]; ++cc) {
                double W = w[0][a] * w[1][bb] * w[2][cc];
                int64_t n = gather_node(s, first[0] + a, first[1] + bb, first[2] + cc);
                for (int d = 0; d < 3; ++d) {
                    E[d] += W * s->E[3 * n + d];
                    B[d] += W * s->Bb[3 * n + d];
                }
            }
}

/* Boris: half electric kick, magnetic rotation, half electric kick (q/m=1).
 * In relativistic mode v is the four-velocity and the rotation vector is
 * divided by the Lorentz factor after the first half kick (reading R11). */
static void boris(const ora_cfg* c, double v[3], const double E[3], const double B[3], double dt)
{
    double h = 0.5 * dt, vm[3], t[3], sv[3], vp[3], vq[3];
    for (int d = 0; d < 3; ++d) vm[d] = v[d] + h * E[d];
    if (relativistic(c)) {
        double g = lorentz_u(c, vm);
        for (int d = 0; d < 3; ++d) t[d] = h * B[d] / g;
    } else {
        for (int d = 0; d < 3; ++d) t[d] = h * B[d];
    }
    double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int d = 0; d < 3; ++d) sv[d] = 2.0 * t[d] / (1.0 + tt);
    vp[0] = vm[0] + (vm[1] * t[2] - vm[2] * t[1]);
    vp[1] = vm[1] + (vm[2] * t[0] - vm[0] * t[2]);
    vp[2] = vm[2] + (vm[0] * t[1] - vm[1] * t[0]);
    vq[0] = vm[0] + (vp[1] * sv[2] - vp[2] * sv[1]);
    vq[1] = vm[1] + (vp[2] * sv[0] - vp[0] * sv[2]);
    vq[2] = vm[2] + (vp[0] * sv[1] - vp[1] * sv[0]);
    for (int d = 0; d < 3; ++d) v[d] = vq[d] + h * E[d];
}

static void push_species(ora_sim* s, int k)
{
    ora_sp* p = &s->sp[k];
    double dtdx = s->c.dt / s->c.dx;
    for (int64_t i = 0; i < p->n; ++i) {
        int64_t* c = &p->c[3 * i];
        double* o = &p->o[3 * i];
        double* v = &p->v[3 * i];
        double E[3], B[3];
        gather(s, c, o, E, B);
        boris(&s->c, v, E, B, s->c.dt);
        double vel[3];
        velocity_of(&s->c, v, vel);
        if (s->c.coupling == 2) {
            /* reading R16: midpoint of the move, where the flux is deposited */
            double hdtdx = 0.5 * dtdx;
            for (int d = 0; d < 3; ++d) { p->ch[3 * i + d] = c[d]; p->oh[3 * i + d] = o[d]; }
            for (int d = 0; d < s->c.dim; ++d) {
                double xh = o[d] + vel[d] * hdtdx;
                double fh = floor(xh);
                p->ch[3 * i + d] = c[d] + (int64_t)fh;
                p->oh[3 * i + d] = xh - fh;
                if (p->oh[3 * i + d] >= 1.0) { p->oh[3 * i + d] = 0.0; p->ch[3 * i + d] += 1; }
            }
        }
        for (int d = 0; d < s->c.dim; ++d) {
            double xi = o[d] + vel[d] * dtdx;
            double fl = floor(xi);
            c[d] += (int64_t)fl;
            o[d] = xi - fl;
            if (o[d] >= 1.0) { o[d] = 0.0; c[d] += 1; }
        }
    }
}

/* ------------------------------------------------------------------ */
/* faux-shock wall (eq. 1, readings R6-R7)                              */
/* ------------------------------------------------------------------ */
/* Reading R11's event: eq. (1) and the R7 kick in the downstream rest
 * frame.  u is the lab four-velocity.  The boost along x with speed u2
 * (Lorentz factor g2) gives the downstream four-velocity W and Lorentz
 * factor Gam; the speed there is |w| = |W| / Gam.  The kick keeps |W|, so
 * Gam and |w| too, and turns W into the R7 direction; the inverse boost
 * takes it back to the lab.  The decision is FP64 in this fixed order. */
static int wall_event_rel(const ora_cfg* c, int64_t step, uint64_t id, double delta,
                          const double u[3], double uout[3], double* back)
{
    double cc = c->c_light * c->c_light;
    double u2 = c->u_sh / c->r;
    double gam = sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / cc);
    double g2 = 1.0 / sqrt(1.0 - (u2 * u2) / cc);
    double Gam = g2 * (gam - u2 * u[0] / cc);
    double Wx = g2 * (u[0] - u2 * gam), Wy = u[1], Wz = u[2];
    double W2 = Wx * Wx + Wy * Wy + Wz * Wz;
    double w2 = W2 / (Gam * Gam);
    double U[4];
    draw(c, ORA_STREAM_WALL, step, id, 0, U);
    double m = U[0] > U[1] ? U[0] : U[1];
    double T = u2 * (1.0 + m) / (1.0 - m);
    if (!(w2 > T * T)) return 0;
    double Wabs = sqrt(W2);
    double a = u2 / (Wabs / Gam);
    double mu = a + (1.0 - a) * sqrt(U[2]);
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double phi = ORA_TWO_PI * U[3];
    double Wxn = -Wabs * mu;
    uout[0] = g2 * (Wxn + u2 * Gam);
    uout[1] = Wabs * st * cos(phi);
    uout[2] = Wabs * st * sin(phi);
    double gn = g2 * (Gam + u2 * Wxn / cc);
    double vx = u[0] / gam, vxn = uout[0] / gn;
    *back = vx > 0.0 ? delta * (-vxn) / vx : 0.0;
    return 1;
}

/* Reading R12: the wall's u2 at a step. */
static double wall_u2(const ora_cfg* c, int64_t step)
{
    double r = c->r + c->r_dot * ((double)step * c->dt);
    return c->u_sh / (r > 1.0 ? r : 1.0);
}

/* Reading R15: the downstream field direction at a step (normal component
 * continuous, tangential one compressed by r(t)), as its x and y parts. */
static void downstream_b(const ora_cfg* c, int64_t step, double* bx, double* by)
{
    double r = c->r + c->r_dot * ((double)step * c->dt);
    if (r < 1.0) r = 1.0;
    double th = c->theta_deg * (ORA_TWO_PI / 360.0);
    double bn = cos(th), bt = r * sin(th);
    double nb = sqrt(bn * bn + bt * bt);
    *bx = bn / nb;
    *by = bt / nb;
}

/* Reading R12's event, in both modes.  W is the crosser's velocity in the
 * downstream frame (its four-velocity there in the relativistic mode, with
 * Lorentz factor Gam), |w| = |W| / Gam its speed.  Uniform U[0] decides;
 * U[2] and U[3] direct the return as in R7. */
static int wall_event_prescribed(const ora_cfg* c, int64_t step, uint64_t id, double delta,
                                 const double v[3], double vout[3], double* back)
{
    int rel = relativistic(c);
    double u2 = wall_u2(c, step);
    double cc = rel ? c->c_light * c->c_light : 1.0;
    double gam = 1.0, g2 = 1.0, Gam = 1.0, Wx;
    if (rel) {
        gam = sqrt(1.0 + (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / cc);
        g2 = 1.0 / sqrt(1.0 - (u2 * u2) / cc);
        Gam = g2 * (gam - u2 * v[0] / cc);
        Wx = g2 * (v[0] - u2 * gam);
    } else {
        Wx = v[0] - u2;
    }
    double Wabs = sqrt(Wx * Wx + v[1] * v[1] + v[2] * v[2]);
    double w = Wabs / Gam;
    if (!(w > u2)) return 0;
    double rho = (w - u2) / (w + u2);
    double f = c->ret_f0;
    if (c->ret_alpha != 0.0) f = f * pow(w / c->cr_w, c->ret_alpha);
    double P = f * (rho * rho);
    if (P > 1.0) P = 1.0;
    double U[4];
    draw(c, ORA_STREAM_WALL, step, id, 0, U);
    if (!(U[0] < P)) return 0;
    double Wn = c->gain * Wabs;
    double Gn = rel ? sqrt(1.0 + (Wn * Wn) / cc) : 1.0;
    double wn = Wn / Gn;
    if (!(wn > u2)) return 0;
    double a = u2 / wn;
    double q = c->kappa == 0.0 ? sqrt(U[2]) : pow(U[2], 1.0 / (2.0 + c->kappa));
    double mu = a + (1.0 - a) * q;
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double phi = ORA_TWO_PI * U[3];
    if (c->lc_depletion > 0.0) {
        /* reading R15: n = (-mu, st cos phi, st sin phi), s = (-cx, -sy, 0) */
        double bx, by;
        downstream_b(c, step, &bx, &by);
        double cx = fabs(bx), sy = bx < 0.0 ? -by : by;
        double ns = mu * cx - (st * cos(phi)) * sy;
        if (!(ns * cx > a) && U[1] < c->lc_depletion) return 0;
    }
    double Wxn = -Wn * mu;
    vout[1] = Wn * st * cos(phi);
    vout[2] = Wn * st * sin(phi);
    if (rel) {
        vout[0] = g2 * (Wxn + u2 * Gn);
        double gl = g2 * (Gn + u2 * Wxn / cc);
        double vx = v[0] / gam, vxn = vout[0] / gl;
        *back = vx > 0.0 ? delta * (-vxn) / vx : 0.0;
    } else {
        vout[0] = u2 + Wxn;
        *back = v[0] > 0.0 ? delta * (-vout[0]) / v[0] : 0.0;
    }
    return 1;
}

/* Returns 1 (reflect) or 0 (transmit).  On reflection writes the new
 * velocity and how far (in cells) the particle travels back from x = L. */
static int wall_event(const ora_cfg* c, int64_t step, uint64_t id, double delta,
                      const double v[3], double vout[3], double* back)
{
    if (c->wall_model == 1) return wall_event_prescribed(c, step, id, delta, v, vout, back);
    if (relativistic(c)) return wall_event_rel(c, step, id, delta, v, vout, back);
    double u2 = c->u_sh / c->r;
    double wx = v[0] - u2, wy = v[1], wz = v[2];
    double w2 = wx * wx + wy * wy + wz * wz;
    double U[4];
    draw(c, ORA_STREAM_WALL, step, id, 0, U);
    double m = U[0] > U[1] ? U[0] : U[1];
    double T = u2 * (1.0 + m) / (1.0 - m);
    if (!(w2 > T * T)) return 0;
    double wabs = sqrt(w2);
    double a = u2 / wabs;
    double mu = a + (1.0 - a) * sqrt(U[2]);
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double phi = ORA_TWO_PI * U[3];
    vout[0] = u2 - wabs * mu;
    vout[1] = wabs * st * cos(phi);
    vout[2] = wabs * st * sin(phi);
    *back = v[0] > 0.0 ? delta * (-vout[0]) / v[0] : 0.0;
    return 1;
}

int ora_wall_list(const ora_cfg* cfg, int64_t step, int32_t species, int64_t n,
                  const uint64_t* id, const double* delta, double* v3,
                  double* xi_new, int32_t* outcome)
{
    int policy = species == 0 ? cfg->wall_th : cfg->wall_cr;
    for (int64_t i = 0; i < n; ++i) {
        double vout[3], back = 0.0;
        int r;
        if (policy == ORA_FAUX_SHOCK) r = wall_event(cfg, step, id[i], delta[i], &v3[3 * i], vout, &back);
        else if (policy == ORA_SPECULAR) {
            vout[0] = -v3[3 * i]; vout[1] = v3[3 * i + 1]; vout[2] = v3[3 * i + 2];
            back = delta[i]; r = 1;
        } else r = 0;
        outcome[i] = r;
        if (r) {
            for (int d = 0; d < 3; ++d) v3[3 * i + d] = vout[d];
            xi_new[i] = (double)cfg->nx - back;
        } else xi_new[i] = 0.0;
    }
    return 0;
}

static void record(ora_sim* s, uint64_t id, int32_t kind)
{
    if (!s->recording) return;
    if (s->nev == s->capev) {
        s->capev = s->capev ? 2 * s->capev : 4096;
        s->ev = (ora_event*)realloc(s->ev, (size_t)s->capev * sizeof(ora_event));
    }
    s->ev[s->nev].step = s->step; s->ev[s->nev].id = id; s->ev[s->nev].kind = kind;
    s->nev++;
}

/* Boundary pass: transverse wrap, open far-upstream boundary, wall. */
static void boundaries(ora_sim* s, int k, ora_stats* st)
{
    ora_sp* p = &s->sp[k];
    int policy = k == 0 ? s->c.wall_th : s->c.wall_cr;
    int64_t nx = s->c.nx, out = 0;
    for (int64_t i = 0; i < p->n; ++i) {
        int64_t* c = &p->c[3 * i];
        double* o = &p->o[3 * i];
        double* v = &p->v[3 * i];
        int keep = 1;
        if (s->c.dim >= 2) c[1] = wrapi(c[1], s->c.ny);
        if (s->c.dim >= 3) c[2] = wrapi(c[2], s->c.nz);
        if (s->c.xbc == ORA_XBC_PERIODIC) {
            c[0] = wrapi(c[0], nx);
        } else if (c[0] >= nx) {
            if (policy == ORA_OPEN) { keep = 0; st->open_removed++; }
            else {
                double delta = (double)(c[0] - nx) + o[0];
                double vout[3], back = 0.0;
                int r;
                if (policy == ORA_FAUX_SHOCK) {
                    r = wall_event(&s->c, s->step, p->id[i], delta, v, vout, &back);
                    st->incident++;
                    record(s, p->id[i], r ? 1 : 2);
                } else {
                    vout[0] = -v[0]; vout[1] = v[1]; vout[2] = v[2]; back = delta; r = 1;
                    st->incident++;
                }
                if (r) {
                    st->reflected++;
                    for (int d = 0; d < 3; ++d) v[d] = vout[d];
                    double xi = (double)nx - back;
                    double fl = floor(xi);
                    c[0] = (int64_t)fl; o[0] = xi - fl;
                    if (c[0] >= nx) { c[0] = nx - 1; o[0] = nextafter(1.0, 0.0); }
                    if (c[0] < 0) { keep = 0; st->escaped++; }
                    /* reading R16: a reflected ion deposits its flux where it ends */
                    for (int d = 0; d < 3; ++d) { p->ch[3 * i + d] = c[d]; p->oh[3 * i + d] = o[d]; }
                } else { keep = 0; st->transmitted++; }
            }
        } else if (c[0] < 0) { keep = 0; st->escaped++; record(s, p->id[i], 3); }
        if (keep) {
            if (out != i) {
                for (int d = 0; d < 3; ++d) {
                    p->c[3 * out + d] = c[d]; p->o[3 * out + d] = o[d]; p->v[3 * out + d] = v[d];
                    p->ch[3 * out + d] = p->ch[3 * i + d]; p->oh[3 * out + d] = p->oh[3 * i + d];
                }
                p->id[out] = p->id[i];
            }
            out++;
        }
    }
    p->n = out;
}

/* ------------------------------------------------------------------ */
/* injection (reading R8)                                               */
/* ------------------------------------------------------------------ */
int ora_inject_counts(const ora_cfg* c, int64_t step, int64_t* out2)
{
    out2[0] = out2[1] = 0;
    if (c->xbc != ORA_XBC_BOX || !c->inject) return 0;
    double F = (double)c->ppc * c->u_sh * c->dt / c->dx;
    if (F > 0.0) out2[0] = (int64_t)(floor(F * (double)(step + 1)) - floor(F * (double)step));
    double u2 = c->u_sh / c->r;
    if (c->n_cr > 0.0 && c->wall_cr == ORA_FAUX_SHOCK && c->cr_w > u2) {
        double Fc = (double)c->ppc_cr * (c->cr_w - u2) * c->dt / (2.0 * c->dx);
        out2[1] = (int64_t)(floor(Fc * (double)(step + 1)) - floor(Fc * (double)step));
    }
    return 0;
}

static void inject(ora_sim* s, ora_stats* st)
{
    int64_t cnt[2];
    ora_inject_counts(&s->c, s->step, cnt);
    int64_t nt = s->nyc * s->nzc;
    double sig = sqrt(0.5 * s->c.beta_i);
    double u2 = s->c.u_sh / s->c.r;
    /* thermal ions enter through x = 0 */
    if (cnt[0] > 0) {
        for (int64_t t = 0; t < nt; ++t)
            for (int64_t q = 0; q < cnt[0]; ++q) {
                uint64_t id = (uint64_t)(s->next_id + t * cnt[0] + q);
                double U[4], V[4], n1, n2, n3, n4;
                draw(&s->c, ORA_STREAM_INJECT_TH, s->step, id, 0, U);
                draw(&s->c, ORA_STREAM_INJECT_TH, s->step, id, 1, V);
                normals(V[0], V[1], &n1, &n2);
                normals(V[2], V[3], &n3, &n4);
                double v[3] = {s->c.u_sh + sig * n1, sig * n2, sig * n3};
                v[0] = fabs(v[0]);
                double xi = v[0] * U[0] * s->c.dt / s->c.dx;
                double fl = floor(xi);
                int64_t c[3] = {(int64_t)fl, t % s->nyc, t / s->nyc};
                double o[3] = {xi - fl, s->c.dim >= 2 ? U[1] : 0.0, s->c.dim >= 3 ? U[2] : 0.0};
                if (c[0] >= s->c.nx) { c[0] = s->c.nx - 1; o[0] = nextafter(1.0, 0.0); }
                if (relativistic(&s->c)) four_velocity(&s->c, v, v);
                sp_append(&s->sp[0], c, o, v, id);
            }
        s->next_id += nt * cnt[0];
        st->injected_th += nt * cnt[0];
    }
    /* CRs enter through the wall, isotropic in the downstream frame */
    if (cnt[1] > 0) {
        double wabs = s->c.cr_w, a = u2 / wabs;
        for (int64_t t = 0; t < nt; ++t)
            for (int64_t q = 0; q < cnt[1]; ++q) {
                uint64_t id = (uint64_t)(s->next_id + t * cnt[1] + q);
                double U[4], V[4];
                draw(&s->c, ORA_STREAM_INJECT_CR, s->step, id, 0, U);
                draw(&s->c, ORA_STREAM_INJECT_CR, s->step, id, 1, V);
                double mu = a + (1.0 - a) * sqrt(U[2]);
                double stt = sqrt(fmax(0.0, 1.0 - mu * mu));
                double phi = ORA_TWO_PI * U[3];
                double v[3] = {u2 - wabs * mu, wabs * stt * cos(phi), wabs * stt * sin(phi)};
                double vx = v[0];
                if (relativistic(&s->c)) {
                    /* downstream four-velocity of speed wabs, boosted to the lab */
                    double cc = s->c.c_light * s->c.c_light;
                    double g2 = 1.0 / sqrt(1.0 - (u2 * u2) / cc);
                    double Gw = 1.0 / sqrt(1.0 - (wabs * wabs) / cc);
                    double Wabs = Gw * wabs, Wx = -Wabs * mu;
                    v[0] = g2 * (Wx + u2 * Gw);
                    v[1] = Wabs * stt * cos(phi);
                    v[2] = Wabs * stt * sin(phi);
                    vx = v[0] / (g2 * (Gw + u2 * Wx / cc));
                }
                double xi = (double)s->c.nx - fabs(vx) * U[0] * s->c.dt / s->c.dx;
                double fl = floor(xi);
                int64_t c[3] = {(int64_t)fl, t % s->nyc, t / s->nyc};
                double o[3] = {xi - fl, s->c.dim >= 2 ? U[1] : 0.0, s->c.dim >= 3 ? V[0] : 0.0};
                if (c[0] >= s->c.nx) { c[0] = s->c.nx - 1; o[0] = nextafter(1.0, 0.0); }
                sp_append(&s->sp[1], c, o, v, id);
            }
        s->next_id += nt * cnt[1];
        st->injected_cr += nt * cnt[1];
    }
}

/* ------------------------------------------------------------------ */
/* moment deposit (reading R9)                                          */
/* ------------------------------------------------------------------ */
static int64_t quant_v(double v, int sv, int64_t* sat)
{
    if (v != v) { (*sat)++; return 0; }
    double t = nearbyint(ldexp(v, sv));
    if (t > (double)ORA_VSAT) { (*sat)++; return ORA_VSAT; }
    if (t < -(double)ORA_VSAT) { (*sat)++; return -ORA_VSAT; }
    return (int64_t)t;
}

static int64_t dep_index(const ora_sim* s, int64_t i, int64_t j, int64_t k)
{
    j = wrapi(j, s->nyc); k = wrapi(k, s->nzc);
    if (s->c.xbc == ORA_XBC_PERIODIC) i = wrapi(i, s->c.nx);
    else {
        i += s->g;
        if (i < 0 || i >= s->ndx) return -1;
    }
    return i + s->ndx * (j + s->nyc * k);
}

/* One particle's moments at (c, o): the density when which & 1, the flux
 * when which & 2. */
static void deposit_at(ora_sim* s, int k, const int64_t c[3], const double o[3], const double v[3],
                       const int64_t vq[3], int which, ora_stats* st)
{
    int64_t* M = s->M[k];
    double* Mc = s->Mc[k];
    int64_t first[3] = {0, 0, 0}, wi[3][3] = {{1, 0, 0}, {1, 0, 0}, {1, 0, 0}};
    double wr[3][3] = {{1, 0, 0}, {1, 0, 0}, {1, 0, 0}};
    int np[3] = {1, 1, 1};
    for (int d = 0; d < s->c.dim; ++d) {
        if (s->c.deposit_mode == 0) np[d] = shape_int(s->c.shape, s->b, c[d], o[d], &first[d], wi[d]);
        else np[d] = shape_real(s->c.shape, c[d], o[d], &first[d], wr[d]);
    }
    for (int a = 0; a < np[0]; ++a)
        for (int bb = 0; bb < np[1]; ++bb)
            for (int cc = 0; cc < np[2]; ++cc) {
                int64_t n = dep_index(s, first[0] + a, first[1] + bb, first[2] + cc);
                if (n < 0) { st->out_of_range++; continue; }
                if (s->c.deposit_mode == 0) {
                    int64_t W = wi[0][a] * wi[1][bb] * wi[2][cc];
                    if (which & 1) M[4 * n + 0] += W;
                    if (which & 2)
                        for (int d = 0; d < 3; ++d) M[4 * n + 1 + d] += W * vq[d];
                } else {
                    double W = wr[0][a] * wr[1][bb] * wr[2][cc];
                    if (which & 1) Mc[4 * n + 0] += W;
                    if (which & 2)
                        for (int d = 0; d < 3; ++d) Mc[4 * n + 1 + d] += W * v[d];
                }
            }
}

/* Moments of one species: density and flux at the particles' positions, or
 * (reading R16) the flux at the midpoints of their last move. */
static void deposit_species(ora_sim* s, int k, ora_stats* st)
{
    ora_sp* p = &s->sp[k];
    memset(s->M[k], 0, (size_t)(4 * s->ndep) * sizeof(int64_t));
    memset(s->Mc[k], 0, (size_t)(4 * s->ndep) * sizeof(double));
    for (int64_t i = 0; i < p->n; ++i) {
        double v[3];
        velocity_of(&s->c, &p->v[3 * i], v);
        int64_t vq[3];
        for (int d = 0; d < 3; ++d) vq[d] = quant_v(v[d], s->sv, &st->saturated);
        if (s->c.coupling == 2) {
            deposit_at(s, k, &p->c[3 * i], &p->o[3 * i], v, vq, 1, st);
            deposit_at(s, k, &p->ch[3 * i], &p->oh[3 * i], v, vq, 2, st);
        } else {
            deposit_at(s, k, &p->c[3 * i], &p->o[3 * i], v, vq, 3, st);
        }
    }
}

static double species_weight(const ora_sim* s, int k)
{
    /* a species with no ions per cell contributes no moments: weight 0 */
    if (k == 0) return s->c.ppc > 0 ? 1.0 / (double)s->c.ppc : 0.0;
    return s->c.alpha_cr * s->c.n_cr / (double)s->c.ppc_cr;
}

static void smooth_fluid(ora_sim* s);

/* Ion density and flux at the field nodes from both species' moments. */
static void fluid_from_moments(ora_sim* s)
{
    double scR = ldexp(1.0, -s->SW), scG = ldexp(1.0, -(s->SW + s->sv));
    for (int64_t n = 0; n < s->nnode; ++n) {
        int64_t i = n % s->nxn, rest = n / s->nxn;
        int64_t dn = (i + s->g) + s->ndx * rest;
        double dens = 0.0, G[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < 2; ++k) {
            double w = species_weight(s, k);
            if (k == 1 && !(s->c.n_cr > 0.0)) continue;
            if (s->c.deposit_mode == 0) {
                dens += w * ((double)s->M[k][4 * dn] * scR);
                for (int d = 0; d < 3; ++d) G[d] += w * ((double)s->M[k][4 * dn + 1 + d] * scG);
            } else {
                dens += w * s->Mc[k][4 * dn];
                for (int d = 0; d < 3; ++d) G[d] += w * s->Mc[k][4 * dn + 1 + d];
            }
        }
        s->fn[n] = dens;
        for (int d = 0; d < 3; ++d) s->fg[3 * n + d] = G[d];
    }
    if (s->c.smooth > 0) smooth_fluid(s);
}

/* Reading R13: N passes of the 1-2-1 filter over n_e and Gamma. */
static void smooth_fluid(ora_sim* s)
{
    int64_t N = s->nnode, nxn = s->nxn, nyc = s->nyc, nzc = s->nzc;
    double* a = (double*)malloc((size_t)(4 * N) * sizeof(double));
    double* b = (double*)malloc((size_t)(4 * N) * sizeof(double));
    for (int64_t n = 0; n < N; ++n) {
        int64_t i = n % nxn, j = (n / nxn) % nyc, k = n / (nxn * nyc);
        int64_t f = fluid_node(s, i, j, k);
        a[n] = fmax(s->fn[f], s->c.n_floor);
        for (int d = 0; d < 3; ++d) a[(1 + d) * N + n] = s->fg[3 * f + d];
    }
    for (int pass = 0; pass < s->c.smooth; ++pass) {
        for (int axis = 0; axis < s->c.dim; ++axis) {
            for (int64_t n = 0; n < N; ++n) {
                int64_t i = n % nxn, j = (n / nxn) % nyc, k = n / (nxn * nyc);
                int64_t m, p;
                int keep = 0;
                if (axis == 0) {
                    if (s->c.xbc == ORA_XBC_PERIODIC) {
                        m = node_idx(s, wrapi(i - 1, s->c.nx), j, k);
                        p = node_idx(s, wrapi(i + 1, s->c.nx), j, k);
                    } else {
                        keep = i == 0 || i == s->c.nx;
                        m = keep ? n : node_idx(s, i - 1, j, k);
                        p = keep ? n : node_idx(s, i + 1, j, k);
                    }
                } else if (axis == 1) {
                    m = node_idx(s, i, wrapi(j - 1, nyc), k);
                    p = node_idx(s, i, wrapi(j + 1, nyc), k);
                } else {
                    m = node_idx(s, i, j, wrapi(k - 1, nzc));
                    p = node_idx(s, i, j, wrapi(k + 1, nzc));
                }
                for (int q = 0; q < 4; ++q) {
                    const double* x = a + q * N;
                    b[q * N + n] = keep ? x[n] : 0.25 * ((x[m] + 2.0 * x[n]) + x[p]);
                }
            }
            double* t = a; a = b; b = t;
        }
    }
    for (int64_t n = 0; n < N; ++n) {
        s->fn[n] = a[n];
        for (int d = 0; d < 3; ++d) s->fg[3 * n + d] = a[(1 + d) * N + n];
    }
    free(a);
    free(b);
}

/* ------------------------------------------------------------------ */
/* fields (readings R3, R5)                                             */
/* ------------------------------------------------------------------ */
static double pressure(const ora_sim* s, int64_t n)
{
    double ne = fmax(s->fn[n], s->c.n_floor);
    return 0.5 * s->c.beta_e * pow(ne, s->c.gamma_e);
}

/* Ohm's law at node (i,j,k) from centre field B; also returns Bbar. */
static void ohm_node(const ora_sim* s, const double* B, int64_t i, int64_t j, int64_t k,
                     double E[3], double bb[3])
{
    int D = s->c.dim;
    int nb = D >= 2 ? 2 : 1, nc = D >= 3 ? 2 : 1;
    double dBx[3] = {0, 0, 0}, dBy[3] = {0, 0, 0}, dBz[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) bb[d] = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b2 = 0; b2 < nb; ++b2)
            for (int c2 = 0; c2 < nc; ++c2)
                for (int d = 0; d < 3; ++d)
                    bb[d] += centre_B(s, B, i - 1 + a, j - 1 + b2, k - 1 + c2, d);
    for (int d = 0; d < 3; ++d) bb[d] /= (double)(2 * nb * nc);
    /* d/dx, averaged over the transverse centre pairs */
    for (int b2 = 0; b2 < nb; ++b2)
        for (int c2 = 0; c2 < nc; ++c2)
            for (int d = 0; d < 3; ++d)
                dBx[d] += centre_B(s, B, i, j - 1 + b2, k - 1 + c2, d)
                        - centre_B(s, B, i - 1, j - 1 + b2, k - 1 + c2, d);
    for (int d = 0; d < 3; ++d) dBx[d] = dBx[d] / (double)(nb * nc) / s->c.dx;
    if (D >= 2) {
        for (int a = 0; a < 2; ++a)
            for (int c2 = 0; c2 < nc; ++c2)
                for (int d = 0; d < 3; ++d)
                    dBy[d] += centre_B(s, B, i - 1 + a, j, k - 1 + c2, d)
                            - centre_B(s, B, i - 1 + a, j - 1, k - 1 + c2, d);
        for (int d = 0; d < 3; ++d) dBy[d] = dBy[d] / (double)(2 * nc) / s->c.dx;
    }
    if (D >= 3) {
        for (int a = 0; a < 2; ++a)
            for (int b2 = 0; b2 < 2; ++b2)
                for (int d = 0; d < 3; ++d)
                    dBz[d] += centre_B(s, B, i - 1 + a, j - 1 + b2, k, d)
                            - centre_B(s, B, i - 1 + a, j - 1 + b2, k - 1, d);
        for (int d = 0; d < 3; ++d) dBz[d] = dBz[d] / 4.0 / s->c.dx;
    }
    double J[3] = {dBy[2] - dBz[1], dBz[0] - dBx[2], dBx[1] - dBy[0]};
    double gp[3] = {0, 0, 0};
    gp[0] = (pressure(s, fluid_node(s, i + 1, j, k)) - pressure(s, fluid_node(s, i - 1, j, k))) / (2.0 * s->c.dx);
    if (D >= 2)
        gp[1] = (pressure(s, fluid_node(s, i, j + 1, k)) - pressure(s, fluid_node(s, i, j - 1, k))) / (2.0 * s->c.dx);
    if (D >= 3)
        gp[2] = (pressure(s, fluid_node(s, i, j, k + 1)) - pressure(s, fluid_node(s, i, j, k - 1))) / (2.0 * s->c.dx);
    int64_t f = fluid_node(s, i, j, k);
    double ne = fmax(s->fn[f], s->c.n_floor);
    double G[3] = {s->fg[3 * f] + s->c.j_ext, s->fg[3 * f + 1], s->fg[3 * f + 2]};
    double num[3];
    num[0] = -(G[1] * bb[2] - G[2] * bb[1]) + (J[1] * bb[2] - J[2] * bb[1]) - gp[0];
    num[1] = -(G[2] * bb[0] - G[0] * bb[2]) + (J[2] * bb[0] - J[0] * bb[2]) - gp[1];
    num[2] = -(G[0] * bb[1] - G[1] * bb[0]) + (J[0] * bb[1] - J[1] * bb[0]) - gp[2];
    for (int d = 0; d < 3; ++d) E[d] = num[d] / ne + s->c.eta * J[d];
    /* Reading R10: the inflow node x = 0 of the box carries the motional
     * field of the unperturbed upstream plasma, E = -u_sh x_hat x B0. */
    if (s->c.xbc != ORA_XBC_PERIODIC && i == 0) {
        E[0] = 0.0;
        E[1] = s->c.u_sh * s->B0[2];
        E[2] = -s->c.u_sh * s->B0[1];
    }
    /* Reading R14: a conducting wall at x = L. */
    if (s->c.xbc != ORA_XBC_PERIODIC && s->c.wall_field == 1 && i == s->c.nx) {
        E[1] = 0.0;
        E[2] = 0.0;
    }
}

static void ohm_all(const ora_sim* s, const double* B, double* E, double* Bb)
{
    for (int64_t k = 0; k < s->nzc; ++k)
        for (int64_t j = 0; j < s->nyc; ++j)
            for (int64_t i = 0; i < s->nxn; ++i) {
                int64_t n = node_idx(s, i, j, k);
                double e[3], b[3];
                ohm_node(s, B, i, j, k, e, b);
                for (int d = 0; d < 3; ++d) {
                    E[3 * n + d] = e[d];
                    if (Bb) Bb[3 * n + d] = b[d];
                }
            }
}

/* -curl E at every centre (node -> centre differences). */
static void faraday_rhs(const ora_sim* s, const double* E, double* F)
{
    int D = s->c.dim;
    int nb = D >= 2 ? 2 : 1, nc = D >= 3 ? 2 : 1;
    for (int64_t k = 0; k < s->nzc; ++k)
        for (int64_t j = 0; j < s->nyc; ++j)
            for (int64_t i = 0; i < s->c.nx; ++i) {
                double dEx[3] = {0, 0, 0}, dEy[3] = {0, 0, 0}, dEz[3] = {0, 0, 0};
                for (int b2 = 0; b2 < nb; ++b2)
                    for (int c2 = 0; c2 < nc; ++c2)
                        for (int d = 0; d < 3; ++d)
                            dEx[d] += node_E(s, E, i + 1, j + b2, k + c2, d) - node_E(s, E, i, j + b2, k + c2, d);
                for (int d = 0; d < 3; ++d) dEx[d] = dEx[d] / (double)(nb * nc) / s->c.dx;
                if (D >= 2) {
                    for (int a = 0; a < 2; ++a)
                        for (int c2 = 0; c2 < nc; ++c2)
                            for (int d = 0; d < 3; ++d)
                                dEy[d] += node_E(s, E, i + a, j + 1, k + c2, d) - node_E(s, E, i + a, j, k + c2, d);
                    for (int d = 0; d < 3; ++d) dEy[d] = dEy[d] / (double)(2 * nc) / s->c.dx;
                }
                if (D >= 3) {
                    for (int a = 0; a < 2; ++a)
                        for (int b2 = 0; b2 < 2; ++b2)
                            for (int d = 0; d < 3; ++d)
                                dEz[d] += node_E(s, E, i + a, j + b2, k + 1, d) - node_E(s, E, i + a, j + b2, k, d);
                    for (int d = 0; d < 3; ++d) dEz[d] = dEz[d] / 4.0 / s->c.dx;
                }
                int64_t n = cent_idx(s, i, j, k);
                F[3 * n + 0] = -(dEy[2] - dEz[1]);
                F[3 * n + 1] = -(dEz[0] - dEx[2]);
                F[3 * n + 2] = -(dEx[1] - dEy[0]);
            }
}

/* SSP-RK3 (Shu-Osher) over dt in n_sub substeps with moments frozen, then
 * the final Ohm's law gives E^{n+1}. */
static void field_update(ora_sim* s)
{
    size_t nb = (size_t)(3 * s->ncent) * sizeof(double);
    double *B0 = (double*)malloc(nb), *B1 = (double*)malloc(nb), *B2 = (double*)malloc(nb);
    double *F = (double*)malloc(nb);
    double* E = (double*)malloc((size_t)(3 * s->nnode) * sizeof(double));
    int64_t N = 3 * s->ncent, nn = s->nnode;
    fluid_from_moments(s);
    double* fn1 = NULL;
    if (s->c.coupling == 2) {
        /* reading R16: moments frozen at t_{n+1/2} during the update: the
         * mean of the two densities, the midpoint flux as deposited */
        fn1 = (double*)malloc((size_t)nn * sizeof(double));
        memcpy(fn1, s->fn, (size_t)nn * sizeof(double));
        for (int64_t q = 0; q < nn; ++q) s->fn[q] = 0.5 * (s->fn_prev[q] + fn1[q]);
    }
    double h = s->c.dt / (double)s->c.n_sub;
    for (int sub = 0; sub < s->c.n_sub; ++sub) {
        memcpy(B0, s->B, nb);
        ohm_all(s, B0, E, NULL); faraday_rhs(s, E, F);
        for (int64_t q = 0; q < N; ++q) B1[q] = B0[q] + h * F[q];
        ohm_all(s, B1, E, NULL); faraday_rhs(s, E, F);
        for (int64_t q = 0; q < N; ++q) B2[q] = 0.75 * B0[q] + 0.25 * (B1[q] + h * F[q]);
        ohm_all(s, B2, E, NULL); faraday_rhs(s, E, F);
        for (int64_t q = 0; q < N; ++q) s->B[q] = (1.0 / 3.0) * B0[q] + (2.0 / 3.0) * (B2[q] + h * F[q]);
    }
    if (s->c.coupling == 2) {
        /* E^{n+1}: n^{n+1} and the flux extrapolated from t_{n-1/2} and
         * t_{n+1/2} to t_{n+1}; both become the previous step's values */
        for (int64_t q = 0; q < nn; ++q) {
            s->fn[q] = fn1[q];
            s->fn_prev[q] = fn1[q];
        }
        for (int64_t q = 0; q < 3 * nn; ++q) {
            double gh = s->fg[q];
            s->fg[q] = 1.5 * gh - 0.5 * s->fg_prev[q];
            s->fg_prev[q] = gh;
        }
        free(fn1);
    }
    ohm_all(s, s->B, s->E, s->Bb);
    free(B0); free(B1); free(B2); free(F); free(E);
}

/* E from the current B and moments.  With reading R16 the moments' density
 * and flux also become the previous step's (a loaded or initial state has
 * no earlier flux: its own stands in for it). */
void ora_compute_E(ora_sim* s)
{
    fluid_from_moments(s);
    if (s->c.coupling == 2) {
        memcpy(s->fn_prev, s->fn, (size_t)s->nnode * sizeof(double));
        memcpy(s->fg_prev, s->fg, (size_t)(3 * s->nnode) * sizeof(double));
    }
    ohm_all(s, s->B, s->E, s->Bb);
}

void ora_leapfrog_start(ora_sim* s)
{
    for (int k = 0; k < 2; ++k) {
        ora_sp* p = &s->sp[k];
        for (int64_t i = 0; i < p->n; ++i) {
            double E[3], B[3];
            gather(s, &p->c[3 * i], &p->o[3 * i], E, B);
            boris(&s->c, &p->v[3 * i], E, B, -0.5 * s->c.dt);
        }
    }
}

/* ------------------------------------------------------------------ */
/* initial load                                                         */
/* ------------------------------------------------------------------ */
int ora_init(ora_sim* s, const double* amps)
{
    double L = (double)s->c.nx * s->c.dx;
    double* phase = (double*)calloc((size_t)(s->c.n_modes + 1), sizeof(double));
    for (int m = 1; m <= s->c.n_modes; ++m) {
        double U[4];
        draw(&s->c, ORA_STREAM_FOURIER, m, 0, 0, U);
        phase[m] = ORA_TWO_PI * U[0];
    }
    for (int64_t k = 0; k < s->nzc; ++k)
        for (int64_t j = 0; j < s->nyc; ++j)
            for (int64_t i = 0; i < s->c.nx; ++i) {
                double x = ((double)i + 0.5) * s->c.dx;
                double by = s->B0[1], bz = s->B0[2];
                for (int m = 1; m <= s->c.n_modes; ++m) {
                    double A = amps ? amps[m - 1] : s->c.mode_amp;
                    double ph = ORA_TWO_PI * (double)m * x / L + phase[m];
                    by += A * cos(ph);
                    bz += A * sin(ph);
                }
                int64_t n = cent_idx(s, i, j, k);
                s->B[3 * n] = s->B0[0]; s->B[3 * n + 1] = by; s->B[3 * n + 2] = bz;
            }
    free(phase);
    double sig = sqrt(0.5 * s->c.beta_i);
    for (int k = 0; k < 2; ++k) s->sp[k].n = 0;
    sp_reserve(&s->sp[0], s->ncent * s->c.ppc);
    for (int64_t cell = 0; cell < s->ncent; ++cell) {
        int64_t i = cell % s->c.nx, j = (cell / s->c.nx) % s->nyc, kk = cell / (s->c.nx * s->nyc);
        for (int64_t q = 0; q < s->c.ppc; ++q) {
            uint64_t id = (uint64_t)(cell * s->c.ppc + q);
            double U[4], V[4], n1, n2, n3, n4;
            draw(&s->c, ORA_STREAM_INIT, 0, id, 0, U);
            draw(&s->c, ORA_STREAM_INIT, 0, id, 1, V);
            normals(V[0], V[1], &n1, &n2);
            normals(V[2], V[3], &n3, &n4);
            int64_t c[3] = {i, j, kk};
            double o[3] = {U[0], s->c.dim >= 2 ? U[1] : 0.0, s->c.dim >= 3 ? U[2] : 0.0};
            double v[3] = {s->c.u_sh + sig * n1, sig * n2, sig * n3};
            if (relativistic(&s->c)) four_velocity(&s->c, v, v);
            sp_append(&s->sp[0], c, o, v, id);
        }
    }
    s->next_id = s->ncent * s->c.ppc;
    s->step = 0;
    ora_stats st;
    memset(&st, 0, sizeof(st));
    for (int k = 0; k < 2; ++k) deposit_species(s, k, &st);
    ora_compute_E(s);
    return (int)(st.out_of_range + st.saturated);
}

/* ------------------------------------------------------------------ */
/* one step                                                             */
/* ------------------------------------------------------------------ */
int ora_step(ora_sim* s, int32_t flags, ora_stats* st_out)
{
    ora_stats st;
    memset(&st, 0, sizeof(st));
    for (int k = 0; k < 2; ++k) {
        if (flags & ORA_PUSH) push_species(s, k);
        if (flags & ORA_BOUNDARY) boundaries(s, k, &st);
    }
    if (flags & ORA_INJECT) inject(s, &st);
    if (flags & ORA_DEPOSIT)
        for (int k = 0; k < 2; ++k) deposit_species(s, k, &st);
    if (flags & ORA_FIELD) field_update(s);
    s->step++;
    if (st_out) *st_out = st;
    return 0;
}

/* ------------------------------------------------------------------ */
/* state access                                                         */
/* ------------------------------------------------------------------ */
int64_t ora_count(const ora_sim* s, int32_t k) { return s->sp[k].n; }
int64_t ora_next_id(const ora_sim* s) { return s->next_id; }
int64_t ora_get_step(const ora_sim* s) { return s->step; }
void ora_set_clock(ora_sim* s, int64_t step, int64_t next_id) { s->step = step; s->next_id = next_id; }

int ora_set_particles(ora_sim* s, int32_t k, int64_t n, const int64_t* cell3, const double* off3,
                      const double* v3, const uint64_t* id)
{
    ora_sp* p = &s->sp[k];
    p->n = 0;
    sp_reserve(p, n);
    memcpy(p->c, cell3, (size_t)(3 * n) * sizeof(int64_t));
    memcpy(p->o, off3, (size_t)(3 * n) * sizeof(double));
    memcpy(p->v, v3, (size_t)(3 * n) * sizeof(double));
    memcpy(p->id, id, (size_t)n * sizeof(uint64_t));
    memcpy(p->ch, cell3, (size_t)(3 * n) * sizeof(int64_t));   /* no move yet: midpoint = position */
    memcpy(p->oh, off3, (size_t)(3 * n) * sizeof(double));
    p->n = n;
    return 0;
}

int ora_get_particles(const ora_sim* s, int32_t k, int64_t* cell3, double* off3, double* v3, uint64_t* id)
{
    const ora_sp* p = &s->sp[k];
    memcpy(cell3, p->c, (size_t)(3 * p->n) * sizeof(int64_t));
    memcpy(off3, p->o, (size_t)(3 * p->n) * sizeof(double));
    memcpy(v3, p->v, (size_t)(3 * p->n) * sizeof(double));
    memcpy(id, p->id, (size_t)p->n * sizeof(uint64_t));
    return 0;
}

void ora_set_B(ora_sim* s, const double* B3) { memcpy(s->B, B3, (size_t)(3 * s->ncent) * sizeof(double)); }
void ora_get_B(const ora_sim* s, double* B3) { memcpy(B3, s->B, (size_t)(3 * s->ncent) * sizeof(double)); }
void ora_set_E(ora_sim* s, const double* E3) { memcpy(s->E, E3, (size_t)(3 * s->nnode) * sizeof(double)); }
void ora_get_E(const ora_sim* s, double* E3) { memcpy(E3, s->E, (size_t)(3 * s->nnode) * sizeof(double)); }
void ora_get_Bbar(const ora_sim* s, double* B3) { memcpy(B3, s->Bb, (size_t)(3 * s->nnode) * sizeof(double)); }
void ora_get_moments(const ora_sim* s, int32_t k, int64_t* m4) { memcpy(m4, s->M[k], (size_t)(4 * s->ndep) * sizeof(int64_t)); }
void ora_set_moments(ora_sim* s, int32_t k, const int64_t* m4) { memcpy(s->M[k], m4, (size_t)(4 * s->ndep) * sizeof(int64_t)); }
void ora_get_cmoments(const ora_sim* s, int32_t k, double* m4) { memcpy(m4, s->Mc[k], (size_t)(4 * s->ndep) * sizeof(double)); }
void ora_get_fluid(const ora_sim* s, double* n, double* g3)
{
    memcpy(n, s->fn, (size_t)s->nnode * sizeof(double));
    memcpy(g3, s->fg, (size_t)(3 * s->nnode) * sizeof(double));
}
void ora_sizes(const ora_sim* s, int64_t* o)
{
    o[0] = s->nxn; o[1] = s->ndx; o[2] = s->nyc; o[3] = s->nzc; o[4] = s->ncent; o[5] = s->nnode;
}
void ora_fixed_point(const ora_sim* s, int32_t* o) { o[0] = s->b; o[1] = s->sv; o[2] = s->SW; }

/* ------------------------------------------------------------------ */
/* diagnostics                                                          */
/* ------------------------------------------------------------------ */
void ora_profile(const ora_sim* s, double* prof)
{
    for (int64_t i = 0; i < s->c.nx; ++i) prof[i] = 0.0;
    for (int64_t k = 0; k < s->nzc; ++k)
        for (int64_t j = 0; j < s->nyc; ++j)
            for (int64_t i = 0; i < s->c.nx; ++i) {
                int64_t n = cent_idx(s, i, j, k);
                prof[i] += s->B[3 * n + 1] * s->B[3 * n + 1] + s->B[3 * n + 2] * s->B[3 * n + 2];
            }
}

/* Precursor magnetic energy: sum of By^2 + Bz^2 over centres in [L/2, L). */
double ora_loss(const ora_sim* s)
{
    double sum = 0.0;
    for (int64_t k = 0; k < s->nzc; ++k)
        for (int64_t j = 0; j < s->nyc; ++j)
            for (int64_t i = s->c.nx / 2; i < s->c.nx; ++i) {
                int64_t n = cent_idx(s, i, j, k);
                sum += s->B[3 * n + 1] * s->B[3 * n + 1] + s->B[3 * n + 2] * s->B[3 * n + 2];
            }
    return sum;
}

/* out: field energy, kinetic energy (thermal, CR), particle counts (thermal,
 * CR), precursor loss, max |div B| over interior nodes, total |B_perp|^2. */
void ora_diag(const ora_sim* s, double* out)
{
    double dV = pow(s->c.dx, (double)s->c.dim);
    double wb = 0.0, bperp = 0.0;
    for (int64_t n = 0; n < s->ncent; ++n) {
        wb += s->B[3 * n] * s->B[3 * n] + s->B[3 * n + 1] * s->B[3 * n + 1] + s->B[3 * n + 2] * s->B[3 * n + 2];
        bperp += s->B[3 * n + 1] * s->B[3 * n + 1] + s->B[3 * n + 2] * s->B[3 * n + 2];
    }
    out[0] = 0.5 * wb * dV;
    for (int k = 0; k < 2; ++k) {
        double ke = 0.0;
        const ora_sp* p = &s->sp[k];
        for (int64_t i = 0; i < p->n; ++i) {
            const double* u = &p->v[3 * i];
            double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
            /* (gamma - 1) c^2 = |u|^2 / (gamma + 1); |v|^2 / 2 without c */
            ke += relativistic(&s->c) ? uu / (lorentz_u(&s->c, u) + 1.0) : 0.5 * uu;
        }
        out[1 + k] = species_weight(s, k) * ke * dV;
        out[3 + k] = (double)p->n;
    }
    out[5] = ora_loss(s);
    int D = s->c.dim;
    int nb = D >= 2 ? 2 : 1, nc = D >= 3 ? 2 : 1;
    double maxdiv = 0.0;
    int64_t ilo = s->c.xbc == ORA_XBC_PERIODIC ? 0 : 1;
    int64_t ihi = s->c.xbc == ORA_XBC_PERIODIC ? s->c.nx : s->c.nx;
    for (int64_t k = 0; k < s->nzc; ++k)
        for (int64_t j = 0; j < s->nyc; ++j)
            for (int64_t i = ilo; i < ihi; ++i) {
                double dx = 0.0, dy = 0.0, dz = 0.0;
                for (int b2 = 0; b2 < nb; ++b2)
                    for (int c2 = 0; c2 < nc; ++c2)
                        dx += centre_B(s, s->B, i, j - 1 + b2, k - 1 + c2, 0) - centre_B(s, s->B, i - 1, j - 1 + b2, k - 1 + c2, 0);
                dx = dx / (double)(nb * nc) / s->c.dx;
                if (D >= 2) {
                    for (int a = 0; a < 2; ++a)
                        for (int c2 = 0; c2 < nc; ++c2)
                            dy += centre_B(s, s->B, i - 1 + a, j, k - 1 + c2, 1) - centre_B(s, s->B, i - 1 + a, j - 1, k - 1 + c2, 1);
                    dy = dy / (double)(2 * nc) / s->c.dx;
                }
                if (D >= 3) {
                    for (int a = 0; a < 2; ++a)
                        for (int b2 = 0; b2 < 2; ++b2)
                            dz += centre_B(s, s->B, i - 1 + a, j - 1 + b2, k, 2) - centre_B(s, s->B, i - 1 + a, j - 1 + b2, k - 1, 2);
                    dz = dz / 4.0 / s->c.dx;
                }
                double dv = fabs(dx + dy + dz);
                if (dv > maxdiv) maxdiv = dv;
            }
    out[6] = maxdiv;
    out[7] = bperp;
}

int ora_record(ora_sim* s, int32_t on) { s->recording = on; s->nev = 0; return 0; }

/* ------------------------------------------------------------------ */
/* sampled evaluation (checks of large runs one particle / node at a   */
/* time)                                                                */
/* ------------------------------------------------------------------ */
/* Gather, Boris and move (readings R3, R4: the push of push_species,
 * without boundaries) of n given particles in given node fields E3, Bb3
 * (nnode x 3, interleaved). */
int ora_push_sample(const ora_cfg* cfg, const double* E3, const double* Bb3, int64_t n, const int64_t* cell3,
                    const double* off3, const double* v3, int64_t* cell_out3, double* off_out3, double* v_out3)
{
    if (cfg->dim < 1 || cfg->dim > 3 || (cfg->shape != 1 && cfg->shape != 2)) return -1;
    ora_sim s;
    memset(&s, 0, sizeof(s));
    s.c = *cfg;
    s.nyc = cfg->dim >= 2 ? cfg->ny : 1;
    s.nzc = cfg->dim >= 3 ? cfg->nz : 1;
    s.nxn = cfg->xbc == ORA_XBC_PERIODIC ? cfg->nx : cfg->nx + 1;
    s.E = (double*)E3;
    s.Bb = (double*)Bb3;
    s.sp[0].n = n;
    s.sp[0].cap = n;
    s.sp[0].c = cell_out3;
    s.sp[0].o = off_out3;
    s.sp[0].v = v_out3;
    memcpy(cell_out3, cell3, (size_t)(3 * n) * sizeof(int64_t));
    memcpy(off_out3, off3, (size_t)(3 * n) * sizeof(double));
    memcpy(v_out3, v3, (size_t)(3 * n) * sizeof(double));
    push_species(&s, 0);
    return 0;
}

/* Ohm's law (reading R5) at n given nodes (node3: i, j, k) from centre
 * field B3 (ncent x 3, interleaved) and the fixed-point moments of both
 * species (ndep x 4; M1 may be NULL without CRs): E and Bbar (n x 3). */
int ora_ohm_sample(const ora_cfg* cfg, const double* B3, const int64_t* M0, const int64_t* M1, int64_t n,
                   const int64_t* node3, double* E_out3, double* Bb_out3)
{
    ora_sim* s = ora_new(cfg);
    if (!s) return -1;
    ora_set_B(s, B3);
    ora_set_moments(s, 0, M0);
    if (M1) ora_set_moments(s, 1, M1);
    fluid_from_moments(s);
    for (int64_t q = 0; q < n; ++q)
        ohm_node(s, s->B, node3[3 * q], node3[3 * q + 1], node3[3 * q + 2], &E_out3[3 * q], &Bb_out3[3 * q]);
    ora_free(s);
    return 0;
}

