/*
 * fsoracle.h -- TEST INFRASTRUCTURE ONLY (never part of the product path).
 *
 * C interface of the plain FP64 CPU oracle for one time step of the
 * faux-shock hybrid particle-in-cell method (Simon, Caprioli, Haggerty &
 * Reville 2025, "A 'Faux-Shock' Method for Hybrid Simulations of
 * Astrophysical Shocks").  Only tests/, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code with the GPU library.
 *
 * Parity note: the hybrid discretisation is not printed in the paper (Sec. 2
 * cites the dHybridR papers for it); the oracle implements the explicit
 * scheme written out in fsoracle.c, whose every reading of the paper is
 * listed at the top of that file.
 */
#ifndef FSORACLE_H
#define FSORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_OPEN = 0, ORA_FAUX_SHOCK = 1, ORA_SPECULAR = 2 };
enum { ORA_XBC_BOX = 0, ORA_XBC_PERIODIC = 1 };
enum { ORA_PUSH = 1, ORA_BOUNDARY = 2, ORA_INJECT = 4, ORA_DEPOSIT = 8,
       ORA_FIELD = 16, ORA_ALL = 31 };
enum { ORA_STREAM_INIT = 1, ORA_STREAM_INJECT_TH = 2, ORA_STREAM_INJECT_CR = 3,
       ORA_STREAM_WALL = 4, ORA_STREAM_FOURIER = 5 };

/* Field order is mirrored by oracle/oracle.py; keep the two in step. */
typedef struct ora_cfg {
    double dx, dt;
    double u_sh, beta_i, beta_e, gamma_e, theta_deg, r;
    double n_cr, cr_w, alpha_cr, j_ext;
    double n_floor, eta, mode_amp, v_max;
    double c_light;   /* c / v_A; 0: non-relativistic (reading R4), > 0: reading R11 */
    uint64_t seed;
    int32_t dim, nx, ny, nz;
    int32_t ppc, ppc_cr, shape, deposit_mode; /* shape 1 CIC 2 TSC; deposit 0 fixed point, 1 continuous */
    int32_t wall_th, wall_cr, xbc, n_sub;
    int32_t n_modes, inject, replay;
    int32_t wall_model;   /* 0: eq. (1) with the R7 kick; 1: the prescribed wall (reading R12) */
    double ret_f0, ret_alpha, gain, kappa, r_dot;
    int32_t smooth;         /* binomial passes on the fluid moments (reading R13) */
    int32_t wall_field;     /* 1: conducting wall at x = L (reading R14) */
    double lc_depletion;    /* prescribed wall: depletion of the return flux outside the loss cone (reading R15) */
    int32_t coupling;       /* ion-field time coupling: 1 first order (R4), 2 time-centred (reading R16) */
} ora_cfg;

typedef struct ora_stats {
    int64_t incident, reflected, transmitted, open_removed, escaped;
    int64_t injected_th, injected_cr, saturated, out_of_range;
} ora_stats;

typedef struct ora_sim ora_sim;

ora_sim* ora_new(const ora_cfg* cfg);
void     ora_free(ora_sim* s);
int      ora_init(ora_sim* s, const double* amps);          /* amps[n_modes] or NULL */
int      ora_step(ora_sim* s, int32_t flags, ora_stats* st); /* one step (or sub-steps) */
int64_t  ora_count(const ora_sim* s, int32_t species);
int64_t  ora_next_id(const ora_sim* s);
int64_t  ora_get_step(const ora_sim* s);
void     ora_set_clock(ora_sim* s, int64_t step, int64_t next_id);
int      ora_set_particles(ora_sim* s, int32_t species, int64_t n, const int64_t* cell3,
                           const double* off3, const double* v3, const uint64_t* id);
int      ora_get_particles(const ora_sim* s, int32_t species, int64_t* cell3, double* off3,
                           double* v3, uint64_t* id);
void     ora_set_B(ora_sim* s, const double* B3);            /* centres, 3 x ncent */
void     ora_get_B(const ora_sim* s, double* B3);
void     ora_set_E(ora_sim* s, const double* E3);            /* nodes, 3 x nnode */
void     ora_get_E(const ora_sim* s, double* E3);
void     ora_get_Bbar(const ora_sim* s, double* B3);
void     ora_compute_E(ora_sim* s);                          /* Ohm from current B, moments */
void     ora_get_moments(const ora_sim* s, int32_t species, int64_t* m4);  /* ndep x 4 */
void     ora_get_cmoments(const ora_sim* s, int32_t species, double* m4);
void     ora_set_moments(ora_sim* s, int32_t species, const int64_t* m4);
void     ora_get_fluid(const ora_sim* s, double* n, double* g3);
void     ora_sizes(const ora_sim* s, int64_t* out6);         /* nxn, ndx, nyn, nzn, ncent, nnode */
void     ora_fixed_point(const ora_sim* s, int32_t* out3);   /* b, s_v, S_W */
void     ora_diag(const ora_sim* s, double* out8);
void     ora_profile(const ora_sim* s, double* prof);        /* nx values */
double   ora_loss(const ora_sim* s);
int      ora_wall_list(const ora_cfg* cfg, int64_t step, int32_t species, int64_t n,
                       const uint64_t* id, const double* delta, double* v3,
                       double* xi_new, int32_t* outcome);
void     ora_philox(const uint64_t ctr[4], uint64_t k0, uint64_t k1, uint64_t out[4]);
int      ora_inject_counts(const ora_cfg* cfg, int64_t step, int64_t* out2);
int      ora_record(ora_sim* s, int32_t on);
/* Start of the leapfrog from velocities given at t = 0: one Boris step of
 * -dt/2 in the current E and Bbar (positions unchanged), so that the stored
 * velocities are v^{-1/2} to second order. */
void     ora_leapfrog_start(ora_sim* s);

/* Sampled evaluation for large runs: the push (gather, Boris, move; no
 * boundaries) of given particles in given node fields (E3, Bb3: nnode x 3),
 * and Ohm's law at given nodes (node3: i, j, k) from B (ncent x 3) and the
 * fixed-point moments (M1 may be NULL). */
int      ora_push_sample(const ora_cfg* cfg, const double* E3, const double* Bb3, int64_t n, const int64_t* cell3,
                         const double* off3, const double* v3, int64_t* cell_out3, double* off_out3, double* v_out3);
int      ora_ohm_sample(const ora_cfg* cfg, const double* B3, const int64_t* M0, const int64_t* M1, int64_t n,
                        const int64_t* node3, double* E_out3, double* Bb_out3);

/* Reverse mode (fsoracle_adj.c): loss = sum over centres i >= nx/2 of
 * By^2 + Bz^2 after nsteps continuous-deposit steps, and its gradient
 * grad[0] = d/du_sh, grad[1] = d/dalpha_cr, grad[1+m] = d/dA_m (m = 1..n_modes),
 * with every discrete decision of the forward run held fixed. */
int      ora_adjoint(const ora_cfg* cfg, const double* amps, int64_t nsteps, double* loss, double* grad);
/* Single transposes, for finite-difference pins. */
void     ora_adj_boris(const double v[3], const double E[3], const double B[3], double dt, const double lo[3],
                       double out[3], double lv[3], double lE[3], double lB[3]);
void     ora_adj_kick(const ora_cfg* cfg, int64_t step, uint64_t id, const double v[3], double delta, double u2,
                      double lxo, const double lvo[3], double out4[4], double lin5[5]);
void     ora_adj_ohm(const ora_cfg* cfg, const double* B, const double* fn, const double* fg, const double* lE,
                     double* E, double* lB, double* lfn, double* lfg);
void     ora_adj_rk3(const ora_cfg* cfg, const double* B, const double* fn, const double* fg, double* Bout,
                     double* lB, double* lfn, double* lfg);

#ifdef __cplusplus
}
#endif
#endif
