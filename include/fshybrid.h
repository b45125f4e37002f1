/*
 * fshybrid.h -- C ABI of the MI355X (gfx950) library for the data-parallel
 * hot path of the faux-shock hybrid particle-in-cell method
 * (Simon, Caprioli, Haggerty & Reville 2025, "A 'Faux-Shock' Method for
 * Hybrid Simulations of Astrophysical Shocks").
 *
 * One time step is: kinetic-ion Boris push with E/B gather, the faux-shock
 * (FS) wall that transmits each crossing ion or reflects it with a
 * downstream-isotropic kick (return probability of eq. 1, Sec. 2), thermal
 * injection at x = 0 and cosmic-ray (CR) injection at the wall (Sec. 2),
 * fixed-point moment deposition, and the massless-electron Ohm's-law E plus
 * Faraday B update of the hybrid model (Sec. 2, first paragraph after
 * Table 1).
 *
 * Conventions
 *  - Units are the paper's (Sec. 2): d_i, 1/Omega_ci, v_A, B0, n_g; q/m = 1.
 *    The upstream plasma enters at x = 0 and flows in +x toward the FS wall
 *    at x = L = nx*dx; y and z are periodic.
 *  - Every call returns an int status: FS_OK (0) or a negative FS_E* code.
 *    fs_last_error() gives a static description of the last error.
 *  - All work is enqueued on the hipStream_t passed in (NULL = default
 *    stream).  Statistics are valid once the stream has been synchronised;
 *    calls that take an fs_step_stats* synchronise the stream themselves.
 *  - Ownership: the caller allocates (e.g. with torch) and owns every
 *    particle, field and moment buffer, with the sizes fs_layout() reports,
 *    and passes raw device pointers.  The library owns only the handle and
 *    its scratch (crosser lists, field stage buffers, counters), freed by
 *    fs_destroy().  The library never reallocates caller memory.
 *  - Errors FS_EINVAL, FS_ECAPACITY and FS_EIDOVERFLOW are detected on the
 *    host before any work is enqueued: the state is unchanged.  FS_ENUMERIC
 *    (NaN, velocity-code saturation), FS_ETILE (a tile or crosser list
 *    overflowed on the device) and FS_EDEVICE (HIP error) leave the state
 *    undefined: restore a checkpoint.
 */
#ifndef FSHYBRID_H
#define FSHYBRID_H
#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FS_OK           0
#define FS_EINVAL      -1   /* bad configuration or argument (state unchanged) */
#define FS_ECAPACITY   -2   /* caller buffer too small (state unchanged) */
#define FS_EIDOVERFLOW -3   /* particle ids would pass 2^32 - 1 (state unchanged) */
#define FS_ENUMERIC    -4   /* NaN or saturated velocity code (state undefined) */
#define FS_EDEVICE     -5   /* HIP runtime error (state undefined) */
#define FS_ETILE       -6   /* device-side tile / crosser overflow (state undefined) */

/* wall policy per species: what happens to an ion that reaches x >= L */
#define FS_WALL_OPEN        0   /* leaves the box (thermal ions in the paper, Sec. 2) */
#define FS_WALL_FAUX_SHOCK  1   /* eq. (1) return probability + downstream-isotropic kick */
#define FS_WALL_SPECULAR    2   /* mirror reflection (reflecting-wall variant) */

#define FS_XBC_BOX       0      /* inflow at x = 0, wall at x = L */
#define FS_XBC_PERIODIC  1      /* periodic x (test boxes) */

/* fs_step flags.  The wall events and the re-binning of the ions are part
 * of FS_PUSH: the wall runs on the crosser list the push builds, within the
 * same call, and every pushed ion is written straight into its destination
 * tile's bin (so there is no separate wall or binning flag, and a push
 * without its wall, which would lose the crossers, cannot be asked for).
 * Diagnostics are their own calls (fs_diagnostics, fs_phase_space,
 * fs_bperp_spectrum). */
#define FS_PUSH    1u   /* gather + Boris + move + boundaries + FS wall + binning */
#define FS_INJECT  4u   /* thermal injection at x = 0, CR injection at x = L */
#define FS_DEPOSIT 8u   /* fixed-point moments at the new positions */
#define FS_FIELD  16u   /* SSP-RK3 Faraday update with frozen moments, then Ohm */
#define FS_ALL    (FS_PUSH | FS_INJECT | FS_DEPOSIT | FS_FIELD)

/* Run configuration.  Field meaning follows the paper's Table 1 and Sec. 2:
 * u_sh is the upstream flow speed in the shock frame, r the compression
 * ratio (u2 = u_sh / r, eq. 1), n_cr the CR density in units of n_g, cr_w
 * the CR speed in the downstream frame at injection, alpha_cr a multiplier
 * on the CR macro-particle weight (the "CR current" parameter), j_ext a
 * rigid external current along x, v_max the largest speed the run expects
 * (it sets the fixed-point velocity scale, see fs_layout_info.sv_bits).
 * Field order is mirrored by the Python binding. */
typedef struct fs_config {
    double dx, dt;
    double u_sh, beta_i, beta_e, gamma_e, theta_deg, r;
    double n_cr, cr_w, alpha_cr, j_ext;
    double n_floor, eta, mode_amp, v_max;
    double cap_factor_th, cap_factor_cr;   /* tile capacity / mean occupancy */
    double c_light;         /* c / v_A.  0: non-relativistic push, velocity arrays
                               hold v.  > 0: relativistic push (the dHybridR code
                               of the paper's 2D runs, Sec. 2), velocity arrays
                               hold the four-velocity u = gamma v; it must exceed
                               every sampled speed (u_sh + 15 sqrt(beta_i / 2),
                               u_sh / r, cr_w with CRs) or FS_EINVAL.  The
                               adjoint entry points refuse it (FS_EINVAL). */
    uint64_t seed;
    int32_t dim, nx, ny, nz;
    int32_t ppc, ppc_cr, shape, precision;  /* shape 1 = CIC, 2 = TSC; precision 32 or 64 */
    int32_t wall_th, wall_cr, xbc, n_sub;
    int32_t n_modes, inject;
    int32_t deposit_mode;   /* 0: int64 fixed point (bit-reproducible); 1: real
                               weights, FP64 sums (the differentiable variant the
                               adjoint needs; moments then hold doubles) */
    int32_t wall_model;     /* 0: the faux-shock event of eq. (1) with the
                               isotropic-flux kick; the five fields below are
                               then ignored.  1: the prescribed wall, the
                               calibration the paper leaves open (Sec. 1: return
                               rate, anisotropy and energy gain prescribed from
                               RW runs; Sec. 4: a boundary that may change in
                               time), for a crosser of downstream-frame speed
                               |w| at step s, u2(s) = u_sh / max(1, r + r_dot s dt):
                                 returns with probability
                                   min(1, ret_f0 (|w| / cr_w)^ret_alpha) rho^2,
                                   rho = (|w| - u2) / (|w| + u2), 0 if |w| <= u2;
                                 leaves with downstream-frame speed gain |w|
                                   (four-velocity gain |W| in the relativistic
                                   mode; no return if that is <= u2);
                                 with direction cosine mu' into the box of pdf
                                   ~ (mu' - a)^(1 + kappa) on (a, 1],
                                   a = u2 / (new speed), azimuth uniform.
                               CR injection keeps u_sh / r.  The adjoint entry
                               points refuse it (FS_EINVAL). */
    double ret_f0, ret_alpha;   /* return-probability factor and its power of |w| / cr_w
                                   (ret_f0 > 0; ret_alpha != 0 needs cr_w > 0) */
    double gain;                /* speed gain of a return, > 0 */
    double kappa;               /* anisotropy exponent of the return direction, > -2 */
    double r_dot;               /* d r / d t of the wall's compression ratio */
    int32_t smooth;         /* passes of the 1-2-1 binomial filter on the ion
                               density (floored) and flux before Ohm's law, each
                               pass along x, then y, then z; 0 (the default) for
                               none.  The paper runs dHybrid(R), which smooths,
                               but does not describe the filter; the 2D
                               reflecting-wall runs need it past t ~ 12.  In the
                               box x boundaries the end nodes keep their values and
                               the nodes within `shape` of them copy the nearest
                               filtered node.  The adjoint entry points refuse it. */
    int32_t wall_field;     /* field boundary at x = L in the box.  0: the last
                               cell's B is copied into the ghost and Ohm's law
                               holds at the wall node (open to the outflowing
                               plasma of the faux-shock runs).  1: a conducting
                               wall at rest, E_y = E_z = 0 at the wall node (the
                               reflecting-wall runs, whose plasma piles up there). */
    double lc_depletion;    /* prescribed wall only (wall_model 1), in [0, 1]:
                               the loss cone of an oblique shock, which the paper
                               expects the downstream CRs not to fill
                               isotropically (Sec. 3.2).  Downstream CRs gyrate
                               about b2 ~ (cos th_Bn, r(t) sin th_Bn, 0) (normal
                               B continuous, tangential B compressed by the
                               wall's ratio); a return direction n whose motion
                               along b2 alone outruns the receding shock,
                               (n . s) |b2_x| > u2 / (return speed) with s the
                               field direction pointing upstream, is in the loss
                               cone and returns as above; any other return is
                               turned into a transmission with probability
                               lc_depletion.  0 (the default) leaves the wall
                               as above, bit for bit; a parallel shock's cone
                               holds every return direction. */
    int32_t coupling;       /* ion-field time coupling.  1 (the default): the
                               moments of the new positions, frozen over the
                               field update, first order in dt.  2: time-centred,
                               second order (the coupling of the dHybridR code
                               the paper runs, Sec. 2; the paper gives no
                               scheme): the density is deposited at x^{n+1} and
                               the flux at the midpoint of the move,
                               x^n + v^{n+1/2} dt / 2 (ions reflected or injected
                               in the step at their new position); B advances
                               with the moments frozen at t_{n+1/2} (the mean of
                               the last two densities, the midpoint flux); E^{n+1}
                               takes n^{n+1} and the flux extrapolated to t_{n+1},
                               (3 Gamma^{n+1/2} - Gamma^{n-1/2}) / 2.  A load or a
                               refresh takes its own flux as Gamma^{-1/2}.  Needs
                               deposit_mode 0 and no smoothing; checkpoints and
                               the adjoint entry points refuse it (FS_EINVAL). */
    int32_t pad_coupling;
} fs_config;

/* Sizes the caller must allocate, reported by fs_layout(). */
typedef struct fs_layout_info {
    int64_t ncent;          /* cell centres: B lives here, 3 planar FP64 arrays */
    int64_t nnode;          /* field nodes: E and the gather grid live here */
    int64_t ndep;           /* deposit nodes (field nodes + TSC ghosts in x) */
    int64_t nxn, ndx, nyc, nzc;
    int64_t ntiles;
    int64_t tile_cap[2];    /* particle slots per tile, per species */
    int64_t capacity[2];    /* ntiles * tile_cap: slots per particle buffer */
    int64_t buf_bytes[2];   /* bytes of one particle buffer (two are needed) */
    int64_t gather_bytes;   /* bytes of the gather grid */
    int32_t tile[3], ntile[3];
    int32_t b_bits, sv_bits, sw_bits;   /* fixed-point format */
    int32_t cell_bits[3];   /* packed cell index: bit widths of x, y, z */
    int32_t real_bytes;     /* 4 (FP32 mode) or 8 (FP64 mode) */
    int32_t pad;
} fs_layout_info;

/* Particles of one species.  Each of the two buffers holds, in this order,
 * sections of `capacity` entries, each section starting on a 256-byte
 * boundary:
 *   int32  cell      packed cell index: ix | iy << cell_bits[0] |
 *                    iz << (cell_bits[0] + cell_bits[1])
 *   real   off[d]    in-cell offset in [0, 1), one section per dimension
 *   real   v[3]      velocity (v^{n-1/2} before a step, v^{n+1/2} after)
 *   uint32 id        unique particle id (keys the wall's random numbers)
 * Tile t owns slots [t*tile_cap, (t+1)*tile_cap) of each buffer.  Its live
 * particles are the bottom run [0, lo) and the top run [tile_cap - hi,
 * tile_cap) of that range, with lo = tile_count[t] and hi =
 * tile_count[ntiles + t]: the tile's own stayers are written bottom-up, ions
 * arriving from elsewhere (neighbour tiles, the wall, injection) top-down.
 * fs_step writes the other buffer and flips cur. */
typedef struct fs_particles {
    void*    buf[2];
    int32_t* tile_count[2]; /* device, 2 * ntiles entries each (lo, then hi) */
    int64_t* count;         /* device, live particles (updated by fs_step) */
    int64_t  capacity;
    int64_t  tile_cap;
    int32_t  cur;
    int32_t  species;       /* 0 thermal ions, 1 CRs */
} fs_particles;

/* Grid state, all device pointers owned by the caller. */
typedef struct fs_fields {
    double*  B;        /* centres: 3 planar arrays of ncent (Bx, By, Bz) */
    double*  E;        /* nodes: 3 planar arrays of nnode, E^n (FP64) */
    void*    gather;   /* nodes: nnode x 6 reals (Ex Ey Ez Bbarx Bbary Bbarz) */
    int64_t* mom[2];   /* per species: ndep x 4 int64 (R, Gx, Gy, Gz) */
} fs_fields;

typedef struct fs_step_stats {
    int64_t incident, reflected, transmitted, open_removed, escaped;
    int64_t injected_th, injected_cr, saturated, out_of_range;
    int64_t count[2];      /* live particles per species after the step */
    int64_t next_id;
    int32_t flags;         /* device error bits (1 tile overflow, 2 crosser
                              overflow, 4 NaN, 8 saturation) */
    int32_t pad;
} fs_step_stats;

typedef struct fs_handle fs_handle;

/* Validates cfg and fills *out with the buffer sizes of the run. */
int fs_layout(const fs_config* cfg, fs_layout_info* out);

/* Creates a handle (validates cfg, allocates library scratch). */
int fs_create(const fs_config* cfg, fs_handle** out);
void fs_destroy(fs_handle* h);
const char* fs_last_error(const fs_handle* h);

/* Loads the box (Sec. 2): B = B0 (cos theta, sin theta, 0) plus n_modes
 * Fourier modes of amplitude amps[m] (device pointer, or NULL for mode_amp)
 * with Philox phases; ppc thermal ions per cell with uniform offsets and a
 * drifting Maxwellian (u_sh, sqrt(beta_i/2)); ids cell-major; deposits the
 * moments and computes E^0 by Ohm's law.  Resets the step clock. */
int fs_init_plasma(fs_handle* h, fs_particles* sp, fs_fields* f, const double* amps,
                   hipStream_t s);

/* One step (or the sub-steps selected by flags) from step index `step`.
 * With stats != NULL the stream is synchronised and device errors are
 * returned; otherwise the call is fully asynchronous. */
int fs_step(fs_handle* h, fs_particles* sp, fs_fields* f, int64_t step, uint32_t flags,
            fs_step_stats* st, hipStream_t s);

/* Deposits both species' moments from the current particles (overwrites). */
int fs_deposit_moments(fs_handle* h, const fs_particles* sp, fs_fields* f, hipStream_t s);

/* FS wall (eq. 1, Sec. 2) applied to a caller list of n crossers (device
 * arrays): id, delta = overshoot beyond x = L in cells, v (3 x n planar,
 * FP64, overwritten for reflected ions).  outcome[i] = 1 reflect, 0
 * transmit; xi_new[i] = new x in cells for reflected ions. */
int fs_apply_faux_shock(fs_handle* h, int32_t species, int64_t step, int64_t n,
                        const uint32_t* id, const double* delta, double* v,
                        int32_t* outcome, double* xi_new, hipStream_t s);

/* Faraday update with SSP-RK3 (moments frozen) and the final Ohm's law:
 * B^n -> B^{n+1}, E^{n+1}, gather grid. */
int fs_field_update(fs_handle* h, fs_fields* f, hipStream_t s);

/* E and the gather grid from the current B and moments (Ohm's law only). */
int fs_refresh_fields(fs_handle* h, fs_fields* f, hipStream_t s);

/* Host-side state access (tests, checkpoints of small runs).  Arrays are
 * host memory: cell3 int64 (n x 3), off3 and v3 double (n x 3), id uint64.
 * fs_read_particles with cell3 == NULL only reports the count in *n. */
int fs_load_particles(fs_handle* h, fs_particles* sp, int64_t n, const int64_t* cell3,
                      const double* off3, const double* v3, const uint64_t* id, hipStream_t s);
int fs_read_particles(fs_handle* h, const fs_particles* sp, int64_t* n, int64_t* cell3,
                      double* off3, double* v3, uint64_t* id, hipStream_t s);

/* Step clock and id counter kept by the handle. */
int fs_set_clock(fs_handle* h, int64_t next_id);
int64_t fs_next_id(const fs_handle* h);

/* Diagnostics (FP64, deterministic): out[8] = field energy, kinetic energy
 * of thermal ions and CRs, particle counts, precursor loss
 * sum_{x >= L/2} (By^2 + Bz^2), max |div B| over interior nodes, total
 * By^2 + Bz^2.  prof (optional, device, nx) = sum over y, z of By^2 + Bz^2. */
int fs_diagnostics(fs_handle* h, const fs_particles* sp, const fs_fields* f, double* out8,
                   double* prof, hipStream_t s);

/* Checkpoint and restore (the restart of long runs).  A checkpoint holds
 * the live ions of both species (packed tile by tile in the particle
 * buffers' own section layout and precision), B at the centres and the id
 * counter, behind a header recording the layout (precision, dim, grid,
 * shape, tile plan), c_light and the seed.
 * fs_checkpoint_bytes: the size of a checkpoint of the current state
 *   (synchronises the stream to read the live counts).
 * fs_checkpoint: writes it to dst, device memory or host memory (pinned or
 *   pageable), cap >= that size else FS_ECAPACITY; the library stages it in
 *   device memory it allocates and frees within the call, and returns after
 *   the copy has completed.
 * fs_restore: loads a checkpoint (device or host src of `bytes` bytes) into a
 *   handle of the same layout, c_light and seed (else FS_EINVAL), into the
 *   current buffers' bins; sets the id counter, deposits the moments and
 *   recomputes E and the gather grid, so that fs_step continues bit for bit
 *   as the checkpointed run would have (ions are matched by id; their order
 *   within a bin is not part of the state).  Every offset and per-tile count
 *   is checked on the host before a kernel reads the blob: a truncated or
 *   corrupt checkpoint gives FS_EINVAL and leaves the state unchanged.  The
 *   step index is the caller's (the argument of fs_step). */
int fs_checkpoint_bytes(fs_handle* h, const fs_particles* sp, int64_t* bytes, hipStream_t s);
int fs_checkpoint(fs_handle* h, const fs_particles* sp, const fs_fields* f, void* dst, int64_t cap,
                  hipStream_t s);
int fs_restore(fs_handle* h, fs_particles* sp, fs_fields* f, const void* src, int64_t bytes, hipStream_t s);

/* Momentum phase space of one species: the paper's phase-space and
 * spectrum figures (Sec. 3, Figs. 2 and 4: x-|p|, x-p_x, x-p_y, x-p_z, and
 * the spectra n(p) summed over x).  p is the stored velocity variable per
 * unit mass: the four-velocity in relativistic mode, the velocity otherwise.
 * sp: both species' particles as for fs_step; species 0 or 1 (1 needs CRs).
 * counts (device, int64, nxb x nb, x-bin major, nxb = ceil(nx /
 * x_cells_per_bin)) is overwritten with the number of ions whose cell x
 * index / x_cells_per_bin is the x bin and whose momentum falls in bin j:
 *   component -1: edges[j]^2 <= |p|^2 < edges[j+1]^2  (edges >= 0);
 *   component 0, 1, 2: edges[j] <= p_c < edges[j+1].
 * |p|^2 = (p_x p_x + p_y p_y) + p_z p_z and the squared edges are FP64 in
 * that order without contraction, so the counts are an exact function of the
 * stored state.  Ions outside the edges are not counted.  edges: device, nb
 * + 1 ascending FP64 values (not checked; counts are undefined otherwise).
 * FS_EINVAL: NULL pointer, bad species, component or bin count. */
int fs_phase_space(fs_handle* h, const fs_particles* sp, int32_t species, int32_t component,
                   int32_t x_cells_per_bin, int32_t nb, const double* edges, int64_t* counts,
                   hipStream_t s);

/* Perpendicular magnetic power spectrum along x (the paper's Sec. 3 power
 * spectra of B_perp, Fig. 3): out (device, nx/2 + 1 FP64) = the mean over
 * the (y, z) lines of |B^_y(k)|^2 + |B^_z(k)|^2 with
 * B^(k) = (1/nx) sum_x B(x) exp(-2 pi i k x / nx), k = 0 .. nx/2, for B at the
 * centres as stored (B0 included at k = 0).  A mode A cos(2 pi m x / nx + phi)
 * of B_y and A sin(...) of B_z gives A^2 / 2 at k = m.  Direct transform with
 * a twiddle table, summed over line groups in a fixed order (deterministic).
 * The handle keeps a scratch of 2 nx + min(lines, 256) (nx/2 + 1) doubles from
 * the first call.  FS_EINVAL: NULL pointer; FS_EDEVICE: scratch allocation. */
int fs_bperp_spectrum(fs_handle* h, const fs_fields* f, double* out, hipStream_t s);

/* The same spectrum for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * same arguments and result as fs_bperp_spectrum, bit for bit, but the call
 * allocates nothing.  Its 2 nx + min(lines, 256) (nx/2 + 1) doubles of
 * scratch live in a static device array of the library, 2^21 doubles
 * (16 MiB), one per GPU for the life of the process; its address on the
 * handle's device is resolved by fs_create.  Every partial is written before
 * it is read, so nothing carries over from the previous call.  All calls on
 * one GPU share that array: calls that overlap in time on one GPU (two
 * streams, two threads) race and give undefined results.
 * FS_EINVAL: NULL pointer, a box whose scratch exceeds 2^21 doubles (e.g.
 * nx = 16384 with 256 or more (y, z) lines), or a current device other than
 * the handle's. */
int fs_bperp_spectrum_noalloc(fs_handle* h, const fs_fields* f, double* out, hipStream_t s);

/* ---------------------------------------------------------------------
 * Reverse mode.  The derivative is that of the continuous-deposit step
 * (deposit_mode 1) with every discrete decision of the forward run held
 * fixed: cells, FS reflections (the eq. 1 decision of Sec. 2), removals,
 * injection counts, the density floor.  The FS kick after a reflection is
 * differentiated, including through u2 = u_sh / r.  Gradients are those of
 * a scalar loss of the final state with respect to u_sh, alpha_cr (the CR
 * macro-weight multiplier) and the initial Fourier amplitudes.
 * --------------------------------------------------------------------- */

/* What a recorded step writes, per species k (k = 1 only with CRs): dst[k]
 * (device, int32, one entry per bin slot of the species' particle buffers,
 * capacity[k] entries, at least the species' capacity) receives, at the bin
 * slot each ion occupied in the step's input buffer, where the step put it:
 * its bin slot in the output buffer (>= 0), -1 if the step removed it (it
 * left through x = 0, or the wall transmitted or dropped it), or -2 - slot
 * if the FS wall reflected it into that slot.  Entries of slots that held
 * no ion keep whatever they held.  id0 receives the first id the step can
 * inject (the injected ions are id0, id0 + 1, ..., thermal first).  stages
 * (NULL for none; n_sub = 1 only) is device memory of 6 x ncent doubles
 * where the step leaves its SSP-RK3 stages B1 and B2 (each planar like B),
 * for fs_adjoint_step to read instead of recomputing them.  B_in and
 * gather_in (both NULL, or both given: device memory laid out like an
 * fs_fields' B and gather) are the input state's B and gather grid, which
 * the step then reads in place of f's: f's B and gather (and E) only
 * receive the output state, so stepping from one state's grids into
 * another's needs no copy first.  They may be f's own (the in-place step).
 * fluid (NULL for none; unfiltered moments only) is device memory of
 * 5 x nnode doubles where the step's field update leaves the fluid state
 * it used (n_e, p_e, Gamma_x, Gamma_y, Gamma_z, each planar over the nodes),
 * for fs_adjoint_step to read instead of recomputing it from the moments. */
typedef struct fs_record {
    int32_t*      dst[2];
    int64_t       capacity[2];
    int64_t       id0;
    double*       stages;
    const double* B_in;
    const void*   gather_in;
    double*       fluid;
} fs_record;

/* A particle state packed to its live ions: the reverse mode's tape, sized
 * to the ions rather than to the bins.  Per species k (k = 1 only with CRs),
 * buf[k] holds the sections of a particle buffer (the layout above) with
 * n[k] entries in place of capacity, tile t's ions at [toff[k][t],
 * toff[k][t + 1]) in the order of its bin (the bottom run, then the top run
 * from the top down); toff[k] has ntiles + 1 entries.  dst[k] (n[k] int32)
 * holds the record of the step that leaves this state, in packed indices of
 * the state after it: >= 0 kept there, -2 - i reflected into i, -1 removed.
 * *status (device int32) is set to 1 by fs_tape_pack (and fs_tape_unpack)
 * when a species had more live ions than n[k] (those beyond are dropped),
 * and to 2 by fs_adjoint_step, on the state after the step, when it did not
 * find every ion the step injected near the boundaries where injection
 * places them.  All arrays are device memory owned by the caller. */
typedef struct fs_packed {
    void*    buf[2];
    int32_t* toff[2];
    int32_t* dst[2];
    int64_t  n[2];
    int32_t* status;
} fs_packed;

/* Adjoint state (device arrays owned by the caller).  Particle adjoints are
 * in the particle precision and laid out like the packed states, one entry
 * per packed index: for species k and buffer b, x[k][b][d] (d < dim; dL
 * per cell of position) and v[k][b][c], capacity[k] entries each (at least
 * the n[k] of the packed states they serve).  Buffer cur holds the adjoints
 * of the state a reverse step starts from; the step writes buffer cur ^ 1
 * in the packed indices of the state before it and flips cur.  Grid
 * adjoints are FP64 planar: lB (3 x ncent) = dL/dB at the centres, lE
 * (6 x nnode) = dL/d(Ex, Ey, Ez, Bbarx, Bbary, Bbarz) of the gather grid. */
typedef struct fs_adjoint {
    void*   x[2][2][3];
    void*   v[2][2][3];
    int64_t capacity[2];
    int32_t cur;
    int32_t pad;
    double* lB;
    double* lE;
} fs_adjoint;

/* One full step (deposit_mode 1, non-relativistic, first-order coupling:
 * the step the reverse mode covers) that also fills *rec (in bin slots, see
 * fs_record).  Same contract as fs_step with flags = FS_ALL.  With pack_in
 * (NULL for none), whose toff fs_tape_pack has already set for the input
 * state (sp's buf[cur]), the push also copies each input ion as it reads it
 * to its packed index in pack_in->buf: the ions of fs_tape_pack with
 * FS_PACK_IONS, without a pass of their own.  FS_EINVAL on another
 * configuration, a NULL dst of a species, rec->stages with n_sub > 1,
 * only one of rec->B_in and rec->gather_in or rec->fluid with filtered
 * moments,
 * FS_ECAPACITY if a dst holds fewer entries than the species' capacity or
 * the capacity does not fit the int32 encoding (above 2^31 - 3 slots). */
int fs_step_record(fs_handle* h, fs_particles* sp, fs_fields* f, int64_t step, fs_record* rec,
                   const fs_packed* pack_in, fs_step_stats* st, hipStream_t s);

/* Packs the live ions of sp (buf[cur], tile_count[cur]) into *out: the tile
 * offsets, and with FS_PACK_IONS in flags the ions (else a recorded step
 * from this state copies them, see fs_step_record).  With prev_sp, rec and
 * prev given, sp is the output of the recorded step *rec whose input
 * prev_sp (as the step read it, packed into *prev) left the record in bin
 * slots; it goes into prev->dst in packed indices of *out.  Asynchronous on
 * s; an overflow of n[k] sets *out->status (*prev->status for a record
 * entry that points past out's n).  FS_EINVAL on a NULL argument (prev_sp,
 * rec and prev are all given or all NULL) or an unknown flag, FS_ECAPACITY
 * if a species' capacity does not fit the int32 tile offsets (above
 * 2^31 - 3 slots). */
#define FS_PACK_IONS 1u
int fs_tape_pack(fs_handle* h, const fs_particles* sp, fs_packed* out, const fs_particles* prev_sp,
                 const fs_record* rec, fs_packed* prev, uint32_t flags, hipStream_t s);

/* The inverse of a pack with FS_PACK_IONS: the ions of *pk (its offsets and
 * ions as fs_tape_pack left them) into the bins of sp (buf[cur],
 * tile_count[cur] and count), tile t's ions in the bottom run of its bin in
 * packed order.  A later fs_tape_pack of sp gives back *pk's ions in the same
 * order; a step from sp moves every ion as it would from the state that
 * was packed.  Asynchronous on s; a tile with more ions than tile_cap sets
 * *pk->status (those beyond are dropped).  FS_EINVAL on a NULL argument,
 * FS_ECAPACITY as fs_step for a particle buffer smaller than the layout. */
int fs_tape_unpack(fs_handle* h, const fs_packed* pk, fs_particles* sp, hipStream_t s);

/* Reverse of step `step` (n -> n+1, recorded with fs_step_record and packed
 * with fs_tape_pack).  pn / f_n: the packed state before the step (with the
 * step's record in pn->dst) and its fields (B, gather grid); pn1 / f_n1: the
 * packed state after it and its B and moment grids (f_n1->mom as the step
 * left them).  stages: the step's RK stages as fs_record.stages kept them
 * (n_sub = 1), or NULL to recompute them from f_n->B.  fluid: the step's
 * fluid state as fs_record.fluid kept it, or NULL to recompute it from
 * f_n1->mom.  id0: the first id the step handed out (fs_record.id0).
 * *lam holds on entry the adjoints after the step (particles in buffer cur,
 * in the packed indices of pn1; lB, lE of B^{n+1} and E^{n+1}) and on exit
 * those before it (particles in the other buffer, in the packed indices of
 * pn, which becomes cur; B^n, E^n).  Every ion of pn is written, zero for
 * one the step removed.  grads (device, 2 + n_modes doubles) accumulates
 * dL/du_sh and dL/dalpha_cr.  FS_EINVAL on a NULL argument (f_n1->mom
 * included) or stages with n_sub > 1, FS_ECAPACITY if an adjoint buffer is
 * shorter than pn or pn1. */
int fs_adjoint_step(fs_handle* h, const fs_packed* pn, const fs_fields* f_n, const fs_packed* pn1,
                    const fs_fields* f_n1, const double* stages, const double* fluid, int64_t id0, int64_t step,
                    fs_adjoint* lam, double* grads, hipStream_t s);

/* Moving the particle adjoints between two packings of one state: a segment
 * of steps re-run from its checkpoint packs its last state in another order
 * than the checkpoint that began the later segment (the push places ions in
 * an order set by the timing of its atomics).  fs_adjoint_park writes the
 * adjoints of buffer lam->cur, at the packed indices of `from`, into scratch
 * by particle id (after zeroing it); fs_adjoint_unpark reads them back into
 * buffer lam->cur at the packed indices of `to` (zero for an id scratch does
 * not hold).  scratch: device, (dim + 3) * nid reals of the particle
 * precision per species (species 1 after species 0), nid above every id;
 * ids >= nid are skipped; its layout between a park and an unpark is the
 * library's own.  FS_EINVAL on a NULL argument or a negative nid,
 * FS_ECAPACITY if an adjoint buffer is shorter than the packed state. */
int fs_adjoint_park(fs_handle* h, const fs_packed* from, fs_adjoint* lam, void* scratch, int64_t nid,
                    hipStream_t s);
int fs_adjoint_unpark(fs_handle* h, const fs_packed* to, fs_adjoint* lam, const void* scratch, int64_t nid,
                      hipStream_t s);

/* Reverse of fs_init_plasma: E^0 = Ohm(B^0, moments of the initial load),
 * the initial velocities (v_x = u_sh + sigma n) and the Fourier modes of
 * B^0.  p0: the initial state packed, f0: its fields (f0->mom: the moments
 * of the initial load).  Adds to dL/du_sh, dL/dalpha_cr and
 * grads[1 + m] = dL/dA_m. */
int fs_adjoint_init(fs_handle* h, const fs_packed* p0, const fs_fields* f0, fs_adjoint* lam, double* grads,
                    hipStream_t s);

/* The loss of the reverse-mode workload: the magnetic energy of the
 * transverse field in the precursor, the region ahead of the shock where
 * the CR current drives the Bell instability (Sec. 3), taken as the
 * downstream half of the box next to the wall,
 *   L = sum over cell centres with x index i >= nx/2 of B_y^2 + B_z^2.
 * f->B: FP64 planar B (3 x ncent, device).  loss: device pointer to one
 * double, written asynchronously on s (valid after a stream sync).  The sum
 * is taken in a fixed order (partials per workgroup of a fixed grid in the
 * handle's scratch, then one workgroup), so repeated calls agree bit for
 * bit.  FS_EINVAL on a NULL argument. */
int fs_precursor_loss(fs_handle* h, const fs_fields* f, double* loss, hipStream_t s);

/* Start of a reverse sweep for that loss.  Zeroes buffer lam->cur of every
 * species' particle adjoints (x[k][cur][d] for d < dim and v[k][cur][c],
 * capacity[k] entries each, in the particle precision), lE and grads
 * (2 + n_modes doubles, device), and sets lB = dL/dB at the final state f->B:
 * (0, 2 B_y, 2 B_z) at the centres with i >= nx/2, 0 elsewhere.  FS_EINVAL
 * on a NULL array, a negative capacity or cur outside {0, 1}. */
int fs_adjoint_seed(fs_handle* h, const fs_fields* f, fs_adjoint* lam, double* grads, hipStream_t s);

/* Phase timing with HIP events recorded on the caller's stream (benchmark
 * support).  While enabled, every fs_step records an event pair around each
 * phase: 0 = push kernels (gather, Boris, move, boundaries, fused deposit),
 * 1 = wall kernels, 2 = injection, 3 = field update, 4 = the whole step.
 * fs_timing_read synchronises the stream, writes the summed milliseconds and
 * the number of recorded intervals per phase (5 entries each) and clears the
 * record.  At most 4096 steps are recorded between reads. */
int fs_timing_enable(fs_handle* h, int32_t on);
int fs_timing_read(fs_handle* h, double* ms5, int64_t* n5, hipStream_t s);

#ifdef __cplusplus
}
#endif
#endif
