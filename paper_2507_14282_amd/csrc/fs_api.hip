// fs_api.hip -- host runtime and C ABI of the faux-shock hybrid library.
//
// Owns the handle (configuration, derived layout, library scratch) and
// enqueues the kernels of fs_kernels.h / fs_field.h on the caller's stream.
// See include/fshybrid.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fs_adjoint.h"
#include "fshybrid.h"

using namespace fsk;

struct fs_handle {
    fs_config cfg;
    fs_layout_info L;
    Geo G;
    FieldGeo F;
    int64_t next_id = 0;
    bool has_cr = false;
    unsigned long long* ctr = nullptr;       // device counters
    unsigned long long* ctr_host = nullptr;  // pinned mirror
    XList xl[2];
    void* xl_mem[2] = {nullptr, nullptr};
    double* B1 = nullptr;
    double* B2 = nullptr;
    double* Etmp = nullptr;
    double* fluid = nullptr;
    double* fluid2 = nullptr;     // second fluid buffer: binomial filter, or the final Ohm of the time-centred coupling
    double* nprev = nullptr;      // time-centred coupling: density of the previous step (nnode)
    double* gprev = nullptr;      // and its midpoint flux (3 x nnode)
    double* phase = nullptr;
    double* part = nullptr;
    int64_t npart = 0;
    double* spec = nullptr;   // B_perp spectrum: twiddles + partial sums (first use)
    int64_t nspec = 0;
    int device = -1;                  // device current at fs_create
    double* static_scratch = nullptr; // device address of `scratch` on that device
    // reverse-mode scratch (deposit_mode 1 only)
    double* alM[2] = {nullptr, nullptr};    // their adjoints
    double* afl = nullptr;                  // fluid state of the reverse step
    double* alfl = nullptr;                 // its adjoint
    double* al[3] = {nullptr, nullptr, nullptr};  // RK3 transpose: l0 and lam_F (two, ping-ponged)
    double* aBs = nullptr;                  // B at the start of each RK substep after the first
    double* aob = nullptr;                  // 1D Ohm transpose: lam(Bbar), lam(J) per node
    unsigned long long* actr = nullptr;     // injected-ion counters of the reverse step (zero between launches)
    long long* scan_part = nullptr;         // chunk sums of the tile-offset scan of a packed state
    std::string err;
    // phase timing: pool of event pairs recorded on the caller's stream
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_phase;
    size_t ev_used = 0;
};

namespace {

thread_local std::string g_err;

int fail(fs_handle* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    g_err = msg;
    return code;
}

int hip_check(fs_handle* h, hipError_t e, const char* what) {
    if (e == hipSuccess) return FS_OK;
    return fail(h, FS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace

// Scratch of the allocation-free B_perp spectrum (fs_bperp_spectrum_noalloc):
// its twiddles and per-group partial sums live in this file-scope device
// array, one copy per GPU for the life of the process.  Host code never
// uses the name itself (on the host it is only a stand-in for the symbol):
// fs_create resolves the device address once per device and the kernels
// receive that address.
constexpr int64_t kStaticScratchDoubles = int64_t(1) << 21;   // 16 MiB
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

namespace {

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
double* g_scratch_dev[kMaxDevices] = {};   // device address of `scratch`, per device

// Records the current device in the handle and the address of `scratch` on
// it, resolving that address with hipGetSymbolAddress on the device's first
// handle.
int resolve_static_scratch(fs_handle* h) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_check(h, e, "current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(h, FS_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_check(h, e, "address of the static scratch");
        if (!p) return fail(h, FS_EDEVICE, "address of the static scratch is NULL");
        g_scratch_dev[dev] = static_cast<double*>(p);
    }
    h->device = dev;
    h->static_scratch = g_scratch_dev[dev];
    return FS_OK;
}

// Workgroups per tile for the per-particle passes that may split a bin: about
// 2048 slots each, at most 16.
int split_of(int64_t tile_cap) { return (int)std::max<int64_t>(1, std::min<int64_t>(16, tile_cap / 2048)); }

// The workgroups per tile of a particle pass that stages its tile's stencil
// and flushes it: split_of for boxes of few tiles, one where the tiles alone
// give some 4096 workgroups (each extra workgroup of a tile stages and
// flushes the whole stencil again: on the 3D box that was four times the
// global atomics of one).
int split_for(const fs_layout_info& L, int64_t tile_cap) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(split_of(tile_cap), (4096 + L.ntiles - 1) / L.ntiles));
}

int bits_for(int64_t n) {
    int b = 1;
    while ((int64_t(1) << b) < n) ++b;
    return b;
}

// s_v = 23 - ceil(log2 v_max): the largest expected speed maps just under 2^23.
int sv_for(double v_max) {
    int e;
    double m = frexp(v_max, &e);
    if (m == 0.5) e -= 1;
    return 23 - e;
}

void tile_shape(int dim, int t[3]) {
    if (dim == 1) { t[0] = TileShape<1>::X; t[1] = 1; t[2] = 1; }
    else if (dim == 2) { t[0] = TileShape<2>::X; t[1] = TileShape<2>::Y; t[2] = 1; }
    else { t[0] = TileShape<3>::X; t[1] = TileShape<3>::Y; t[2] = TileShape<3>::Z; }
}

int lds_bytes(int dim, int shape, int rb, bool gather) {
    int t[3];
    tile_shape(dim, t);
    int w = shape == 2 ? 3 : 1;
    int gx = t[0] + w, gy = dim >= 2 ? t[1] + w : 1, gz = dim >= 3 ? t[2] + w : 1;
    int dx = t[0] + 2 + w, dy = dim >= 2 ? t[1] + 2 + w : 1, dz = dim >= 3 ? t[2] + 2 + w : 1;
    return (gather ? 6 * rb * gx * gy * gz : 0) + 32 * dx * dy * dz;  // upper bound of both deposit paths
}

int compute_layout(const fs_config* c, fs_layout_info* L, std::string& err) {
    std::memset(L, 0, sizeof(*L));
    if (c->dim < 1 || c->dim > 3) { err = "dim must be 1, 2 or 3"; return FS_EINVAL; }
    if (c->shape != 1 && c->shape != 2) { err = "shape must be 1 (CIC) or 2 (TSC)"; return FS_EINVAL; }
    if (c->precision != 32 && c->precision != 64) { err = "precision must be 32 or 64"; return FS_EINVAL; }
    if (c->xbc != FS_XBC_BOX && c->xbc != FS_XBC_PERIODIC) { err = "bad x boundary"; return FS_EINVAL; }
    if (c->nx < 2 * c->shape + 2) { err = "nx too small"; return FS_EINVAL; }
    if (c->dim >= 2 && c->ny < 2) { err = "ny must be >= 2"; return FS_EINVAL; }
    if (c->dim >= 3 && c->nz < 2) { err = "nz must be >= 2"; return FS_EINVAL; }
    if (!(c->dx > 0) || !(c->dt > 0)) { err = "dx and dt must be positive"; return FS_EINVAL; }
    if (c->ppc < 0 || c->ppc_cr < 0) { err = "ppc must be non-negative"; return FS_EINVAL; }
    if (!(c->v_max > 0)) { err = "v_max must be positive"; return FS_EINVAL; }
    if (!(c->r > 0)) { err = "compression ratio must be positive"; return FS_EINVAL; }
    if (c->n_sub < 1) { err = "n_sub must be >= 1"; return FS_EINVAL; }
    if (c->deposit_mode != 0 && c->deposit_mode != 1) { err = "deposit_mode must be 0 or 1"; return FS_EINVAL; }
    for (int w : {c->wall_th, c->wall_cr})
        if (w < FS_WALL_OPEN || w > FS_WALL_SPECULAR) { err = "bad wall policy"; return FS_EINVAL; }
    if (c->n_modes < 0) { err = "n_modes must be >= 0"; return FS_EINVAL; }
    const bool has_cr = c->n_cr > 0.0;
    if (has_cr && c->ppc_cr < 1) { err = "ppc_cr must be >= 1 with CRs"; return FS_EINVAL; }
    if (!(c->c_light >= 0.0)) { err = "c_light must be >= 0"; return FS_EINVAL; }
    if (c->c_light > 0.0) {
        // every sampled speed below c: a Box-Muller normal stays below 8.66,
        // so a thermal velocity below u_sh + 15 sigma
        if (!(c->u_sh + 15.0 * std::sqrt(0.5 * c->beta_i) < c->c_light) || !(c->u_sh / c->r < c->c_light) ||
            (has_cr && !(c->cr_w < c->c_light))) {
            err = "c_light must exceed every sampled speed";
            return FS_EINVAL;
        }
    }
    if (c->wall_model != 0 && c->wall_model != 1) { err = "wall_model must be 0 or 1"; return FS_EINVAL; }
    if (c->wall_model == 1) {
        if (!(c->ret_f0 > 0.0) || !std::isfinite(c->ret_f0) || !std::isfinite(c->ret_alpha) || !(c->gain > 0.0) ||
            !std::isfinite(c->gain) || !(c->kappa > -2.0) || !std::isfinite(c->kappa) || !std::isfinite(c->r_dot)) {
            err = "prescribed wall needs ret_f0 > 0, gain > 0, kappa > -2, all finite";
            return FS_EINVAL;
        }
        if (c->ret_alpha != 0.0 && !(c->cr_w > 0.0)) { err = "ret_alpha != 0 needs cr_w > 0"; return FS_EINVAL; }
    }
    if (!(c->lc_depletion >= 0.0 && c->lc_depletion <= 1.0)) { err = "lc_depletion must be in [0, 1]"; return FS_EINVAL; }
    if (c->coupling != 1 && c->coupling != 2) { err = "coupling must be 1 or 2"; return FS_EINVAL; }
    if (c->coupling == 2 && (c->deposit_mode != 0 || c->smooth != 0)) {
        err = "the time-centred coupling needs deposit_mode 0 and no smoothing";
        return FS_EINVAL;
    }
    if (c->lc_depletion > 0.0 && c->wall_model != 1) { err = "lc_depletion needs the prescribed wall"; return FS_EINVAL; }
    if (c->smooth < 0 || c->smooth > 64) { err = "smooth must be in [0, 64]"; return FS_EINVAL; }
    if (c->wall_field != 0 && c->wall_field != 1) { err = "wall_field must be 0 or 1"; return FS_EINVAL; }
    int t[3];
    tile_shape(c->dim, t);
    L->tile[0] = t[0]; L->tile[1] = t[1]; L->tile[2] = t[2];
    L->nyc = c->dim >= 2 ? c->ny : 1;
    L->nzc = c->dim >= 3 ? c->nz : 1;
    L->nxn = c->xbc == FS_XBC_PERIODIC ? c->nx : c->nx + 1;
    const int g = (c->xbc == FS_XBC_BOX && c->shape == 2) ? 1 : 0;
    L->ndx = L->nxn + 2 * g;
    L->ncent = (int64_t)c->nx * L->nyc * L->nzc;
    L->nnode = L->nxn * L->nyc * L->nzc;
    L->ndep = L->ndx * L->nyc * L->nzc;
    L->ntile[0] = (c->nx + t[0] - 1) / t[0];
    L->ntile[1] = (int32_t)((L->nyc + t[1] - 1) / t[1]);
    L->ntile[2] = (int32_t)((L->nzc + t[2] - 1) / t[2]);
    L->ntiles = (int64_t)L->ntile[0] * L->ntile[1] * L->ntile[2];
    L->cell_bits[0] = bits_for(c->nx);
    L->cell_bits[1] = c->dim >= 2 ? bits_for(c->ny) : 0;
    L->cell_bits[2] = c->dim >= 3 ? bits_for(c->nz) : 0;
    if (L->cell_bits[0] + L->cell_bits[1] + L->cell_bits[2] > 31) { err = "grid too large for a packed int32 cell"; return FS_EINVAL; }
    // device index arithmetic uses 24-bit products and 32-bit node indices
    if (L->ndx >= (1 << 24) || L->nyc * L->nzc >= (1 << 24) || L->ndep >= INT32_MAX ||
        L->ntile[0] >= (1 << 24) || (int64_t)L->ntile[1] * L->ntile[2] >= (1 << 24)) {
        err = "grid too large for 32-bit node indices";
        return FS_EINVAL;
    }
    const int64_t cells = (int64_t)t[0] * t[1] * t[2];
    const int rb = c->precision == 64 ? 8 : 4;
    L->real_bytes = rb;
    double cf0 = c->cap_factor_th > 0 ? c->cap_factor_th : 2.0;
    double cf1 = c->cap_factor_cr > 0 ? c->cap_factor_cr : 4.0;
    L->tile_cap[0] = round_up(std::max<int64_t>((int64_t)std::ceil(cf0 * c->ppc * cells), c->ppc * cells + 64), 64);
    L->tile_cap[1] = has_cr ? round_up(std::max<int64_t>((int64_t)std::ceil(cf1 * c->ppc_cr * cells), 64), 64) : 0;
    for (int s = 0; s < 2; ++s) {
        L->capacity[s] = L->ntiles * L->tile_cap[s];
        int64_t cap = L->capacity[s];
        int64_t bytes = round_up(cap * 4, 256) + c->dim * round_up(cap * rb, 256) + 3 * round_up(cap * rb, 256) +
                        round_up(cap * 4, 256);
        L->buf_bytes[s] = cap ? bytes : 0;
    }
    if (L->tile_cap[0] > INT32_MAX || L->tile_cap[1] > INT32_MAX) { err = "tile capacity too large"; return FS_EINVAL; }
    L->gather_bytes = L->nnode * 6 * rb;
    static const int cic[4] = {0, 22, 11, 7}, tsc[4] = {0, 10, 5, 3};
    L->b_bits = c->shape == 2 ? tsc[c->dim] : cic[c->dim];
    L->sv_bits = sv_for(c->v_max);
    L->sw_bits = c->shape == 2 ? c->dim * (2 * L->b_bits + 1) : c->dim * L->b_bits;
    if (lds_bytes(c->dim, c->shape, rb, true) > 160 * 1024) { err = "tile does not fit in LDS"; return FS_EINVAL; }
    return FS_OK;
}

void inject_counts(const fs_config& c, int64_t step, int64_t& th, int64_t& cr) {
    th = cr = 0;
    if (c.xbc != FS_XBC_BOX || !c.inject) return;
    double F = (double)c.ppc * c.u_sh * c.dt / c.dx;
    if (F > 0.0) th = (int64_t)(std::floor(F * (double)(step + 1)) - std::floor(F * (double)step));
    double u2 = c.u_sh / c.r;
    if (c.n_cr > 0.0 && c.wall_cr == FS_WALL_FAUX_SHOCK && c.cr_w > u2) {
        double Fc = (double)c.ppc_cr * (c.cr_w - u2) * c.dt / (2.0 * c.dx);
        cr = (int64_t)(std::floor(Fc * (double)(step + 1)) - std::floor(Fc * (double)step));
    }
}

template <typename R> PBuf<R> sections(void* base, int64_t cap, int dim) {
    char* p = static_cast<char*>(base);
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        char* q = p + off;
        off += round_up(bytes, 256);
        return q;
    };
    PBuf<R> b;
    b.cell = reinterpret_cast<int32_t*>(take(cap * 4));
    for (int d = 0; d < 3; ++d) b.off[d] = d < dim ? reinterpret_cast<R*>(take(cap * sizeof(R))) : nullptr;
    for (int c = 0; c < 3; ++c) b.v[c] = reinterpret_cast<R*>(take(cap * sizeof(R)));
    b.id = reinterpret_cast<uint32_t*>(take(cap * 4));
    return b;
}

// Dynamic LDS above the default limit must be requested per kernel.
template <typename K> void allow_lds(K kernel, size_t bytes) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)bytes);
}

constexpr size_t kMaxTimed = 4096 * 8;

// Records an event pair bracketing one phase; returns the index of the pair
// or -1 when timing is off or the pool is exhausted.
int timing_begin(fs_handle* h, int phase, hipStream_t s) {
    if (!h->timing || h->ev_used + 2 > h->ev_pool.size()) return -1;
    int k = (int)h->ev_used;
    h->ev_used += 2;
    h->ev_phase[k / 2] = phase;
    (void)hipEventRecord(h->ev_pool[k], s);
    return k;
}
void timing_end(fs_handle* h, int k, hipStream_t s) {
    if (k >= 0) (void)hipEventRecord(h->ev_pool[k + 1], s);
}

unsigned grid_for(int64_t n, int block = 256) { return (unsigned)std::max<int64_t>(1, (n + block - 1) / block); }

int policy_of(const fs_handle* h, int s) { return s == 0 ? h->cfg.wall_th : h->cfg.wall_cr; }

// The wall's parameters at a step: with the prescribed wall, u2 follows the
// drifting compression ratio u_sh / max(1, r + r_dot t), t = step dt.
WallModel wall_model_at(const fs_handle* h, int64_t step) {
#pragma clang fp contract(off)
    const fs_config& c = h->cfg;
    WallModel m{};
    m.on = c.wall_model == 1;
    const double r = c.r + c.r_dot * ((double)step * c.dt);
    m.u2 = m.on ? c.u_sh / (r > 1.0 ? r : 1.0) : h->G.u2;
    m.f0 = c.ret_f0; m.alpha = c.ret_alpha; m.wref = c.cr_w; m.gain = c.gain; m.kappa = c.kappa;
    // loss cone: downstream field b2 ~ (cos th, r sin th, 0) at this step's r,
    // its upstream-pointing direction (-lc_cx, -lc_sy, 0)
    m.lc_dep = c.lc_depletion;
    const double th = c.theta_deg * (kTwoPi / 360.0);
    const double bn = std::cos(th), bt = (r > 1.0 ? r : 1.0) * std::sin(th);
    const double nb = std::sqrt(bn * bn + bt * bt);
    const double bx = bn / nb, by = bt / nb;
    m.lc_cx = std::fabs(bx);
    m.lc_sy = bx < 0.0 ? -by : by;
    return m;
}

void zero_u64(void* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill_u64<<<std::min<unsigned>(grid_for(n), 4096u), 256, 0, s>>>(static_cast<unsigned long long*>(p), 0ull, n);
}
void zero_i32(int32_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill_i32<<<std::min<unsigned>(grid_for(n), 4096u), 256, 0, s>>>(p, 0, n);
}

// ------------------------------------------------------------------------
// field update (FP64)
// ------------------------------------------------------------------------
// stages: NULL, or (one sub-step) where the RK stages B1 and B2 go instead
// of the handle's scratch (3 x ncent doubles each, B1 first).  Bin: NULL,
// or B^n to step from instead of f->B (which then only receives B^{n+1}).
// fluid_out: NULL, or where the fluid state goes instead of the handle's
// buffer (5 x nnode doubles; never given with the filter or the
// time-centred coupling).
template <typename R, int D> void field_update_d(fs_handle* h, fs_fields* f, hipStream_t s, bool rk,
                                                 double* stages = nullptr, const double* Bin = nullptr,
                                                 double* fluid_out = nullptr) {
    const long nn = h->L.nnode, nc = h->L.ncent;
    const dim3 blk(kFX, kFY, 1);
    const dim3 gn((unsigned)((h->L.nxn + kFX - 1) / kFX), (unsigned)((h->L.nyc + kFY - 1) / kFY), (unsigned)h->L.nzc);
    // the time-centred coupling: the step's field update takes the moments at
    // t_{n+1/2} (h->fluid) and its final Ohm those at t_{n+1} (h->fluid2); a
    // refresh (Ohm only) makes the current moments the previous step's
    const int tc = h->cfg.coupling == 2 ? (rk ? 2 : 1) : 0;
    k_fluid<<<gn, blk, 0, s>>>(h->F, reinterpret_cast<const long long*>(f->mom[0]),
                               reinterpret_cast<const long long*>(h->has_cr ? f->mom[1] : f->mom[0]),
                               fluid_out ? fluid_out : h->fluid, nn,
                               h->fluid2, h->nprev, h->gprev, tc);
    if (h->cfg.smooth > 0) {
        // passes ping-pong between the two buffers; the finish writes the
        // other one, which then becomes h->fluid
        double* a = h->fluid;
        double* b = h->fluid2;
        for (int pass = 0; pass < h->cfg.smooth; ++pass)
            for (int axis = 0; axis < D; ++axis) {
                k_smooth_axis<<<gn, blk, 0, s>>>(h->F, a, b, axis, nn);
                std::swap(a, b);
            }
        k_smooth_finish<<<gn, blk, 0, s>>>(h->F, a, b, nn);
        if (b != h->fluid) std::swap(h->fluid, h->fluid2);
    }
    // taken after the filter, which may have swapped the buffers (the
    // time-centred coupling, which uses fluid2, runs without it)
    const double* fl = fluid_out ? fluid_out : h->fluid;
    const double* fl_ohm = tc == 2 ? h->fluid2 : fl;
    const double hs = h->cfg.dt / (double)h->cfg.n_sub;
    if constexpr (D == 3) {
        // z-marching kernels: 32 x 8 columns over runs of at most 32 z planes
        const int gx = (h->cfg.nx + ZMarch::X - 1) / ZMarch::X, gxo = (int)((h->L.nxn + ZMarch::X - 1) / ZMarch::X);
        const int gy = (int)((h->L.nyc + ZMarch::Y - 1) / ZMarch::Y);
        const int zc = (int)std::min<int64_t>(h->L.nzc, 32), gz = (int)((h->L.nzc + zc - 1) / zc);
        if (rk) {
            const unsigned nb = (unsigned)(gx * gy * gz);
            double* B1 = stages ? stages : h->B1;
            double* B2 = stages ? stages + 3 * nc : h->B2;
            for (int sub = 0; sub < h->cfg.n_sub; ++sub) {
                const double* B0 = (sub == 0 && Bin) ? Bin : f->B;
                k_stage3<<<nb, 256, 0, s>>>(h->F, B0, B0, B1, fl, 0.0, 1.0, hs, nn, nc, gx, gy, zc);
                k_stage3<<<nb, 256, 0, s>>>(h->F, B1, B0, B2, fl, 0.75, 0.25, hs, nn, nc, gx, gy, zc);
                k_stage3<<<nb, 256, 0, s>>>(h->F, B2, B0, f->B, fl, 1.0 / 3.0, 2.0 / 3.0, hs, nn, nc, gx, gy,
                                            zc);
            }
        }
        k_ohm3<R><<<(unsigned)(gxo * gy * gz), 256, 0, s>>>(h->F, f->B, fl_ohm, f->E, static_cast<R*>(f->gather), nn,
                                                           nc, gxo, gy, zc);
        return;
    }
    using FB = FieldBlock<D>;
    const int gy = (int)((h->L.nyc + FB::Y - 1) / FB::Y), gz = (int)((h->L.nzc + FB::Z - 1) / FB::Z);
    if (rk) {
        const int gx = (h->cfg.nx + FB::X - 1) / FB::X;
        const unsigned nb = (unsigned)(gx * gy * gz);
        double* B1 = stages ? stages : h->B1;
        double* B2 = stages ? stages + 3 * nc : h->B2;
        for (int sub = 0; sub < h->cfg.n_sub; ++sub) {
            // SSP-RK3 (Shu-Osher): B1 = B + h F(B); B2 = 3/4 B + 1/4 (B1 + h F(B1));
            // B <- 1/3 B + 2/3 (B2 + h F(B2)); the last stage writes f->B
            const double* B0 = (sub == 0 && Bin) ? Bin : f->B;
            k_stage<D><<<nb, 256, 0, s>>>(h->F, B0, B0, B1, fl, 0.0, 1.0, hs, nn, nc, gx, gy);
            k_stage<D><<<nb, 256, 0, s>>>(h->F, B1, B0, B2, fl, 0.75, 0.25, hs, nn, nc, gx, gy);
            k_stage<D><<<nb, 256, 0, s>>>(h->F, B2, B0, f->B, fl, 1.0 / 3.0, 2.0 / 3.0, hs, nn, nc, gx, gy);
        }
    }
    const int gxo = (int)((h->L.nxn + FB::X - 1) / FB::X);
    k_ohm<R, D><<<(unsigned)(gxo * gy * gz), 256, 0, s>>>(h->F, f->B, fl_ohm, f->E, static_cast<R*>(f->gather), nn, nc,
                                                        gxo, gy);
}

template <typename R>
void field_update(fs_handle* h, fs_fields* f, hipStream_t s, bool rk, double* stages = nullptr,
                  const double* Bin = nullptr, double* fluid_out = nullptr) {
    if (h->cfg.dim == 1) field_update_d<R, 1>(h, f, s, rk, stages, Bin, fluid_out);
    else if (h->cfg.dim == 2) field_update_d<R, 2>(h, f, s, rk, stages, Bin, fluid_out);
    else field_update_d<R, 3>(h, f, s, rk, stages, Bin, fluid_out);
}

// ------------------------------------------------------------------------
// one step, templated on precision, dimensionality and shape
// ------------------------------------------------------------------------
template <typename R, int D, int S>
void deposit_continuous(fs_handle* h, const fs_particles* sp, double* const mom[2], hipStream_t s) {
    using X = Extent<D, S>;
    const size_t lds = 32 * X::DN;
    for (int k = 0; k < (h->has_cr ? 2 : 1); ++k) {
        const fs_particles& P = sp[k];
        PBuf<R> in = sections<R>(P.buf[P.cur], P.capacity, D);
        zero_u64(reinterpret_cast<unsigned long long*>(mom[k]), 4 * h->L.ndep, s);
        allow_lds(k_deposit_c<R, D, S>, lds);
        const int sp_ = split_for(h->L, P.tile_cap);
        k_deposit_c<R, D, S><<<(unsigned)(h->L.ntiles * sp_), 256, lds, s>>>(h->G, in, P.tile_count[P.cur], P.tile_cap,
                                                                            mom[k], h->ctr, sp_);
    }
}

template <typename R, int D, int S>
int step_impl(fs_handle* h, fs_particles* sp, fs_fields* f, int64_t step, uint32_t flags, hipStream_t s,
              const fs_record* rec = nullptr, const fs_packed* pk = nullptr) {
    const bool push = flags & FS_PUSH, inj = flags & FS_INJECT, fld = flags & FS_FIELD;
    const bool cont = h->cfg.deposit_mode == 1;
    const bool rel = h->cfg.c_light > 0.0;
    // the continuous deposit is fused into the push, the wall and the
    // injection of a non-relativistic 2D or 3D step that moves the ions;
    // otherwise it runs as its own pass over the bins after the moves.  In 1D
    // all ions injected in a step land on the same two nodes, where their
    // direct FP64 atomics serialise, and the separate pass is the cheaper one.
    const bool dep = (flags & FS_DEPOSIT) && !cont;
    const bool cdep = (flags & FS_DEPOSIT) && cont;
    const bool fcd = cdep && push && !rel && D >= 2;
    const int nsp = h->has_cr ? 2 : 1;
    const fs_config& c = h->cfg;
    int64_t cth = 0, ccr = 0;
    if (inj) inject_counts(c, step, cth, ccr);
    const int64_t ntr = h->L.nyc * h->L.nzc;
    const int64_t ninj = (cth + ccr) * ntr;
    if (h->next_id + ninj > (int64_t)UINT32_MAX + 1) return fail(h, FS_EIDOVERFLOW, "particle ids would overflow 32 bits");
    Geo G = h->G;
    const int t_step = timing_begin(h, 4, s);
    zero_u64(h->ctr, C_N, s);
    if (dep || fcd)
        for (int k = 0; k < nsp; ++k) zero_u64(f->mom[k], 4 * h->L.ndep, s);
    using X = Extent<D, S>;
    const size_t lds_push = PushLds<R, D, S>::bytes(dep || fcd);
    // a recorded step may read its input state's grids from elsewhere
    const R* gather_in = static_cast<const R*>(rec && rec->gather_in ? rec->gather_in : f->gather);
    if (push) {
        for (int k = 0; k < nsp; ++k) {
            zero_i32(sp[k].tile_count[sp[k].cur ^ 1], 2 * h->L.ntiles, s);
            zero_i32(h->xl[k].count, 1, s);
        }
        const int t_push = timing_begin(h, 0, s);
        for (int k = 0; k < nsp; ++k) {
            fs_particles& P = sp[k];
            PBuf<R> in = sections<R>(P.buf[P.cur], P.capacity, D);
            PBuf<R> out = sections<R>(P.buf[P.cur ^ 1], P.capacity, D);
            auto* mom = reinterpret_cast<unsigned long long*>(f->mom[k]);
            // a recorded step with a packed state: the push copies its input there
            PBuf<R> pko{};
            const int32_t* pk_toff = nullptr;
            int64_t pk_n = 0;
            if (pk) {
                pko = sections<R>(pk->buf[k], pk->n[k], D);
                pk_toff = pk->toff[k];
                pk_n = pk->n[k];
            }
            auto launch = [&](auto kern) {
                allow_lds(kern, lds_push);
                kern<<<(unsigned)h->L.ntiles, PUSH_THREADS, lds_push, s>>>(
                    G, in, out, P.tile_count[P.cur], P.tile_count[P.cur ^ 1], P.tile_cap, gather_in,
                    mom, h->xl[k], h->ctr, policy_of(h, k), k, rec ? rec->dst[k] : nullptr, pko, pk_toff, pk_n);
            };
            // a recorded step is a continuous-deposit, non-relativistic one
            if (rec) fcd ? launch(k_push<R, D, S, true, false, false, true, true>)
                         : launch(k_push<R, D, S, false, false, false, true>);
            else if (fcd) launch(k_push<R, D, S, true, false, false, false, true>);
            else if (dep && h->cfg.coupling == 2)
                rel ? launch(k_push<R, D, S, true, true, true>) : launch(k_push<R, D, S, true, false, true>);
            else if (dep) rel ? launch(k_push<R, D, S, true, true>) : launch(k_push<R, D, S, true, false>);
            else rel ? launch(k_push<R, D, S, false, true>) : launch(k_push<R, D, S, false, false>);
        }
        timing_end(h, t_push, s);
        const int t_wall = timing_begin(h, 1, s);
        if (c.xbc == FS_XBC_BOX) {
            for (int k = 0; k < nsp; ++k) {
                if (policy_of(h, k) == FS_WALL_OPEN) continue;
                fs_particles& P = sp[k];
                PBuf<R> out = sections<R>(P.buf[P.cur ^ 1], P.capacity, D);
                unsigned gw = std::min<unsigned>(grid_for(h->xl[k].cap), 1024u);
                auto* mom = reinterpret_cast<unsigned long long*>(f->mom[k]);
                int32_t* rd = rec ? rec->dst[k] : nullptr;
                const WallModel wm = wall_model_at(h, step);
                if (dep)
                    k_wall<R, D, S, true><<<gw, 256, 0, s>>>(G, h->xl[k], out, P.tile_count[P.cur ^ 1], P.tile_cap, mom,
                                                            h->ctr, policy_of(h, k), k, (uint64_t)step, rd, wm);
                else if (fcd)
                    k_wall<R, D, S, true, true><<<gw, 256, 0, s>>>(G, h->xl[k], out, P.tile_count[P.cur ^ 1], P.tile_cap,
                                                                  mom, h->ctr, policy_of(h, k), k, (uint64_t)step, rd,
                                                                  wm);
                else
                    k_wall<R, D, S, false><<<gw, 256, 0, s>>>(G, h->xl[k], out, P.tile_count[P.cur ^ 1], P.tile_cap, mom,
                                                             h->ctr, policy_of(h, k), k, (uint64_t)step, rd, wm);
            }
        }
        timing_end(h, t_wall, s);
    }
    const int t_inj = timing_begin(h, 2, s);
    if (inj && ninj > 0) {
        fs_particles& P0 = sp[0];
        const int t0 = push ? P0.cur ^ 1 : P0.cur;
        PBuf<R> o0 = sections<R>(P0.buf[t0], P0.capacity, D);
        PBuf<R> o1 = o0;
        int32_t* c1 = P0.tile_count[t0];
        int64_t cap1 = P0.tile_cap;
        unsigned long long* m1 = reinterpret_cast<unsigned long long*>(f->mom[0]);
        if (h->has_cr) {
            fs_particles& P1 = sp[1];
            const int t1 = push ? P1.cur ^ 1 : P1.cur;
            o1 = sections<R>(P1.buf[t1], P1.capacity, D);
            c1 = P1.tile_count[t1];
            cap1 = P1.tile_cap;
            m1 = reinterpret_cast<unsigned long long*>(f->mom[1]);
        }
        auto* m0 = reinterpret_cast<unsigned long long*>(f->mom[0]);
        if (dep && push)
            k_inject<R, D, S, true><<<grid_for(ninj), 256, 0, s>>>(G, o0, P0.tile_count[t0], P0.tile_cap, m0, o1, c1, cap1, m1,
                                                                  h->ctr, (uint64_t)step, h->next_id, cth, ccr, ntr);
        else if (fcd)
            k_inject<R, D, S, true, true><<<grid_for(ninj), 256, 0, s>>>(G, o0, P0.tile_count[t0], P0.tile_cap, m0, o1, c1,
                                                                        cap1, m1, h->ctr, (uint64_t)step, h->next_id,
                                                                        cth, ccr, ntr);
        else
            k_inject<R, D, S, false><<<grid_for(ninj), 256, 0, s>>>(G, o0, P0.tile_count[t0], P0.tile_cap, m0, o1, c1, cap1, m1,
                                                                   h->ctr, (uint64_t)step, h->next_id, cth, ccr, ntr);
    }
    timing_end(h, t_inj, s);
    if (push)
        for (int k = 0; k < nsp; ++k) sp[k].cur ^= 1;
    if (cdep && !fcd) {
        double* const mom[2] = {reinterpret_cast<double*>(f->mom[0]), h->has_cr ? reinterpret_cast<double*>(f->mom[1]) : nullptr};
        deposit_continuous<R, D, S>(h, sp, mom, s);
    }
    if (dep && !push) {
        const size_t lds_dep = 32 * X::DN;
        for (int k = 0; k < nsp; ++k) {
            fs_particles& P = sp[k];
            PBuf<R> in = sections<R>(P.buf[P.cur], P.capacity, D);
            allow_lds(k_deposit<R, D, S>, lds_dep);
            k_deposit<R, D, S><<<(unsigned)h->L.ntiles, 256, lds_dep, s>>>(
                G, in, P.tile_count[P.cur], P.tile_cap, reinterpret_cast<unsigned long long*>(f->mom[k]), h->ctr);
        }
    }
    if (fld) {
        const int t_fld = timing_begin(h, 3, s);
        field_update<R>(h, f, s, true, rec ? rec->stages : nullptr, rec ? rec->B_in : nullptr,
                        rec ? rec->fluid : nullptr);
        timing_end(h, t_fld, s);
    }
    if (push || inj)
        for (int k = 0; k < nsp; ++k)
            k_check_bins<<<grid_for(h->L.ntiles), 256, 0, s>>>(sp[k].tile_count[sp[k].cur], (int)h->L.ntiles, sp[k].tile_cap, h->ctr);
    k_count_update<<<1, 64, 0, s>>>(sp[0].count, h->has_cr ? sp[1].count : nullptr, h->ctr);
    timing_end(h, t_step, s);
    h->next_id += ninj;
    int rc = hip_check(h, hipGetLastError(), "kernel launch");
    if (rc) return rc;
    return hip_check(h, hipMemcpyAsync(h->ctr_host, h->ctr, C_N * sizeof(unsigned long long), hipMemcpyDeviceToHost, s),
                     "stats copy");
}

template <typename R, int D>
int init_impl(fs_handle* h, fs_particles* sp, fs_fields* f, const double* amps, hipStream_t s) {
    const fs_config& c = h->cfg;
    const long nc = h->L.ncent;
    if (c.n_modes > 0) k_phases<<<grid_for(c.n_modes), 256, 0, s>>>(c.seed, c.n_modes, h->phase);
    k_init_B<<<grid_for(nc), 256, 0, s>>>(h->F, c.n_modes, amps, c.mode_amp, h->phase, (double)c.nx * c.dx, f->B, nc);
    const long np = nc * (long)c.ppc;
    fs_particles& P = sp[0];
    P.cur = 0;
    PBuf<R> out = sections<R>(P.buf[0], P.capacity, D);
    if (np > 0) k_init_particles<R, D><<<grid_for(np), 256, 0, s>>>(h->G, out, P.tile_cap, c.ppc, np);
    k_init_counts<D><<<grid_for(h->L.ntiles), 256, 0, s>>>(h->G, P.tile_count[0], c.ppc);
    k_set_i64<<<1, 1, 0, s>>>(P.count, np);
    if (h->has_cr) {
        sp[1].cur = 0;
        zero_i32(sp[1].tile_count[0], 2 * h->L.ntiles, s);
        k_set_i64<<<1, 1, 0, s>>>(sp[1].count, 0);
    }
    h->next_id = np;
    return FS_OK;
}

template <typename R, int D, int S> int deposit_impl(fs_handle* h, const fs_particles* sp, fs_fields* f, hipStream_t s) {
    using X = Extent<D, S>;
    const int nsp = h->has_cr ? 2 : 1;
    zero_u64(h->ctr, C_N, s);
    if (h->cfg.deposit_mode == 1) {
        double* const mom[2] = {reinterpret_cast<double*>(f->mom[0]), h->has_cr ? reinterpret_cast<double*>(f->mom[1]) : nullptr};
        deposit_continuous<R, D, S>(h, sp, mom, s);
        return hip_check(h, hipGetLastError(), "deposit launch");
    }
    for (int k = 0; k < nsp; ++k) {
        zero_u64(f->mom[k], 4 * h->L.ndep, s);
        const fs_particles& P = sp[k];
        PBuf<R> in = sections<R>(P.buf[P.cur], P.capacity, D);
        allow_lds(k_deposit<R, D, S>, 32 * X::DN);
        k_deposit<R, D, S><<<(unsigned)h->L.ntiles, 256, 32 * X::DN, s>>>(
            h->G, in, P.tile_count[P.cur], P.tile_cap, reinterpret_cast<unsigned long long*>(f->mom[k]), h->ctr);
    }
    return hip_check(h, hipGetLastError(), "deposit launch");
}

// ------------------------------------------------------------------------
// reverse mode
// ------------------------------------------------------------------------
// One SSP-RK3 stage Bout = c0 Bn + c1 (Bin + h F(Bin)) with fluid state fl.
template <int D>
void stage_launch(fs_handle* h, const double* Bin, const double* Bn, double* Bout, const double* fl, double c0,
                  double c1, double hs, hipStream_t s) {
    const long nn = h->L.nnode, nc = h->L.ncent;
    if constexpr (D == 3) {
        const int gx = (h->cfg.nx + ZMarch::X - 1) / ZMarch::X;
        const int gy = (int)((h->L.nyc + ZMarch::Y - 1) / ZMarch::Y);
        const int zc = (int)std::min<int64_t>(h->L.nzc, 32), gz = (int)((h->L.nzc + zc - 1) / zc);
        k_stage3<<<(unsigned)(gx * gy * gz), 256, 0, s>>>(h->F, Bin, Bn, Bout, fl, c0, c1, hs, nn, nc, gx, gy, zc);
    } else {
        using FB = FieldBlock<D>;
        const int gx = (h->cfg.nx + FB::X - 1) / FB::X;
        const int gy = (int)((h->L.nyc + FB::Y - 1) / FB::Y), gz = (int)((h->L.nzc + FB::Z - 1) / FB::Z);
        k_stage<D><<<(unsigned)(gx * gy * gz), 256, 0, s>>>(h->F, Bin, Bn, Bout, fl, c0, c1, hs, nn, nc, gx, gy);
    }
}

// Particle adjoints of species k in buffer b.
template <typename R> PLam<R> plam(const fs_adjoint* a, int k, int b, int D) {
    PLam<R> L;
    for (int d = 0; d < 3; ++d) {
        L.x[d] = d < D ? static_cast<R*>(a->x[k][b][d]) : nullptr;
        L.v[d] = static_cast<R*>(a->v[k][b][d]);
    }
    return L;
}

// Fluid state of a tape state into the reverse scratch; the moments are read
// in place from `mom` (the tape's grids of that state), which the reverse
// step only reads.
void fluid_of(fs_handle* h, int64_t* const* mom, hipStream_t s) {
    const dim3 blk(kFX, kFY, 1);
    const dim3 gn((unsigned)((h->L.nxn + kFX - 1) / kFX), (unsigned)((h->L.nyc + kFY - 1) / kFY), (unsigned)h->L.nzc);
    k_fluid<<<gn, blk, 0, s>>>(h->F, reinterpret_cast<const long long*>(mom[0]),
                               reinterpret_cast<const long long*>(h->has_cr ? mom[1] : mom[0]), h->afl,
                               h->L.nnode, nullptr, nullptr, nullptr, 0);
}

// Transpose of Ohm's law at every node (see k_ohm_adj_node) evaluated at B:
// the node pass from lam_E (lE, or with curl the Faraday transpose of lam_F
// in lE), then the centre pass into o as EMIT says; in 2D and 3D both in one
// pass that marches through y rows or z planes.
template <int D, bool CURL, int EMIT>
void ohm_adj(fs_handle* h, const double* fl, const double* B, const double* lE, const double* lBb, const RkOut& o,
             double* grads, hipStream_t s) {
    const long nn = h->L.nnode, nc = h->L.ncent;
    if constexpr (D == 3) {
        // one z-marching pass over 32 x 8 block columns and runs of at most
        // 32 z planes, as the forward stage kernels
        const int gx = (h->cfg.nx + ZMarch::X - 1) / ZMarch::X, gy = (int)((h->L.nyc + ZMarch::Y - 1) / ZMarch::Y);
        const int zc = (int)std::min<int64_t>(h->L.nzc, 32), gz = (int)((h->L.nzc + zc - 1) / zc);
        k_ohm_adj3<CURL, EMIT><<<(unsigned)(gx * gy * gz), 256, 0, s>>>(h->F, B, fl, lE, lBb, h->alfl, o, grads,
                                                                         nn, nc, gx, gy, zc);
        return;
    }
    if constexpr (D == 2) {
        // the same in 2D through runs of at most 16 y rows: 255 centre
        // columns and 256 node columns (one per thread) per block
        const int gx = (h->cfg.nx + YMarch::RX - 1) / YMarch::RX;
        const int yc = (int)std::min<int64_t>(h->L.nyc, 16), gy = (int)((h->L.nyc + yc - 1) / yc);
        k_ohm_adj2<CURL, EMIT><<<(unsigned)(gx * gy), 256, 0, s>>>(h->F, B, fl, lE, lBb, h->alfl, o, grads, nn, nc,
                                                                    gx, yc);
        return;
    }
    k_ohm_adj_node<D, CURL><<<grid_for(nn), 256, 0, s>>>(h->F, B, fl, lE, lBb, h->aob, h->alfl, grads, nn, nc);
    k_ohm_adj_centre<D, EMIT><<<grid_for(nc), 256, 0, s>>>(h->F, h->aob, o, nn, nc);
}

// Transpose of the field update of one step (the SSP-RK3 sub-steps from
// B^n, then Ohm's law at B^{n+1}) with the fluid state fl: lam_B
// (in: lam(B^{n+1}), out: lam(B^n)), lam(E^{n+1}) in lE, lam(Bbar^{n+1})
// in lBb; fluid adjoints into h->alfl (its n_e and Gamma planes stored by
// the first pass, its p_e plane, zeroed before, added to).  The stages are
// recomputed unless the recorded step kept them.
// Each stage's F(B) = -curl Ohm(B, fl) is transposed by one node pass (the
// Faraday transpose gathered in it) and one centre pass that also does the
// RK vector update that follows it, fused into one marching pass in 2D and 3D.
template <int D>
void field_adj(fs_handle* h, const double* fl, const double* Bn1, const double* lE, const double* lBb,
               const double* Bn, double* lB, const double* stages, double* grads, hipStream_t s) {
    const long N = 3 * h->L.ncent;
    const int ns = h->cfg.n_sub;
    const double hs = h->cfg.dt / (double)ns;
    // the start of each sub-step (B^n for the first)
    double* Bs = h->aBs;
    for (int sub = 0; sub + 1 < ns; ++sub) {
        const double* B0 = sub == 0 ? Bn : Bs + (size_t)sub * N;
        stage_launch<D>(h, B0, B0, h->B1, fl, 0.0, 1.0, hs, s);
        stage_launch<D>(h, h->B1, B0, h->B2, fl, 0.75, 0.25, hs, s);
        stage_launch<D>(h, h->B2, B0, Bs + (size_t)(sub + 1) * N, fl, 1.0 / 3.0, 2.0 / 3.0, hs, s);
    }
    RkOut o{};
    o.l0 = h->al[0]; o.out = lB; o.h = hs;
    // lam_F alternates between two buffers: a pass reads the one the pass
    // before wrote (with halos, in the marching forms) and writes the other
    double* lFs[2] = {h->al[1], h->al[2]};
    int lfw = 0;
    auto next_lF = [&]() -> const double* {
        const double* in = lFs[lfw];
        lfw ^= 1;
        o.lF = lFs[lfw];
        return in;
    };
    o.lF = lFs[lfw];
    // Ohm at B^{n+1}; its centre pass starts the last sub-step's transpose
    // B3 = 1/3 B0 + 2/3 (B2 + h F(B2))
    o.base = lB;
    ohm_adj<D, false, kEmitStage3>(h, fl, Bn1, lE, lBb, o, grads, s);
    for (int sub = ns - 1; sub >= 0; --sub) {
        const double* B0 = sub == 0 ? Bn : Bs + (size_t)sub * N;
        // the stages, as the recorded step kept them or recomputed
        const double *B1 = h->B1, *B2 = h->B2;
        if (stages) {
            B1 = stages;
            B2 = stages + N;
        } else {
            stage_launch<D>(h, B0, B0, h->B1, fl, 0.0, 1.0, hs, s);
            stage_launch<D>(h, h->B1, B0, h->B2, fl, 0.75, 0.25, hs, s);
        }
        // lam(B2) = 2/3 lam(B3) + (dF/dB2)^T lF, where 2/3 lam(B3) = lF / h,
        // then B2 = 3/4 B0 + 1/4 (B1 + h F(B1))
        const double* lF2 = next_lF();
        o.lFin = lF2;
        ohm_adj<D, true, kEmitStage2>(h, fl, B2, lF2, nullptr, o, grads, s);
        // lam(B1) = 1/4 lam(B2) + (dF/dB1)^T lF, where 1/4 lam(B2) = lF / h,
        // then B1 = B0 + h F(B0)
        const double* lF1 = next_lF();
        o.lFin = lF1;
        ohm_adj<D, true, kEmitStage1>(h, fl, B1, lF1, nullptr, o, grads, s);
        // lam(B0) = l0 + (dF/dB0)^T lF: the start of this sub-step, which
        // ends the previous one (or is lam(B^n))
        o.base = o.l0;
        const double* lF0 = next_lF();
        if (sub > 0) ohm_adj<D, true, kEmitStage3>(h, fl, B0, lF0, nullptr, o, grads, s);
        else ohm_adj<D, true, kEmitOut>(h, fl, B0, lF0, nullptr, o, grads, s);
    }
}

// Fluid transpose: lam of the fluid state in h->alfl -> the moment adjoints
// h->alM[k] at the deposit nodes (and the alpha_cr adjoint), at the moment
// grids `mom` the fluid state came from.
void fluid_adj(fs_handle* h, int64_t* const* mom, double* grads, hipStream_t s) {
    const long nn = h->L.nnode;
    // k_fluid_adj stores every entry of a periodic grid once; in a box only
    // the entries at the x ends need clearing first
    if (h->cfg.xbc == FS_XBC_BOX) {
        const int g = (int)((h->L.ndx - h->L.nxn) / 2), mc = h->cfg.shape;
        const int lo = mc + g, hi = h->cfg.nx - mc + g;
        const long rows = h->L.nyc * h->L.nzc;
        const unsigned nb = std::min<unsigned>(grid_for(rows * (lo + 1 + (h->L.ndx - hi)) * 4), 4096u);
        for (int k = 0; k < (h->has_cr ? 2 : 1); ++k)
            k_zero_dep_ends<<<nb, 256, 0, s>>>(h->alM[k], (int)h->L.ndx, rows, lo, hi);
    }
    const double dwcr = h->has_cr ? h->cfg.n_cr / (double)h->cfg.ppc_cr : 0.0;
    const double* m0 = reinterpret_cast<const double*>(mom[0]);
    const double* m1 = reinterpret_cast<const double*>(h->has_cr ? mom[1] : mom[0]);
    k_fluid_adj<<<grid_for(nn), 256, 0, s>>>(h->F, m0, m1, h->alfl, h->alM[0],
                                             h->alM[1], nn, dwcr, grads + 1);
}

template <typename R, int D, int S>
int adjoint_step_impl(fs_handle* h, const fs_packed* pn, const fs_fields* f_n, const fs_packed* pn1,
                      const fs_fields* f_n1, const double* stages, const double* fluid, int64_t id0, int64_t step,
                      fs_adjoint* lam, double* grads, hipStream_t s) {
    const long nn = h->L.nnode;
    // fluid state the step's field update used (from the moments of the
    // particles after it), as the recorded step kept it or recomputed
    const double* fl = fluid;
    if (!fl) {
        fluid_of(h, f_n1->mom, s);
        fl = h->afl;
    }
    // the p_e adjoints are gathered by atomics; the first (curl-free) Ohm
    // transpose stores the n_e and Gamma ones
    zero_u64(reinterpret_cast<unsigned long long*>(h->alfl + nn), nn, s);
    // final Ohm, then the RK3 sub-steps
    field_adj<D>(h, fl, f_n1->B, lam->lE, lam->lE + 3 * nn, f_n->B, lam->lB, stages, grads, s);
    // fluid at n+1: the moment adjoints the deposit transpose reads
    fluid_adj(h, f_n1->mom, grads, s);
    const int post = lam->cur, pre = lam->cur ^ 1;
    // the ions the step injected: their adjoint after it into dL/du_sh
    int64_t cth = 0, ccr = 0;
    inject_counts(h->cfg, step, cth, ccr);
    const int64_t ntr = h->L.nyc * h->L.nzc, nth = cth * ntr, ncr = ccr * ntr;
    // injection puts a thermal ion at x = |u_sh + sigma n| U dt/dx and a CR at
    // x = nx - |u2 - cr_w mu| U dt/dx (U < 1, |n| < 8.7 for the 53-bit
    // uniforms of the Box-Muller pair), so only the tile columns within
    // those depths of their boundary (and one more) are read
    const fs_config& c = h->cfg;
    const int TX = h->L.tile[0], ntx = h->L.ntile[0];
    const double dtdx = c.dt / c.dx, sigma = std::sqrt(0.5 * c.beta_i);
    const double dth = (std::fabs(c.u_sh) + 8.7 * sigma) * dtdx;
    const double dcr = (std::fabs(c.u_sh / c.r) + c.cr_w) * dtdx;
    for (int k = 0; k < (h->has_cr ? 2 : 1) && nth + ncr > 0; ++k) {
        const int64_t expect = k == 0 ? nth : ncr;
        int cx0, cx1;
        if (k == 0) {
            const int cmax = (int)std::min<double>(c.nx - 1, std::floor(dth));
            cx0 = 0;
            cx1 = std::min(ntx - 1, cmax / TX + 1);
        } else {
            const int cmin = (int)std::max<double>(0.0, std::floor((double)c.nx - dcr));
            cx0 = std::max(0, cmin / TX - 1);
            cx1 = ntx - 1;
        }
        const int ncols = cx1 - cx0 + 1;
        PBuf<R> in1 = sections<R>(pn1->buf[k], pn1->n[k], D);
        const unsigned g = (unsigned)(ncols * (h->L.ntiles / ntx));
        k_inject_adj<R, D, S><<<g, 256, 0, s>>>(h->G, in1, pn1->toff[k], pn1->n[k], h->alM[k],
                                                plam<R>(lam, k, post, D), (uint64_t)step, id0, nth, nth + ncr, cx0,
                                                ncols, h->actr, expect, pn1->status, grads);
    }
    // deposit at n+1, then push, wall and gather of the ions that lived
    // before the step: buffer cur (indices after the step) -> cur ^ 1
    // (indices before it)
    zero_u64(reinterpret_cast<unsigned long long*>(lam->lE), 6 * nn, s);
    for (int k = 0; k < (h->has_cr ? 2 : 1); ++k) {
        PBuf<R> in = sections<R>(pn->buf[k], pn->n[k], D);
        PBuf<R> in1 = sections<R>(pn1->buf[k], pn1->n[k], D);
        const int sp_ = split_for(h->L, h->L.tile_cap[k]);
        k_push_adj<R, D, S><<<(unsigned)(h->L.ntiles * sp_), AdjPush<R, D, S>::threads, 0, s>>>(
            h->G, in, pn->toff[k], pn->n[k], in1, h->alM[k], static_cast<const R*>(f_n->gather), pn->dst[k],
            plam<R>(lam, k, post, D), plam<R>(lam, k, pre, D), lam->lE, nn, (uint64_t)step, grads, sp_,
            policy_of(h, k) == FS_WALL_SPECULAR ? 1 : 0);
    }
    lam->cur = pre;
    return hip_check(h, hipGetLastError(), "adjoint step launch");
}

template <typename R, int D, int S>
int adjoint_init_impl(fs_handle* h, const fs_packed* p0, const fs_fields* f0, fs_adjoint* lam, double* grads,
                      hipStream_t s) {
    const long nn = h->L.nnode, nc = h->L.ncent;
    fluid_of(h, f0->mom, s);
    // the p_e adjoints are gathered by atomics; the first (curl-free) Ohm
    // transpose stores the n_e and Gamma ones
    zero_u64(reinterpret_cast<unsigned long long*>(h->alfl + nn), nn, s);
    RkOut o{};
    o.base = o.out = lam->lB;
    ohm_adj<D, false, kEmitOut>(h, h->afl, f0->B, lam->lE, lam->lE + 3 * nn, o, grads, s);
    fluid_adj(h, f0->mom, grads, s);
    for (int k = 0; k < (h->has_cr ? 2 : 1); ++k) {
        PBuf<R> in = sections<R>(p0->buf[k], p0->n[k], D);
        const int sp_ = split_for(h->L, h->L.tile_cap[k]);
        k_deposit_adj<R, D, S><<<(unsigned)(h->L.ntiles * sp_), 256, 0, s>>>(
            h->G, in, p0->toff[k], p0->n[k], h->alM[k], plam<R>(lam, k, lam->cur, D), sp_);
    }
    k_init_adj<R><<<std::min<unsigned>(grid_for(p0->n[0]), 2048u), 256, 0, s>>>(
        p0->toff[0], (int)h->L.ntiles, p0->n[0], plam<R>(lam, 0, lam->cur, D), grads);
    const fs_config& c = h->cfg;
    if (c.n_modes > 0) {
        k_phases<<<grid_for(c.n_modes), 256, 0, s>>>(c.seed, c.n_modes, h->phase);
        const int parts = (int)std::min<int64_t>(64, std::max<int64_t>(1, nc / 4096));
        k_amps_adj<<<dim3((unsigned)parts, (unsigned)c.n_modes), 256, 0, s>>>(h->F, lam->lB, h->phase,
                                                                           (double)c.nx * c.dx, nc, grads);
    }
    return hip_check(h, hipGetLastError(), "adjoint init launch");
}

// The tile offsets of sp's live ions into out, with `ions` the ions
// themselves, and with a record its conversion into prev->dst.
template <typename R, int D>
int tape_pack_impl(fs_handle* h, const fs_particles* sp, fs_packed* out, const fs_particles* prev_sp,
                   const fs_record* rec, fs_packed* prev, bool ions, hipStream_t s) {
    const int nt = (int)h->L.ntiles;
    for (int k = 0; k < (h->has_cr ? 2 : 1); ++k) {
        const fs_particles& P = sp[k];
        const unsigned nch = (unsigned)((nt + kScanChunk - 1) / kScanChunk);
        k_tape_chunks<<<nch, 1024, 0, s>>>(P.tile_count[P.cur], nt, P.tile_cap, h->scan_part);
        k_tape_offsets<<<nch, 1024, 0, s>>>(P.tile_count[P.cur], nt, P.tile_cap, h->scan_part, out->toff[k], out->n[k],
                                            out->status);
        PBuf<R> in = sections<R>(P.buf[P.cur], P.capacity, D);
        PBuf<R> o = sections<R>(out->buf[k], out->n[k], D);
        // boxes with few tiles (large ones) split each over workgroups of
        // about 1024 ions, up to some 4096 workgroups in all
        const int sp_ = (int)std::max<int64_t>(1, std::min<int64_t>(P.tile_cap / 1024, 4096 / nt));
        if (ions)
            k_tape_pack<R, D><<<(unsigned)(nt * sp_), 256, 0, s>>>(h->G, in, P.tile_count[P.cur], P.tile_cap,
                                                                   out->toff[k], out->n[k], o, sp_);
        if (rec) {
            const fs_particles& Q = prev_sp[k];
            k_tape_record<<<(unsigned)(nt * sp_), 256, 0, s>>>(h->G, Q.tile_count[Q.cur], Q.tile_cap, prev->toff[k],
                                                               prev->n[k], rec->dst[k], P.tile_count[P.cur],
                                                               out->toff[k], out->n[k], prev->dst[k], prev->status,
                                                               sp_);
        }
    }
    return hip_check(h, hipGetLastError(), "tape pack launch");
}

// The packed state pk into the bins of sp (buf[cur], tile_count[cur], count).
template <typename R, int D>
int tape_unpack_impl(fs_handle* h, const fs_packed* pk, fs_particles* sp, hipStream_t s) {
    const int nt = (int)h->L.ntiles;
    for (int k = 0; k < (h->has_cr ? 2 : 1); ++k) {
        fs_particles& P = sp[k];
        PBuf<R> in = sections<R>(pk->buf[k], pk->n[k], D);
        PBuf<R> out = sections<R>(P.buf[P.cur], P.capacity, D);
        const int sp_ = (int)std::max<int64_t>(1, std::min<int64_t>(P.tile_cap / 1024, 4096 / nt));
        k_tape_unpack<R, D><<<(unsigned)(nt * sp_), 256, 0, s>>>(h->G, in, pk->toff[k], pk->n[k], out,
                                                                 P.tile_count[P.cur], P.tile_cap,
                                                                 reinterpret_cast<long long*>(P.count), sp_,
                                                                 pk->status);
    }
    return hip_check(h, hipGetLastError(), "tape unpack launch");
}

// Dispatch a templated implementation on (precision, dim).
#define FS_DISPATCH_RD(h, CALL)                                                  \
    do {                                                                         \
        const int _d = (h)->cfg.dim;                                             \
        if ((h)->cfg.precision == 32) {                                          \
            using R = float;                                                     \
            if (_d == 1) { constexpr int D = 1; return CALL; }                   \
            if (_d == 2) { constexpr int D = 2; return CALL; }                   \
            if (_d == 3) { constexpr int D = 3; return CALL; }                   \
        } else {                                                                 \
            using R = double;                                                    \
            if (_d == 1) { constexpr int D = 1; return CALL; }                   \
            if (_d == 2) { constexpr int D = 2; return CALL; }                   \
            if (_d == 3) { constexpr int D = 3; return CALL; }                   \
        }                                                                        \
        return fail(h, FS_EINVAL, "unsupported configuration");                  \
    } while (0)

// Dispatch a templated implementation on (precision, dim, shape).
#define FS_DISPATCH(h, CALL)                                                           \
    do {                                                                               \
        const int _d = (h)->cfg.dim, _s = (h)->cfg.shape;                              \
        if ((h)->cfg.precision == 32) {                                                \
            using R = float;                                                           \
            if (_d == 1 && _s == 1) { constexpr int D = 1, S = 1; return CALL; }       \
            if (_d == 1 && _s == 2) { constexpr int D = 1, S = 2; return CALL; }       \
            if (_d == 2 && _s == 1) { constexpr int D = 2, S = 1; return CALL; }       \
            if (_d == 2 && _s == 2) { constexpr int D = 2, S = 2; return CALL; }       \
            if (_d == 3 && _s == 1) { constexpr int D = 3, S = 1; return CALL; }       \
            if (_d == 3 && _s == 2) { constexpr int D = 3, S = 2; return CALL; }       \
        } else {                                                                       \
            using R = double;                                                          \
            if (_d == 1 && _s == 1) { constexpr int D = 1, S = 1; return CALL; }       \
            if (_d == 1 && _s == 2) { constexpr int D = 1, S = 2; return CALL; }       \
            if (_d == 2 && _s == 1) { constexpr int D = 2, S = 1; return CALL; }       \
            if (_d == 2 && _s == 2) { constexpr int D = 2, S = 2; return CALL; }       \
            if (_d == 3 && _s == 1) { constexpr int D = 3, S = 1; return CALL; }       \
            if (_d == 3 && _s == 2) { constexpr int D = 3, S = 2; return CALL; }       \
        }                                                                              \
        return fail(h, FS_EINVAL, "unsupported configuration");                        \
    } while (0)

int check_particles(fs_handle* h, const fs_particles* sp) {
    const int nsp = h->has_cr ? 2 : 1;
    for (int k = 0; k < nsp; ++k) {
        const fs_particles& P = sp[k];
        if (!P.buf[0] || !P.buf[1] || !P.tile_count[0] || !P.tile_count[1] || !P.count)
            return fail(h, FS_EINVAL, "particle buffer pointer is NULL");
        if (P.capacity < h->L.capacity[k] || P.tile_cap != h->L.tile_cap[k])
            return fail(h, FS_ECAPACITY, "particle buffer smaller than fs_layout reports");
        if (P.cur != 0 && P.cur != 1) return fail(h, FS_EINVAL, "cur must be 0 or 1");
    }
    return FS_OK;
}

int check_fields(fs_handle* h, const fs_fields* f) {
    if (!f || !f->B || !f->E || !f->gather || !f->mom[0] || (h->has_cr && !f->mom[1]))
        return fail(h, FS_EINVAL, "field pointer is NULL");
    return FS_OK;
}

}  // namespace

// ==========================================================================
// C ABI
// ==========================================================================
// Id-indexed parking of the adjoints of buffer lam->cur (see the header).
template <typename R, int D>
int park_impl(fs_handle* h, const fs_packed* pk, fs_adjoint* lam, void* scratch, const void* cscratch, int64_t nid,
              bool park, hipStream_t s) {
    for (int k = 0; k < (h->has_cr ? 2 : 1); ++k) {
        PBuf<R> p = sections<R>(pk->buf[k], pk->n[k], D);
        const unsigned g = std::min<unsigned>(grid_for(std::max<int64_t>(pk->n[k], 1)), 4096u);
        if (park) {
            R* sc = static_cast<R*>(scratch) + (int64_t)k * (D + 3) * nid;
            if (sizeof(R) == 8) zero_u64(sc, (int64_t)(D + 3) * nid, s);
            else zero_i32(reinterpret_cast<int32_t*>(sc), (int64_t)(D + 3) * nid, s);
            k_lam_park<R, D><<<g, 256, 0, s>>>(p.id, pk->toff[k], (int)h->L.ntiles, pk->n[k],
                                               plam<R>(lam, k, lam->cur, D), sc, nid);
        } else {
            const R* sc = static_cast<const R*>(cscratch) + (int64_t)k * (D + 3) * nid;
            k_lam_unpark<R, D><<<g, 256, 0, s>>>(p.id, pk->toff[k], (int)h->L.ntiles, pk->n[k],
                                                 plam<R>(lam, k, lam->cur, D), sc, nid);
        }
    }
    return hip_check(h, hipGetLastError(), "adjoint park launch");
}

extern "C" {

int fs_layout(const fs_config* cfg, fs_layout_info* out) {
    if (!cfg || !out) return fail(nullptr, FS_EINVAL, "NULL argument");
    std::string err;
    int rc = compute_layout(cfg, out, err);
    if (rc) g_err = err;
    return rc;
}

int fs_create(const fs_config* cfg, fs_handle** out) {
    if (!cfg || !out) return fail(nullptr, FS_EINVAL, "NULL argument");
    *out = nullptr;
    fs_handle* h = new fs_handle();
    h->cfg = *cfg;
    std::string err;
    int rc = compute_layout(cfg, &h->L, err);
    if (rc) { g_err = err; delete h; return rc; }
    const fs_config& c = h->cfg;
    h->has_cr = c.n_cr > 0.0;
    Geo& G = h->G;
    G.dim = c.dim; G.nx = c.nx; G.nyc = (int)h->L.nyc; G.nzc = (int)h->L.nzc;
    G.nxn = (int)h->L.nxn; G.ndx = (int)h->L.ndx; G.g = (int)((h->L.ndx - h->L.nxn) / 2);
    G.xbc = c.xbc;
    G.ntx = h->L.ntile[0]; G.nty = h->L.ntile[1]; G.ntz = h->L.ntile[2]; G.ntiles = (int)h->L.ntiles;
    G.bx = h->L.cell_bits[0]; G.by = h->L.cell_bits[1];
    G.b = h->L.b_bits; G.sv = h->L.sv_bits; G.mclamp = c.shape;
    G.dt = c.dt; G.dx = c.dx; G.u_sh = c.u_sh; G.u2 = c.u_sh / c.r; G.sigma = std::sqrt(0.5 * c.beta_i);
    G.cr_w = c.cr_w; G.dtdx = c.dt / c.dx; G.seed = c.seed; G.rinv = 1.0 / c.r;
    G.c_light = c.c_light; G.ic2 = c.c_light > 0.0 ? 1.0 / (c.c_light * c.c_light) : 0.0;
    FieldGeo& F = h->F;
    F.dim = c.dim; F.nx = c.nx; F.nyc = G.nyc; F.nzc = G.nzc; F.nxn = G.nxn; F.ndx = G.ndx; F.g = G.g;
    F.xbc = c.xbc; F.mclamp = c.shape; F.dx = c.dx; F.rdx = 1.0 / c.dx;
    const double th = c.theta_deg * (kTwoPi / 360.0);
    F.B0[0] = std::cos(th); F.B0[1] = std::sin(th); F.B0[2] = 0.0;
    F.n_floor = c.n_floor; F.beta_e = c.beta_e; F.gamma_e = c.gamma_e; F.eta = c.eta; F.j_ext = c.j_ext;
    F.smooth = c.smooth;
    F.conduct = c.xbc == FS_XBC_BOX && c.wall_field == 1;
    F.u_sh = c.u_sh;
    F.wth = c.ppc > 0 ? 1.0 / (double)c.ppc : 0.0;
    F.wcr = h->has_cr ? c.alpha_cr * c.n_cr / (double)c.ppc_cr : 0.0;
    F.scR = std::ldexp(1.0, -h->L.sw_bits);
    F.scG = std::ldexp(1.0, -(h->L.sw_bits + h->L.sv_bits));
    F.has_cr = h->has_cr ? 1 : 0;
    F.cont = c.deposit_mode == 1 ? 1 : 0;

    auto dmalloc = [&](void** p, size_t bytes) -> bool {
        return hipMalloc(p, std::max<size_t>(bytes, 256)) == hipSuccess;
    };
    bool ok = true;
    ok = ok && dmalloc((void**)&h->ctr, C_N * sizeof(unsigned long long));
    ok = ok && hipHostMalloc((void**)&h->ctr_host, C_N * sizeof(unsigned long long), hipHostMallocDefault) == hipSuccess;
    const long nc = h->L.ncent, nn = h->L.nnode;
    ok = ok && dmalloc((void**)&h->B1, 3 * nc * sizeof(double));
    ok = ok && dmalloc((void**)&h->B2, 3 * nc * sizeof(double));
    ok = ok && dmalloc((void**)&h->Etmp, 3 * nn * sizeof(double));
    ok = ok && dmalloc((void**)&h->fluid, 5 * nn * sizeof(double));
    if (c.smooth > 0 || c.coupling == 2) ok = ok && dmalloc((void**)&h->fluid2, 5 * nn * sizeof(double));
    if (c.coupling == 2) {
        ok = ok && dmalloc((void**)&h->nprev, nn * sizeof(double));
        ok = ok && dmalloc((void**)&h->gprev, 3 * nn * sizeof(double));
    }
    ok = ok && dmalloc((void**)&h->phase, (c.n_modes + 1) * sizeof(double));
    h->npart = std::max<int64_t>(grid_for(nc), h->L.ntiles) * 4;
    ok = ok && dmalloc((void**)&h->part, h->npart * sizeof(double));
    ok = ok && dmalloc((void**)&h->scan_part, (size_t)((h->L.ntiles + kScanChunk - 1) / kScanChunk) * sizeof(long long));
    if (c.deposit_mode == 1) {
        const long nd = h->L.ndep;
        for (int k = 0; k < (h->has_cr ? 2 : 1) && ok; ++k) ok = ok && dmalloc((void**)&h->alM[k], 4 * nd * sizeof(double));
        ok = ok && dmalloc((void**)&h->afl, 5 * nn * sizeof(double));
        ok = ok && dmalloc((void**)&h->alfl, 5 * nn * sizeof(double));
        for (int k = 0; k < 3 && ok; ++k) ok = ok && dmalloc((void**)&h->al[k], 3 * nc * sizeof(double));
        // the starts of RK sub-steps after the first (slot 0, B^n itself, unused)
        if (c.n_sub > 1) ok = ok && dmalloc((void**)&h->aBs, (size_t)c.n_sub * 3 * nc * sizeof(double));
        // the node pass's (lam_Bbar, lam_J) for the centre pass (1D only: the
        // 2D and 3D transposes keep a node row or plane in LDS)
        if (c.dim == 1) ok = ok && dmalloc((void**)&h->aob, 6 * nn * sizeof(double));
        ok = ok && dmalloc((void**)&h->actr, 2 * sizeof(unsigned long long));
        if (ok) ok = hipMemset(h->actr, 0, 2 * sizeof(unsigned long long)) == hipSuccess;
    }
    // crosser lists: a generous bound on the ions that can reach the wall in one step
    for (int k = 0; k < 2 && ok; ++k) {
        int64_t ppc = k == 0 ? c.ppc : c.ppc_cr;
        int64_t cap = (k == 1 && !h->has_cr) ? 64 : h->L.nyc * h->L.nzc * std::max<int64_t>(ppc, 1) * 8 + 4096;
        size_t bytes = 256 + 3 * round_up(cap * 8, 256) + round_up(3 * cap * 8, 256) + 4 * round_up(cap * 4, 256);
        ok = dmalloc(&h->xl_mem[k], bytes);
        if (!ok) break;
        char* p = static_cast<char*>(h->xl_mem[k]);
        XList& x = h->xl[k];
        x.cap = cap;
        x.count = reinterpret_cast<int32_t*>(p); p += 256;
        x.delta = reinterpret_cast<double*>(p); p += round_up(cap * 8, 256);
        x.oy = reinterpret_cast<double*>(p); p += round_up(cap * 8, 256);
        x.oz = reinterpret_cast<double*>(p); p += round_up(cap * 8, 256);
        x.v = reinterpret_cast<double*>(p); p += round_up(3 * cap * 8, 256);
        x.id = reinterpret_cast<uint32_t*>(p); p += round_up(cap * 4, 256);
        x.cy = reinterpret_cast<int32_t*>(p); p += round_up(cap * 4, 256);
        x.cz = reinterpret_cast<int32_t*>(p); p += round_up(cap * 4, 256);
        x.src = reinterpret_cast<int32_t*>(p);
    }
    if (!ok) {
        fs_destroy(h);
        return fail(nullptr, FS_EDEVICE, "device allocation of library scratch failed");
    }
    if (int rc = resolve_static_scratch(h)) {
        const std::string msg = h->err;
        fs_destroy(h);
        return fail(nullptr, rc, msg);
    }
    *out = h;
    return FS_OK;
}

void fs_destroy(fs_handle* h) {
    if (!h) return;
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    hipFree(h->ctr);
    if (h->ctr_host) hipHostFree(h->ctr_host);
    hipFree(h->B1); hipFree(h->B2); hipFree(h->Etmp); hipFree(h->fluid); hipFree(h->fluid2); hipFree(h->nprev); hipFree(h->gprev); hipFree(h->phase); hipFree(h->part); hipFree(h->scan_part); hipFree(h->spec);
    for (int k = 0; k < 2; ++k) hipFree(h->xl_mem[k]);
    for (int k = 0; k < 2; ++k) hipFree(h->alM[k]);
    hipFree(h->afl); hipFree(h->alfl); hipFree(h->aBs); hipFree(h->aob); hipFree(h->actr);
    for (int k = 0; k < 3; ++k) hipFree(h->al[k]);
    delete h;
}

const char* fs_last_error(const fs_handle* h) {
    if (h && !h->err.empty()) return h->err.c_str();
    return g_err.c_str();
}

int fs_init_plasma(fs_handle* h, fs_particles* sp, fs_fields* f, const double* amps, hipStream_t s) {
    if (!h || !sp || !f) return fail(h, FS_EINVAL, "NULL argument");
    int rc = check_particles(h, sp);
    if (!rc) rc = check_fields(h, f);
    if (rc) return rc;
    if ((int64_t)h->L.ncent * h->cfg.ppc > (int64_t)UINT32_MAX) return fail(h, FS_EIDOVERFLOW, "too many particles for 32-bit ids");
    auto init = [&]() -> int { FS_DISPATCH(h, (init_impl<R, D>(h, sp, f, amps, s))); };
    rc = init();
    if (rc) return rc;
    rc = fs_deposit_moments(h, sp, f, s);
    if (rc) return rc;
    return fs_refresh_fields(h, f, s);
}

static int step_common(fs_handle* h, fs_particles* sp, fs_fields* f, int64_t step, uint32_t flags, fs_step_stats* st,
                       hipStream_t s, const fs_record* rec, const fs_packed* pk = nullptr) {
    if (!h || !sp || !f) return fail(h, FS_EINVAL, "NULL argument");
    if (flags & ~FS_ALL) return fail(h, FS_EINVAL, "unknown step flags");
    if (step < 0) return fail(h, FS_EINVAL, "negative step");
    int rc = check_particles(h, sp);
    if (!rc) rc = check_fields(h, f);
    if (rc) return rc;
    auto run = [&]() -> int { FS_DISPATCH(h, (step_impl<R, D, S>(h, sp, f, step, flags, s, rec, pk))); };
    rc = run();
    if (rc) return rc;
    if (!st) return FS_OK;
    rc = hip_check(h, hipStreamSynchronize(s), "stream synchronise");
    if (rc) return rc;
    const unsigned long long* c = h->ctr_host;
    std::memset(st, 0, sizeof(*st));
    st->incident = (int64_t)c[C_INC];
    st->reflected = (int64_t)c[C_REFL];
    st->transmitted = (int64_t)c[C_TRANS];
    st->open_removed = (int64_t)c[C_OPEN];
    st->escaped = (int64_t)c[C_ESC];
    st->injected_th = (int64_t)c[C_INJ_TH];
    st->injected_cr = (int64_t)c[C_INJ_CR];
    st->saturated = (int64_t)c[C_SAT];
    st->out_of_range = (int64_t)c[C_OOR];
    st->flags = (int32_t)c[C_FLAGS];
    st->next_id = h->next_id;
    for (int k = 0; k < (h->has_cr ? 2 : 1); ++k) {
        rc = hip_check(h, hipMemcpy(&st->count[k], sp[k].count, sizeof(int64_t), hipMemcpyDeviceToHost), "count copy");
        if (rc) return rc;
    }
    if (st->flags & (F_TILE | F_XLIST)) return fail(h, FS_ETILE, "a tile bin or the crosser list overflowed");
    if (st->flags & (F_NAN | F_SAT)) return fail(h, FS_ENUMERIC, "NaN or saturated velocity code in the deposit");
    return FS_OK;
}

int fs_step(fs_handle* h, fs_particles* sp, fs_fields* f, int64_t step, uint32_t flags, fs_step_stats* st, hipStream_t s) {
    return step_common(h, sp, f, step, flags, st, s, nullptr);
}

static int check_adjoint(fs_handle* h, const fs_adjoint* lam) {
    if (!lam || !lam->lB || !lam->lE) return fail(h, FS_EINVAL, "NULL adjoint array");
    if (lam->cur != 0 && lam->cur != 1) return fail(h, FS_EINVAL, "adjoint buffer index outside {0, 1}");
    for (int k = 0; k < (h->has_cr ? 2 : 1); ++k) {
        for (int b = 0; b < 2; ++b)
            for (int d = 0; d < 3; ++d)
                if ((d < h->cfg.dim && !lam->x[k][b][d]) || !lam->v[k][b][d])
                    return fail(h, FS_EINVAL, "NULL particle adjoint array");
        if (lam->capacity[k] < 0) return fail(h, FS_EINVAL, "negative adjoint capacity");
    }
    return FS_OK;
}

// A packed state: arrays given, sizes within the int32 indices, and (with
// lam) adjoint buffers at least as long.
static int check_packed(fs_handle* h, const fs_packed* pk, const fs_adjoint* lam, bool need_dst) {
    if (!pk || !pk->status) return fail(h, FS_EINVAL, "NULL packed state");
    for (int k = 0; k < (h->has_cr ? 2 : 1); ++k) {
        if (!pk->buf[k] || !pk->toff[k] || (need_dst && !pk->dst[k])) return fail(h, FS_EINVAL, "NULL packed array");
        if (pk->n[k] < 0 || pk->n[k] > (int64_t)INT32_MAX - 2) return fail(h, FS_EINVAL, "packed size out of range");
        if (lam && lam->capacity[k] < pk->n[k])
            return fail(h, FS_ECAPACITY, "particle adjoint arrays shorter than the packed state");
    }
    return FS_OK;
}

static int check_record(fs_handle* h, const fs_record* rec) {
    for (int k = 0; k < (h->has_cr ? 2 : 1); ++k) {
        if (!rec->dst[k]) return fail(h, FS_EINVAL, "NULL record array");
        if (rec->capacity[k] < h->L.capacity[k]) return fail(h, FS_ECAPACITY, "record smaller than the particle buffers");
        if (h->L.capacity[k] > (int64_t)INT32_MAX - 2)
            return fail(h, FS_ECAPACITY, "particle buffers too large for the int32 step record");
    }
    return FS_OK;
}

static int check_reverse_cfg(fs_handle* h) {
    if (h->cfg.deposit_mode != 1) return fail(h, FS_EINVAL, "the adjoint needs deposit_mode 1");
    if (h->cfg.c_light != 0.0) return fail(h, FS_EINVAL, "the adjoint covers the non-relativistic push only");
    if (h->cfg.wall_model != 0) return fail(h, FS_EINVAL, "the adjoint covers the eq. (1) wall only");
    if (h->cfg.coupling != 1) return fail(h, FS_EINVAL, "the adjoint covers the first-order coupling only");
    if (h->cfg.smooth != 0) return fail(h, FS_EINVAL, "the adjoint covers the unfiltered moments only");
    return FS_OK;
}

int fs_step_record(fs_handle* h, fs_particles* sp, fs_fields* f, int64_t step, fs_record* rec,
                   const fs_packed* pack_in, fs_step_stats* st, hipStream_t s) {
    if (!h || !rec) return fail(h, FS_EINVAL, "NULL argument");
    if (h->cfg.deposit_mode != 1) return fail(h, FS_EINVAL, "a recorded step needs deposit_mode 1");
    if (h->cfg.c_light != 0.0 || h->cfg.coupling != 1)
        return fail(h, FS_EINVAL, "a recorded step covers the non-relativistic first-order step only");
    if (int rc = check_record(h, rec)) return rc;
    if (rec->stages && h->cfg.n_sub != 1) return fail(h, FS_EINVAL, "kept RK stages need n_sub = 1");
    if ((rec->B_in == nullptr) != (rec->gather_in == nullptr))
        return fail(h, FS_EINVAL, "B_in and gather_in go together");
    if (rec->fluid && h->cfg.smooth > 0) return fail(h, FS_EINVAL, "a kept fluid state needs the unfiltered moments");
    if (pack_in)
        if (int rc = check_packed(h, pack_in, nullptr, false)) return rc;
    rec->id0 = h->next_id;
    return step_common(h, sp, f, step, FS_ALL, st, s, rec, pack_in);
}

int fs_tape_pack(fs_handle* h, const fs_particles* sp, fs_packed* out, const fs_particles* prev_sp,
                 const fs_record* rec, fs_packed* prev, uint32_t flags, hipStream_t s) {
    if (!h || !sp || !out) return fail(h, FS_EINVAL, "NULL argument");
    if (flags & ~(uint32_t)FS_PACK_IONS) return fail(h, FS_EINVAL, "unknown pack flags");
    const bool with = prev_sp || rec || prev;
    if (with && !(prev_sp && rec && prev)) return fail(h, FS_EINVAL, "prev_sp, rec and prev go together");
    int rc = check_particles(h, sp);
    for (int k = 0; !rc && k < (h->has_cr ? 2 : 1); ++k)
        if (h->L.capacity[k] > (int64_t)INT32_MAX - 2)
            rc = fail(h, FS_ECAPACITY, "particle buffers too large for the int32 tile offsets");
    if (!rc) rc = check_packed(h, out, nullptr, false);
    if (!rc && with) rc = check_particles(h, prev_sp);
    if (!rc && with) rc = check_packed(h, prev, nullptr, true);
    if (!rc && with) rc = check_record(h, rec);
    if (rc) return rc;
    auto run = [&]() -> int {
        FS_DISPATCH_RD(h, (tape_pack_impl<R, D>(h, sp, out, prev_sp, rec, prev, (flags & FS_PACK_IONS) != 0, s)));
    };
    return run();
}

int fs_tape_unpack(fs_handle* h, const fs_packed* pk, fs_particles* sp, hipStream_t s) {
    if (!h || !pk || !sp) return fail(h, FS_EINVAL, "NULL argument");
    int rc = check_particles(h, sp);
    if (!rc) rc = check_packed(h, pk, nullptr, false);
    if (rc) return rc;
    auto run = [&]() -> int { FS_DISPATCH_RD(h, (tape_unpack_impl<R, D>(h, pk, sp, s))); };
    return run();
}

int fs_adjoint_step(fs_handle* h, const fs_packed* pn, const fs_fields* f_n, const fs_packed* pn1,
                    const fs_fields* f_n1, const double* stages, const double* fluid, int64_t id0, int64_t step,
                    fs_adjoint* lam, double* grads, hipStream_t s) {
    if (!h || !pn || !f_n || !pn1 || !f_n1 || !lam || !grads) return fail(h, FS_EINVAL, "NULL argument");
    if (int rc = check_reverse_cfg(h)) return rc;
    if (!f_n->B || !f_n->gather || !f_n1->B || !f_n1->mom[0] || (h->has_cr && !f_n1->mom[1]))
        return fail(h, FS_EINVAL, "NULL field array");
    if (step < 0 || id0 < 0) return fail(h, FS_EINVAL, "negative step or id");
    if (stages && h->cfg.n_sub != 1) return fail(h, FS_EINVAL, "kept RK stages need n_sub = 1");
    int rc = check_adjoint(h, lam);
    if (!rc) rc = check_packed(h, pn, lam, true);
    if (!rc) rc = check_packed(h, pn1, lam, false);
    if (rc) return rc;
    auto run = [&]() -> int {
        FS_DISPATCH(h, (adjoint_step_impl<R, D, S>(h, pn, f_n, pn1, f_n1, stages, fluid, id0, step, lam, grads, s)));
    };
    return run();
}

int fs_adjoint_park(fs_handle* h, const fs_packed* from, fs_adjoint* lam, void* scratch, int64_t nid, hipStream_t s) {
    if (!h || !from || !lam || !scratch) return fail(h, FS_EINVAL, "NULL argument");
    if (nid < 0) return fail(h, FS_EINVAL, "negative id range");
    int rc = check_adjoint(h, lam);
    if (!rc) rc = check_packed(h, from, lam, false);
    if (rc) return rc;
    auto run = [&]() -> int { FS_DISPATCH_RD(h, (park_impl<R, D>(h, from, lam, scratch, nullptr, nid, true, s))); };
    return run();
}

int fs_adjoint_unpark(fs_handle* h, const fs_packed* to, fs_adjoint* lam, const void* scratch, int64_t nid,
                      hipStream_t s) {
    if (!h || !to || !lam || !scratch) return fail(h, FS_EINVAL, "NULL argument");
    if (nid < 0) return fail(h, FS_EINVAL, "negative id range");
    int rc = check_adjoint(h, lam);
    if (!rc) rc = check_packed(h, to, lam, false);
    if (rc) return rc;
    auto run = [&]() -> int { FS_DISPATCH_RD(h, (park_impl<R, D>(h, to, lam, nullptr, scratch, nid, false, s))); };
    return run();
}

int fs_adjoint_init(fs_handle* h, const fs_packed* p0, const fs_fields* f0, fs_adjoint* lam, double* grads,
                    hipStream_t s) {
    if (!h || !p0 || !f0 || !lam || !grads) return fail(h, FS_EINVAL, "NULL argument");
    if (int rc = check_reverse_cfg(h)) return rc;
    if (!f0->B || !f0->mom[0] || (h->has_cr && !f0->mom[1])) return fail(h, FS_EINVAL, "NULL field array");
    int rc = check_adjoint(h, lam);
    if (!rc) rc = check_packed(h, p0, lam, false);
    if (rc) return rc;
    auto run = [&]() -> int { FS_DISPATCH(h, (adjoint_init_impl<R, D, S>(h, p0, f0, lam, grads, s))); };
    return run();
}

int fs_deposit_moments(fs_handle* h, const fs_particles* sp, fs_fields* f, hipStream_t s) {
    if (!h || !sp || !f) return fail(h, FS_EINVAL, "NULL argument");
    int rc = check_particles(h, sp);
    if (!rc) rc = check_fields(h, f);
    if (rc) return rc;
    auto run = [&]() -> int { FS_DISPATCH(h, (deposit_impl<R, D, S>(h, sp, f, s))); };
    return run();
}

int fs_field_update(fs_handle* h, fs_fields* f, hipStream_t s) {
    if (!h) return fail(h, FS_EINVAL, "NULL handle");
    int rc = check_fields(h, f);
    if (rc) return rc;
    if (h->cfg.precision == 32) field_update<float>(h, f, s, true);
    else field_update<double>(h, f, s, true);
    return hip_check(h, hipGetLastError(), "field update launch");
}

int fs_refresh_fields(fs_handle* h, fs_fields* f, hipStream_t s) {
    if (!h) return fail(h, FS_EINVAL, "NULL handle");
    int rc = check_fields(h, f);
    if (rc) return rc;
    if (h->cfg.precision == 32) field_update<float>(h, f, s, false);
    else field_update<double>(h, f, s, false);
    return hip_check(h, hipGetLastError(), "field refresh launch");
}

}  // extern "C"

namespace {
__global__ void k_wall_list(Geo G, WallModel wm, int policy, uint64_t step, int64_t n, const uint32_t* id,
                            const double* delta, double* v, int32_t* outcome, double* xi_new) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double vin[3] = {v[i], v[n + i], v[2 * n + i]}, vout[3], back = 0.0;
    int r = 0;
    if (policy == FS_WALL_FAUX_SHOCK)
        r = wm.on ? faux_shock_event_prescribed(wm, G.seed, step, id[i], G.c_light, delta[i], vin, vout, back)
                  : faux_shock_event(G.seed, step, id[i], G.u2, G.c_light, delta[i], vin, vout, back);
    else if (policy == FS_WALL_SPECULAR) {
        vout[0] = -vin[0]; vout[1] = vin[1]; vout[2] = vin[2];
        back = delta[i];
        r = 1;
    }
    outcome[i] = r;
    if (r) {
        v[i] = vout[0]; v[n + i] = vout[1]; v[2 * n + i] = vout[2];
        xi_new[i] = (double)G.nx - back;
    } else {
        xi_new[i] = 0.0;
    }
}
}  // namespace

extern "C" {

int fs_apply_faux_shock(fs_handle* h, int32_t species, int64_t step, int64_t n, const uint32_t* id, const double* delta,
                        double* v, int32_t* outcome, double* xi_new, hipStream_t s) {
    if (!h) return fail(h, FS_EINVAL, "NULL handle");
    if (species < 0 || species > 1 || n < 0) return fail(h, FS_EINVAL, "bad species or count");
    if (n == 0) return FS_OK;
    if (!id || !delta || !v || !outcome || !xi_new) return fail(h, FS_EINVAL, "NULL array");
    k_wall_list<<<grid_for(n), 256, 0, s>>>(h->G, wall_model_at(h, step), policy_of(h, species), (uint64_t)step, n, id,
                                            delta, v, outcome, xi_new);
    return hip_check(h, hipGetLastError(), "wall launch");
}

int fs_set_clock(fs_handle* h, int64_t next_id) {
    if (!h || next_id < 0) return fail(h, FS_EINVAL, "bad argument");
    h->next_id = next_id;
    return FS_OK;
}

int64_t fs_next_id(const fs_handle* h) { return h ? h->next_id : -1; }

int fs_timing_enable(fs_handle* h, int32_t on) {
    if (!h) return fail(h, FS_EINVAL, "NULL handle");
    if (on && h->ev_pool.empty()) {
        h->ev_pool.resize(kMaxTimed);
        h->ev_phase.assign(kMaxTimed / 2, 0);
        for (auto& e : h->ev_pool)
            if (hipEventCreate(&e) != hipSuccess) return fail(h, FS_EDEVICE, "event creation failed");
    }
    h->timing = on != 0;
    h->ev_used = 0;
    return FS_OK;
}

int fs_timing_read(fs_handle* h, double* ms5, int64_t* n5, hipStream_t s) {
    if (!h || !ms5 || !n5) return fail(h, FS_EINVAL, "bad argument");
    for (int i = 0; i < 5; ++i) { ms5[i] = 0.0; n5[i] = 0; }
    int rc = hip_check(h, hipStreamSynchronize(s), "stream synchronise");
    if (rc) return rc;
    for (size_t k = 0; k + 1 < h->ev_used; k += 2) {
        float ms = 0.f;
        rc = hip_check(h, hipEventElapsedTime(&ms, h->ev_pool[k], h->ev_pool[k + 1]), "event timing");
        if (rc) return rc;
        int ph = h->ev_phase[k / 2];
        ms5[ph] += ms;
        n5[ph] += 1;
    }
    h->ev_used = 0;
    return FS_OK;
}

}  // extern "C"

// --------------------------------------------------------------------------
// host-side state access
// --------------------------------------------------------------------------
namespace {

template <typename R, int D>
int load_impl(fs_handle* h, fs_particles* sp, int64_t n, const int64_t* cell3, const double* off3, const double* v3,
              const uint64_t* id, hipStream_t s) {
    fs_particles& P = *sp;
    const int64_t cap = P.tile_cap, ntiles = h->L.ntiles;
    std::vector<int32_t> counts(2 * ntiles, 0);
    std::vector<int64_t> slot(n);
    std::vector<int32_t> tile(n);
    const int* T = h->L.tile;
    for (int64_t i = 0; i < n; ++i) {
        int64_t x = cell3[3 * i], y = cell3[3 * i + 1], z = cell3[3 * i + 2];
        if (x < 0 || x >= h->cfg.nx || y < 0 || y >= h->L.nyc || z < 0 || z >= h->L.nzc)
            return fail(h, FS_EINVAL, "particle cell out of the box");
        for (int d = 0; d < 3; ++d)
            if (!(off3[3 * i + d] >= 0.0 && off3[3 * i + d] < 1.0)) return fail(h, FS_EINVAL, "offset outside [0, 1)");
        if (id[i] > UINT32_MAX) return fail(h, FS_EIDOVERFLOW, "id does not fit 32 bits");
        int t = (int)(x / T[0] + h->L.ntile[0] * (y / T[1] + (int64_t)h->L.ntile[1] * (z / T[2])));
        tile[i] = t;
        slot[i] = counts[t]++;
        if (counts[t] > cap) return fail(h, FS_ECAPACITY, "too many particles in one tile");
    }
    const int64_t C = P.capacity;
    std::vector<int32_t> hcell(C, 0);
    std::vector<uint32_t> hid(C, 0);
    std::vector<R> hoff[3], hv[3];
    for (int d = 0; d < D; ++d) hoff[d].assign(C, (R)0);
    for (int c = 0; c < 3; ++c) hv[c].assign(C, (R)0);
    const int bx = h->L.cell_bits[0], by = h->L.cell_bits[1];
    for (int64_t i = 0; i < n; ++i) {
        int64_t dst = (int64_t)tile[i] * cap + slot[i];
        hcell[dst] = (int32_t)(cell3[3 * i] | (cell3[3 * i + 1] << bx) | (cell3[3 * i + 2] << (bx + by)));
        for (int d = 0; d < D; ++d) {
            R o = (R)off3[3 * i + d];
            hoff[d][dst] = o >= (R)1 ? std::nextafter((R)1, (R)0) : o;
        }
        for (int c = 0; c < 3; ++c) hv[c][dst] = (R)v3[3 * i + c];
        hid[dst] = (uint32_t)id[i];
    }
    PBuf<R> b = sections<R>(P.buf[P.cur], C, D);
    hipError_t e = hipMemcpyAsync(b.cell, hcell.data(), C * 4, hipMemcpyHostToDevice, s);
    for (int d = 0; d < D && e == hipSuccess; ++d)
        e = hipMemcpyAsync(b.off[d], hoff[d].data(), C * sizeof(R), hipMemcpyHostToDevice, s);
    for (int c = 0; c < 3 && e == hipSuccess; ++c)
        e = hipMemcpyAsync(b.v[c], hv[c].data(), C * sizeof(R), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b.id, hid.data(), C * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(P.tile_count[P.cur], counts.data(), 2 * ntiles * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(P.count, &n, sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return hip_check(h, e, "particle upload");
}

template <typename R, int D>
int read_impl(fs_handle* h, const fs_particles* sp, int64_t* n_out, int64_t* cell3, double* off3, double* v3, uint64_t* id,
              hipStream_t s) {
    const fs_particles& P = *sp;
    const int64_t ntiles = h->L.ntiles;
    std::vector<int32_t> counts(2 * ntiles);
    hipError_t e = hipMemcpyAsync(counts.data(), P.tile_count[P.cur], 2 * ntiles * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_check(h, e, "count copy");
    std::vector<int64_t> offs(ntiles);
    int64_t tot = 0;
    for (int64_t t = 0; t < ntiles; ++t) {
        offs[t] = tot;
        tot += std::min<int64_t>((int64_t)counts[t] + counts[ntiles + t], P.tile_cap);
    }
    if (!cell3) { *n_out = tot; return FS_OK; }
    if (*n_out < tot) { *n_out = tot; return fail(h, FS_ECAPACITY, "host arrays too small"); }
    *n_out = tot;
    if (tot == 0) return FS_OK;
    char* dmem = nullptr;
    size_t bytes = ntiles * 8 + tot * (24 + 24 + 24 + 8) + 1024;
    e = hipMalloc(&dmem, bytes);
    if (e != hipSuccess) return hip_check(h, e, "readback scratch");
    int64_t* doffs = reinterpret_cast<int64_t*>(dmem);
    int64_t* dcell = reinterpret_cast<int64_t*>(dmem + round_up(ntiles * 8, 256));
    double* doff = reinterpret_cast<double*>(reinterpret_cast<char*>(dcell) + round_up(tot * 24, 256));
    double* dv = reinterpret_cast<double*>(reinterpret_cast<char*>(doff) + round_up(tot * 24, 256));
    uint64_t* did = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(dv) + round_up(tot * 24, 256));
    if (reinterpret_cast<char*>(did) + tot * 8 > dmem + bytes) {
        hipFree(dmem);
        bytes = round_up(ntiles * 8, 256) + 3 * round_up(tot * 24, 256) + round_up(tot * 8, 256);
        if (hipMalloc(&dmem, bytes) != hipSuccess) return fail(h, FS_EDEVICE, "readback scratch");
        doffs = reinterpret_cast<int64_t*>(dmem);
        dcell = reinterpret_cast<int64_t*>(dmem + round_up(ntiles * 8, 256));
        doff = reinterpret_cast<double*>(reinterpret_cast<char*>(dcell) + round_up(tot * 24, 256));
        dv = reinterpret_cast<double*>(reinterpret_cast<char*>(doff) + round_up(tot * 24, 256));
        did = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(dv) + round_up(tot * 24, 256));
    }
    e = hipMemcpyAsync(doffs, offs.data(), ntiles * 8, hipMemcpyHostToDevice, s);
    PBuf<R> b = sections<R>(P.buf[P.cur], P.capacity, D);
    if (e == hipSuccess) {
        k_compact<R, D><<<(unsigned)ntiles, 256, 0, s>>>(h->G, b, P.tile_count[P.cur], doffs, P.tile_cap, dcell, doff, dv, did);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(cell3, dcell, tot * 24, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(off3, doff, tot * 24, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(v3, dv, tot * 24, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(id, did, tot * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(dmem);
    return hip_check(h, e, "particle readback");
}


// ---------------------------------------------------------------------------
// checkpoints: header, then per species the per-tile offsets and the live
// ions packed tile after tile (particle-buffer section layout), then B
// ---------------------------------------------------------------------------
struct CkptHeader {
    char magic[8];
    int32_t version, precision, dim, nx, ny, nz, shape, nsp;
    int64_t ntiles, tile_cap[2], ncent;
    double c_light;
    uint64_t seed;
    int64_t next_id;
    int64_t n[2];
    int64_t off_toff[2], off_part[2], off_B, total;
};
constexpr char kCkptMagic[8] = {'F', 'S', 'C', 'K', 'P', 'T', '0', '1'};
constexpr int64_t kCkptHead = 256;
static_assert(sizeof(CkptHeader) <= kCkptHead, "checkpoint header must fit its slot");

int64_t part_block_bytes(int64_t n, int dim, int rb) {
    return round_up(n * 4, 256) + (int64_t)(dim + 3) * round_up(n * rb, 256) + round_up(n * 4, 256);
}

// Header and per-tile offsets of a checkpoint of the current state.
int ckpt_plan(fs_handle* h, const fs_particles* sp, CkptHeader& H, std::vector<int64_t> toff[2], hipStream_t s) {
    std::memset(&H, 0, sizeof(H));
    std::memcpy(H.magic, kCkptMagic, 8);
    const fs_config& c = h->cfg;
    H.version = 1; H.precision = c.precision; H.dim = c.dim; H.nx = c.nx;
    H.ny = (int32_t)h->L.nyc; H.nz = (int32_t)h->L.nzc; H.shape = c.shape;
    H.nsp = h->has_cr ? 2 : 1;
    H.ntiles = h->L.ntiles; H.tile_cap[0] = h->L.tile_cap[0]; H.tile_cap[1] = h->L.tile_cap[1];
    H.ncent = h->L.ncent; H.c_light = c.c_light; H.seed = c.seed; H.next_id = h->next_id;
    const int64_t nt = h->L.ntiles;
    const int rb = c.precision == 64 ? 8 : 4;
    int64_t off = kCkptHead;
    for (int k = 0; k < H.nsp; ++k) {
        std::vector<int32_t> cnt(2 * nt);
        hipError_t e = hipMemcpyAsync(cnt.data(), sp[k].tile_count[sp[k].cur], 2 * nt * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_check(h, e, "checkpoint counts");
        toff[k].assign(nt + 1, 0);
        for (int64_t t = 0; t < nt; ++t)
            toff[k][t + 1] = toff[k][t] + std::min<int64_t>((int64_t)cnt[t] + cnt[nt + t], sp[k].tile_cap);
        H.n[k] = toff[k][nt];
        H.off_toff[k] = off;
        off += round_up((nt + 1) * 8, 256);
        H.off_part[k] = off;
        off += part_block_bytes(H.n[k], c.dim, rb);
    }
    H.off_B = off;
    off += round_up(3 * h->L.ncent * 8, 256);
    H.total = off;
    return FS_OK;
}

template <typename R, int D>
int checkpoint_impl(fs_handle* h, const fs_particles* sp, const fs_fields* f, void* dst, int64_t cap_bytes,
                    hipStream_t s) {
    CkptHeader H;
    std::vector<int64_t> toff[2];
    if (int rc = ckpt_plan(h, sp, H, toff, s)) return rc;
    if (cap_bytes < H.total) return fail(h, FS_ECAPACITY, "checkpoint buffer smaller than fs_checkpoint_bytes");
    char* st = nullptr;
    if (hipMalloc((void**)&st, H.total) != hipSuccess) return fail(h, FS_EDEVICE, "checkpoint staging");
    hipError_t e = hipMemcpyAsync(st, &H, sizeof(H), hipMemcpyHostToDevice, s);
    for (int k = 0; k < H.nsp && e == hipSuccess; ++k) {
        const fs_particles& P = sp[k];
        int64_t* dtoff = reinterpret_cast<int64_t*>(st + H.off_toff[k]);
        e = hipMemcpyAsync(dtoff, toff[k].data(), toff[k].size() * 8, hipMemcpyHostToDevice, s);
        if (e != hipSuccess || H.n[k] == 0) continue;
        PBuf<R> in = sections<R>(P.buf[P.cur], P.capacity, D);
        PBuf<R> out = sections<R>(st + H.off_part[k], H.n[k], D);
        k_ckpt_pack<R, D><<<(unsigned)h->L.ntiles, 256, 0, s>>>(h->G, in, P.tile_count[P.cur], dtoff, P.tile_cap, out);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(st + H.off_B, f->B, 3 * h->L.ncent * 8, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dst, st, H.total, hipMemcpyDefault, s);
    hipError_t e2 = hipStreamSynchronize(s);
    hipFree(st);
    if (e == hipSuccess) e = e2;
    return hip_check(h, e, "checkpoint");
}

template <typename R, int D>
int restore_impl(fs_handle* h, fs_particles* sp, fs_fields* f, const void* src, int64_t bytes, hipStream_t s) {
    CkptHeader H;
    if (bytes < kCkptHead) return fail(h, FS_EINVAL, "checkpoint too short");
    hipError_t e = hipMemcpy(&H, src, sizeof(H), hipMemcpyDefault);
    if (e != hipSuccess) return hip_check(h, e, "checkpoint header");
    const fs_config& c = h->cfg;
    const int nsp = h->has_cr ? 2 : 1;
    if (std::memcmp(H.magic, kCkptMagic, 8) != 0 || H.version != 1) return fail(h, FS_EINVAL, "not a checkpoint");
    if (H.precision != c.precision || H.dim != c.dim || H.nx != c.nx || H.ny != (int32_t)h->L.nyc ||
        H.nz != (int32_t)h->L.nzc || H.shape != c.shape || H.nsp != nsp || H.ntiles != h->L.ntiles ||
        H.tile_cap[0] != h->L.tile_cap[0] || H.tile_cap[1] != h->L.tile_cap[1] || H.ncent != h->L.ncent ||
        H.c_light != c.c_light || H.seed != c.seed)
        return fail(h, FS_EINVAL, "checkpoint of a different configuration");
    if (H.total > bytes || H.next_id < 0 || H.next_id > (int64_t)UINT32_MAX + 1)
        return fail(h, FS_EINVAL, "checkpoint truncated or corrupt");
    // every offset and count is checked here, before a kernel reads the blob
    const int64_t nt = h->L.ntiles;
    const int rb = c.precision == 64 ? 8 : 4;
    std::vector<int64_t> toff[2];
    int64_t end = kCkptHead;
    for (int k = 0; k < nsp; ++k) {
        if (H.n[k] < 0 || H.off_toff[k] != end) return fail(h, FS_EINVAL, "checkpoint corrupt");
        end += round_up((nt + 1) * 8, 256);
        if (H.off_part[k] != end) return fail(h, FS_EINVAL, "checkpoint corrupt");
        end += part_block_bytes(H.n[k], c.dim, rb);
        if (end > H.total) return fail(h, FS_EINVAL, "checkpoint corrupt");
        toff[k].resize(nt + 1);
        e = hipMemcpy(toff[k].data(), static_cast<const char*>(src) + H.off_toff[k], (nt + 1) * 8, hipMemcpyDefault);
        if (e != hipSuccess) return hip_check(h, e, "checkpoint offsets");
        if (toff[k][0] != 0 || toff[k][nt] != H.n[k]) return fail(h, FS_EINVAL, "checkpoint corrupt");
        for (int64_t t = 0; t < nt; ++t)
            if (toff[k][t + 1] < toff[k][t] || toff[k][t + 1] - toff[k][t] > sp[k].tile_cap)
                return fail(h, FS_EINVAL, "checkpoint corrupt");
    }
    if (H.off_B != end || end + round_up(3 * h->L.ncent * 8, 256) != H.total)
        return fail(h, FS_EINVAL, "checkpoint corrupt");
    char* st = nullptr;
    if (hipMalloc((void**)&st, H.total) != hipSuccess) return fail(h, FS_EDEVICE, "restore staging");
    e = hipMemcpyAsync(st, src, H.total, hipMemcpyDefault, s);
    for (int k = 0; k < nsp && e == hipSuccess; ++k) {
        fs_particles& P = sp[k];
        PBuf<R> in = sections<R>(st + H.off_part[k], H.n[k], D);
        PBuf<R> out = sections<R>(P.buf[P.cur], P.capacity, D);
        k_ckpt_unpack<R, D><<<(unsigned)nt, 256, 0, s>>>(h->G, in, reinterpret_cast<const int64_t*>(st + H.off_toff[k]),
                                                         P.tile_cap, out, P.tile_count[P.cur]);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(P.count, &H.n[k], 8, hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(f->B, st + H.off_B, 3 * h->L.ncent * 8, hipMemcpyDeviceToDevice, s);
    hipError_t e2 = hipStreamSynchronize(s);
    hipFree(st);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return hip_check(h, e, "restore");
    h->next_id = H.next_id;
    return FS_OK;
}

// Scratch of the B_perp spectrum: 2 nx twiddles, then one partial sum per
// (line group, wavenumber) with up to 256 groups of (y, z) lines.
int spectrum_groups(const fs_handle* h) { return (int)std::min<int64_t>(h->L.nyc * h->L.nzc, 256); }
int64_t spectrum_scratch_doubles(const fs_handle* h) {
    const int nx = h->cfg.nx, nk = nx / 2 + 1;
    return 2 * (int64_t)nx + (int64_t)spectrum_groups(h) * nk;
}

// The spectrum's three kernels with their scratch at `scr`: every partial
// is written before it is read, so the scratch needs no clearing.
int spectrum_launch(fs_handle* h, const fs_fields* f, double* out, double* scr, hipStream_t s) {
    const int nx = h->cfg.nx, nk = nx / 2 + 1;
    const int64_t nlines = h->L.nyc * h->L.nzc;
    const int ngroups = spectrum_groups(h);
    double* tw = scr;
    double* part = scr + 2 * (int64_t)nx;
    k_twiddles<<<grid_for(nx), 256, 0, s>>>(nx, tw);
    k_bperp_dft<<<dim3((unsigned)((nk + 255) / 256), (unsigned)ngroups), 256, 0, s>>>(h->F, f->B, h->L.ncent, tw, nk,
                                                                                      ngroups, part);
    k_bperp_reduce<<<grid_for(nk), 256, 0, s>>>(nk, ngroups, 1.0 / ((double)nlines * (double)nx * (double)nx), part,
                                                out);
    return hip_check(h, hipGetLastError(), "spectrum launch");
}

template <typename R> int diag_impl(fs_handle* h, const fs_particles* sp, const fs_fields* f, double* out, double* prof,
                                    hipStream_t s) {
    const long nc = h->L.ncent;
    const unsigned gb = grid_for(nc);
    k_diag_field<<<gb, 256, 0, s>>>(h->F, f->B, nc, h->part);
    std::vector<double> part(4 * (size_t)gb);
    hipError_t e = hipMemcpyAsync(part.data(), h->part, part.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_check(h, e, "diagnostics");
    double b2 = 0, bp = 0, loss = 0, dv = 0;
    for (unsigned i = 0; i < gb; ++i) {
        b2 += part[4 * i]; bp += part[4 * i + 1]; loss += part[4 * i + 2]; dv = std::max(dv, part[4 * i + 3]);
    }
    const double dV = std::pow(h->cfg.dx, (double)h->cfg.dim);
    out[0] = 0.5 * b2 * dV;
    const int nsp = h->has_cr ? 2 : 1;
    for (int k = 0; k < 2; ++k) {
        out[1 + k] = 0.0;
        out[3 + k] = 0.0;
        if (k >= nsp) continue;
        const fs_particles& P = sp[k];
        PBuf<R> b = sections<R>(P.buf[P.cur], P.capacity, h->cfg.dim);
        k_diag_kin<R><<<(unsigned)h->L.ntiles, 256, 0, s>>>(b, P.tile_count[P.cur], (int)h->L.ntiles, P.tile_cap,
                                                            h->G.ic2, h->part);
        std::vector<double> kp(h->L.ntiles);
        int64_t cnt = 0;
        e = hipMemcpyAsync(kp.data(), h->part, kp.size() * 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&cnt, P.count, 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_check(h, e, "diagnostics");
        double ke = 0;
        for (double x : kp) ke += x;
        const double w = k == 0 ? h->F.wth : h->F.wcr;
        out[1 + k] = w * ke * dV;
        out[3 + k] = (double)cnt;
    }
    out[5] = loss;
    out[6] = dv;
    out[7] = bp;
    if (prof) {
        k_profile<<<grid_for(h->cfg.nx), 256, 0, s>>>(h->F, f->B, nc, prof);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_check(h, e, "profile");
    }
    return FS_OK;
}

}  // namespace

extern "C" {

int fs_load_particles(fs_handle* h, fs_particles* sp, int64_t n, const int64_t* cell3, const double* off3,
                      const double* v3, const uint64_t* id, hipStream_t s) {
    if (!h || !sp || n < 0) return fail(h, FS_EINVAL, "bad argument");
    if (n > 0 && (!cell3 || !off3 || !v3 || !id)) return fail(h, FS_EINVAL, "NULL array");
    if (sp->species == 1 && !h->has_cr) return fail(h, FS_EINVAL, "run has no CR species");
    const fs_particles& P = *sp;
    if (!P.buf[0] || !P.tile_count[0] || !P.count) return fail(h, FS_EINVAL, "NULL particle buffer");
    if (P.tile_cap != h->L.tile_cap[sp->species] || P.capacity < h->L.capacity[sp->species])
        return fail(h, FS_ECAPACITY, "particle buffer smaller than fs_layout reports");
    FS_DISPATCH_RD(h, (load_impl<R, D>(h, sp, n, cell3, off3, v3, id, s)));
}

int fs_read_particles(fs_handle* h, const fs_particles* sp, int64_t* n, int64_t* cell3, double* off3, double* v3,
                      uint64_t* id, hipStream_t s) {
    if (!h || !sp || !n) return fail(h, FS_EINVAL, "bad argument");
    if (cell3 && (!off3 || !v3 || !id)) return fail(h, FS_EINVAL, "NULL array");
    FS_DISPATCH_RD(h, (read_impl<R, D>(h, sp, n, cell3, off3, v3, id, s)));
}

int fs_checkpoint_bytes(fs_handle* h, const fs_particles* sp, int64_t* bytes, hipStream_t s) {
    if (!h || !sp || !bytes) return fail(h, FS_EINVAL, "NULL argument");
    if (h->cfg.coupling == 2) return fail(h, FS_EINVAL, "checkpoints do not carry the time-centred coupling's previous moments");
    if (int rc = check_particles(h, sp)) return rc;
    CkptHeader H;
    std::vector<int64_t> toff[2];
    if (int rc = ckpt_plan(h, sp, H, toff, s)) return rc;
    *bytes = H.total;
    return FS_OK;
}

int fs_checkpoint(fs_handle* h, const fs_particles* sp, const fs_fields* f, void* dst, int64_t cap_bytes,
                  hipStream_t s) {
    if (!h || !sp || !f || !dst) return fail(h, FS_EINVAL, "NULL argument");
    if (h->cfg.coupling == 2) return fail(h, FS_EINVAL, "checkpoints do not carry the time-centred coupling's previous moments");
    if (int rc = check_particles(h, sp)) return rc;
    if (int rc = check_fields(h, f)) return rc;
    FS_DISPATCH_RD(h, (checkpoint_impl<R, D>(h, sp, f, dst, cap_bytes, s)));
}

int fs_restore(fs_handle* h, fs_particles* sp, fs_fields* f, const void* src, int64_t bytes, hipStream_t s) {
    if (!h || !sp || !f || !src) return fail(h, FS_EINVAL, "NULL argument");
    if (h->cfg.coupling == 2) return fail(h, FS_EINVAL, "checkpoints do not carry the time-centred coupling's previous moments");
    if (int rc = check_particles(h, sp)) return rc;
    if (int rc = check_fields(h, f)) return rc;
    auto load = [&]() -> int { FS_DISPATCH_RD(h, (restore_impl<R, D>(h, sp, f, src, bytes, s))); };
    if (int rc = load()) return rc;
    if (int rc = fs_deposit_moments(h, sp, f, s)) return rc;
    return fs_refresh_fields(h, f, s);
}

int fs_phase_space(fs_handle* h, const fs_particles* sp, int32_t species, int32_t component,
                   int32_t x_cells_per_bin, int32_t nb, const double* edges, int64_t* counts, hipStream_t s) {
    if (!h || !sp || !edges || !counts) return fail(h, FS_EINVAL, "NULL argument");
    if (species < 0 || species > (h->has_cr ? 1 : 0)) return fail(h, FS_EINVAL, "no such species");
    if (component < -1 || component > 2) return fail(h, FS_EINVAL, "component must be -1, 0, 1 or 2");
    if (x_cells_per_bin < 1 || nb < 1 || nb > (1 << 24)) return fail(h, FS_EINVAL, "bad bin counts");
    if (int rc = check_particles(h, sp)) return rc;
    const fs_particles& P = sp[species];
    const int64_t nxb = (h->cfg.nx + x_cells_per_bin - 1) / x_cells_per_bin;
    zero_u64(counts, nxb * nb, s);
    auto run = [&](auto tag) {
        using R = decltype(tag);
        PBuf<R> b = sections<R>(P.buf[P.cur], P.capacity, h->cfg.dim);
        k_phase_space<R><<<(unsigned)h->L.ntiles, 256, 0, s>>>(h->G, b, P.tile_count[P.cur], (int)h->L.ntiles,
                                                              P.tile_cap, component, x_cells_per_bin, (int)nxb, nb,
                                                              edges,
                                                              reinterpret_cast<unsigned long long*>(counts));
    };
    if (h->cfg.precision == 32) run(float());
    else run(double());
    return hip_check(h, hipGetLastError(), "phase space launch");
}

int fs_bperp_spectrum(fs_handle* h, const fs_fields* f, double* out, hipStream_t s) {
    if (!h || !f || !f->B || !out) return fail(h, FS_EINVAL, "NULL argument");
    const int64_t need = spectrum_scratch_doubles(h);
    if (h->nspec < need) {
        hipFree(h->spec);
        h->spec = nullptr;
        h->nspec = 0;
        if (hipMalloc((void**)&h->spec, need * sizeof(double)) != hipSuccess) return fail(h, FS_EDEVICE, "spectrum scratch");
        h->nspec = need;
    }
    return spectrum_launch(h, f, out, h->spec, s);
}

int fs_bperp_spectrum_noalloc(fs_handle* h, const fs_fields* f, double* out, hipStream_t s) {
    if (!h || !f || !f->B || !out) return fail(h, FS_EINVAL, "NULL argument");
    const int64_t need = spectrum_scratch_doubles(h);
    if (need > kStaticScratchDoubles)
        return fail(h, FS_EINVAL, "box too large for the allocation-free spectrum: it needs " + std::to_string(need) +
                                      " doubles of scratch, the static array holds " +
                                      std::to_string(kStaticScratchDoubles));
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_check(h, e, "current device");
    if (dev != h->device || !h->static_scratch)
        return fail(h, FS_EINVAL, "the handle was created on device " + std::to_string(h->device) +
                                      ", the current device is " + std::to_string(dev));
    return spectrum_launch(h, f, out, h->static_scratch, s);
}

int fs_precursor_loss(fs_handle* h, const fs_fields* f, double* loss, hipStream_t s) {
    if (!h || !f || !f->B || !loss) return fail(h, FS_EINVAL, "NULL argument");
    const long nc = h->L.ncent;
    const int64_t total = (int64_t)(h->cfg.nx - h->cfg.nx / 2) * (nc / h->cfg.nx);
    const unsigned g = std::min<unsigned>(grid_for(total), (unsigned)std::min<int64_t>(kLossParts, h->npart));
    k_loss_part<<<g, 256, 0, s>>>(h->F, f->B, nc, h->part);
    k_loss_final<<<1, 256, 0, s>>>(h->part, (int)g, loss);
    return hip_check(h, hipGetLastError(), "loss launch");
}

int fs_adjoint_seed(fs_handle* h, const fs_fields* f, fs_adjoint* lam, double* grads, hipStream_t s) {
    if (!h || !f || !f->B || !grads) return fail(h, FS_EINVAL, "NULL argument");
    int rc = check_adjoint(h, lam);
    if (rc) return rc;
    const int rb = h->cfg.precision == 64 ? 8 : 4;
    for (int k = 0; k < (h->has_cr ? 2 : 1); ++k)
        for (int d = 0; d < 3; ++d) {
            void* arr[2] = {d < h->cfg.dim ? lam->x[k][lam->cur][d] : nullptr, lam->v[k][lam->cur][d]};
            for (void* a : arr) {
                if (!a) continue;
                if (rb == 8) zero_u64(a, lam->capacity[k], s);
                else zero_i32(static_cast<int32_t*>(a), lam->capacity[k], s);
            }
        }
    zero_u64(lam->lE, 6 * h->L.nnode, s);
    zero_u64(grads, 2 + (int64_t)h->cfg.n_modes, s);
    k_loss_seed<<<grid_for(h->L.ncent), 256, 0, s>>>(h->F, f->B, h->L.ncent, lam->lB);
    return hip_check(h, hipGetLastError(), "adjoint seed launch");
}

int fs_diagnostics(fs_handle* h, const fs_particles* sp, const fs_fields* f, double* out8, double* prof, hipStream_t s) {
    if (!h || !sp || !f || !out8) return fail(h, FS_EINVAL, "bad argument");
    if (h->cfg.precision == 32) return diag_impl<float>(h, sp, f, out8, prof, s);
    return diag_impl<double>(h, sp, f, out8, prof, s);
}

}  // extern "C"
