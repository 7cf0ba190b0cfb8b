// C ABI of the double-MRT lattice Boltzmann phase-change solver: argument
// checking, the dimensionless-to-lattice parameter mapping (Sec. 4.3 of
// Liu & He, arXiv:1503.08406), device memory, launches, checkpoints.
#include "../../include/dmrt.h"
#include "dmrt_device.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using dmrtk::Geom;
using dmrtk::Phys;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(e_ == hipErrorOutOfMemory ? DMRT_ENOMEM : DMRT_EDEVICE, "%s: %s",  \
                        #expr, hipGetErrorString(e_));                                      \
    } while (0)

constexpr uint64_t kMagic = 0x324d52544d444d44ull;  // checkpoint tag (layout 2: ten f planes)

bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

}  // namespace

// Device scratch of dmrt_diag_noalloc: the block partials of the diagnostics
// (at most 65536 blocks of 8 doubles, 4 MiB), the row fronts and the ten
// reduced results (64 KiB).  Each device the library runs on holds one copy
// until the process ends; every call on that device shares it.
constexpr size_t kScratchBytes = (size_t(4) << 20) + (size_t(64) << 10);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, found once per device
// with that device current (the array's name is a host-side stand-in and
// must not be passed to kernels).
int scratch_setup(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(DMRT_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return DMRT_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(DMRT_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
    return DMRT_OK;
}

void* scratch_of(int dev)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
}

}  // namespace

struct dmrt {
    int dev = 0;
    hipStream_t stream = nullptr;
    Geom G{};
    Phys P{};
    dmrt_derived D{};
    double Ste = 1;
    bool flow = false;
    int cur = 0;  // buffer index holding the current state
    int64_t t = 0;
    int check_every = 0, graph_steps = 0;
    char* base = nullptr;
    float *f[2]{}, *g[2]{}, *fl[2]{};
    float* u[2]{};  // u_x plane then u_y plane of the state in buffer parity 0 / 1
    float *eps = nullptr, *Ac = nullptr, *Bc = nullptr;
    char* work = nullptr;  // device work space of the field, population and diagnostics copies
    size_t work_bytes = 0;
    int *it_sum = nullptr, *it_max = nullptr;
    hipGraphExec_t graph[2]{};
    int graph_flip[2]{};  // buffer parity changes of a replay of graph[p]
    bool two_step = false;  // steps run two per launch (k_step2) where possible
    double ergun_c = 175.0;
    bool feps_given = false;
    // recorded run for the adjoint: checkpoints every rec_S steps, the ring
    // of states of one segment, the adjoint buffers
    int64_t rec_n = 0, rec_S = 0, rec_cap = 0;  // rec_cap: n the buffers are sized for
    char* rec_base = nullptr;
    float *ckpt = nullptr, *ring = nullptr, *ls = nullptr, *la = nullptr, *ga = nullptr;
    float* flnext = nullptr;  // f_l of the state after a segment's end
    float* stage = nullptr;   // two packed nx*ny planes: terminal adjoints in, gradients out
    hipGraphExec_t adj_graph = nullptr;  // the reversed pass for rec_cap steps
    bool adj_flow = false;
    int record_mode = 0;
    bool rec_all = false;  // every state of the recorded run kept (no recomputation)
    int rec_flip = 0;      // buffer parity change of a recorded run (checkpoint mode)
    hipGraphExec_t rec_graph[2]{};  // the recording's launches from buffer parity 0 / 1
    bool rec_graph_flow = false;
    // latent source at the pre-stream site: T*, two f_l iterates, sweep flags
    bool r2 = false;
    char* r2_base = nullptr;
    dmrtk::R2Bufs R{};
};

// Tiling constants for tiles of w x h nodes (see dmrt_internal.h).
namespace dmrtk {
void set_tiling(Geom& G, int w, int h)
{
    G.st_tx = (G.nx + w - 1) / w;
    G.st_ntiles = G.st_tx * ((G.ny + h - 1) / h);
    G.st_per_xcd = (G.st_ntiles + NXCD - 1) / NXCD;
    G.st_rot = G.st_tx % 8 == 0 ? 1 : 0;
    const uint32_t d = (uint32_t)G.st_tx;
    if (d == 1) {
        G.st_magic = 0;
        G.st_shift = 0;
    } else {
        int l = 0;
        while ((1ull << l) < d) ++l;
        G.st_magic = (uint32_t)(((((uint64_t)1 << l) - d) << 32) / d + 1);
        G.st_shift = l;
    }
}
}  // namespace dmrtk

namespace {

int derive_impl(const dmrt_grid* grid, double Ra, double Da, double Pr, double Ste,
                const dmrt_opts& o, dmrt_derived* d)
{
    if (!grid || !d) return fail(DMRT_EINVAL, "null argument");
    if (grid->nx <= 0 || grid->ny <= 0) return fail(DMRT_EINVAL, "grid must be at least 1x1");
    if (!(Ra >= 0) || !std::isfinite(Ra)) return fail(DMRT_EINVAL, "Ra must be >= 0");
    if (!finite_pos(Pr) || !finite_pos(Ste)) return fail(DMRT_EINVAL, "Pr and Ste must be > 0");
    if (!(Da > 0)) return fail(DMRT_EINVAL, "Da must be > 0");
    if (!finite_pos(o.J) || !finite_pos(o.lambda) || !finite_pos(o.alpha_ratio) ||
        !finite_pos(o.sigma_s) || !finite_pos(o.sigma_l))
        return fail(DMRT_EINVAL, "J, lambda, alpha_ratio, sigma_s, sigma_l must be > 0");
    if (!(o.varpi > -4 && o.varpi < 1)) return fail(DMRT_EINVAL, "varpi must lie in (-4, 1)");
    d->H = grid->H > 0 ? grid->H : (double)grid->ny;
    d->csT2 = (4.0 + o.varpi) / 10.0;
    if (Ra > 0) {
        if (!finite_pos(o.Ma)) return fail(DMRT_EINVAL, "Ma must be > 0");
        // tau_nu from Ra, Pr, Ma and H; u_c = Ma c_s = sqrt(g beta DT H)
        d->tau_nu = 0.5 + o.Ma * o.J * d->H * std::sqrt(3.0 * Pr) / std::sqrt(Ra);
        d->nu_e = (d->tau_nu - 0.5) / 3.0;
        d->nu_l = d->nu_e / o.J;
        d->alpha_l = d->nu_l / Pr;
        d->gbeta = o.Ma * o.Ma / (3.0 * d->H);
    } else {
        if (!finite_pos(o.alpha_l)) return fail(DMRT_EINVAL, "alpha_l must be > 0 when Ra == 0");
        d->alpha_l = o.alpha_l;
        d->nu_l = Pr * o.alpha_l;
        d->nu_e = o.J * d->nu_l;
        d->tau_nu = 0.5 + 3.0 * d->nu_e;
        d->gbeta = 0.0;
    }
    d->alpha_s = d->alpha_l / o.alpha_ratio;
    d->K_default = Da * d->H * d->H;
    d->tau_T_liquid = 0.5 + o.lambda * d->alpha_l / (o.sigma_l * d->csT2);
    d->tau_T_solid = 0.5 + o.lambda * d->alpha_s / (o.sigma_s * d->csT2);
    if (!(d->tau_nu > 0.5) || !std::isfinite(d->tau_nu))
        return fail(DMRT_EINVAL, "tau_nu = %g is not above 1/2", d->tau_nu);
    if (!(d->tau_T_liquid > 0.5) || !(d->tau_T_solid > 0.5))
        return fail(DMRT_EINVAL, "tau_T is not above 1/2");
    return DMRT_OK;
}

int check_opts(const dmrt_opts& o)
{
    if (!(o.T_l > o.T_s)) return fail(DMRT_EINVAL, "T_l must exceed T_s");
    if (!(o.fl_tol >= 0) || o.fl_maxit < 1) return fail(DMRT_EINVAL, "bad enthalpy iteration limits");
    const double r[] = {o.s_e, o.s_eps, o.s_q, o.zeta_e, o.zeta_nu};
    for (double v : r)
        if (!(v > 0 && v < 2)) return fail(DMRT_EINVAL, "relaxation rates must lie in (0, 2)");
    if (!finite_pos(o.ergun_c)) return fail(DMRT_EINVAL, "ergun_c must be > 0");
    if (o.check_every < 0 || o.graph_steps < 0 || (o.graph_steps & 1))
        return fail(DMRT_EINVAL, "check_every must be >= 0 and graph_steps even and >= 0");
    if (o.block_rows != 0 && o.block_rows != 4 && o.block_rows != 8)
        return fail(DMRT_EINVAL, "block_rows must be 0, 4 or 8");
    if (o.cells_per_lane < 0 || o.cells_per_lane > 2)
        return fail(DMRT_EINVAL, "cells_per_lane must be 0, 1 or 2");
    if (o.sigma_mode < 0 || o.sigma_mode > 1 || o.ke_mode < 0 || o.ke_mode > 1 ||
        o.latent_mode < 0 || o.latent_mode > 1)
        return fail(DMRT_EINVAL, "sigma_mode, ke_mode and latent_mode must be 0 or 1");
    if (o.store_hint < 0 || o.store_hint > 3)
        return fail(DMRT_EINVAL, "store_hint must be 0, 1, 2 or 3");
    if (o.record_mode < 0 || o.record_mode > 2)
        return fail(DMRT_EINVAL, "record_mode must be 0, 1 or 2");
    if (o.steps_per_launch < 0 || o.steps_per_launch > 2)
        return fail(DMRT_EINVAL, "steps_per_launch must be 0, 1 or 2");
    if (o.addressing < 0 || o.addressing > 1) return fail(DMRT_EINVAL, "addressing must be 0 or 1");
    if (!finite_pos(o.cps_ratio) || !finite_pos(o.cm_ratio) || !finite_pos(o.ks_ratio) ||
        !finite_pos(o.km_ratio))
        return fail(DMRT_EINVAL, "cps_ratio, cm_ratio, ks_ratio, km_ratio must be > 0");
    return DMRT_OK;
}

int check_bc(const dmrt_bc* bc)
{
    if (!bc) return fail(DMRT_EINVAL, "null boundary spec");
    for (int k = 0; k < 4; ++k)
        if (bc->kind[k] < DMRT_PERIODIC || bc->kind[k] > DMRT_WALL_ADIABATIC)
            return fail(DMRT_EINVAL, "unknown boundary kind on side %d", k);
    if ((bc->kind[0] == DMRT_PERIODIC) != (bc->kind[1] == DMRT_PERIODIC) ||
        (bc->kind[2] == DMRT_PERIODIC) != (bc->kind[3] == DMRT_PERIODIC))
        return fail(DMRT_EINVAL, "periodic sides must come in pairs");
    return DMRT_OK;
}

void fill_phys(Phys& P, const dmrt_derived& d, double Ste, const dmrt_opts& o)
{
    P.s_e = (float)o.s_e;
    P.s_eps = (float)o.s_eps;
    P.s_q = (float)o.s_q;
    P.s_nu = (float)(1.0 / d.tau_nu);
    P.zeta_e = (float)o.zeta_e;
    P.zeta_nu = (float)o.zeta_nu;
    P.w5_0 = (float)((1.0 - o.varpi) / 5.0);
    P.w5_1 = (float)((4.0 + o.varpi) / 20.0);
    P.varpi = (float)o.varpi;
    P.csT2 = (float)d.csT2;
    P.inv_csT2 = (float)(1.0 / d.csT2);
    P.sig_s = (float)o.sigma_s;
    P.dsig = (float)(o.sigma_l - o.sigma_s);
    P.isig_s = (float)(1.0 / o.sigma_s);
    P.lam_as = (float)(o.lambda * d.alpha_s);
    P.dlam = (float)(o.lambda * (d.alpha_l - d.alpha_s));
    P.T_s = (float)o.T_s;
    P.inv_St = (float)(1.0 / Ste);
    P.inv_den = (float)(1.0 / (o.T_l - o.T_s + 1.0 / Ste));
    P.inv_dTm = (float)(1.0 / (o.T_l - o.T_s));
    P.gbeta = (float)d.gbeta;
    P.T0 = (float)o.T0;
    P.fl_tol = (float)o.fl_tol;
    P.fl_maxit = o.fl_maxit;
    P.conv = o.convective ? 1.0f : 0.0f;
    P.zeta_uniform =
        (o.alpha_ratio == 1.0 && o.sigma_s == o.sigma_l && !o.sigma_mode && !o.ke_mode) ? 1 : 0;
    P.zeta_a = (float)(1.0 / d.tau_T_liquid);
    P.T_init = (float)o.T_init;
    P.sig_mode = o.sigma_mode;
    P.cps = (float)o.cps_ratio;
    P.cm = (float)o.cm_ratio;
    P.Es = (float)(o.cps_ratio * o.T_s);
    P.inv_den_c = (float)(1.0 / (o.T_l + 1.0 / Ste - o.cps_ratio * o.T_s));
    P.ke_mode = o.ke_mode;
    P.ks = (float)o.ks_ratio;
    P.km = (float)o.km_ratio;
    P.alpha_l = (float)d.alpha_l;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Cache policy of the state stores for a state of `bytes` (both buffers):
// write-through the die's L2 while the state fits the 256 MB Infinity Cache
// with room to spare (the next step reads it back from there), streaming
// stores beyond.
int store_policy(int hint, size_t bytes)
{
    if (hint == 1) return dmrtk::ST_PLAIN;
    if (hint == 2) return dmrtk::ST_WT;
    if (hint == 3) return dmrtk::ST_NT;
    return bytes <= (size_t)192 << 20 ? dmrtk::ST_WT : dmrtk::ST_NT;
}

void set_step_tiling(Geom& G);

// Lattice geometry, boundary description and launch shape of one lattice.
void fill_geom(Geom& G, int nx, int ny, const dmrt_bc& bc, const dmrt_opts& o)
{
    G.nx = nx;
    G.ny = ny;
    G.pitch = (nx + 63) / 64 * 64;
    G.plane = (long long)ny * G.pitch;
    G.per_x = bc.kind[0] == DMRT_PERIODIC;
    G.per_y = bc.kind[2] == DMRT_PERIODIC;
    for (int k = 0; k < 4; ++k) {
        G.wall_T[k] = bc.kind[k] == DMRT_WALL_T;
        G.T_wall[k] = (float)bc.T_wall[k];
    }
    G.block_rows = o.block_rows ? o.block_rows : 4;
    G.store = store_policy(o.store_hint, (size_t)G.plane * 4 * (2 * dmrtk::FQ + 2 * 5 + 2 + 4 + 3));
    // the thermal-model variants run one node per lane
    const bool variant = o.sigma_mode || o.ke_mode || o.latent_mode;
    G.cells_per_lane = (o.cells_per_lane && !variant) ? o.cells_per_lane : 1;
    // 32-bit buffer addressing while the largest array (9 planes) fits 4 GB
    G.wide = (uint64_t)G.plane * 4 * dmrtk::FQ >= (1ull << 32) ? 1 : 0;
    G.per_array = o.addressing == 1;
    set_step_tiling(G);
}

// Tiling constants of the step kernel, including the magic number that
// divides a tile index by the tiles per row (Granlund & Montgomery, unsigned
// 32-bit "add" form: l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1).
void set_step_tiling(Geom& G)
{
    dmrtk::set_tiling(G, dmrtk::TX, G.block_rows * G.cells_per_lane);
}

int copy_in(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, s));
    HIPCHK(hipStreamSynchronize(s));
    return DMRT_OK;
}

dmrtk::StepBufs bufs(dmrt* h, bool counted)
{
    dmrtk::StepBufs B;
    const int a = h->cur, b = 1 - h->cur;
    B.fin = h->f[a];
    B.fout = h->f[b];
    B.gin = h->g[a];
    B.gout = h->g[b];
    B.flin = h->fl[a];
    B.flout = h->fl[b];
    B.ux = h->u[b];
    B.uy = h->u[b] + h->G.plane;
    B.uin = h->u[a];
    B.eps = h->eps;
    B.Ac = h->Ac;
    B.Bc = h->Bc;
    B.it_sum = counted ? h->it_sum : nullptr;
    B.it_max = counted ? h->it_max : nullptr;
    B.r2f = nullptr;
    B.r2_its = 0;
    return B;
}

int ensure_work(dmrt* h, size_t bytes)
{
    if (h->work_bytes >= bytes) return DMRT_OK;
    if (h->work) HIPCHK(hipFree(h->work));
    h->work = nullptr;
    h->work_bytes = 0;
    HIPCHK(hipMalloc(&h->work, bytes));
    h->work_bytes = bytes;
    return DMRT_OK;
}

// The launches of one step from buffer parity h->cur.
hipError_t enqueue_step(dmrt* h, bool counted)
{
    if (h->r2) return dmrtk::launch_step_r2(h->G, h->P, bufs(h, counted), h->R, h->flow, counted, h->stream);
    return dmrtk::launch_step(h->G, h->P, bufs(h, counted), h->flow, counted, h->stream);
}

// Two steps in one launch (k_step2) from buffer parity h->cur into the other.
bool use_two_step(const dmrt* h) { return h->two_step && !h->r2; }

hipError_t enqueue_step2(dmrt* h)
{
    return dmrtk::launch_step2(h->G, h->P, bufs(h, false), h->flow, h->stream);
}

// One plain step; flips the buffer index.
int step_once(dmrt* h, bool counted)
{
    HIPCHK(enqueue_step(h, counted));
    h->cur = 1 - h->cur;
    h->t += 1;
    return DMRT_OK;
}

// Capture graph_steps launches starting from buffer parity p.
int build_graph(dmrt* h, int p)
{
    const int save = h->cur;
    const int64_t tsave = h->t;
    h->cur = p;
    HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    const bool two = use_two_step(h);
    const int launches = two ? h->graph_steps / 2 : h->graph_steps;
    for (int k = 0; k < launches; ++k) {
        hipError_t e = two ? enqueue_step2(h) : enqueue_step(h, false);
        h->cur = 1 - h->cur;
        if (e != hipSuccess) {
            hipGraph_t gdrop = nullptr;
            (void)hipStreamEndCapture(h->stream, &gdrop);
            if (gdrop) (void)hipGraphDestroy(gdrop);
            h->cur = save;
            return fail(DMRT_EDEVICE, "launch during capture: %s", hipGetErrorString(e));
        }
    }
    h->cur = save;
    h->t = tsave;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(h->stream, &graph);
    if (e != hipSuccess) return fail(DMRT_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&h->graph[p], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        h->graph[p] = nullptr;
        return fail(DMRT_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    h->graph_flip[p] = launches & 1;
    return DMRT_OK;
}

int diag_impl(dmrt* h, dmrt_diag_t* out)
{
    const Geom& G = h->G;
    const int nblk = dmrtk::tile_blocks(G, dmrtk::TY);
    const size_t pbytes = align256((size_t)nblk * dmrtk::DIAG_SLOTS * sizeof(double));
    const size_t fbytes = (size_t)G.ny * sizeof(float);
    int rc = ensure_work(h, pbytes + align256(fbytes));
    if (rc) return rc;
    double* part = (double*)h->work;
    float* front = (float*)(h->work + pbytes);
    int nb = 0;
    const int a = h->cur;
    HIPCHK(dmrtk::launch_diag(G, h->P, h->f[a], h->g[a], h->fl[a], h->u[a], h->u[a] + G.plane, h->eps, h->flow,
                             part, &nb, h->stream));
    HIPCHK(dmrtk::launch_front(G, h->fl[a], front, h->stream));
    std::vector<double> hp((size_t)nb * dmrtk::DIAG_SLOTS);
    std::vector<float> hf(G.ny);
    HIPCHK(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipMemcpyAsync(hf.data(), front, fbytes, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    double s[dmrtk::DIAG_SLOTS] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < dmrtk::DIAG_SLOTS; ++k) {
            const double v = hp[(size_t)b * dmrtk::DIAG_SLOTS + k];
            s[k] = (k == 4) ? std::fmax(s[k], v) : s[k] + v;
        }
    double fm = 0, fx = 0;
    for (int r = 0; r < G.ny; ++r) {
        fm += hf[r];
        fx = std::fmax(fx, (double)hf[r]);
    }
    out->mass = s[0];
    out->enthalpy = s[1];
    out->liquid = s[2];
    out->T_sum = s[3];
    out->u_max = s[4];
    out->active = (int64_t)llround(s[5]);
    out->nonfinite = (int64_t)llround(s[6]);
    out->front_mean = fm / G.ny;
    out->front_max = fx;
    out->step = h->t;
    return DMRT_OK;
}

// Porosity and drag-coefficient planes (pitched) from the caller's per-cell
// eps, K, Feps (K NULL: Da H^2; Feps NULL: the Ergun relation of Eq. 6).
int porous_planes(dmrt* h, const float* eps, const float* K, const float* Feps,
                  std::vector<float>& pe, std::vector<float>& pa, std::vector<float>& pb)
{
    const Geom& G = h->G;
    const size_t nx = (size_t)G.nx, ny = (size_t)G.ny, pitch = (size_t)G.pitch;
    const size_t ncell = nx * ny;
    std::vector<float> he(ncell), hk, hf;
    int rc = copy_in(he.data(), eps, ncell * sizeof(float), h->stream);
    if (rc) return rc;
    if (K) {
        hk.resize(ncell);
        if ((rc = copy_in(hk.data(), K, ncell * sizeof(float), h->stream))) return rc;
    }
    if (Feps) {
        hf.resize(ncell);
        if ((rc = copy_in(hf.data(), Feps, ncell * sizeof(float), h->stream))) return rc;
    }
    const size_t pcell = (size_t)G.plane;
    pe.assign(pcell, 1.0f);
    pa.assign(pcell, 0.0f);
    pb.assign(pcell, 0.0f);
    for (size_t y = 0; y < ny; ++y)
        for (size_t x = 0; x < nx; ++x) {
            const size_t i = y * nx + x, j = y * pitch + x;
            const double ep = he[i];
            if (!(ep > 0.0 && ep <= 1.0))
                return fail(DMRT_EINVAL, "eps[%zu] = %g outside (0, 1]", i, ep);
            const double k = K ? (double)hk[i] : h->D.K_default;
            if (!(k > 0) || !std::isfinite(k)) return fail(DMRT_EINVAL, "K[%zu] = %g must be > 0", i, k);
            const double cf = Feps ? (double)hf[i] : 1.75 / std::sqrt(h->ergun_c * ep * ep * ep);
            if (!(cf >= 0) || !std::isfinite(cf))
                return fail(DMRT_EINVAL, "Feps[%zu] = %g must be finite and >= 0", i, cf);
            pe[j] = (float)ep;
            if (ep < 1.0) {  // eps = 1: clear fluid, no porous drag
                pa[j] = (float)(ep * h->D.nu_l / (k * (1 - ep) * (1 - ep)));
                pb[j] = (float)(ep * cf / (std::sqrt(k) * (1 - ep)));
            }
        }
    return DMRT_OK;
}

void drop_record_graphs(dmrt* h)
{
    for (auto& g : h->rec_graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

void drop_recording(dmrt* h)
{
    if (h->adj_graph) (void)hipGraphExecDestroy(h->adj_graph);
    h->adj_graph = nullptr;
    drop_record_graphs(h);
    h->rec_all = false;
    if (h->rec_base) (void)hipFree(h->rec_base);
    h->rec_base = nullptr;
    h->ckpt = h->ring = h->ls = h->la = h->ga = h->flnext = h->stage = nullptr;
    h->rec_n = h->rec_S = h->rec_cap = 0;
}

dmrtk::StepBufs ring_bufs(const dmrt* h, const float* a, float* b);

// Steps from ring state a at slot k into the following slots up to slot
// end: two per launch where the handle runs two steps per launch (the state
// between them stored too), else one.
hipError_t ring_steps(dmrt* h, const float* a, int64_t k, int64_t end, float* ring, size_t sb)
{
    const bool two = use_two_step(h);
    while (k < end) {
        hipError_t e;
        if (two && k + 2 <= end) {
            const dmrtk::StepBufs mid = ring_bufs(h, a, ring + (size_t)(k + 1) * sb);
            e = dmrtk::launch_step2(h->G, h->P, ring_bufs(h, a, ring + (size_t)(k + 2) * sb), h->flow,
                                    h->stream, &mid);
            k += 2;
        } else {
            e = dmrtk::launch_step(h->G, h->P, ring_bufs(h, a, ring + (size_t)(k + 1) * sb), h->flow,
                                   false, h->stream);
            k += 1;
        }
        if (e != hipSuccess) return e;
        a = ring + (size_t)k * sb;
    }
    return hipSuccess;
}

// Enqueue the reversed pass over a recorded run of n steps: per segment,
// last segment first, recompute its states into the ring (the first read
// from its checkpoint), then one adjoint launch per step, last step first;
// the local adjoints alternate between two buffers.  When the recording kept
// every state (one segment of n steps, already in the ring) nothing is
// recomputed.
int enqueue_adjoint(dmrt* h)
{
    const Geom& G = h->G;
    const size_t pl = (size_t)G.plane, sb = (size_t)dmrtk::ADJ_STATE * pl, fq = dmrtk::FQ;
    const size_t la_n = (size_t)dmrtk::ADJ_LA * pl;
    const int64_t n = h->rec_n, S = h->rec_S, C = (n + S - 1) / S;
    int64_t r = 0;  // reversed steps enqueued so far
    for (int64_t c = C - 1; c >= 0; --c) {
        const int64_t len = std::min(S, n - c * S);
        const float* ck = h->ckpt + (size_t)c * sb;
        auto state = [&](int64_t j) { return j == 0 ? ck : h->ring + (size_t)j * sb; };
        if (c < C - 1 && !h->rec_all) {
            // f_l of the state after this segment's end is the later
            // segment's state 1, about to be overwritten in the ring
            hipError_t e = dmrtk::launch_copy(h->flnext, h->ring + sb + (fq + 5) * pl, pl, h->stream);
            if (e != hipSuccess) return fail(DMRT_EDEVICE, "copy launch: %s", hipGetErrorString(e));
        }
        if (!h->rec_all) {
            hipError_t e = ring_steps(h, ck, 0, len, h->ring, sb);
            if (e != hipSuccess) return fail(DMRT_EDEVICE, "recompute launch: %s", hipGetErrorString(e));
        }
        for (int64_t j = len - 1; j >= 0; --j, ++r) {
            const float* a = state(j);
            dmrtk::AdjBufs A;
            A.f0 = a;
            A.g0 = a + fq * pl;
            A.fl0 = a + (fq + 5) * pl;
            A.u0 = a + (fq + 6) * pl;
            A.fl1 = h->ring + (size_t)(j + 1) * sb + (fq + 5) * pl;
            A.fl2 = j + 2 <= len ? h->ring + (size_t)(j + 2) * sb + (fq + 5) * pl : h->flnext;
            A.eps = h->eps;
            A.Ac = h->Ac;
            A.Bc = h->Bc;
            A.ls = h->ls;
            A.la_prev = h->la + (size_t)((r + 1) & 1) * la_n;
            A.la = h->la + (size_t)(r & 1) * la_n;
            A.ga = h->ga;
            hipError_t e = dmrtk::launch_adjoint_step(G, h->P, A, h->flow, r == 0, h->stream);
            if (e != hipSuccess) return fail(DMRT_EDEVICE, "adjoint launch: %s", hipGetErrorString(e));
        }
    }
    return DMRT_OK;
}

// Buffers of one step from ring state a into ring slot b (u^k read from a).
dmrtk::StepBufs ring_bufs(const dmrt* h, const float* a, float* b)
{
    const size_t pl = (size_t)h->G.plane, fq = dmrtk::FQ;
    dmrtk::StepBufs B;
    B.fin = a;
    B.fout = b;
    B.gin = a + fq * pl;
    B.gout = b + fq * pl;
    B.flin = a + (fq + 5) * pl;
    B.flout = b + (fq + 5) * pl;
    B.ux = b + (fq + 6) * pl;
    B.uy = b + (fq + 7) * pl;
    B.uin = a + (fq + 6) * pl;
    B.eps = h->eps;
    B.Ac = h->Ac;
    B.Bc = h->Bc;
    B.it_sum = B.it_max = nullptr;
    B.r2f = nullptr;
    B.r2_its = 0;
    return B;
}

// Copy the handle's state at buffer parity p into a snapshot of ADJ_STATE
// planes (f, g, f_l, u), or back (copy kernels, so that a graph can hold them).
hipError_t state_copy(dmrt* h, int p, float* snap, bool to_snapshot)
{
    const size_t pl = (size_t)h->G.plane, fq = dmrtk::FQ;
    float* const parts[4] = {h->f[p], h->g[p], h->fl[p], h->u[p]};  // u_y follows u_x
    const size_t planes[4] = {fq, 5, 1, 2};
    float* q = snap;
    for (int k = 0; k < 4; ++k) {
        const size_t n = planes[k] * pl;
        hipError_t e = to_snapshot ? dmrtk::launch_copy(q, parts[k], n, h->stream)
                                   : dmrtk::launch_copy(parts[k], q, n, h->stream);
        if (e != hipSuccess) return e;
        q += n;
    }
    return hipSuccess;
}

// The launches of a recorded run of rec_n steps from buffer parity p.  With
// every state kept: the state into checkpoint 0, each step from one ring
// slot into the next, the last state back into the buffers at parity p.
// With checkpoints: per segment, the state into its checkpoint, then its
// steps in the handle's buffers.
int enqueue_record(dmrt* h, int p)
{
    const size_t sb = (size_t)dmrtk::ADJ_STATE * h->G.plane;
    const int64_t n = h->rec_n, S = h->rec_S;
    if (h->rec_all) {
        HIPCHK(state_copy(h, p, h->ckpt, true));
        HIPCHK(ring_steps(h, h->ckpt, 0, n, h->ring, sb));
        HIPCHK(state_copy(h, p, h->ring + (size_t)n * sb, false));
        return DMRT_OK;
    }
    const int save = h->cur;
    h->cur = p;
    const bool two = use_two_step(h);
    int launches = 0;
    for (int64_t c = 0, k = 0; k < n; ++c) {
        hipError_t e = state_copy(h, h->cur, h->ckpt + (size_t)c * sb, true);
        for (int64_t j = 0; j < S && k < n && e == hipSuccess;) {
            const int st = (two && j + 2 <= S && k + 2 <= n) ? 2 : 1;
            e = st == 2 ? enqueue_step2(h) : enqueue_step(h, false);
            h->cur = 1 - h->cur;
            j += st;
            k += st;
            ++launches;
        }
        if (e != hipSuccess) {
            h->cur = save;
            return fail(DMRT_EDEVICE, "record launch: %s", hipGetErrorString(e));
        }
    }
    h->cur = save;
    h->rec_flip = launches & 1;
    return DMRT_OK;
}

// The replay graphs hold the launches of one flow mode (flow kernels or the
// conduction-only ones): drop them when the mode changes.
void set_flow(dmrt* h, bool flow)
{
    if (flow == h->flow) return;
    h->flow = flow;
    for (auto& g : h->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

int check_finite(dmrt* h)
{
    dmrt_diag_t d;
    int rc = diag_impl(h, &d);
    if (rc) return rc;
    if (d.nonfinite > 0 || !std::isfinite(d.enthalpy))
        return fail(DMRT_ENONFINITE, "non-finite state detected at step %lld (%lld values)",
                    (long long)h->t, (long long)d.nonfinite);
    return DMRT_OK;
}

}  // namespace

extern "C" {

void dmrt_opts_default(dmrt_opts* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->Ma = 0.1;
    o->J = 1.0;
    o->lambda = 1.0;
    o->alpha_ratio = 1.0;
    o->sigma_s = o->sigma_l = 1.0;
    o->T_s = -0.02;
    o->T_l = 0.02;
    o->T0 = 0.0;
    o->T_init = 0.0;
    o->alpha_l = 0.02;
    o->varpi = -2.0;
    o->s_e = 1.1;
    o->s_eps = 1.1;
    o->s_q = 1.2;
    o->zeta_e = 1.5;
    o->zeta_nu = 1.5;
    o->ergun_c = 175.0;
    o->fl_tol = 1e-6;
    o->fl_maxit = 64;
    o->convective = 1;
    o->check_every = 0;
    o->graph_steps = 0;
    o->block_rows = 0;
    o->cells_per_lane = 0;
    o->stream = nullptr;
    o->sigma_mode = 0;
    o->ke_mode = 0;
    o->latent_mode = 0;
    o->store_hint = 0;
    o->cps_ratio = 1.0;
    o->cm_ratio = 1.0;
    o->ks_ratio = 1.0;
    o->km_ratio = 1.0;
    o->record_mode = 0;
    o->steps_per_launch = 2;
    o->addressing = 0;
}

int dmrt_derive(const dmrt_grid* grid, double Ra, double Da, double Pr, double Ste,
                const dmrt_opts* opts, dmrt_derived* out)
{
    dmrt_opts o;
    if (opts) o = *opts; else dmrt_opts_default(&o);
    return derive_impl(grid, Ra, Da, Pr, Ste, o, out);
}

int dmrt_create(const dmrt_grid* grid, const float* eps, const float* K, const float* Feps,
                double Ra, double Da, double Pr, double Ste, const dmrt_bc* bc,
                const dmrt_opts* opts, dmrt_t** out)
{
    g_err.clear();
    if (!out) return fail(DMRT_EINVAL, "null output handle");
    *out = nullptr;
    if (!grid || !eps) return fail(DMRT_EINVAL, "grid and eps are required");
    dmrt_opts o;
    if (opts) o = *opts; else dmrt_opts_default(&o);
    dmrt_derived d;
    int rc = derive_impl(grid, Ra, Da, Pr, Ste, o, &d);
    if (rc) return rc;
    if ((rc = check_opts(o)) || (rc = check_bc(bc))) return rc;
    if (o.sigma_mode && !(o.T_l + 1.0 / Ste > o.cps_ratio * o.T_s))
        return fail(DMRT_EINVAL, "sigma_mode 1 needs T_l + 1/St > cps_ratio T_s");
    if (o.latent_mode && o.fl_maxit > 4096)
        return fail(DMRT_EINVAL, "latent_mode 1 launches fl_maxit sweeps per step: fl_maxit <= 4096");
    const long long nx = grid->nx, ny = grid->ny;
    const long long pitch = (nx + 63) / 64 * 64;
    if (ny * pitch >= (1ll << 31)) return fail(DMRT_EINVAL, "lattice too large (%lld x %lld)", nx, ny);

    dmrt* h = new (std::nothrow) dmrt;
    if (!h) return fail(DMRT_ENOMEM, "host allocation");
    h->D = d;
    h->Ste = Ste;
    h->check_every = o.check_every;
    h->graph_steps = o.graph_steps;
    h->record_mode = o.record_mode;
    h->stream = (hipStream_t)o.stream;
    Geom& G = h->G;
    fill_geom(G, (int)nx, (int)ny, *bc, o);
    fill_phys(h->P, h->D, h->Ste, o);
    h->flow = d.gbeta != 0.0;
    h->two_step = o.steps_per_launch == 2 && !o.latent_mode && dmrtk::step2_supported(G, h->P);

    auto bail = [&](int code) {
        dmrt_destroy(h);
        return code;
    };
    hipError_t e = hipGetDevice(&h->dev);
    if (e != hipSuccess) return bail(fail(DMRT_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e)));
    if ((rc = scratch_setup(h->dev))) return bail(rc);

    // Inputs: stage through host memory, validate, derive the drag coefficients.
    h->ergun_c = o.ergun_c;
    h->feps_given = Feps != nullptr;
    const size_t pcell = (size_t)G.plane;
    std::vector<float> pe, pa, pb;
    if ((rc = porous_planes(h, eps, K, Feps, pe, pa, pb))) return bail(rc);

    // Device memory: one allocation, 256-byte aligned sub-arrays.
    const size_t plane_b = align256(pcell * sizeof(float));
    const size_t total = plane_b * (2 * dmrtk::FQ + 2 * 5 + 2 + 4 + 3);
    e = hipMalloc(&h->base, total);
    if (e != hipSuccess)
        return bail(fail(e == hipErrorOutOfMemory ? DMRT_ENOMEM : DMRT_EDEVICE,
                         "hipMalloc(%zu): %s", total, hipGetErrorString(e)));
    char* p = h->base;
    auto take = [&](size_t planes) {
        float* r = (float*)p;
        p += planes * plane_b;
        return r;
    };
    h->f[0] = take(dmrtk::FQ);
    h->f[1] = take(dmrtk::FQ);
    h->g[0] = take(5);
    h->g[1] = take(5);
    h->fl[0] = take(1);
    h->fl[1] = take(1);
    h->u[0] = take(2);
    h->u[1] = take(2);
    h->eps = take(1);
    h->Ac = take(1);
    h->Bc = take(1);
    // Zero everything once: padding columns and inactive slots stay finite.
    e = hipMemsetAsync(h->base, 0, total, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h->eps, pe.data(), pcell * 4, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h->Ac, pa.data(), pcell * 4, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h->Bc, pb.data(), pcell * 4, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return bail(fail(DMRT_EDEVICE, "upload: %s", hipGetErrorString(e)));

    if (o.latent_mode) {
        // T*, two f_l iterates and the sweep flags of the global iteration
        const size_t r2_bytes = 3 * plane_b + align256((size_t)o.fl_maxit * sizeof(int));
        e = hipMalloc(&h->r2_base, r2_bytes);
        if (e != hipSuccess)
            return bail(fail(e == hipErrorOutOfMemory ? DMRT_ENOMEM : DMRT_EDEVICE,
                             "hipMalloc(%zu): %s", r2_bytes, hipGetErrorString(e)));
        h->r2 = true;
        h->R.ts = (float*)h->r2_base;
        h->R.r2a = (float*)(h->r2_base + plane_b);
        h->R.r2b = (float*)(h->r2_base + 2 * plane_b);
        h->R.flags = (int*)(h->r2_base + 3 * plane_b);
        e = hipMemsetAsync(h->r2_base, 0, r2_bytes, h->stream);
        if (e != hipSuccess) return bail(fail(DMRT_EDEVICE, "memset: %s", hipGetErrorString(e)));
    }

    // Initial state: uniform T_init at rest.
    if ((rc = dmrt_set_state(h, nullptr, nullptr, nullptr))) return bail(rc);
    *out = h;
    return DMRT_OK;
}

int dmrt_set_state(dmrt_t* h, const float* f, const float* g, const float* fl)
{
    if (!h) return fail(DMRT_EINVAL, "null handle");
    HIPCHK(hipSetDevice(h->dev));
    const Geom& G = h->G;
    const size_t ncell = (size_t)G.nx * G.ny;
    const size_t need = (f ? 9 : 0) * ncell + (g ? 5 : 0) * ncell + (fl ? 1 : 0) * ncell;
    float *df = nullptr, *dg = nullptr, *dfl = nullptr;
    if (need) {
        int rc = ensure_work(h, need * sizeof(float));
        if (rc) return rc;
        float* s = (float*)h->work;
        if (f) { df = s; s += 9 * ncell; HIPCHK(hipMemcpyAsync(df, f, 9 * ncell * 4, hipMemcpyDefault, h->stream)); }
        if (g) { dg = s; s += 5 * ncell; HIPCHK(hipMemcpyAsync(dg, g, 5 * ncell * 4, hipMemcpyDefault, h->stream)); }
        if (fl) { dfl = s; HIPCHK(hipMemcpyAsync(dfl, fl, ncell * 4, hipMemcpyDefault, h->stream)); }
    }
    if (f) set_flow(h, true);  // a given velocity field may move without gravity
    const int a = h->cur;
    HIPCHK(dmrtk::launch_load_state(G, h->P, df, dg, dfl, h->f[a], h->g[a], h->fl[a], h->u[a],
                                   h->u[a] + G.plane, h->eps, h->Ac, h->Bc, h->flow, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return DMRT_OK;
}

int dmrt_step(dmrt_t* h, int64_t n)
{
    if (!h) return fail(DMRT_EINVAL, "null handle");
    if (n < 0) return fail(DMRT_EINVAL, "negative step count");
    HIPCHK(hipSetDevice(h->dev));
    int64_t since_check = 0;
    while (n > 0) {
        int64_t chunk = 1;
        if (h->graph_steps > 0 && h->stream && n >= h->graph_steps &&
            (h->check_every == 0 || h->check_every - since_check >= h->graph_steps)) {
            const int p = h->cur;
            if (!h->graph[p]) {
                int rc = build_graph(h, p);
                if (rc) return rc;
            }
            HIPCHK(hipGraphLaunch(h->graph[p], h->stream));
            h->cur = p ^ h->graph_flip[p];
            h->t += h->graph_steps;
            chunk = h->graph_steps;
        } else if (n >= 2 && use_two_step(h)) {
            HIPCHK(enqueue_step2(h));
            h->cur = 1 - h->cur;
            h->t += 2;
            chunk = 2;
        } else {
            int rc = step_once(h, false);
            if (rc) return rc;
        }
        n -= chunk;
        since_check += chunk;
        if (h->check_every > 0 && since_check >= h->check_every) {
            since_check = 0;
            int rc = check_finite(h);
            if (rc) return rc;
        }
    }
    return DMRT_OK;
}

int dmrt_step_counted(dmrt_t* h, int64_t n, int32_t* max_it, double* mean_it)
{
    if (!h) return fail(DMRT_EINVAL, "null handle");
    if (n < 0) return fail(DMRT_EINVAL, "negative step count");
    HIPCHK(hipSetDevice(h->dev));
    const size_t pb = (size_t)h->G.plane * sizeof(int);
    if (!h->it_sum) {
        HIPCHK(hipMalloc(&h->it_sum, 2 * pb));
        h->it_max = h->it_sum + h->G.plane;
    }
    HIPCHK(hipMemsetAsync(h->it_sum, 0, 2 * pb, h->stream));
    for (int64_t k = 0; k < n; ++k) {
        int rc = step_once(h, true);
        if (rc) return rc;
    }
    std::vector<int> hs(h->G.plane), hm(h->G.plane);
    HIPCHK(hipMemcpyAsync(hs.data(), h->it_sum, pb, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(hm.data(), h->it_max, pb, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    long long tot = 0;
    int mx = 0;
    for (int y = 0; y < h->G.ny; ++y)
        for (int x = 0; x < h->G.nx; ++x) {
            const size_t j = (size_t)y * h->G.pitch + x;
            tot += hs[j];
            mx = hm[j] > mx ? hm[j] : mx;
        }
    if (max_it) *max_it = mx;
    if (mean_it) *mean_it = n > 0 ? (double)tot / ((double)n * h->G.nx * h->G.ny) : 0.0;
    return DMRT_OK;
}

int dmrt_fields(dmrt_t* h, float* T, float* ux, float* uy, float* fl)
{
    if (!h) return fail(DMRT_EINVAL, "null handle");
    HIPCHK(hipSetDevice(h->dev));
    const Geom& G = h->G;
    const size_t ncell = (size_t)G.nx * G.ny;
    int rc = ensure_work(h, 4 * ncell * sizeof(float));
    if (rc) return rc;
    float* s = (float*)h->work;
    const int a = h->cur;
    HIPCHK(dmrtk::launch_fields(G, h->g[a], h->fl[a], h->u[a], h->u[a] + G.plane, h->flow, s,
                                h->stream));
    float* dst[4] = {T, ux, uy, fl};
    for (int k = 0; k < 4; ++k)
        if (dst[k]) HIPCHK(hipMemcpyAsync(dst[k], s + k * ncell, ncell * 4, hipMemcpyDefault, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return DMRT_OK;
}

int dmrt_get_populations(dmrt_t* h, float* fpost, float* gpost)
{
    if (!h) return fail(DMRT_EINVAL, "null handle");
    HIPCHK(hipSetDevice(h->dev));
    const Geom& G = h->G;
    const size_t ncell = (size_t)G.nx * G.ny;
    int rc = ensure_work(h, 14 * ncell * sizeof(float));
    if (rc) return rc;
    float* s = (float*)h->work;
    const int a = h->cur;
    HIPCHK(dmrtk::launch_populations(G, h->f[a], h->g[a], h->fl[a], h->flow, s, s + 9 * ncell,
                                    h->stream));
    if (fpost) HIPCHK(hipMemcpyAsync(fpost, s, 9 * ncell * 4, hipMemcpyDefault, h->stream));
    if (gpost) HIPCHK(hipMemcpyAsync(gpost, s + 9 * ncell, 5 * ncell * 4, hipMemcpyDefault, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return DMRT_OK;
}

int dmrt_diag(dmrt_t* h, dmrt_diag_t* out)
{
    if (!h || !out) return fail(DMRT_EINVAL, "null argument");
    HIPCHK(hipSetDevice(h->dev));
    return diag_impl(h, out);
}

int dmrt_diag_noalloc(dmrt_t* h, dmrt_diag_t* out)
{
    if (!h || !out) return fail(DMRT_EINVAL, "null argument");
    const Geom& G = h->G;
    const int nblk = dmrtk::tile_blocks(G, dmrtk::TY);
    const size_t pbytes = align256((size_t)nblk * dmrtk::DIAG_SLOTS * sizeof(double));
    const size_t fbytes = align256((size_t)G.ny * sizeof(float));
    const size_t rbytes = 16 * sizeof(double);
    if (pbytes + fbytes + rbytes > kScratchBytes)
        return fail(DMRT_ESIZE,
                    "dmrt_diag_noalloc: a %d x %d lattice needs %zu bytes of scratch, the "
                    "fixed array holds %zu (use dmrt_diag)",
                    G.nx, G.ny, pbytes + fbytes + rbytes, kScratchBytes);
    HIPCHK(hipSetDevice(h->dev));
    char* base = (char*)scratch_of(h->dev);
    if (!base) return fail(DMRT_EDEVICE, "no scratch address for device %d", h->dev);
    double* part = (double*)base;
    float* front = (float*)(base + pbytes);
    double* res = (double*)(base + pbytes + fbytes);
    int nb = 0;
    const int a = h->cur;
    // every partial, row front and result is written before it is read: no
    // clearing is needed between calls
    HIPCHK(dmrtk::launch_diag(G, h->P, h->f[a], h->g[a], h->fl[a], h->u[a], h->u[a] + G.plane, h->eps, h->flow,
                             part, &nb, h->stream));
    HIPCHK(dmrtk::launch_front(G, h->fl[a], front, h->stream));
    HIPCHK(dmrtk::launch_diag_reduce(part, nb, front, G.ny, res, h->stream));
    double r[16];
    HIPCHK(hipMemcpyAsync(r, res, rbytes, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    out->mass = r[0];
    out->enthalpy = r[1];
    out->liquid = r[2];
    out->T_sum = r[3];
    out->u_max = r[4];
    out->active = (int64_t)llround(r[5]);
    out->nonfinite = (int64_t)llround(r[6]);
    out->front_mean = r[8] / G.ny;
    out->front_max = r[9];
    out->step = h->t;
    return DMRT_OK;
}

int dmrt_get_derived(const dmrt_t* h, dmrt_derived* out)
{
    if (!h || !out) return fail(DMRT_EINVAL, "null argument");
    *out = h->D;
    return DMRT_OK;
}

int32_t dmrt_launch_steps(const dmrt_t* h)
{
    if (!h) return fail(DMRT_EINVAL, "null handle");
    return use_two_step(h) ? 2 : 1;
}

int64_t dmrt_state_bytes(const dmrt_t* h)
{
    if (!h) return fail(DMRT_EINVAL, "null handle");
    return (int64_t)(64 + (size_t)h->G.plane * (dmrtk::FQ + 8) * sizeof(float));
}

int dmrt_save(dmrt_t* h, void* buf, size_t cap)
{
    if (!h || !buf) return fail(DMRT_EINVAL, "null argument");
    const int64_t need = dmrt_state_bytes(h);
    if ((int64_t)cap < need) return fail(DMRT_ESIZE, "buffer holds %zu bytes, %lld needed", cap, (long long)need);
    HIPCHK(hipSetDevice(h->dev));
    uint64_t hdr[8] = {kMagic, (uint64_t)h->G.nx, (uint64_t)h->G.ny, (uint64_t)h->G.pitch,
                       (uint64_t)h->t, (uint64_t)h->flow, 0, 0};
    std::memcpy(buf, hdr, sizeof hdr);
    char* p = (char*)buf + 64;
    const size_t pb = (size_t)h->G.plane * sizeof(float);
    const int a = h->cur;
    const size_t fq = dmrtk::FQ;
    HIPCHK(hipMemcpyAsync(p, h->f[a], fq * pb, hipMemcpyDefault, h->stream));
    HIPCHK(hipMemcpyAsync(p + fq * pb, h->g[a], 5 * pb, hipMemcpyDefault, h->stream));
    HIPCHK(hipMemcpyAsync(p + (fq + 5) * pb, h->fl[a], pb, hipMemcpyDefault, h->stream));
    HIPCHK(hipMemcpyAsync(p + (fq + 6) * pb, h->u[a], 2 * pb, hipMemcpyDefault, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return DMRT_OK;
}

int dmrt_load(dmrt_t* h, const void* buf, size_t n)
{
    if (!h || !buf) return fail(DMRT_EINVAL, "null argument");
    if ((int64_t)n < dmrt_state_bytes(h)) return fail(DMRT_EINVAL, "checkpoint too short");
    uint64_t hdr[8];
    std::memcpy(hdr, buf, sizeof hdr);
    if (hdr[0] != kMagic || hdr[1] != (uint64_t)h->G.nx || hdr[2] != (uint64_t)h->G.ny ||
        hdr[3] != (uint64_t)h->G.pitch)
        return fail(DMRT_EINVAL, "checkpoint does not match this lattice");
    HIPCHK(hipSetDevice(h->dev));
    const char* p = (const char*)buf + 64;
    const size_t pb = (size_t)h->G.plane * sizeof(float);
    const int a = h->cur;
    const size_t fq = dmrtk::FQ;
    HIPCHK(hipMemcpyAsync(h->f[a], p, fq * pb, hipMemcpyDefault, h->stream));
    HIPCHK(hipMemcpyAsync(h->g[a], p + fq * pb, 5 * pb, hipMemcpyDefault, h->stream));
    HIPCHK(hipMemcpyAsync(h->fl[a], p + (fq + 5) * pb, pb, hipMemcpyDefault, h->stream));
    HIPCHK(hipMemcpyAsync(h->u[a], p + (fq + 6) * pb, 2 * pb, hipMemcpyDefault, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->t = (int64_t)hdr[4];
    if (hdr[5] != 0) set_flow(h, true);
    return DMRT_OK;
}

int dmrt_set_porous(dmrt_t* h, const float* eps, const float* K, const float* Feps)
{
    if (!h || !eps) return fail(DMRT_EINVAL, "handle and eps are required");
    HIPCHK(hipSetDevice(h->dev));
    std::vector<float> pe, pa, pb;
    int rc = porous_planes(h, eps, K, Feps, pe, pa, pb);
    if (rc) return rc;
    const size_t n = (size_t)h->G.plane * sizeof(float);
    HIPCHK(hipMemcpyAsync(h->eps, pe.data(), n, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->Ac, pa.data(), n, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->Bc, pb.data(), n, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->feps_given = Feps != nullptr;
    h->rec_n = 0;  // the recorded run no longer matches; buffers and graph are kept
    return DMRT_OK;
}

int dmrt_record(dmrt_t* h, int64_t n)
{
    if (!h) return fail(DMRT_EINVAL, "null handle");
    if (n < 1) return fail(DMRT_EINVAL, "record at least one step");
    if (h->P.dsig != 0.0f || !h->P.zeta_uniform || h->P.sig_mode || h->P.ke_mode || h->r2)
        return fail(DMRT_EINVAL, "the adjoint needs uniform sigma and tau_T (sigma_s == sigma_l, "
                                 "alpha_ratio == 1, no thermal-model variant)");
    HIPCHK(hipSetDevice(h->dev));
    const size_t pl = (size_t)h->G.plane, sb = (size_t)dmrtk::ADJ_STATE * pl;
    const size_t extra = ((size_t)(dmrtk::ADJ_LS + 2 * dmrtk::ADJ_LA + dmrtk::ADJ_GA + 1) * pl +
                          2 * (size_t)h->G.nx * h->G.ny) * sizeof(float);
    // every state: one checkpoint (state 0) and n + 1 ring slots (states 1..n)
    const size_t all_bytes = (size_t)(n + 2) * sb * sizeof(float) + extra;
    bool keep_all = h->record_mode == 2;
    if (h->record_mode == 0) {
        size_t freeb = 0, totb = 0;
        HIPCHK(hipMemGetInfo(&freeb, &totb));
        const size_t held = (h->rec_cap == n && h->rec_all) ? all_bytes : 0;  // ours already
        keep_all = all_bytes <= (freeb + held) / 2;
    }
    int64_t S = n;
    if (!keep_all) {
        S = 1;
        while (S * S < n) ++S;
    }
    const int64_t C = (n + S - 1) / S;
    if (h->rec_cap != n || h->rec_all != keep_all) {
        drop_recording(h);
        const size_t total = (size_t)C * sb * sizeof(float) + (size_t)(S + 1) * sb * sizeof(float) + extra;
        hipError_t e = hipMalloc(&h->rec_base, total);
        if (e != hipSuccess) {
            h->rec_base = nullptr;
            return fail(e == hipErrorOutOfMemory ? DMRT_ENOMEM : DMRT_EDEVICE, "hipMalloc(%zu): %s",
                        total, hipGetErrorString(e));
        }
        float* p = (float*)h->rec_base;
        h->ckpt = p;
        h->ring = p + (size_t)C * sb;
        h->ls = h->ring + (size_t)(S + 1) * sb;
        h->la = h->ls + (size_t)dmrtk::ADJ_LS * pl;
        h->ga = h->la + (size_t)2 * dmrtk::ADJ_LA * pl;
        h->flnext = h->ga + (size_t)dmrtk::ADJ_GA * pl;
        h->stage = h->flnext + pl;
        h->rec_cap = n;
        h->rec_all = keep_all;
    }
    if (h->rec_graph_flow != h->flow) drop_record_graphs(h);
    h->rec_n = n;
    h->rec_S = S;
    const int p = h->cur;
    if (h->stream) {
        if (!h->rec_graph[p]) {
            HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
            int rc = enqueue_record(h, p);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(h->stream, &graph);
            if (rc || e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                h->rec_n = 0;
                return rc ? rc : fail(DMRT_EDEVICE, "capture of the recording: %s", hipGetErrorString(e));
            }
            e = hipGraphInstantiate(&h->rec_graph[p], graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                h->rec_graph[p] = nullptr;
                h->rec_n = 0;
                return fail(DMRT_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
            }
            h->rec_graph_flow = h->flow;
        }
        HIPCHK(hipGraphLaunch(h->rec_graph[p], h->stream));
    } else {
        int rc = enqueue_record(h, p);
        if (rc) {
            h->rec_n = 0;
            return rc;
        }
    }
    if (!keep_all) h->cur ^= h->rec_flip;  // every-state mode ends back at parity p
    h->t += n;
    if (h->check_every > 0) return check_finite(h);
    return DMRT_OK;
}

int dmrt_adjoint(dmrt_t* h, const float* dL_dT, const float* dL_dfl, float* grad_logK,
                 float* grad_eps)
{
    if (!h) return fail(DMRT_EINVAL, "null handle");
    if (!h->rec_n) return fail(DMRT_EINVAL, "no recorded run (call dmrt_record first)");
    HIPCHK(hipSetDevice(h->dev));
    const Geom& G = h->G;
    const size_t pl = (size_t)G.plane;
    // terminal adjoint (staged through two packed planes: one contiguous copy
    // each, from host or device memory)
    HIPCHK(hipMemsetAsync(h->ls, 0,
                          (size_t)(dmrtk::ADJ_LS + 2 * dmrtk::ADJ_LA + dmrtk::ADJ_GA) * pl * sizeof(float),
                          h->stream));
    const size_t ncell = (size_t)G.nx * G.ny;
    float* sT = h->stage;
    float* sF = h->stage + ncell;
    if (dL_dT) HIPCHK(hipMemcpyAsync(sT, dL_dT, ncell * sizeof(float), hipMemcpyDefault, h->stream));
    if (dL_dfl) HIPCHK(hipMemcpyAsync(sF, dL_dfl, ncell * sizeof(float), hipMemcpyDefault, h->stream));
    HIPCHK(dmrtk::launch_adjoint_terminal(G, dL_dT ? sT : nullptr, dL_dfl ? sF : nullptr, h->ls,
                                          h->stream));
    // the reversed pass: captured once per recording size and flow mode,
    // replayed afterwards
    if (h->adj_graph && h->adj_flow != h->flow) {
        (void)hipGraphExecDestroy(h->adj_graph);
        h->adj_graph = nullptr;
    }
    if (!h->adj_graph) {
        HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_adjoint(h);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(h->stream, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(DMRT_EDEVICE, "capture of the adjoint: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&h->adj_graph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            h->adj_graph = nullptr;
            return fail(DMRT_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
        h->adj_flow = h->flow;
    }
    HIPCHK(hipGraphLaunch(h->adj_graph, h->stream));
    // gradients, assembled on the device into the two staging planes
    HIPCHK(dmrtk::launch_adjoint_grads(G, h->ga, h->eps, h->Ac, h->Bc, !h->feps_given, sT, sF,
                                       h->stream));
    if (grad_logK) HIPCHK(hipMemcpyAsync(grad_logK, sT, ncell * 4, hipMemcpyDefault, h->stream));
    if (grad_eps) HIPCHK(hipMemcpyAsync(grad_eps, sF, ncell * 4, hipMemcpyDefault, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return DMRT_OK;
}

int64_t dmrt_time(const dmrt_t* h) { return h ? h->t : fail(DMRT_EINVAL, "null handle"); }

int dmrt_sync(dmrt_t* h)
{
    if (!h) return fail(DMRT_EINVAL, "null handle");
    HIPCHK(hipSetDevice(h->dev));
    HIPCHK(hipStreamSynchronize(h->stream));
    return DMRT_OK;
}

void dmrt_destroy(dmrt_t* h)
{
    if (!h) return;
    (void)hipSetDevice(h->dev);
    if (h->stream || h->base) (void)hipStreamSynchronize(h->stream);
    for (auto& g : h->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (h->base) (void)hipFree(h->base);
    if (h->work) (void)hipFree(h->work);
    if (h->it_sum) (void)hipFree(h->it_sum);
    if (h->r2_base) (void)hipFree(h->r2_base);
    drop_recording(h);
    delete h;
}

const char* dmrt_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of independent cavities.
//
// Every cavity keeps its own planes, laid out as for a single lattice (row
// pitch a multiple of 64), inside one arena per array kind: f (10 planes:
// the populations and rho - 1), g (5), f_l (1) and u (2), each
// double-buffered.  A device table of
// Cavity headers gives each cavity's geometry, constants, uniform porous
// values and plane offsets; a device tile list names (cavity, x0, y0) for
// every 64 x rows tile, and a second one every 62 x 6 tile of the two-step
// kernel.  One launch covers the whole list: one time step, or two.
// ---------------------------------------------------------------------------

struct dmrt_batch {
    int dev = 0;
    hipStream_t stream = nullptr;
    int ncav = 0;
    std::vector<dmrtk::Cavity> cav;
    std::vector<dmrt_derived> D;
    int64_t cells = 0;
    int cur = 0;
    int64_t t = 0;
    int check_every = 0, graph_steps = 0;
    int rows = 4, blocks = 0, launch_blocks = 0;  // one-step launch shape
    int store = 0;  // cache policy of the state stores
    int die[dmrtk::NXCD + 1]{};
    size_t f_len = 0, g_len = 0, fl_len = 0, u_len = 0;  // arena lengths in floats
    char* base = nullptr;
    float *f[2]{}, *g[2]{}, *fl[2]{}, *u[2]{};  // u[p]: the velocity of state parity p
    dmrtk::Cavity* dcav = nullptr;
    int4* dtiles = nullptr;
    size_t tiles_cap = 0;
    // two steps per launch: allowed (steps_per_launch 2), in effect, and its
    // tile list cut into die parts, launched with one block per tile
    bool two_ok = false, two = false;
    bool per_array = false;  // one buffer resource per array (addressing 1)
    bool cavity_form = false;  // every cavity: uniform thermal properties, walls all round
    int4* dtiles2 = nullptr;
    int die2[dmrtk::NXCD + 1]{};
    int blocks2 = 0;
    long long* partials = nullptr;
    hipGraphExec_t graph[2]{};
    int graph_flip[2]{};  // buffer parity changes of a replay of graph[p]
};

namespace {

constexpr int kCountBlocks = 16;  // partial-count blocks per cavity

void drop_graphs(dmrt_batch* b)
{
    for (auto& g : b->graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

// Cut a tile list (node counts w) into NXCD contiguous parts of about equal
// node count: die d takes tiles [die[d], die[d + 1]).  Returns the largest
// part's tile count.
int cut_dies(const std::vector<long long>& w, int* die)
{
    const int nt = (int)w.size();
    long long total = 0;
    for (long long v : w) total += v;
    int d = 1;
    long long acc = 0;
    die[0] = 0;
    for (int k = 0; k < nt && d < dmrtk::NXCD; ++k) {
        acc += w[k];
        while (d < dmrtk::NXCD && acc * dmrtk::NXCD >= total * d) die[d++] = k + 1;
    }
    while (d <= dmrtk::NXCD) die[d++] = nt;
    int most = 0;
    for (int k = 0; k < dmrtk::NXCD; ++k) most = std::max(most, die[k + 1] - die[k]);
    return most;
}

// Tile list of the two-step kernel, cavity by cavity, one block per tile:
// wide tiles row-major, then, where a cavity's last column chunk is no wider
// than a narrow tile, that column in narrow tiles (rows of 32 lanes: half
// the idle lanes of a ragged last column).
int batch_layout2(dmrt_batch* b)
{
    int tw = 0, th = 0, nw = 0, nh = 0;
    dmrtk::batch_step2_tile(&tw, &th, &nw, &nh);
    std::vector<int4> tl;
    std::vector<long long> w;
    for (int c = 0; c < b->ncav; ++c) {
        const Geom& G = b->cav[c].G;
        const int last = G.nx - (G.nx - 1) / tw * tw;  // width of the last column chunk
        const int xw = last <= nw ? G.nx - last : G.nx;  // end of the wide tiles
        for (int y0 = 0; y0 < G.ny; y0 += th)
            for (int x0 = 0; x0 < xw; x0 += tw) {
                tl.push_back(make_int4(c, x0, y0, 0));
                w.push_back((long long)std::min(tw, xw - x0) * std::min(th, G.ny - y0));
            }
        if (xw < G.nx)
            for (int y0 = 0; y0 < G.ny; y0 += nh) {
                tl.push_back(make_int4(c, xw, y0, 1));
                w.push_back((long long)(G.nx - xw) * std::min(nh, G.ny - y0));
            }
    }
    const int most = cut_dies(w, b->die2);
    b->blocks2 = dmrtk::NXCD * std::max(1, most);
    HIPCHK(hipMalloc(&b->dtiles2, tl.size() * sizeof(int4)));
    HIPCHK(hipMemcpyAsync(b->dtiles2, tl.data(), tl.size() * sizeof(int4), hipMemcpyHostToDevice,
                          b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    return DMRT_OK;
}

// Tile list for tiles of 64 x rows nodes, cut into one contiguous part per
// die with about equal node counts; block count of the launch.
int batch_layout(dmrt_batch* b, int rows, int blocks)
{
    std::vector<int4> tl;
    std::vector<long long> w;
    for (int c = 0; c < b->ncav; ++c) {
        const Geom& G = b->cav[c].G;
        // 64-wide tiles, except a last column chunk of 1-32 nodes, which is
        // covered by 32-wide tiles twice as tall (half the idle lanes)
        const int rem = G.nx % dmrtk::TX;
        const bool narrow = rem > 0 && rem <= dmrtk::TX / 2;
        const int xw = narrow ? G.nx - rem : G.nx;  // end of the wide tiles
        for (int yb = 0; yb < G.ny; yb += 2 * rows) {
            for (int y0 = yb; y0 < std::min(yb + 2 * rows, G.ny); y0 += rows)
                for (int x0 = 0; x0 < xw; x0 += dmrtk::TX) {
                    tl.push_back(make_int4(c, x0, y0, 0));
                    w.push_back((long long)std::min(dmrtk::TX, G.nx - x0) * std::min(rows, G.ny - y0));
                }
            if (narrow) {
                tl.push_back(make_int4(c, xw, yb, 1));
                w.push_back((long long)rem * std::min(2 * rows, G.ny - yb));
            }
        }
    }
    const int nt = (int)tl.size();
    const int most = cut_dies(w, b->die);
    int nb = blocks;
    if (nb == 0) {
        int ncu = 0;
        HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->dev));
        nb = dmrtk::batch_blocks_per_cu(rows) * ncu / dmrtk::NXCD * dmrtk::NXCD;
    }
    // no die needs more blocks than it has tiles
    nb = std::max(dmrtk::NXCD, std::min(nb, dmrtk::NXCD * most));
    if ((size_t)nt > b->tiles_cap) {
        if (b->dtiles) HIPCHK(hipFree(b->dtiles));
        b->dtiles = nullptr;
        b->tiles_cap = 0;
        HIPCHK(hipMalloc(&b->dtiles, (size_t)nt * sizeof(int4)));
        b->tiles_cap = (size_t)nt;
    }
    HIPCHK(hipMemcpyAsync(b->dtiles, tl.data(), (size_t)nt * sizeof(int4), hipMemcpyHostToDevice,
                          b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    drop_graphs(b);
    b->rows = rows;
    b->blocks = blocks;
    b->launch_blocks = nb;
    return DMRT_OK;
}

// Arguments of a launch from state parity p: of the one-step kernel, or of
// the two-step kernel (its tile list) when two is set.
dmrtk::BatchArgs batch_args(const dmrt_batch* b, int p, bool two = false)
{
    dmrtk::BatchArgs a;
    a.cav = b->dcav;
    a.tiles = two ? b->dtiles2 : b->dtiles;
    for (int k = 0; k <= dmrtk::NXCD; ++k) a.die[k] = two ? b->die2[k] : b->die[k];
    a.fin = b->f[p];
    a.fout = b->f[1 - p];
    a.gin = b->g[p];
    a.gout = b->g[1 - p];
    a.flin = b->fl[p];
    a.flout = b->fl[1 - p];
    a.uin = b->u[p];
    a.uout = b->u[1 - p];
    a.store = b->store;
    // parity p's f, g, f_l and u arenas lie in one half of the allocation
    const uint64_t half = (uint64_t)((const char*)b->f[1] - (const char*)b->f[0]);
    a.win = (const char*)b->f[p];
    a.wout = (const char*)b->f[1 - p];
    a.win_bytes = !b->per_array && half < (1ull << 32) ? (uint32_t)half : 0u;
    a.uniform_thermal = b->cavity_form ? 1 : 0;
    return a;
}

// One launch from parity b->cur: two steps (two-step kernel in effect and
// at least two steps wanted) or one.  Flips the parity; returns the steps.
hipError_t batch_launch(dmrt_batch* b, int64_t n, int* steps)
{
    const bool two = b->two && n >= 2;
    hipError_t e = two ? dmrtk::launch_batch_step2(batch_args(b, b->cur, true), b->blocks2, b->stream)
                       : dmrtk::launch_batch_step(batch_args(b, b->cur), b->rows, b->launch_blocks,
                                                  b->stream);
    b->cur = 1 - b->cur;
    *steps = two ? 2 : 1;
    return e;
}

int batch_graph(dmrt_batch* b, int p)
{
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const int save = b->cur;
    b->cur = p;
    int launches = 0;
    for (int k = 0; k < b->graph_steps;) {
        int st = 1;
        hipError_t e = batch_launch(b, b->graph_steps - k, &st);
        k += st;
        ++launches;
        if (e != hipSuccess) {
            b->cur = save;
            hipGraph_t gdrop = nullptr;
            (void)hipStreamEndCapture(b->stream, &gdrop);
            if (gdrop) (void)hipGraphDestroy(gdrop);
            return fail(DMRT_EDEVICE, "launch during capture: %s", hipGetErrorString(e));
        }
    }
    b->cur = save;
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamEndCapture(b->stream, &graph));
    hipError_t e = hipGraphInstantiate(&b->graph[p], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        b->graph[p] = nullptr;
        return fail(DMRT_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    b->graph_flip[p] = launches & 1;
    return DMRT_OK;
}

int batch_counts(dmrt_batch* b, std::vector<long long>& liq, std::vector<long long>& bad)
{
    const int a = b->cur;
    HIPCHK(dmrtk::launch_batch_count(b->dcav, b->ncav, b->fl[a], b->g[a], b->partials,
                                     kCountBlocks, b->stream));
    std::vector<long long> hp((size_t)2 * kCountBlocks * b->ncav);
    HIPCHK(hipMemcpyAsync(hp.data(), b->partials, hp.size() * sizeof(long long),
                          hipMemcpyDeviceToHost, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    liq.assign(b->ncav, 0);
    bad.assign(b->ncav, 0);
    for (int c = 0; c < b->ncav; ++c)
        for (int k = 0; k < kCountBlocks; ++k) {
            liq[c] += hp[2 * ((size_t)c * kCountBlocks + k)];
            bad[c] += hp[2 * ((size_t)c * kCountBlocks + k) + 1];
        }
    return DMRT_OK;
}

int batch_check_finite(dmrt_batch* b)
{
    std::vector<long long> liq, bad;
    int rc = batch_counts(b, liq, bad);
    if (rc) return rc;
    for (int c = 0; c < b->ncav; ++c)
        if (bad[c])
            return fail(DMRT_ENONFINITE, "cavity %d: non-finite state at step %lld (%lld values)",
                        c, (long long)b->t, bad[c]);
    return DMRT_OK;
}

int batch_step_impl(dmrt_batch* b, int64_t n)
{
    int64_t since_check = 0;
    while (n > 0) {
        int64_t chunk = 1;
        if (b->graph_steps > 0 && b->stream && n >= b->graph_steps &&
            (b->check_every == 0 || b->check_every - since_check >= b->graph_steps)) {
            const int p = b->cur;
            if (!b->graph[p]) {
                int rc = batch_graph(b, p);
                if (rc) return rc;
            }
            HIPCHK(hipGraphLaunch(b->graph[p], b->stream));
            b->cur = p ^ b->graph_flip[p];
            chunk = b->graph_steps;
        } else {
            int st = 1;
            HIPCHK(batch_launch(b, n, &st));
            chunk = st;
        }
        b->t += chunk;
        n -= chunk;
        since_check += chunk;
        if (b->check_every > 0 && since_check >= b->check_every) {
            since_check = 0;
            int rc = batch_check_finite(b);
            if (rc) return rc;
        }
    }
    return DMRT_OK;
}

}  // namespace

extern "C" {

int dmrt_batch_create(int32_t ncav, const dmrt_cavity* cav, const dmrt_opts* opts,
                      dmrt_batch_t** out)
{
    g_err.clear();
    if (!out) return fail(DMRT_EINVAL, "null output handle");
    *out = nullptr;
    if (ncav < 1 || !cav) return fail(DMRT_EINVAL, "need at least one cavity");
    dmrt_opts o;
    if (opts) o = *opts; else dmrt_opts_default(&o);
    int rc = check_opts(o);
    if (rc) return rc;
    if (o.sigma_mode || o.ke_mode || o.latent_mode)
        return fail(DMRT_EINVAL, "the thermal-model variants are for single lattices only");

    dmrt_batch* b = new (std::nothrow) dmrt_batch;
    if (!b) return fail(DMRT_ENOMEM, "host allocation");
    auto bail = [&](int code) {
        dmrt_batch_destroy(b);
        return code;
    };
    b->ncav = ncav;
    b->stream = (hipStream_t)o.stream;
    b->check_every = o.check_every;
    b->graph_steps = o.graph_steps;
    b->cav.resize(ncav);
    b->D.resize(ncav);
    for (int c = 0; c < ncav; ++c) {
        const dmrt_cavity& in = cav[c];
        dmrt_derived& d = b->D[c];
        if ((rc = derive_impl(&in.grid, in.Ra, in.Da, in.Pr, in.Ste, o, &d)) || (rc = check_bc(&in.bc))) {
            const std::string why = g_err;
            return bail(fail(rc, "cavity %d: %s", c, why.c_str()));
        }
        const long long pitch = ((long long)in.grid.nx + 63) / 64 * 64;
        if ((long long)in.grid.ny * pitch * 4 * dmrtk::FQ >= (1ll << 32))
            return bail(fail(DMRT_EINVAL, "cavity %d: lattice too large for a batch", c));
        // the porous values of a single lattice with this porosity everywhere
        const double ep = (double)(float)in.eps;
        if (!(ep > 0.0 && ep <= 1.0))
            return bail(fail(DMRT_EINVAL, "cavity %d: eps = %g outside (0, 1]", c, in.eps));
        dmrtk::Cavity& C = b->cav[c];
        std::memset(&C, 0, sizeof C);
        fill_geom(C.G, in.grid.nx, in.grid.ny, in.bc, o);
        fill_phys(C.P, d, in.Ste, o);
        C.eps = (float)ep;
        if (ep < 1.0) {
            const double k = d.K_default, cf = 1.75 / std::sqrt(o.ergun_c * ep * ep * ep);
            C.Ac = (float)(ep * d.nu_l / (k * (1 - ep) * (1 - ep)));
            C.Bc = (float)(ep * cf / (std::sqrt(k) * (1 - ep)));
        }
        const size_t pl = (size_t)C.G.plane;  // a multiple of 64 floats
        C.f_off = b->f_len;
        C.g_off = b->g_len;
        C.fl_off = b->fl_len;
        C.u_off = b->u_len;
        b->f_len += dmrtk::FQ * pl;
        b->g_len += 5 * pl;
        b->fl_len += pl;
        b->u_len += 2 * pl;
        b->cells += (int64_t)in.grid.nx * in.grid.ny;
    }
    hipError_t e = hipGetDevice(&b->dev);
    if (e != hipSuccess) return bail(fail(DMRT_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e)));

    const size_t bytes_f = align256(b->f_len * 4), bytes_g = align256(b->g_len * 4);
    const size_t bytes_fl = align256(b->fl_len * 4), bytes_u = align256(b->u_len * 4);
    const size_t bytes_c = align256((size_t)ncav * sizeof(dmrtk::Cavity));
    const size_t bytes_p = align256((size_t)2 * kCountBlocks * ncav * sizeof(long long));
    const size_t total = 2 * (bytes_f + bytes_g + bytes_fl + bytes_u) + bytes_c + bytes_p;
    b->store = store_policy(o.store_hint, 2 * (bytes_f + bytes_g + bytes_fl + bytes_u));
    e = hipMalloc(&b->base, total);
    if (e != hipSuccess)
        return bail(fail(e == hipErrorOutOfMemory ? DMRT_ENOMEM : DMRT_EDEVICE,
                         "hipMalloc(%zu): %s", total, hipGetErrorString(e)));
    char* p = b->base;
    auto take = [&](size_t n) {
        char* r = p;
        p += n;
        return r;
    };
    for (int k = 0; k < 2; ++k) {
        b->f[k] = (float*)take(bytes_f);
        b->g[k] = (float*)take(bytes_g);
        b->fl[k] = (float*)take(bytes_fl);
        b->u[k] = (float*)take(bytes_u);
    }
    b->dcav = (dmrtk::Cavity*)take(bytes_c);
    b->partials = (long long*)take(bytes_p);
    e = hipMemsetAsync(b->base, 0, total, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->dcav, b->cav.data(), (size_t)ncav * sizeof(dmrtk::Cavity),
                           hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return bail(fail(DMRT_EDEVICE, "upload: %s", hipGetErrorString(e)));
    // initial state of every cavity: uniform T_init at rest
    for (int c = 0; c < ncav; ++c) {
        const dmrtk::Cavity& C = b->cav[c];
        e = dmrtk::launch_load_state(C.G, C.P, nullptr, nullptr, nullptr, b->f[0] + C.f_off,
                                     b->g[0] + C.g_off, b->fl[0] + C.fl_off, b->u[0] + C.u_off,
                                     b->u[0] + C.u_off + C.G.plane, nullptr, nullptr, nullptr, true,
                                     b->stream, C.eps, C.Ac, C.Bc);
        if (e != hipSuccess) return bail(fail(DMRT_EDEVICE, "initial state: %s", hipGetErrorString(e)));
    }
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bail(fail(DMRT_EDEVICE, "initial state: %s", hipGetErrorString(e)));
    if ((rc = batch_layout(b, o.block_rows ? o.block_rows : 4, 0))) return bail(rc);
    b->two_ok = o.steps_per_launch == 2;
    b->per_array = o.addressing == 1;
    b->cavity_form = true;
    for (const dmrtk::Cavity& c : b->cav)
        if (!c.P.zeta_uniform || c.P.dsig != 0.0f || c.G.per_x || c.G.per_y) b->cavity_form = false;
    if (b->two_ok && (rc = batch_layout2(b))) return bail(rc);
    b->two = b->two_ok;
    *out = b;
    return DMRT_OK;
}

int dmrt_batch_step(dmrt_batch_t* b, int64_t n)
{
    if (!b) return fail(DMRT_EINVAL, "null handle");
    if (n < 0) return fail(DMRT_EINVAL, "negative step count");
    HIPCHK(hipSetDevice(b->dev));
    return batch_step_impl(b, n);
}

int dmrt_batch_fields(dmrt_batch_t* b, int32_t i, float* T, float* ux, float* uy, float* fl)
{
    if (!b) return fail(DMRT_EINVAL, "null handle");
    if (i < 0 || i >= b->ncav) return fail(DMRT_EINVAL, "cavity %d out of range", i);
    HIPCHK(hipSetDevice(b->dev));
    const dmrtk::Cavity& C = b->cav[i];
    const size_t ncell = (size_t)C.G.nx * C.G.ny;
    float* s = nullptr;
    HIPCHK(hipMalloc(&s, 4 * ncell * sizeof(float)));
    const int a = b->cur;
    hipError_t e = dmrtk::launch_fields(C.G, b->g[a] + C.g_off, b->fl[a] + C.fl_off,
                                        b->u[a] + C.u_off, b->u[a] + C.u_off + C.G.plane, true, s,
                                        b->stream);
    float* dst[4] = {T, ux, uy, fl};
    for (int k = 0; k < 4 && e == hipSuccess; ++k)
        if (dst[k]) e = hipMemcpyAsync(dst[k], s + k * ncell, ncell * 4, hipMemcpyDefault, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    (void)hipFree(s);
    if (e != hipSuccess) return fail(DMRT_EDEVICE, "fields: %s", hipGetErrorString(e));
    return DMRT_OK;
}

int dmrt_batch_check(dmrt_batch_t* b, int64_t* liquid, int64_t* nonfinite)
{
    if (!b) return fail(DMRT_EINVAL, "null handle");
    HIPCHK(hipSetDevice(b->dev));
    std::vector<long long> liq, bad;
    int rc = batch_counts(b, liq, bad);
    if (rc) return rc;
    for (int c = 0; c < b->ncav; ++c) {
        if (liquid) liquid[c] = liq[c];
        if (nonfinite) nonfinite[c] = bad[c];
    }
    return DMRT_OK;
}

int dmrt_batch_set_launch(dmrt_batch_t* b, int32_t rows, int32_t blocks)
{
    if (!b) return fail(DMRT_EINVAL, "null handle");
    if (rows == 0) {
        if (!b->two_ok) return fail(DMRT_EINVAL, "rows 0 (two steps per launch) needs steps_per_launch 2");
        HIPCHK(hipSetDevice(b->dev));
        HIPCHK(hipStreamSynchronize(b->stream));
        if (!b->two) drop_graphs(b);
        b->two = true;
        return DMRT_OK;
    }
    if (rows != 4 && rows != 8) return fail(DMRT_EINVAL, "rows must be 0, 4 or 8");
    if (blocks < 0 || blocks % dmrtk::NXCD)
        return fail(DMRT_EINVAL, "blocks must be 0 or a positive multiple of 8");
    HIPCHK(hipSetDevice(b->dev));
    HIPCHK(hipStreamSynchronize(b->stream));
    b->two = false;
    return batch_layout(b, rows, blocks);
}

int dmrt_batch_get_launch(const dmrt_batch_t* b, int32_t* rows, int32_t* blocks)
{
    if (!b) return fail(DMRT_EINVAL, "null handle");
    if (rows) *rows = b->two ? 0 : b->rows;
    if (blocks) *blocks = b->two ? b->blocks2 : b->launch_blocks;
    return DMRT_OK;
}

int dmrt_batch_tune(dmrt_batch_t* b, int32_t trial_steps, int32_t* rows, int32_t* blocks,
                    double* ms_per_step)
{
    if (!b) return fail(DMRT_EINVAL, "null handle");
    if (trial_steps < 1) return fail(DMRT_EINVAL, "trial_steps must be >= 1");
    HIPCHK(hipSetDevice(b->dev));
    // candidates: tile rows x (resident blocks, twice that, one block per
    // tile) of the one-step kernel, and the two-step kernel (rows 0) where
    // it is allowed
    int ncu = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->dev));
    struct Cand { int rows, blocks; };
    std::vector<Cand> cands;
    for (int r : {4, 8}) {
        const int res = dmrtk::batch_blocks_per_cu(r) * ncu / dmrtk::NXCD * dmrtk::NXCD;
        for (int nb : {res, 2 * res, 1 << 30}) cands.push_back({r, nb / dmrtk::NXCD * dmrtk::NXCD});
    }
    if (b->two_ok) cands.push_back({0, 0});
    // snapshot of the current state (the trial steps overwrite both buffers)
    const int a = b->cur;
    const size_t nf = b->f_len * 4, ng = b->g_len * 4, nfl = b->fl_len * 4, nu = b->u_len * 4;
    char* snap = nullptr;
    HIPCHK(hipMalloc(&snap, nf + ng + nfl + nu));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto save = [&](bool restore) {
        char* q = snap;
        hipError_t r = hipSuccess;
        const std::pair<char*, size_t> parts[4] = {{(char*)b->f[a], nf}, {(char*)b->g[a], ng},
                                                   {(char*)b->fl[a], nfl}, {(char*)b->u[a], nu}};
        for (const auto& pr : parts) {
            if (r == hipSuccess)
                r = restore ? hipMemcpyAsync(pr.first, q, pr.second, hipMemcpyDeviceToDevice, b->stream)
                            : hipMemcpyAsync(q, pr.first, pr.second, hipMemcpyDeviceToDevice, b->stream);
            q += pr.second;
        }
        return r;
    };
    if (e == hipSuccess) e = save(false);
    const int keep_rows = b->rows, keep_blocks = b->blocks;
    const bool keep_two = b->two;
    int best = -1, best1 = -1, rc = DMRT_OK;  // best1: fastest one-step shape
    float best_ms = 0, best1_ms = 0;
    auto run = [&](int steps) {
        for (int s = 0; s < steps && e == hipSuccess;) {
            int st = 1;
            e = batch_launch(b, steps - s, &st);
            s += st;
        }
    };
    for (size_t k = 0; k < cands.size() && e == hipSuccess && rc == DMRT_OK; ++k) {
        b->two = cands[k].rows == 0;
        if (!b->two && (rc = batch_layout(b, cands[k].rows, cands[k].blocks))) break;
        b->cur = a;
        // trial_steps untimed steps (the state moves past its first steps,
        // which are not representative), then trial_steps timed ones
        run(trial_steps);
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        run(trial_steps);
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && (best < 0 || ms < best_ms)) {
            best = (int)k;
            best_ms = ms;
        }
        if (e == hipSuccess && !b->two && (best1 < 0 || ms < best1_ms)) {
            best1 = (int)k;
            best1_ms = ms;
        }
        b->cur = a;
        if (e == hipSuccess) e = save(true);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(snap);
    b->cur = a;
    if (e != hipSuccess) rc = fail(DMRT_EDEVICE, "tune: %s", hipGetErrorString(e));
    if (rc || best < 0 || best1 < 0) {
        b->two = keep_two;
        (void)batch_layout(b, keep_rows, keep_blocks);
        return rc ? rc : fail(DMRT_EDEVICE, "tune: no candidate ran");
    }
    // the fastest one-step shape stays the shape of single launches
    if ((rc = batch_layout(b, cands[best1].rows, cands[best1].blocks))) return rc;
    b->two = cands[best].rows == 0;
    if ((rc = dmrt_batch_get_launch(b, rows, blocks))) return rc;
    if (ms_per_step) *ms_per_step = best_ms / trial_steps;
    return DMRT_OK;
}

int dmrt_batch_get_derived(const dmrt_batch_t* b, int32_t i, dmrt_derived* out)
{
    if (!b || !out) return fail(DMRT_EINVAL, "null argument");
    if (i < 0 || i >= b->ncav) return fail(DMRT_EINVAL, "cavity %d out of range", i);
    *out = b->D[i];
    return DMRT_OK;
}

int64_t dmrt_batch_cells(const dmrt_batch_t* b) { return b ? b->cells : fail(DMRT_EINVAL, "null handle"); }

int64_t dmrt_batch_time(const dmrt_batch_t* b) { return b ? b->t : fail(DMRT_EINVAL, "null handle"); }

int dmrt_batch_sync(dmrt_batch_t* b)
{
    if (!b) return fail(DMRT_EINVAL, "null handle");
    HIPCHK(hipSetDevice(b->dev));
    HIPCHK(hipStreamSynchronize(b->stream));
    return DMRT_OK;
}

void dmrt_batch_destroy(dmrt_batch_t* b)
{
    if (!b) return;
    (void)hipSetDevice(b->dev);
    if (b->base) (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    if (b->dtiles) (void)hipFree(b->dtiles);
    if (b->dtiles2) (void)hipFree(b->dtiles2);
    if (b->base) (void)hipFree(b->base);
    delete b;
}

}  // extern "C"
