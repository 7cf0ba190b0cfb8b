// Internal types shared by the HIP kernels and the C ABI of the double-MRT
// lattice Boltzmann solver (Liu & He, arXiv:1503.08406).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dmrtk {

// Launch geometry of the fused step: one lattice node per lane, a tile is a
// 64-wide row segment (one wavefront) times TY rows.
constexpr int TX = 64;
constexpr int TY = 4;   // block rows of the auxiliary kernels
constexpr int NXCD = 8;  // MI355X: 8 accelerator dies, each with its own L2
// Planes of an f array: the nine post-collision deviations f+_i - w_i and,
// for liquid nodes, rho - 1 = their sum (what a melting neighbour restarts
// from).
constexpr int FQ = 10;

// Uniform model constants of one run, in the form the kernels use them.
struct Phys {
    float s_e, s_eps, s_q, s_nu;  // D2Q9 rates, Eq. (23)
    float zeta_e, zeta_nu;        // D2Q5 rates zeta_3, zeta_4, Eq. (37)
    float w5_0, w5_1;             // D2Q5 weights below Eq. (39)
    float varpi, csT2, inv_csT2;  // Eq. (34) parameter, c_sT^2, 1/c_sT^2
    float sig_s, dsig, isig_s;    // sigma(f_l) = sig_s + f_l dsig, 1/sig_s
    float lam_as, dlam;           // lambda alpha_e(f_l) = lam_as + f_l dlam
    float T_s, inv_St, inv_den;   // inv_den = 1 / (T_l - T_s + 1/St)
    float inv_dTm;                // 1 / (T_l - T_s)
    float gbeta, T0;              // buoyancy, Eq. (5)
    float fl_tol;
    int fl_maxit;
    float conv;                   // vartheta of Eq. (34)
    int zeta_uniform;             // 1 when zeta_alpha does not depend on f_l
    float zeta_a;                 // that uniform zeta_alpha
    float T_init;
    // literal variants of the thermal model (0 = the default readings)
    int sig_mode;                 // 1: sigma of each node from Eq. (7)
    float cps, cm;                // c_ps / c_pl, (rho c_p)_m / (rho c_pl)
    float Es, inv_den_c;          // c_ps T_s, 1 / (T_l + 1/St - c_ps T_s)
    int ke_mode;                  // 1: alpha_e = alpha_l k_e / k_l with k_e of Eq. (8)
    float ks, km, alpha_l;        // k_s / k_l, k_m / k_l, alpha_l
};

// Lattice geometry and boundary description.
struct Geom {
    int nx, ny, pitch;  // pitch: row stride in elements (multiple of 64)
    long long plane;    // elements per population plane = ny * pitch
    int per_x, per_y;   // periodic axes
    int wall_T[4];      // side x-, x+, y-, y+: 1 fixed temperature, 0 adiabatic
    float T_wall[4];
    int block_rows;     // rows of a step-kernel block (4 or 8)
    int cells_per_lane; // nodes per lane in the step kernel (1 or 2)
    // tiling of the step kernel (tiles of 64 x block_rows*cells_per_lane):
    // tiles per row, tiles in total, tiles per die, and the Granlund-
    // Montgomery magic (multiplier, shift) dividing a tile index by st_tx
    int st_tx, st_ntiles, st_per_xcd;
    uint32_t st_magic;
    int st_shift;
    int wide;           // 1: 64-bit addressing (arrays beyond a 4 GB window)
    int store;          // cache policy of the default step's stores (ST_*)
    int per_array;      // 1: the two-step kernel uses one buffer resource per array
    int st_rot;         // 1: rows of st_tx tiles, a multiple of 8: rotated tile groups
};

// Device buffers of one step (deviation populations for f).
struct StepBufs {
    const float* __restrict__ fin;
    float* __restrict__ fout;
    const float* __restrict__ gin;
    float* __restrict__ gout;
    const float* __restrict__ flin;
    float* __restrict__ flout;
    float* __restrict__ ux;        // u^{k+1} (ux plane, then the uy plane)
    float* __restrict__ uy;
    const float* __restrict__ uin; // u^k when it lives elsewhere; null: read ux/uy (in place)
    const float* __restrict__ eps;
    const float* __restrict__ Ac;  // phi nu_l / (K (1-phi)^2): Darcy coefficient
    const float* __restrict__ Bc;  // phi F_eps / (sqrt(K) (1-phi)): Forchheimer
    int* __restrict__ it_sum;      // enthalpy-iteration counters (counted mode)
    int* __restrict__ it_max;
    const float* __restrict__ r2f; // R2: f_l^{k+1} from the global iteration
    int r2_its;                    // R2: its sweeps
    // A window of device memory of fewer than 4 GB that holds every array
    // above, for kernels that address them all through one buffer resource
    // (null where they do not fit one); with a window pair, win holds the
    // arrays read (state k, the porous planes) and wout those written.
    const char* win = nullptr;
    const char* wout = nullptr;
    uint32_t win_bytes = 0, wout_bytes = 0;
};

// Sets G's tiling constants (st_*) for tiles of w x h nodes: tiles per row,
// in total and per die, and the magic number dividing a tile index by the
// tiles per row.
void set_tiling(Geom& G, int w, int h);

hipError_t launch_step(const Geom& G, const Phys& P, const StepBufs& B, bool flow,
                       bool counted, hipStream_t s);

// Two time steps in one launch (dmrt_step2.hip): reads the state in B's
// input buffers, writes the state two steps later into its output buffers
// (u double-buffered: B.uin holds u^k).  For the default thermal model,
// 32-bit offsets, the 4-row launch shape and one node per lane.
bool step2_supported(const Geom& G, const Phys& P);
// Two steps per launch: B's inputs hold state k, its outputs receive state
// k+2; with mid, its outputs receive state k+1 as well.
hipError_t launch_step2(const Geom& G, const Phys& P, const StepBufs& B, bool flow, hipStream_t s,
                        const StepBufs* mid = nullptr);

// One step with the latent source at the pre-stream site (R2): T* of every
// node (ts), at most P.fl_maxit Jacobi sweeps of f_l over the lattice
// (iterates in r2a / r2b; flags[j] = 1 when sweep j changed some f_l by more
// than P.fl_tol, and a sweep after an unchanged one does nothing), then the
// step kernel with the converged f_l.  ts, r2a, r2b: one plane each;
// flags: P.fl_maxit ints.
struct R2Bufs {
    float* ts;
    float* r2a;
    float* r2b;
    int* flags;
};
hipError_t launch_step_r2(const Geom& G, const Phys& P, const StepBufs& B, const R2Bufs& R,
                          bool flow, bool counted, hipStream_t s);

// One cavity of a batch: its lattice, its model constants, its uniform
// porous fields and the element offsets of its planes in the shared arenas.
struct Cavity {
    Geom G;
    Phys P;
    float eps, Ac, Bc, pad;
    unsigned long long f_off, g_off, fl_off, u_off;
};

// Arguments of one batched step (buffers of the current and next state).
struct BatchArgs {
    const Cavity* __restrict__ cav;
    const int4* __restrict__ tiles;  // (cavity, x0, y0, narrow): 64 x rows nodes, or
                                     // 32 x 2*rows nodes when narrow != 0
    int die[NXCD + 1];               // die d works on tiles [die[d], die[d + 1])
    const float* fin;
    float* fout;
    const float* gin;
    float* gout;
    const float* flin;
    float* flout;
    const float* uin;  // u^k (two planes per cavity at its u_off)
    float* uout;       // u^{k+1}, or u^{k+2} after two steps
    int store;  // cache policy of the state stores (ST_*)
    // the halves of the state arena that hold the arrays read and written
    // (f, g, f_l, u of one parity each), when a half is under 4 GB; else
    // win_bytes is 0
    const char* win;
    const char* wout;
    uint32_t win_bytes;
    int uniform_thermal;  // 1: every cavity has sigma_s = sigma_l, one tau_T and walls
                          // on every side
};

// Persistent batched step: `blocks` blocks (a multiple of 8) of 64 x rows
// lanes; the blocks of die d walk that die's part of the tile list.
hipError_t launch_batch_step(const BatchArgs& a, int rows, int blocks, hipStream_t s);
// Two steps per launch over a list of two-step tiles (a.tiles, a.die): one
// block per tile, `blocks` = 8 x the largest part of a die.
hipError_t launch_batch_step2(const BatchArgs& a, int blocks, hipStream_t s);
// Two-step tiles: pass-B width and rows; returns the waves of a block.
int batch_step2_tile(int* width, int* rows, int* narrow_width = nullptr, int* narrow_rows = nullptr);
// Blocks of 64 x rows lanes that fit on one compute unit at once.
int batch_blocks_per_cu(int rows);
// Per-cavity partial counts of liquid nodes (f_l > 0) and of non-finite f_l
// and g values: partials[2 * (cavity * nblk + block) + {0, 1}].
hipError_t launch_batch_count(const Cavity* cav, int ncav, const float* fl, const float* g,
                              long long* partials, int nblk, hipStream_t s);

// Buffers of one reversed step k+1 -> k of the discrete adjoint.  A state
// snapshot is ADJ_STATE planes: f (FQ), g (5), f_l, u_x, u_y.
constexpr int ADJ_STATE = FQ + 5 + 1 + 2;
constexpr int ADJ_LS = 18;  // state adjoint: d+ (9), rho - 1, g+ (5), f_l, u (2)
constexpr int ADJ_LA = 32;  // local adjoints of one receiving node (double-buffered)
constexpr int ADJ_GA = 3;   // accumulated adjoints of porosity, Ac, Bc
struct AdjBufs {
    const float* f0;   // state k
    const float* g0;
    const float* fl0;
    const float* u0;
    const float* fl1;  // f_l^{k+1}
    const float* eps;
    const float* Ac;
    const float* Bc;
    const float* fl2;  // f_l^{k+2} (unused by the first reversed step)
    const float* ls;   // terminal adjoint (first reversed step only)
    const float* la_prev;  // local adjoints of step k+1
    float* la;         // local adjoints of step k
    float* ga;         // accumulators
};
hipError_t launch_adjoint_step(const Geom& G, const Phys& P, const AdjBufs& B, bool flow,
                               bool first, hipStream_t s);
// Terminal state adjoint from packed dL/dT, dL/df_l (either may be null).
hipError_t launch_adjoint_terminal(const Geom& G, const float* dT, const float* dfl, float* ls,
                                   hipStream_t s);
// Packed gradients with respect to log K and porosity from the accumulators.
hipError_t launch_adjoint_grads(const Geom& G, const float* ga, const float* eps, const float* Ac,
                                const float* Bc, bool ergun, float* gk, float* ge, hipStream_t s);

// Load a pre-collision state (planar, row stride nx; any of f/g/fl may be
// null) and store its post-collision populations into the current buffers.
// eps/Ac/Bc may be null: the lattice then has the uniform values eps_u,
// Ac_u, Bc_u.
hipError_t launch_load_state(const Geom& G, const Phys& P, const float* f_pre,
                             const float* g_pre, const float* fl_pre, float* fcur,
                             float* gcur, float* flcur, float* ux, float* uy,
                             const float* eps, const float* Ac, const float* Bc,
                             bool flow, hipStream_t s, float eps_u = 0.0f, float Ac_u = 0.0f,
                             float Bc_u = 0.0f);

// dst[0..n) = src[0..n) (a kernel, so that it can be captured in a graph).
hipError_t launch_copy(float* dst, const float* src, size_t n, hipStream_t s);

// T, ux, uy, f_l into out[4][ny][nx].
hipError_t launch_fields(const Geom& G, const float* gcur, const float* flcur,
                         const float* ux, const float* uy, bool flow, float* out,
                         hipStream_t s);

// Full post-collision populations into fpost[9][ny][nx], gpost[5][ny][nx].
hipError_t launch_populations(const Geom& G, const float* fcur, const float* gcur,
                              const float* flcur, bool flow, float* fpost, float* gpost,
                              hipStream_t s);

constexpr int DIAG_SLOTS = 8;  // doubles per block partial
hipError_t launch_diag(const Geom& G, const Phys& P, const float* fcur, const float* gcur,
                       const float* flcur, const float* ux, const float* uy,
                       const float* eps, bool flow, double* partials, int* nblocks,
                       hipStream_t s);
hipError_t launch_front(const Geom& G, const float* flcur, float* front, hipStream_t s);
// res[0..7] = the block partials of launch_diag summed (slot 4: max) in block
// order, res[8] = the sum of the ny row fronts, res[9] = their max: the
// host-side reduction of dmrt_diag, in the same order, on the device.
hipError_t launch_diag_reduce(const double* partials, int nblocks, const float* front, int ny,
                              double* res, hipStream_t s);

}  // namespace dmrtk
