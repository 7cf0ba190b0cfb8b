// The fused time step of the double-MRT lattice Boltzmann phase-change model
// (Liu & He, arXiv:1503.08406) for gfx950.  One launch = one time step; one
// lane owns one node (or two, rows apart, with cells_per_lane = 2).
//
// Per node, with start-of-step state (post-collision populations f+, g+ of
// step k, liquid fraction f_l^k, the node's own velocity u^k):
//   1. pull g_i(x) = g+_i(x - e_i) (Eq. 36); a wall source gives
//      g_i^eq(T_w, 0) + g+_i(x) - g_i^eq(T^k(x), u^k(x)).
//   2. iterate the enthalpy update (Eqs. 38, 40-42) to f_l^{k+1}, T^{k+1} and
//      add the latent source w~_i S~_0 to g (Eq. 38 through N^-1).
//   3. where f_l^{k+1} > 0: pull f_i(x) = f+_i(x - e_i) from liquid sources;
//      a wall or solid source gives f_i^eq(rho, 0) + f+_i(x) - f_i^eq(rho,
//      u^k; varphi^k) (rho cancels); a node that just melted restarts at
//      rest at the mean density of its liquid neighbours; then the closure
//      and the MRT collision with forcing.
//   4. D2Q5 MRT collision, store f+, g+, f_l^{k+1}, u^{k+1}.
//
// Memory phases of a block of 64 x rows nodes: every lane issues its first
// batch (f_l^k, porosity, the five g pulls; a wall node also its own g+ and
// u^k) and finishes the thermal part; the nodes whose flow is solved are
// then handed to the lowest lanes of the block, which issue all their flow
// loads in one batch (neighbour f_l, f pulls, own f+, u^k; or neighbour
// f_l and rho - 1 for a node that just melted), so a wavefront never waits
// behind a data-dependent load; last, the thermal collision and stores.
#include "dmrt_node.h"

namespace dmrtk {
namespace {

template <class IO, bool FLOW, bool COUNT, int TYB, int CPT, int TM>
__global__ __launch_bounds__(TX * TYB) void k_step(Geom G, Phys P, StepBufs B)
{
    // a tile of 64 x (TYB * CPT) nodes
    int x0 = 0, y0 = 0;
    const bool tile = step_tile_origin<TYB * CPT, TX, true>(G, x0, y0);
    const Arrays<IO> A(G, B);
    const int x = x0 + (int)threadIdx.x;
    if (CPT == 1) {
        // one node per lane, flow work gathered onto the lowest lanes.  A
        // block past the last tile runs with no valid lane rather than
        // returning early: with no branch before it, the compiler issues all
        // kernel-argument loads at once instead of in dependent rounds.
        __shared__ FlowStage<TX * TYB> S;
        const int y = y0 + (int)threadIdx.y;
        block_step<IO, FLOW, COUNT, false, TX * TYB, TM>(G, P, B, A, x, y,
                                                         tile && x < G.nx && y < G.ny, S, 0);
        return;
    }
    if (!tile) return;
    // CPT nodes per lane, TYB rows apart: the first load batch of all of
    // them is issued before any is finished
    Node<IO> n[CPT];
    bool ok[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int y = y0 + (int)threadIdx.y + j * TYB;
        ok[j] = x < G.nx && y < G.ny;
        if (ok[j]) node_load<IO, FLOW>(G, A, x, y, n[j]);
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j)
        if (ok[j]) node_finish<IO, FLOW, COUNT, false, TM>(G, P, B, A, n[j]);
}

template <class IO, bool FLOW, bool COUNT>
hipError_t launch_rows(const Geom& G, const Phys& P, const StepBufs& B, hipStream_t s)
{
    const int rows = G.block_rows, cpt = G.cells_per_lane;
    const dim3 grd(NXCD * G.st_per_xcd);
    if (P.sig_mode || P.ke_mode) {
        // the thermal-model variants: one node per lane, rows of the tiling
        if (rows == 8)
            hipLaunchKernelGGL((k_step<IO, FLOW, COUNT, 8, 1, TM_VARIANT>), grd, dim3(TX, 8), 0, s,
                               G, P, B);
        else
            hipLaunchKernelGGL((k_step<IO, FLOW, COUNT, 4, 1, TM_VARIANT>), grd, dim3(TX, 4), 0, s,
                               G, P, B);
    } else if (rows == 8 && cpt == 2)
        hipLaunchKernelGGL((k_step<IO, FLOW, COUNT, 8, 2, TM_DEFAULT>), grd, dim3(TX, 8), 0, s, G, P, B);
    else if (rows == 8)
        hipLaunchKernelGGL((k_step<IO, FLOW, COUNT, 8, 1, TM_DEFAULT>), grd, dim3(TX, 8), 0, s, G, P, B);
    else if (cpt == 2)
        hipLaunchKernelGGL((k_step<IO, FLOW, COUNT, 4, 2, TM_DEFAULT>), grd, dim3(TX, 4), 0, s, G, P, B);
    else
        hipLaunchKernelGGL((k_step<IO, FLOW, COUNT, 4, 1, TM_DEFAULT>), grd, dim3(TX, 4), 0, s, G, P, B);
    return hipGetLastError();
}

template <class IO>
hipError_t launch_io(const Geom& G, const Phys& P, const StepBufs& B, bool flow, bool counted,
                     hipStream_t s)
{
    if (flow)
        return counted ? launch_rows<IO, true, true>(G, P, B, s)
                       : launch_rows<IO, true, false>(G, P, B, s);
    return counted ? launch_rows<IO, false, true>(G, P, B, s)
                   : launch_rows<IO, false, false>(G, P, B, s);
}

// ---------------------------------------------------------------------------
// Latent source at the pre-stream site (R2).  The source N^-1 S~ of Eq. (30)
// is added to the post-collision populations of x before they stream, so
// node y receives w~_i S~_0(y - e_i) through each pull, and S~_0 of a node
// needs its own f_l^{k+1} (Eq. 38): the f_l of all nodes are coupled.  The
// step becomes
//   k_r2_pre:   T*(y) = sum_i g_i(y) of the pulled populations (Eq. 36 with
//               the wall sources), for every node;
//   k_r2_sweep: Jacobi sweeps f^{j+1}(y) = f_l(T(En)) (Eqs. 40-42) with
//               T = T*(y) + w~_0 S~_0(y; f^j) + sum_i w~_i S~_0(y - e_i; f^j),
//               starting from f^0 = f_l^k, until no node changes by more
//               than the tolerance (at most fl_maxit sweeps; a sweep after
//               an unchanged one returns at once);
//   k_step<TM_R2>: the step with the converged f_l^{k+1}.
// ---------------------------------------------------------------------------
template <class IO, bool FLOW>
__global__ __launch_bounds__(TX * TY) void k_r2_pre(Geom G, Phys P, StepBufs B, R2Bufs R)
{
    if (blockIdx.x == 0) {
        const int tid = (int)(threadIdx.y * TX + threadIdx.x);
        for (int j = tid; j < P.fl_maxit; j += TX * TY) R.flags[j] = 0;
    }
    int x, y;
    if (!tile_coords<TY>(G, x, y)) return;
    const Arrays<IO> A(G, B);
    Node<IO> n;
    node_load<IO, FLOW>(G, A, x, y, n);
    float sg0, dsg;
    node_sigma<true>(P, n.eps, sg0, dsg);
    node_wall_g<IO, FLOW>(G, P, n, sg0, dsg);
    R.ts[(size_t)y * G.pitch + x] = n.g[0] + ((n.g[1] + n.g[3]) + (n.g[2] + n.g[4]));
}

template <class IO>
__global__ __launch_bounds__(TX * TY) void k_r2_sweep(Geom G, Phys P, StepBufs B, R2Bufs R, int j)
{
    if (j > 0 && R.flags[j - 1] == 0) return;  // converged in an earlier sweep
    int x, y;
    const bool valid = tile_coords<TY>(G, x, y);
    bool changed = false;
    if (valid) {
        using off_t = typename IO::off_t;
        const off_t pb = (off_t)G.plane * 4u;
        const IO fj(j == 0 ? B.flin : ((j - 1) & 1) ? R.r2b : R.r2a, pb);
        const IO fk(B.flin, pb), st(B.eps, pb);
        Node<IO> n;
        node_geometry(G, x, y, n);
        const off_t src[4] = {n.o1, n.o2, n.o3, n.o4};
        float f1s[4], fks[4], es[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f1s[i] = fj.ld(src[i], 0);
            fks[i] = fk.ld(src[i], 0);
            es[i] = st.ld(src[i], 0);
        }
        const float f = fj.ld(n.o, 0), flk = fk.ld(n.o, 0), eps = st.ld(n.o, 0);
        const size_t c = (size_t)y * G.pitch + x;
        float T = R.ts[c] + P.w5_0 * latent_S0<true>(P, eps, flk, f);
        float side = 0.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) side += latent_S0<true>(P, es[i], fks[i], f1s[i]);
        T += P.w5_1 * side;
        float fn;
        if (P.sig_mode) {
            const float En = (P.cps + f * (1.0f - P.cps)) * T + f * P.inv_St;
            fn = fminf(fmaxf((En - P.Es) * P.inv_den_c, 0.0f), 1.0f);
        } else {
            fn = fminf(fmaxf((T + f * P.inv_St - P.T_s) * P.inv_den, 0.0f), 1.0f);
        }
        ((j & 1) ? R.r2b : R.r2a)[c] = fn;
        changed = fabsf(fn - f) > P.fl_tol;
    }
    if (__ballot(changed) != 0ull && threadIdx.x == 0) R.flags[j] = 1;
}

// The converged iterate: sweep j* is the first that changed nothing (or the
// last one), and it wrote r2a when j* is even.
template <class IO, bool FLOW, bool COUNT, int TYB>
__global__ __launch_bounds__(TX * TYB) void k_step_r2(Geom G, Phys P, StepBufs B, R2Bufs R)
{
    int js = P.fl_maxit - 1;
    for (int j = 0; j < P.fl_maxit; ++j)
        if (R.flags[j] == 0) {
            js = j;
            break;
        }
    B.r2f = (js & 1) ? R.r2b : R.r2a;
    B.r2_its = js + 1;
    int x0, y0;
    if (!step_tile_origin<TYB, TX, true>(G, x0, y0)) return;
    const Arrays<IO> A(G, B);
    const int x = x0 + (int)threadIdx.x;
    __shared__ FlowStage<TX * TYB> S;
    const int y = y0 + (int)threadIdx.y;
    block_step<IO, FLOW, COUNT, false, TX * TYB, TM_R2>(G, P, B, A, x, y, x < G.nx && y < G.ny, S,
                                                        0);
}

template <class IO, bool FLOW, bool COUNT>
hipError_t launch_r2(const Geom& G, const Phys& P, const StepBufs& B, const R2Bufs& R,
                     hipStream_t s)
{
    const dim3 aux(tile_blocks(G, TY));
    hipLaunchKernelGGL((k_r2_pre<IO, FLOW>), aux, dim3(TX, TY), 0, s, G, P, B, R);
    for (int j = 0; j < P.fl_maxit; ++j)
        hipLaunchKernelGGL((k_r2_sweep<IO>), aux, dim3(TX, TY), 0, s, G, P, B, R, j);
    const dim3 grd(NXCD * G.st_per_xcd);
    if (G.block_rows == 8)
        hipLaunchKernelGGL((k_step_r2<IO, FLOW, COUNT, 8>), grd, dim3(TX, 8), 0, s, G, P, B, R);
    else
        hipLaunchKernelGGL((k_step_r2<IO, FLOW, COUNT, 4>), grd, dim3(TX, 4), 0, s, G, P, B, R);
    return hipGetLastError();
}

template <class IO>
hipError_t launch_r2_io(const Geom& G, const Phys& P, const StepBufs& B, const R2Bufs& R,
                        bool flow, bool counted, hipStream_t s)
{
    if (flow)
        return counted ? launch_r2<IO, true, true>(G, P, B, R, s)
                       : launch_r2<IO, true, false>(G, P, B, R, s);
    return counted ? launch_r2<IO, false, true>(G, P, B, R, s)
                   : launch_r2<IO, false, false>(G, P, B, R, s);
}

}  // namespace

namespace {
// The default shape (4 rows, one node per lane) with a store cache policy.
template <class IO>
hipError_t launch_hinted(const Geom& G, const Phys& P, const StepBufs& B, bool flow, bool counted,
                         hipStream_t s)
{
    const dim3 grd(NXCD * G.st_per_xcd), blk(TX, 4);
    if (flow && counted)
        hipLaunchKernelGGL((k_step<IO, true, true, 4, 1, TM_DEFAULT>), grd, blk, 0, s, G, P, B);
    else if (flow)
        hipLaunchKernelGGL((k_step<IO, true, false, 4, 1, TM_DEFAULT>), grd, blk, 0, s, G, P, B);
    else if (counted)
        hipLaunchKernelGGL((k_step<IO, false, true, 4, 1, TM_DEFAULT>), grd, blk, 0, s, G, P, B);
    else
        hipLaunchKernelGGL((k_step<IO, false, false, 4, 1, TM_DEFAULT>), grd, blk, 0, s, G, P, B);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_step(const Geom& G, const Phys& P, const StepBufs& B, bool flow, bool counted,
                       hipStream_t s)
{
    const bool dflt = G.block_rows == 4 && G.cells_per_lane == 1 && !P.sig_mode && !P.ke_mode;
    if (G.wide) {
        // arrays past 4 GB never fit the Infinity Cache: streaming stores
        if (dflt && G.store == ST_NT) return launch_hinted<PtrIOT<ST_NT>>(G, P, B, flow, counted, s);
        return launch_io<PtrIO>(G, P, B, flow, counted, s);
    }
    if (dflt && G.store == ST_WT) return launch_hinted<BufIOT<ST_WT>>(G, P, B, flow, counted, s);
    if (dflt && G.store == ST_NT) return launch_hinted<BufIOT<ST_NT>>(G, P, B, flow, counted, s);
    return launch_io<BufIO>(G, P, B, flow, counted, s);
}

hipError_t launch_step_r2(const Geom& G, const Phys& P, const StepBufs& B, const R2Bufs& R,
                          bool flow, bool counted, hipStream_t s)
{
    if (G.wide) return launch_r2_io<PtrIO>(G, P, B, R, flow, counted, s);
    return launch_r2_io<BufIO>(G, P, B, R, flow, counted, s);
}

}  // namespace dmrtk
