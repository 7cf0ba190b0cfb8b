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

template <class IO, bool FLOW, bool COUNT, int TYB, int CPT>
__global__ __launch_bounds__(TX * TYB) void k_step(Geom G, Phys P, StepBufs B)
{
    // a tile of 64 x (TYB * CPT) nodes
    int x0, y0;
    if (!step_tile_origin<TYB * CPT>(G, x0, y0)) return;
    const Arrays<IO> A(G, B);
    const int x = x0 + (int)threadIdx.x;
    if (CPT == 1) {
        // one node per lane, flow work gathered onto the lowest lanes
        __shared__ FlowStage<TX * TYB> S;
        const int y = y0 + (int)threadIdx.y;
        block_step<IO, FLOW, COUNT, false, TX * TYB>(G, P, B, A, x, y, x < G.nx && y < G.ny, S, 0);
        return;
    }
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
        if (ok[j]) node_finish<IO, FLOW, COUNT>(G, P, B, A, n[j]);
}

template <class IO, bool FLOW, bool COUNT>
hipError_t launch_rows(const Geom& G, const Phys& P, const StepBufs& B, hipStream_t s)
{
    const int rows = G.block_rows, cpt = G.cells_per_lane;
    const dim3 grd(NXCD * G.st_per_xcd);
    if (rows == 8 && cpt == 2)
        hipLaunchKernelGGL((k_step<IO, FLOW, COUNT, 8, 2>), grd, dim3(TX, 8), 0, s, G, P, B);
    else if (rows == 8)
        hipLaunchKernelGGL((k_step<IO, FLOW, COUNT, 8, 1>), grd, dim3(TX, 8), 0, s, G, P, B);
    else if (cpt == 2)
        hipLaunchKernelGGL((k_step<IO, FLOW, COUNT, 4, 2>), grd, dim3(TX, 4), 0, s, G, P, B);
    else
        hipLaunchKernelGGL((k_step<IO, FLOW, COUNT, 4, 1>), grd, dim3(TX, 4), 0, s, G, P, B);
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

}  // namespace

hipError_t launch_step(const Geom& G, const Phys& P, const StepBufs& B, bool flow, bool counted,
                       hipStream_t s)
{
    if (G.wide) return launch_io<PtrIO>(G, P, B, flow, counted, s);
    return launch_io<BufIO>(G, P, B, flow, counted, s);
}

}  // namespace dmrtk
