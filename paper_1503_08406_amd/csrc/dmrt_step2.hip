// Two time steps of the double-MRT lattice Boltzmann phase-change model
// (Liu & He, arXiv:1503.08406) in one launch on a single lattice, for gfx950:
// the tiles of dmrt_tile2.h over the whole lattice.
#include "dmrt_tile2.h"

namespace dmrtk {
namespace {

// Tiles numbered row-major; blocks are handed to the dies round-robin and
// die d takes a contiguous run of tiles, so neighbouring tiles (which share
// their ring of nodes and the rows they pull from) run on the same die.
// MID: the state k+1 is stored too, into the arrays of B1 (recorded runs).
template <class IO, bool FLOW, int NW, bool MID>
__global__ __launch_bounds__(TX * NW) void k_step2(Geom G, Phys P, StepBufs B, StepBufs B1)
{
    constexpr int RB = NW - 2;
    __shared__ float tl[TPLANES * NW * TX];
    const int nsx = (G.nx + T2_W - 1) / T2_W;
    const int ntiles = nsx * ((G.ny + RB - 1) / RB);
    const int per = (ntiles + NXCD - 1) / NXCD;
    const int b = (int)blockIdx.x;
    const int tile = (b % NXCD) * per + b / NXCD;
    if (tile >= ntiles) return;  // the whole block: no barrier is left waiting
    const Arrays<IO> A(G, B);
    const int x0 = (tile % nsx) * T2_W, y0 = (tile / nsx) * RB;
    if (MID) {
        const Arrays<IO> A1(G, B1);
        tile_step2<IO, FLOW, NW, false, true>(G, P, B, A, x0, y0, tl, &A1);
    } else {
        tile_step2<IO, FLOW, NW, false>(G, P, B, A, x0, y0, tl);
    }
}

template <class IO, bool FLOW>
hipError_t launch_io2(const Geom& G, const Phys& P, const StepBufs& B, const StepBufs* mid,
                      hipStream_t s)
{
    constexpr int NW = T2_WAVES;
    const int nsx = (G.nx + T2_W - 1) / T2_W;
    const int ntiles = nsx * ((G.ny + NW - 3) / (NW - 2));
    const dim3 grd(NXCD * ((ntiles + NXCD - 1) / NXCD));
    if (mid)
        hipLaunchKernelGGL((k_step2<IO, FLOW, NW, true>), grd, dim3(TX, NW), 0, s, G, P, B, *mid);
    else
        hipLaunchKernelGGL((k_step2<IO, FLOW, NW, false>), grd, dim3(TX, NW), 0, s, G, P, B, B);
    return hipGetLastError();
}

}  // namespace

bool step2_supported(const Geom& G, const Phys& P)
{
    return !G.wide && G.block_rows == 4 && G.cells_per_lane == 1 && !P.sig_mode && !P.ke_mode;
}

hipError_t launch_step2(const Geom& G, const Phys& P, const StepBufs& B, bool flow, hipStream_t s,
                        const StepBufs* mid)
{
    if (G.store == ST_WT)
        return flow ? launch_io2<BufIOT<ST_WT>, true>(G, P, B, mid, s)
                    : launch_io2<BufIOT<ST_WT>, false>(G, P, B, mid, s);
    if (G.store == ST_NT)
        return flow ? launch_io2<BufIOT<ST_NT>, true>(G, P, B, mid, s)
                    : launch_io2<BufIOT<ST_NT>, false>(G, P, B, mid, s);
    return flow ? launch_io2<BufIO, true>(G, P, B, mid, s) : launch_io2<BufIO, false>(G, P, B, mid, s);
}

}  // namespace dmrtk
