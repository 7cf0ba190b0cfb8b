// Two time steps of the double-MRT lattice Boltzmann phase-change model
// (Liu & He, arXiv:1503.08406) in one launch on a single lattice, for gfx950:
// the tiles of dmrt_tile2.h over the whole lattice.
#include "dmrt_tile2.h"

namespace dmrtk {
namespace {

// Tiles numbered row-major; blocks are handed to the dies round-robin and
// die d takes a contiguous run of tiles, so neighbouring tiles (which share
// their ring of nodes and the rows they pull from) run on the same die.  The
// tile of a block comes from host-computed constants (no division on the
// device).
// ILV: tile rows interleaved over the dies instead (die d takes rows d,
// d + 8, d + 16, ...; G.st_ntiles then counts tile rows).  Contiguous runs
// keep the rows two tiles share in one die's L2; on wide lattices, whose
// tile rows overflow it anyway, the interleaved rows measured faster
// (launch_io2 picks by tiles per row).  ROT: each die's tiles taken in
// the rotated groups of rotated_tile (rows of tiles a multiple of 8 long).
// MID: the state k+1 is stored too, into the arrays of B1 (recorded runs).
// UT: compiled for the cavity form (launch_io2 checks it): uniform thermal
// properties (sigma_s = sigma_l and one tau_T), without the per-node
// relaxation rate and 1/sigma of the general case, and walls on every side,
// with neighbour offsets one column or row away: the same values, fewer
// instructions.
// With one buffer resource for all arrays (WinIOT) the kernel is compiled
// for 7 waves per SIMD, which fits its scalar registers into 94 with the
// same few spills as without the bound: measured 3-7 % faster than the
// unbounded build (106 scalar registers), the liquid-started lattice
// unchanged; a bound of 8 spills 33 and is slower where flow dominates.
template <class IO, bool FLOW, int NW, bool MID, bool ILV, bool ROT = false, bool UT = false>
__global__ __launch_bounds__(TX * NW) __attribute__((amdgpu_waves_per_eu(InWindow<IO>::value ? 7 : 1)))
void k_step2(Geom G, Phys P, StepBufs B, StepBufs B1)
{
    __shared__ float tl[TPLANES * NW * TX];
    int x0, y0;
    // G's tiling constants are those of the tiles of this kernel
    if (ROT && !ILV) {
        const int d = (int)(blockIdx.x & (NXCD - 1)), first = d * G.st_per_xcd;
        const int j = (int)(blockIdx.x >> 3), n = min(G.st_per_xcd, G.st_ntiles - first);
        if (j >= n) return;  // the whole block
        const uint32_t tile = (uint32_t)(first + rotated_tile(j, n));
        const uint32_t hi = __umulhi(tile, G.st_magic);
        const uint32_t qd = (hi + ((tile - hi) >> 1)) >> ((uint32_t)(G.st_shift - 1) & 31u);
        const uint32_t q = G.st_shift == 0 ? tile : qd;
        x0 = (int)(tile - q * (uint32_t)G.st_tx) * T2_W;
        y0 = (int)q * (NW - 2);
    } else if (ILV) {
        const uint32_t b = blockIdx.x, d = b & (NXCD - 1);
        uint32_t j = b >> 3;
        if (ROT) {
            // the die's rows d, d + 8, ...: a prefix of its index range
            const int n = ((G.st_ntiles - (int)d + NXCD - 1) / NXCD) * G.st_tx;
            if ((int)j >= n) return;  // the whole block
            j = (uint32_t)rotated_tile((int)j, n);
        }
        const uint32_t hi = __umulhi(j, G.st_magic);
        const uint32_t qd = (hi + ((j - hi) >> 1)) >> ((uint32_t)(G.st_shift - 1) & 31u);
        const uint32_t rd = G.st_shift == 0 ? j : qd;  // the die's row of tiles
        const uint32_t row = rd * NXCD + d;
        if (row >= (uint32_t)G.st_ntiles) return;  // the whole block
        x0 = (int)(j - rd * (uint32_t)G.st_tx) * T2_W;
        y0 = (int)row * (NW - 2);
    } else if (!step_tile_origin<NW - 2, T2_W>(G, x0, y0)) {
        return;  // the whole block
    }
    const Arrays<IO> A(G, B);
    if (MID) {
        const Arrays<IO> A1(G, B1);
        tile_step2<IO, FLOW, NW, false, true, TX, UT>(G, P, B, A, x0, y0, tl, &A1);
    } else {
        tile_step2<IO, FLOW, NW, false, false, TX, UT>(G, P, B, A, x0, y0, tl);
    }
}

template <class IO, bool FLOW, bool UT>
hipError_t launch_tiles2(const Geom& Gt, const Phys& P, const StepBufs& B, const StepBufs* mid,
                         bool ilv, bool rot, hipStream_t s)
{
    constexpr int NW = T2_WAVES;
    const dim3 grd(NXCD * Gt.st_per_xcd), blk(TX, NW);
    if (rot && ilv)
        hipLaunchKernelGGL((k_step2<IO, FLOW, NW, false, true, true, UT>), grd, blk, 0, s, Gt, P, B, B);
    else if (rot)
        hipLaunchKernelGGL((k_step2<IO, FLOW, NW, false, false, true, UT>), grd, blk, 0, s, Gt, P, B, B);
    else if (mid && ilv)
        hipLaunchKernelGGL((k_step2<IO, FLOW, NW, true, true, false, UT>), grd, blk, 0, s, Gt, P, B, *mid);
    else if (mid)
        hipLaunchKernelGGL((k_step2<IO, FLOW, NW, true, false, false, UT>), grd, blk, 0, s, Gt, P, B, *mid);
    else if (ilv)
        hipLaunchKernelGGL((k_step2<IO, FLOW, NW, false, true, false, UT>), grd, blk, 0, s, Gt, P, B, B);
    else
        hipLaunchKernelGGL((k_step2<IO, FLOW, NW, false, false, false, UT>), grd, blk, 0, s, Gt, P, B, B);
    return hipGetLastError();
}

template <class IO, bool FLOW>
hipError_t launch_io2(const Geom& G, const Phys& P, const StepBufs& B, const StepBufs* mid,
                      hipStream_t s)
{
    Geom Gt = G;
    set_tiling(Gt, T2_W, T2_WAVES - 2);
    // rows interleaved over the dies from 48 tiles per row (lattices about
    // 3000 nodes wide and more; measured at 1024-6144 nodes)
    const bool ilv = Gt.st_tx >= 48;
    if (ilv) {
        Gt.st_ntiles /= Gt.st_tx;  // tile rows
        Gt.st_per_xcd = (Gt.st_ntiles + NXCD - 1) / NXCD * Gt.st_tx;
    }
    // rows of tiles a multiple of 8 long: rotated groups (flow runs only)
    const bool rot = FLOW && !mid && Gt.st_tx % 8 == 0;
    if (P.zeta_uniform && P.dsig == 0.0f && !G.per_x && !G.per_y)
        return launch_tiles2<IO, FLOW, true>(Gt, P, B, mid, ilv, rot, s);
    return launch_tiles2<IO, FLOW, false>(Gt, P, B, mid, ilv, rot, s);
}

}  // namespace

bool step2_supported(const Geom& G, const Phys& P)
{
    return !G.wide && G.block_rows == 4 && G.cells_per_lane == 1 && !P.sig_mode && !P.ke_mode;
}

namespace {

// Sets the window of B (and of mid, the same one) when every array of the
// launch lies within 4 GB of the lowest; false otherwise.
bool set_window(const Geom& G, StepBufs& B, StepBufs* mid)
{
    const uint64_t pb = (uint64_t)G.plane * 4u;
    struct Span {
        const void* p;
        uint64_t n;
    };
    const Span in[] = {{B.fin, FQ * pb},  {B.fout, FQ * pb}, {B.gin, 5 * pb},
                       {B.gout, 5 * pb},  {B.flin, pb},      {B.flout, pb},
                       {B.ux, 2 * pb},    {B.uin ? B.uin : B.ux, 2 * pb}, {B.eps, 3 * pb}};
    uint64_t lo = ~0ull, hi = 0;
    auto add = [&](const void* p, uint64_t n) {
        const uint64_t a = (uint64_t)(uintptr_t)p;
        lo = a < lo ? a : lo;
        hi = a + n > hi ? a + n : hi;
    };
    for (const Span& sp : in) add(sp.p, sp.n);
    if (mid) {
        add(mid->fout, FQ * pb);
        add(mid->gout, 5 * pb);
        add(mid->flout, pb);
        add(mid->ux, 2 * pb);
    }
    if (hi - lo >= (1ull << 32)) return false;
    B.win = (const char*)(uintptr_t)lo;
    B.win_bytes = (uint32_t)(hi - lo);
    if (mid) {
        mid->win = B.win;
        mid->win_bytes = B.win_bytes;
    }
    return true;
}

template <int SP>
using WinIO1 = WinIOT<SP, false>;

template <template <int> class IOT>
hipError_t launch_policy(const Geom& G, const Phys& P, const StepBufs& B, bool flow,
                         hipStream_t s, const StepBufs* mid)
{
    if (G.store == ST_WT)
        return flow ? launch_io2<IOT<ST_WT>, true>(G, P, B, mid, s)
                    : launch_io2<IOT<ST_WT>, false>(G, P, B, mid, s);
    if (G.store == ST_NT)
        return flow ? launch_io2<IOT<ST_NT>, true>(G, P, B, mid, s)
                    : launch_io2<IOT<ST_NT>, false>(G, P, B, mid, s);
    return flow ? launch_io2<IOT<ST_PLAIN>, true>(G, P, B, mid, s)
                : launch_io2<IOT<ST_PLAIN>, false>(G, P, B, mid, s);
}

}  // namespace

hipError_t launch_step2(const Geom& G, const Phys& P, const StepBufs& B, bool flow, hipStream_t s,
                        const StepBufs* mid)
{
    StepBufs Bw = B, Mw;
    if (mid) Mw = *mid;
    if (!G.per_array && set_window(G, Bw, mid ? &Mw : nullptr))
        return launch_policy<WinIO1>(G, P, Bw, flow, s, mid ? &Mw : nullptr);
    return launch_policy<BufIOT>(G, P, B, flow, s, mid);
}

}  // namespace dmrtk
