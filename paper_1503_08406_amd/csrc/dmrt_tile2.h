// Two time steps of the double-MRT lattice Boltzmann phase-change model
// (Liu & He, arXiv:1503.08406) in one launch, for gfx950: the tile
// step shared by the single-lattice and the batched two-step kernels.
//
// A block of 64 x NW lanes owns a tile of 62 columns [x0, x0 + 62) and
// NW - 2 rows [y0, y0 + NW - 2).  Lane (lane, w) holds node
// (x0 - 1 + lane, y0 - 1 + w): the tile and a ring of one node around it,
// which the neighbouring tiles also compute.
//   pass A: every lane steps its node from k to k+1, reading the state in
//           memory, and leaves in LDS what the neighbours pull in the next
//           step (f+_1..8, rho - 1, g+_1..4, f_l);
//   pass B: after one barrier, the lanes of the tile (waves 1 .. NW-2,
//           lanes 1 .. 62) step the same node from k+1 to k+2, pulling from
//           LDS and keeping the node's own values in registers, and write the
//           state k+2 to memory.
// Both passes run the per-node step of one launch per step (dmrt_node.h: the
// enthalpy update, the flow part with its wall and solid extrapolation or
// restart, both collisions) with the same arithmetic, so one launch gives
// the bits of two single steps.  That holds because multiply-adds are fused
// within a source expression only (-ffp-contract=on): values that the second
// pass takes from the first in registers are rounded as the single step's
// values read back from memory are.  The intermediate state never leaves the
// chip; all NW rows of a tile load at once, so a block waits for memory
// twice per launch (the first load batch, then the flow loads) like a block
// of the single step.  The flow part runs in the node's own lane (no
// hand-over of work between lanes: it would cost barriers and the own
// values would have to follow the work).
#pragma once

#include "dmrt_node.h"

namespace dmrtk {
namespace {

constexpr int T2_W = 62;    // tile width (pass-B columns)
// Waves of a block: tile rows + 2 (a build-time knob; 8 measured best of
// 6 to 16).
#ifndef DMRT_T2_WAVES
#define DMRT_T2_WAVES 8
#endif
constexpr int T2_WAVES = DMRT_T2_WAVES;
constexpr int T2_ROWS = T2_WAVES - 2;
// LDS planes of a tile: f+_i at TF + i - 1 (i = 1..8), rho - 1, g+_i at
// TG + i - 1 (i = 1..4), f_l^{k+1}.
enum { TF = 0, TRHO = 8, TG = 9, TFL = 13, TPLANES = 14 };

// Coordinate of a pass-A node on an axis: wrapped on a periodic axis, out
// of the lattice (false) behind a wall.
__device__ __forceinline__ bool axis_node(int& v, int n, int periodic)
{
    if (v >= 0 && v < n) return true;
    if (!periodic) return false;
    v %= n;
    if (v < 0) v += n;
    return true;
}

// Tile slots of the sources x - e_i (i = 0..8) of the pass-B node at `slot`
// (R slots per tile row); a source behind a wall is the node's own slot.
template <int R>
__device__ __forceinline__ void tile_sources(const FlowWalls& W, int slot, int (&s)[9])
{
    s[0] = slot;
    s[1] = W.w[1] ? slot : slot - 1;
    s[2] = W.w[2] ? slot : slot - R;
    s[3] = W.w[3] ? slot : slot + 1;
    s[4] = W.w[4] ? slot : slot + R;
    s[5] = W.w[5] ? slot : slot - R - 1;
    s[6] = W.w[6] ? slot : slot - R + 1;
    s[7] = W.w[7] ? slot : slot + R + 1;
    s[8] = W.w[8] ? slot : slot + R - 1;
}

// Both steps of the tile at (x0, y0) for a block of 64 x NW lanes with the
// LDS planes `tl` (TPLANES x NW x 64 floats).  The lanes form rows of TWD:
// 64 (a wavefront per row, a tile of 62 x (NW - 2) nodes) or 32 (a
// wavefront spans two rows, a tile of 30 x (2 NW - 2) nodes, for a narrow
// last column of a lattice).  USTAT: uniform porous fields (A.eps_u,
// A.Ac_u, A.Bc_u) instead of the per-node planes.  MID: the tile's state
// k+1 is also stored, through A1 (its output arrays), with the stores of a
// single step.  UT: compiled for the cavity form, uniform thermal
// properties (zeta_alpha) and walls on every side (node_geometry).
template <class IO, bool FLOW, int NW, bool USTAT, bool MID = false, int TWD = TX, bool UT = false>
__device__ __forceinline__ void tile_step2(const Geom& G, const Phys& P, const StepBufs& B,
                                           const Arrays<IO>& A, int x0, int y0, float* tl,
                                           const Arrays<IO>* A1 = nullptr)
{
    using off_t = typename IO::off_t;
    static_assert(TWD == TX || TWD == TX / 2, "rows of 64 or 32 lanes");
    constexpr int PS = NW * TX;        // floats per plane
    constexpr int RB = PS / TWD - 2;   // pass-B rows
    const int yend = min(y0 + RB, G.ny);
    const off_t pb = A.pb;
    // lane (column) and row of this thread in the tile's lane grid
    const int tid = (int)threadIdx.y * TX + (int)threadIdx.x;
    const int lane = TWD == TX ? (int)threadIdx.x : tid % TWD;
    const int w = TWD == TX ? (int)threadIdx.y : tid / TWD;
    const int slot = tid;
    // the lanes of the tile (pass B), where (xa, ya) below is (xb, yb)
    const int xb = x0 - 1 + lane, yb = y0 - 1 + w;
    const bool vb = w >= 1 && w <= RB && lane >= 1 && lane <= TWD - 2 && xb < G.nx && yb < yend;

    // ---- pass A: step k -> k+1 of the tile and its ring (rows y0-1 .. yend)
    int xa = x0 - 1 + lane, ya = y0 - 1 + w;
    bool va = ya <= yend;
    va = va && axis_node(xa, G.nx, G.per_x);
    va = va && axis_node(ya, G.ny, G.per_y);
    Node<IO> n;
    float T1 = 0.0f, fl1 = 0.0f, isig1 = 0.0f, ux = 0.0f, uy = 0.0f;
    float f0 = 0.0f, Ac = 0.0f, Bc = 0.0f;  // f+_0 and drag of a flow node
    n.eps = 0.0f;
    n.g[0] = 0.0f;
    // first load batch at raised wave priority (as in block_step)
    __builtin_amdgcn_s_setprio(2);
    if (va) {
        node_load<IO, FLOW, USTAT, UT>(G, A, xa, ya, n);
        __builtin_amdgcn_s_setprio(0);
        node_enthalpy<IO, FLOW, false, TM_DEFAULT, UT>(G, P, B, A, n, T1, fl1, isig1);
        if (FLOW && fl1 > 0.0f) {
            float d[9];
            off_t o;
            node_flow_core<IO, USTAT, UT>(G, P, A, xa, ya, n.flk, fl1, T1, n.eps, d, ux, uy, o, Ac,
                                      Bc);
#pragma unroll
            for (int i = 1; i < 9; ++i) tl[(TF + i - 1) * PS + slot] = d[i];
            tl[TRHO * PS + slot] = rho_dev(d);
            f0 = d[0];
            if (MID && vb) {
#pragma unroll
                for (int i = 0; i < 9; ++i) A1->fout.st(o, (off_t)i * pb, d[i]);
                A1->fout.st(o, 9 * pb, rho_dev(d));
                A1->uv.st(o, 0, ux);
                A1->uv.st(o, pb, uy);
            }
        }
        thermal_collide<false, UT>(n.g, fl1, isig1, T1, ux, uy, n.eps, P);
#pragma unroll
        for (int i = 1; i < 5; ++i) tl[(TG + i - 1) * PS + slot] = n.g[i];
        tl[TFL * PS + slot] = fl1;
        if (MID && vb) {
            const off_t o = n.o;
#pragma unroll
            for (int i = 0; i < 5; ++i) A1->gout.st(o, (off_t)i * pb, n.g[i]);
            A1->flout.st(o, 0, fl1);
        }
    }
    __syncthreads();

    // ---- pass B: step k+1 -> k+2 of the tile, from LDS into memory.  A
    // lane of the tile holds the same node in both passes (no wrap: xb, yb
    // are in the lattice).
    if (!vb) return;
    const FlowWalls W(G, xb, yb);
    int s[9];
    tile_sources<TWD>(W, slot, s);
    const off_t o = ((off_t)yb * (off_t)G.pitch + (off_t)xb) * 4u;
    Node<IO> m;
    m.x = xb;
    m.y = yb;
    m.flk = fl1;
    m.eps = n.eps;
    m.g[0] = n.g[0];
#pragma unroll
    for (int i = 1; i < 5; ++i) m.g[i] = tl[(TG + i - 1) * PS + s[i]];
    if (W.w[1] | W.w[2] | W.w[3] | W.w[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) m.q[i] = tl[(TG + i) * PS + slot];
        if (FLOW) {
            m.uk[0] = ux;
            m.uk[1] = uy;
        }
    }
    float T2, fl2, isig2, vx = 0.0f, vy = 0.0f;
    node_enthalpy<IO, FLOW, false, TM_DEFAULT, UT>(G, P, B, A, m, T2, fl2, isig2);
    if (FLOW && fl2 > 0.0f) {
        float d[9];
        if (fl1 > 0.0f) {
            float v[27];  // as node_flow_core: neighbour f_l, pulls, own f+_1..8, u
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = tl[TFL * PS + s[k + 1]];
            v[8] = f0;
#pragma unroll
            for (int i = 1; i < 9; ++i) v[8 + i] = tl[(TF + i - 1) * PS + s[i]];
#pragma unroll
            for (int i = 1; i < 9; ++i) v[16 + i] = tl[(TF + i - 1) * PS + slot];
            v[25] = ux;
            v[26] = uy;
            flow_gather_liquid(v, W, m.eps, fl1, d);
        } else {
            // melted in the second step: drag coefficients from memory
            Ac = USTAT ? A.Ac_u : A.stat.ld(o, pb);
            Bc = USTAT ? A.Bc_u : A.stat.ld(o, 2 * pb);
            float nf[8], nr[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                nf[k] = tl[TFL * PS + s[k + 1]];
                nr[k] = tl[TRHO * PS + s[k + 1]];
            }
            flow_gather_restart(nf, nr, W, d);
        }
        flow_collide(d, fl2, m.eps, Ac, Bc, T2, P, vx, vy);
#pragma unroll
        for (int i = 0; i < 9; ++i) A.fout.st(o, (off_t)i * pb, d[i]);
        A.fout.st(o, 9 * pb, rho_dev(d));
        A.uv.st(o, 0, vx);
        A.uv.st(o, pb, vy);
    }
    thermal_collide<false, UT>(m.g, fl2, isig2, T2, vx, vy, m.eps, P);
#pragma unroll
    for (int i = 0; i < 5; ++i) A.gout.st(o, (off_t)i * pb, m.g[i]);
    A.flout.st(o, 0, fl2);
}

}  // namespace
}  // namespace dmrtk
