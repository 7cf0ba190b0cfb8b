// Two time steps of the double-MRT lattice Boltzmann phase-change model
// (Liu & He, arXiv:1503.08406) in one launch, for gfx950.
//
// A block of 64 x 2 lanes owns a strip of 62 columns [x0, x0 + 62) and R
// rows [y0, y0 + R) and marches down it two rows at a time:
//   pass A: step k -> k+1 of two rows of 64 nodes, columns x0 - 1 .. x0 + 62
//           (the strip plus one column on each side, which the neighbouring
//           strips also compute), read from the state in memory and written
//           into a ring of four rows in LDS;
//   pass B: step k+1 -> k+2 of two rows of the strip, read from the ring and
//           written to memory.
// Every node of the strip runs the per-node step of one launch per step
// (dmrt_node.h: the enthalpy update, the flow part with its wall and solid
// extrapolation or restart, both collisions) twice, with the same arithmetic,
// so two launches of this kernel give the bits of four single steps.  The
// intermediate state k+1 never leaves the chip: a node update moves half the
// bytes of the single step.
//
// Ring: logical row r of pass A lives in ring row r & 3; a node holds f+
// (nine deviations), rho - 1, g+ (five), f_l and u (two planes).  Before a
// pass B of rows b, b + 1 the ring holds pass-A rows b - 1 .. b + 2; the
// next pass A writes rows b + 3, b + 4 over b - 1, b.
#include "dmrt_node.h"

namespace dmrtk {
namespace {

constexpr int S2_W = 62;                // strip width (pass-B columns)
constexpr int S2_WAVES = 2;             // rows per pass
constexpr int S2_NT = TX * S2_WAVES;    // lanes per block
constexpr int RING_ROWS = 4;
constexpr int RPS = RING_ROWS * TX;     // floats per ring plane
enum { RF = 0, RRHO = 9, RG = 10, RFL = 15, RUX = 16, RUY = 17, RP = 18 };

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

// Handing the flow work of a pass to the lowest lanes of the block: the
// ballot and the owner of lane tid's work (as in block_step).
__device__ __forceinline__ int flow_owner(const FlowStage<S2_NT>& S, int parity, int tid)
{
    int j = tid, owner = 0;
#pragma unroll
    for (int k = 0; k < S2_WAVES; ++k) {
        const unsigned long long mk = S.mask[parity][k];
        const int c = __popcll(mk);
        if (j >= 0 && j < c) owner = k * 64 + nth_set_bit(mk, j);
        j -= c;
    }
    return owner;
}

// Pass A: step k -> k+1 of logical rows ra0, ra0 + 1 (only those in
// [ylo, yhi) are needed), columns x0 - 1 + lane, into the ring.
template <class IO, bool FLOW>
__device__ __forceinline__ void pass_A(const Geom& G, const Phys& P, const StepBufs& B,
                                       const Arrays<IO>& A, float* ring, FlowStage<S2_NT>& S,
                                       int x0, int ra0, int ylo, int yhi, int parity)
{
    const int lane = (int)threadIdx.x, w = (int)threadIdx.y;
    const int tid = w * 64 + lane;
    const int ra = ra0 + w;
    int xa = x0 - 1 + lane, ya = ra;
    const bool valid = ra >= ylo && ra < yhi && axis_node(xa, G.nx, G.per_x) &&
                       axis_node(ya, G.ny, G.per_y);
    const int slot = (ra & (RING_ROWS - 1)) * TX + lane;
    Node<IO> n;
    float T1 = 0.0f, fl1 = 0.0f, isig1 = 0.0f, ux = 0.0f, uy = 0.0f;
    __builtin_amdgcn_s_setprio(2);
    if (valid) {
        node_load<IO, FLOW>(G, A, xa, ya, n);
        __builtin_amdgcn_s_setprio(0);
        node_enthalpy<IO, FLOW, false>(G, P, B, A, n, T1, fl1, isig1);
    }
    if (FLOW) {
        const bool act = valid && fl1 > 0.0f;
        const unsigned long long m = __ballot(act);
        if (act) {
            S.x[tid] = xa;
            S.y[tid] = ya;
            S.flk[tid] = n.flk;
            S.fl1[tid] = fl1;
            S.T1[tid] = T1;
            S.eps[tid] = n.eps;
        }
        if (lane == 0) S.mask[parity][w] = m;
        __syncthreads();
        int total = 0;
#pragma unroll
        for (int k = 0; k < S2_WAVES; ++k) total += __popcll(S.mask[parity][k]);
        total = __builtin_amdgcn_readfirstlane(total);
        if (total > 0) {
            if (tid < total) {
                const int owner = flow_owner(S, parity, tid);
                float d[9], wx, wy;
                typename IO::off_t o;
                node_flow_core<IO, false>(G, P, A, S.x[owner], S.y[owner], S.flk[owner],
                                          S.fl1[owner], S.T1[owner], S.eps[owner], d, wx, wy, o);
                const int so = (((ra0 + (owner >> 6)) & (RING_ROWS - 1)) * TX) + (owner & 63);
#pragma unroll
                for (int i = 0; i < 9; ++i) ring[(RF + i) * RPS + so] = d[i];
                ring[RRHO * RPS + so] = rho_dev(d);
                ring[RUX * RPS + so] = wx;
                ring[RUY * RPS + so] = wy;
                S.ux[owner] = wx;
                S.uy[owner] = wy;
            }
            __syncthreads();
            if (act) {
                ux = S.ux[tid];
                uy = S.uy[tid];
            }
        }
    }
    if (valid) {
        thermal_collide<false>(n.g, fl1, isig1, T1, ux, uy, n.eps, P);
#pragma unroll
        for (int i = 0; i < 5; ++i) ring[(RG + i) * RPS + slot] = n.g[i];
        ring[RFL * RPS + slot] = fl1;
    }
}

// Ring slots of the sources x - e_i (i = 0..8) of the pass-B node at ring
// row rr and lane `lane`; a source behind a wall is the node's own slot.
__device__ __forceinline__ void ring_sources(const FlowWalls& W, int rr, int lane, int (&s)[9])
{
    const int r0 = (rr & (RING_ROWS - 1)) * TX;
    const int rm = ((rr - 1) & (RING_ROWS - 1)) * TX;
    const int rp = ((rr + 1) & (RING_ROWS - 1)) * TX;
    const int own = r0 + lane;
    s[0] = own;
    s[1] = W.w[1] ? own : r0 + lane - 1;
    s[2] = W.w[2] ? own : rm + lane;
    s[3] = W.w[3] ? own : r0 + lane + 1;
    s[4] = W.w[4] ? own : rp + lane;
    s[5] = W.w[5] ? own : rm + lane - 1;
    s[6] = W.w[6] ? own : rm + lane + 1;
    s[7] = W.w[7] ? own : rp + lane + 1;
    s[8] = W.w[8] ? own : rp + lane - 1;
}

// Pass B: step k+1 -> k+2 of rows rb0, rb0 + 1 (those below yend), columns
// x0 - 1 + lane for lanes 1..62, from the ring into memory.
template <class IO, bool FLOW>
__device__ __forceinline__ void pass_B(const Geom& G, const Phys& P, const StepBufs& B,
                                       const Arrays<IO>& A, const float* ring,
                                       FlowStage<S2_NT>& S, int x0, int rb0, int yend, int parity)
{
    using off_t = typename IO::off_t;
    const int lane = (int)threadIdx.x, w = (int)threadIdx.y;
    const int tid = w * 64 + lane;
    const int yb = rb0 + w, xb = x0 - 1 + lane;
    const bool valid = lane >= 1 && lane <= S2_W && xb < G.nx && yb < yend;
    const off_t pb = A.pb;
    const off_t og = ((off_t)yb * (off_t)G.pitch + (off_t)(valid ? xb : 0)) * 4u;
    Node<IO> n;
    float T1 = 0.0f, fl1 = 0.0f, isig1 = 0.0f, ux = 0.0f, uy = 0.0f;
    if (valid) {
        const FlowWalls W(G, xb, yb);
        int s[9];
        ring_sources(W, yb, lane, s);
        n.x = xb;
        n.y = yb;
        n.flk = ring[RFL * RPS + s[0]];
        n.eps = A.stat.ld(og, 0);
        n.g[0] = ring[(RG + 0) * RPS + s[0]];
        n.g[1] = ring[(RG + 1) * RPS + s[1]];
        n.g[2] = ring[(RG + 2) * RPS + s[2]];
        n.g[3] = ring[(RG + 3) * RPS + s[3]];
        n.g[4] = ring[(RG + 4) * RPS + s[4]];
        if (W.w[1] | W.w[2] | W.w[3] | W.w[4]) {
#pragma unroll
            for (int i = 0; i < 4; ++i) n.q[i] = ring[(RG + 1 + i) * RPS + s[0]];
            if (FLOW) {
                n.uk[0] = ring[RUX * RPS + s[0]];
                n.uk[1] = ring[RUY * RPS + s[0]];
            }
        }
        node_enthalpy<IO, FLOW, false>(G, P, B, A, n, T1, fl1, isig1);
    }
    if (FLOW) {
        const bool act = valid && fl1 > 0.0f;
        const unsigned long long m = __ballot(act);
        if (act) {
            S.x[tid] = xb;
            S.y[tid] = yb;
            S.flk[tid] = n.flk;
            S.fl1[tid] = fl1;
            S.T1[tid] = T1;
            S.eps[tid] = n.eps;
        }
        if (lane == 0) S.mask[parity][w] = m;
        __syncthreads();
        int total = 0;
#pragma unroll
        for (int k = 0; k < S2_WAVES; ++k) total += __popcll(S.mask[parity][k]);
        total = __builtin_amdgcn_readfirstlane(total);
        if (total > 0) {
            if (tid < total) {
                const int owner = flow_owner(S, parity, tid);
                const int x = S.x[owner], y = S.y[owner];
                const int olane = owner & 63;
                const FlowWalls W(G, x, y);
                int s[9];
                ring_sources(W, y, olane, s);
                const float flk = S.flk[owner], eps = S.eps[owner];
                const off_t o = ((off_t)y * (off_t)G.pitch + (off_t)x) * 4u;
                const float Ac = A.stat.ld(o, pb), Bc = A.stat.ld(o, 2 * pb);
                float d[9];
                if (flk > 0.0f) {
                    float v[27];
#pragma unroll
                    for (int k = 0; k < 8; ++k) v[k] = ring[RFL * RPS + s[k + 1]];
#pragma unroll
                    for (int i = 0; i < 9; ++i) v[8 + i] = ring[(RF + i) * RPS + s[i]];
#pragma unroll
                    for (int i = 1; i < 9; ++i) v[16 + i] = ring[(RF + i) * RPS + s[0]];
                    v[25] = ring[RUX * RPS + s[0]];
                    v[26] = ring[RUY * RPS + s[0]];
                    flow_gather_liquid(v, W, eps, flk, d);
                } else {
                    float nf[8], nr[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        nf[k] = ring[RFL * RPS + s[k + 1]];
                        nr[k] = ring[RRHO * RPS + s[k + 1]];
                    }
                    flow_gather_restart(nf, nr, W, d);
                }
                float wx, wy;
                flow_collide(d, S.fl1[owner], eps, Ac, Bc, S.T1[owner], P, wx, wy);
#pragma unroll
                for (int i = 0; i < 9; ++i) A.fout.st(o, (off_t)i * pb, d[i]);
                A.fout.st(o, 9 * pb, rho_dev(d));
                A.uv.st(o, 0, wx);
                A.uv.st(o, pb, wy);
                S.ux[owner] = wx;
                S.uy[owner] = wy;
            }
            __syncthreads();
            if (act) {
                ux = S.ux[tid];
                uy = S.uy[tid];
            }
        }
    }
    if (valid) {
        thermal_collide<false>(n.g, fl1, isig1, T1, ux, uy, n.eps, P);
#pragma unroll
        for (int i = 0; i < 5; ++i) A.gout.st(og, (off_t)i * pb, n.g[i]);
        A.flout.st(og, 0, fl1);
    }
}

// Strips of 62 x R nodes, numbered row-major; blocks are handed to the dies
// round-robin and die d takes a contiguous run of strips, so neighbouring
// strips (which share halo columns and rows) run on the same die.
template <class IO, bool FLOW, int R>
__global__ __launch_bounds__(S2_NT) void k_step2(Geom G, Phys P, StepBufs B)
{
    __shared__ float ring[RP * RPS];
    __shared__ FlowStage<S2_NT> S;
    const int nsx = (G.nx + S2_W - 1) / S2_W;
    const int ntiles = nsx * ((G.ny + R - 1) / R);
    const int per = (ntiles + NXCD - 1) / NXCD;
    const int b = (int)blockIdx.x;
    const int tile = (b % NXCD) * per + b / NXCD;
    if (tile >= ntiles) return;  // the whole block: no barrier is left waiting
    const int x0 = (tile % nsx) * S2_W, y0 = (tile / nsx) * R;
    const int yend = min(y0 + R, G.ny);
    const Arrays<IO> A(G, B);
    // pass-A rows needed: y0 - 1 .. yend
    const int ylo = y0 - 1, yhi = yend + 1;
    int parity = 0;
    pass_A<IO, FLOW>(G, P, B, A, ring, S, x0, y0 - 1, ylo, yhi, parity);
    parity ^= 1;
    __syncthreads();
    pass_A<IO, FLOW>(G, P, B, A, ring, S, x0, y0 + 1, ylo, yhi, parity);
    parity ^= 1;
    __syncthreads();
    for (int b0 = y0; b0 < yend; b0 += 2) {
        pass_B<IO, FLOW>(G, P, B, A, ring, S, x0, b0, yend, parity);
        parity ^= 1;
        __syncthreads();
        if (b0 + 2 < yend) {
            pass_A<IO, FLOW>(G, P, B, A, ring, S, x0, b0 + 3, ylo, yhi, parity);
            parity ^= 1;
            __syncthreads();
        }
    }
}

// Rows of a strip (a build-time tuning knob).
#ifndef DMRT_STEP2_ROWS
#define DMRT_STEP2_ROWS 16
#endif

template <class IO, bool FLOW>
hipError_t launch_io2(const Geom& G, const Phys& P, const StepBufs& B, hipStream_t s)
{
    constexpr int R = DMRT_STEP2_ROWS;
    static_assert(R % 2 == 0 && R >= 2, "strips hold an even number of rows");
    const int nsx = (G.nx + S2_W - 1) / S2_W;
    const int ntiles = nsx * ((G.ny + R - 1) / R);
    const dim3 grd(NXCD * ((ntiles + NXCD - 1) / NXCD));
    hipLaunchKernelGGL((k_step2<IO, FLOW, R>), grd, dim3(TX, S2_WAVES), 0, s, G, P, B);
    return hipGetLastError();
}

}  // namespace

bool step2_supported(const Geom& G, const Phys& P)
{
    return !G.wide && G.block_rows == 4 && G.cells_per_lane == 1 && !P.sig_mode && !P.ke_mode;
}

hipError_t launch_step2(const Geom& G, const Phys& P, const StepBufs& B, bool flow, hipStream_t s)
{
    if (G.store == ST_WT)
        return flow ? launch_io2<BufIOT<ST_WT>, true>(G, P, B, s) : launch_io2<BufIOT<ST_WT>, false>(G, P, B, s);
    if (G.store == ST_NT)
        return flow ? launch_io2<BufIOT<ST_NT>, true>(G, P, B, s) : launch_io2<BufIOT<ST_NT>, false>(G, P, B, s);
    return flow ? launch_io2<BufIO, true>(G, P, B, s) : launch_io2<BufIO, false>(G, P, B, s);
}

}  // namespace dmrtk
