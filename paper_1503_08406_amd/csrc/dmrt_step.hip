// The fused time step of the double-MRT lattice Boltzmann phase-change model
// (Liu & He, arXiv:1503.08406) for gfx950.  One launch = one time step; one
// lane owns one node.
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
// Memory phases: f_l^k first; then every pull of the node in one batch (g,
// the neighbour liquid fractions, and f from all lattice neighbours when the
// node was liquid, discarding the values of solid sources afterwards); the
// node's own post-collision values are read only where an extrapolation
// needs them.
#include "dmrt_device.h"

namespace dmrtk {
namespace {

// The state arrays of one launch.
template <class IO>
struct Arrays {
    typename IO::off_t pb;  // bytes per population plane
    IO fin, fout, gin, gout, flin, flout, uv, stat;
    __device__ __forceinline__ Arrays(const Geom& G, const StepBufs& B)
        : pb((typename IO::off_t)G.plane * 4u),
          fin(B.fin, 9 * (uint64_t)pb), fout(B.fout, 9 * (uint64_t)pb),
          gin(B.gin, 5 * (uint64_t)pb), gout(B.gout, 5 * (uint64_t)pb),
          flin(B.flin, pb), flout(B.flout, pb),
          uv(B.ux, 2 * (uint64_t)pb),    // ux plane, then uy plane
          stat(B.eps, 3 * (uint64_t)pb)  // eps, Ac, Bc planes
    {
    }
};

// A node between its first load batch and the rest of its step.
template <class IO>
struct Node {
    typename IO::off_t o, o1, o2, o3, o4;
    int xm, xp, ym, yp;
    float flk, eps, g[5];
    int x, y;
};

// Offsets of node (x, y) and its first load batch: f_l^k, porosity and the
// five g pulls (every node needs them, liquid or solid).
template <class IO>
__device__ __forceinline__ void node_load(const Geom& G, const Arrays<IO>& A, int x, int y,
                                          Node<IO>& n)
{
    using off_t = typename IO::off_t;
    n.x = x;
    n.y = y;
    // neighbour indices without branches: wrap on periodic axes, a wall flag
    // (and any in-bounds index) otherwise
    const bool xlo = x == 0, xhi = x == G.nx - 1, ylo = y == 0, yhi = y == G.ny - 1;
    const bool wxm = xlo & !G.per_x, wxp = xhi & !G.per_x;
    const bool wym = ylo & !G.per_y, wyp = yhi & !G.per_y;
    const int xm = xlo ? G.nx - 1 : x - 1, xp = xhi ? 0 : x + 1;
    const int ym = ylo ? G.ny - 1 : y - 1, yp = yhi ? 0 : y + 1;
    const off_t pitch = (off_t)G.pitch;
    const off_t r0 = (off_t)y * pitch;
    const off_t o = (r0 + (off_t)x) * 4u;
    // byte offsets of the sources x - e_i; a source behind a wall is pointed
    // at the node itself (always in bounds) and its value is replaced later,
    // so every pull is an unconditional load.  Diagonal offsets are formed
    // only for liquid nodes (node_finish).
    n.o = o;
    n.o1 = wxm ? o : (r0 + (off_t)xm) * 4u;
    n.o3 = wxp ? o : (r0 + (off_t)xp) * 4u;
    n.o2 = wym ? o : ((off_t)ym * pitch + (off_t)x) * 4u;
    n.o4 = wyp ? o : ((off_t)yp * pitch + (off_t)x) * 4u;
    n.xm = xm;
    n.xp = xp;
    n.ym = ym;
    n.yp = yp;
    const off_t pb = A.pb;
    n.flk = A.flin.ld(o, 0);
    n.eps = A.stat.ld(o, 0);
    n.g[0] = A.gin.ld(o, 0);
    n.g[1] = A.gin.ld(n.o1, pb);
    n.g[2] = A.gin.ld(n.o2, 2 * pb);
    n.g[3] = A.gin.ld(n.o3, 3 * pb);
    n.g[4] = A.gin.ld(n.o4, 4 * pb);
}

// The rest of the step of one node (see the top of this file).
template <class IO, bool FLOW, bool COUNT>
__device__ __forceinline__ void node_finish(const Geom& G, const Phys& P, const StepBufs& B,
                                            const Arrays<IO>& A, Node<IO>& n)
{
    using off_t = typename IO::off_t;
    const off_t pb = A.pb;
    const IO &fin = A.fin, &fout = A.fout, &gin = A.gin, &gout = A.gout;
    const IO &flin = A.flin, &flout = A.flout, &uv = A.uv, &stat = A.stat;
    const off_t o = n.o, o1 = n.o1, o2 = n.o2, o3 = n.o3, o4 = n.o4;
    const bool wxm = (n.x == 0) & !G.per_x, wxp = (n.x == G.nx - 1) & !G.per_x;
    const bool wym = (n.y == 0) & !G.per_y, wyp = (n.y == G.ny - 1) & !G.per_y;
    const bool w5 = wxm | wym, w6 = wxp | wym, w7 = wxp | wyp, w8 = wxm | wyp;
    off_t o5 = o, o6 = o, o7 = o, o8 = o;  // diagonal sources, formed where needed
    const auto diag_offsets = [&]() {
        const off_t pitch = (off_t)G.pitch;
        const off_t rm = (off_t)n.ym * pitch, rp = (off_t)n.yp * pitch;
        o5 = w5 ? o : (rm + (off_t)n.xm) * 4u;
        o6 = w6 ? o : (rm + (off_t)n.xp) * 4u;
        o7 = w7 ? o : (rp + (off_t)n.xp) * 4u;
        o8 = w8 ? o : (rp + (off_t)n.xm) * 4u;
    };
    const bool wall = wxm | wxp | wym | wyp;
    const int x = n.x, y = n.y;
    const float flk = n.flk, eps = n.eps;
    float (&g)[5] = n.g;
    const bool act0 = FLOW && flk > 0.0f;

    float d[9];
    bool nee_f = false;
    unsigned liq = 0;  // bit i set: source of direction i is a liquid node
    float Ac = 0.0f, Bc = 0.0f;
    if (act0) {
        diag_offsets();
        const float n1 = flin.ld(o1, 0), n2 = flin.ld(o2, 0), n3 = flin.ld(o3, 0);
        const float n4 = flin.ld(o4, 0), n5 = flin.ld(o5, 0), n6 = flin.ld(o6, 0);
        const float n7 = flin.ld(o7, 0), n8 = flin.ld(o8, 0);
        d[0] = fin.ld(o, 0);
        d[1] = fin.ld(o1, pb);
        d[2] = fin.ld(o2, 2 * pb);
        d[3] = fin.ld(o3, 3 * pb);
        d[4] = fin.ld(o4, 4 * pb);
        d[5] = fin.ld(o5, 5 * pb);
        d[6] = fin.ld(o6, 6 * pb);
        d[7] = fin.ld(o7, 7 * pb);
        d[8] = fin.ld(o8, 8 * pb);
        Ac = stat.ld(o, pb);
        Bc = stat.ld(o, 2 * pb);
        liq = (unsigned)(!wxm & (n1 > 0.0f)) << 1 | (unsigned)(!wym & (n2 > 0.0f)) << 2 |
              (unsigned)(!wxp & (n3 > 0.0f)) << 3 | (unsigned)(!wyp & (n4 > 0.0f)) << 4 |
              (unsigned)(!w5 & (n5 > 0.0f)) << 5 | (unsigned)(!w6 & (n6 > 0.0f)) << 6 |
              (unsigned)(!w7 & (n7 > 0.0f)) << 7 | (unsigned)(!w8 & (n8 > 0.0f)) << 8;
        nee_f = liq != 0x1FEu;
    }
    float uxk = 0.0f, uyk = 0.0f;
    if (act0 & (wall | nee_f)) {
        uxk = uv.ld(o, 0);
        uyk = uv.ld(o, pb);
    }

    // ---- wall sources of g (start-of-step values of this node)
    if (wall) {
        const float q1 = gin.ld(o, pb), q2 = gin.ld(o, 2 * pb);
        const float q3 = gin.ld(o, 3 * pb), q4 = gin.ld(o, 4 * pb);
        const float Tk = g[0] + ((q1 + q3) + (q2 + q4));
        const float cu = frcp((P.sig_s + flk * P.dsig) * P.csT2);
        const float wTk = P.w5_1 * Tk;
        if (wxm) g[1] = P.w5_1 * (G.wall_T[0] ? G.T_wall[0] : Tk) + q1 - wTk * (1.0f + uxk * cu);
        if (wym) g[2] = P.w5_1 * (G.wall_T[2] ? G.T_wall[2] : Tk) + q2 - wTk * (1.0f + uyk * cu);
        if (wxp) g[3] = P.w5_1 * (G.wall_T[1] ? G.T_wall[1] : Tk) + q3 - wTk * (1.0f - uxk * cu);
        if (wyp) g[4] = P.w5_1 * (G.wall_T[3] ? G.T_wall[3] : Tk) + q4 - wTk * (1.0f - uyk * cu);
    }

    // ---- iterated enthalpy update (Eqs. 38, 40-42) at the receiving node;
    // the wavefront loops until every lane has converged.
    const float Tstar = g[0] + ((g[1] + g[3]) + (g[2] + g[4]));
    const float alat = eps * P.inv_St;  // phi L_a / c_p
    float f = flk;
    int it = 0;
    if (P.dsig == 0.0f) {
        const float a = alat * P.isig_s;
        for (;;) {
            ++it;
            const float En = (Tstar - a * (f - flk)) + f * P.inv_St;
            const float fn = fminf(fmaxf((En - P.T_s) * P.inv_den, 0.0f), 1.0f);
            const bool done = fabsf(fn - f) <= P.fl_tol || it >= P.fl_maxit;
            f = fn;
            if (done) break;
        }
    } else {
        for (;;) {
            ++it;
            const float T = Tstar - alat * (f - flk) * frcp(P.sig_s + f * P.dsig);
            const float fn = fminf(fmaxf((T + f * P.inv_St - P.T_s) * P.inv_den, 0.0f), 1.0f);
            const bool done = fabsf(fn - f) <= P.fl_tol || it >= P.fl_maxit;
            f = fn;
            if (done) break;
        }
    }
    const float fl1 = f;
    const float isig1 = P.dsig == 0.0f ? P.isig_s : frcp(P.sig_s + fl1 * P.dsig);
    const float dT = -alat * (fl1 - flk) * isig1;  // S~_0 (Eq. 38)
    const float T1 = Tstar + dT;
    g[0] += P.w5_0 * dT;
    g[1] += P.w5_1 * dT;
    g[2] += P.w5_1 * dT;
    g[3] += P.w5_1 * dT;
    g[4] += P.w5_1 * dT;
    if (COUNT) {
        const size_t ci = (size_t)y * G.pitch + x;
        B.it_sum[ci] += it;
        if (it > B.it_max[ci]) B.it_max[ci] = it;
    }

    // ---- flow where f_l^{k+1} > 0 (Sec. 4)
    float ux = 0.0f, uy = 0.0f;
    if (FLOW && fl1 > 0.0f) {
        if (act0) {
            if (nee_f) {
                const float iph = frcp(eps * flk);
                const float uu = 1.5f * (uxk * uxk + uyk * uyk) * iph;
#define DMRT_NEE(I, N, EU, W)                                                          \
    if (!(liq & (1u << I))) {                                                         \
        const float eu = (EU);                                                        \
        d[I] = fin.ld(o, I * pb) - (W) * (3.0f * eu + 4.5f * eu * eu * iph - uu);     \
    }
                DMRT_NEE(1, n1, uxk, W9_1)
                DMRT_NEE(2, n2, uyk, W9_1)
                DMRT_NEE(3, n3, -uxk, W9_1)
                DMRT_NEE(4, n4, -uyk, W9_1)
                DMRT_NEE(5, n5, uxk + uyk, W9_2)
                DMRT_NEE(6, n6, uyk - uxk, W9_2)
                DMRT_NEE(7, n7, -uxk - uyk, W9_2)
                DMRT_NEE(8, n8, uxk - uyk, W9_2)
#undef DMRT_NEE
            }
        } else {
            // the node melted in this step: restart at rest at the mean
            // start-of-step density of its liquid neighbours (rho0 if none),
            // f_i = w_i rho_bar; rho - 1 of a neighbour is the sum of its
            // stored post-collision deviations (collision conserves mass)
            diag_offsets();
            const off_t on[8] = {o1, o2, o3, o4, o5, o6, o7, o8};
            const bool wn[8] = {wxm, wym, wxp, wyp, w5, w6, w7, w8};
            float rsum = 0.0f;
            int cnt = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (!wn[k] && flin.ld(on[k], 0) > 0.0f) {
                    float r = 0.0f;
#pragma unroll
                    for (int i = 0; i < 9; ++i) r += fin.ld(on[k], (off_t)i * pb);
                    rsum += r;
                    ++cnt;
                }
            }
            const float drho = cnt ? rsum * frcp((float)cnt) : 0.0f;
#pragma unroll
            for (int i = 0; i < 9; ++i) d[i] = w9(i) * drho;
            Ac = stat.ld(o, pb);
            Bc = stat.ld(o, 2 * pb);
        }
        flow_collide(d, fl1, eps, Ac, Bc, T1, P, ux, uy);
#pragma unroll
        for (int i = 0; i < 9; ++i) fout.st(o, (off_t)i * pb, d[i]);
        uv.st(o, 0, ux);
        uv.st(o, pb, uy);
    }

    thermal_collide(g, fl1, isig1, T1, ux, uy, P);
#pragma unroll
    for (int i = 0; i < 5; ++i) gout.st(o, (off_t)i * pb, g[i]);
    flout.st(o, 0, fl1);
}


template <class IO, bool FLOW, bool COUNT, int TYB, int CPT>
__global__ __launch_bounds__(TX * TYB) void k_step(Geom G, Phys P, StepBufs B)
{
    // a tile of 64 x (TYB * CPT) nodes; a lane owns CPT nodes TYB rows apart
    // and issues the first load batch of all of them before finishing any
    int x0, y0;
    if (!step_tile_origin<TYB * CPT>(G, x0, y0)) return;
    const Arrays<IO> A(G, B);
    const int x = x0 + (int)threadIdx.x;
    Node<IO> n[CPT];
    bool ok[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int y = y0 + (int)threadIdx.y + j * TYB;
        ok[j] = x < G.nx && y < G.ny;
        if (ok[j]) node_load<IO>(G, A, x, y, n[j]);
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
