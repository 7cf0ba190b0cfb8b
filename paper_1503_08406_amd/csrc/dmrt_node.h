// Per-node step of the double-MRT lattice Boltzmann phase-change model
// (Liu & He, arXiv:1503.08406), shared by the single-lattice and the batched
// step kernels.  See dmrt_step.hip for the order of the operations.
#pragma once

#include "dmrt_device.h"

namespace dmrtk {

// An access object of kind IO for the array of nbytes at p (WinIOT: inside
// the window of B).
template <class IO, class = void>
struct InWindow {
    static constexpr bool value = false;
};
template <class IO>
struct InWindow<IO, decltype((void)IO::in_window)> {
    static constexpr bool value = true;
};

template <class IO, bool OUT>
__device__ __forceinline__ IO array_io(const StepBufs& B, const float* p, uint64_t nbytes)
{
    if constexpr (InWindow<IO>::value) {
        if constexpr (OUT && IO::pair)
            return IO(B.wout, B.wout_bytes, p);
        else
            return IO(B.win, B.win_bytes, p);
    } else {
        return IO(p, nbytes);
    }
}

// The state arrays of one launch.
template <class IO>
struct Arrays {
    typename IO::off_t pb;  // bytes per population plane
    IO fin, fout, gin, gout, flin, flout, uv, uvin, stat;
    // porosity and drag coefficients of a lattice with uniform porous fields
    // (used instead of the stat planes when the node functions are told so)
    float eps_u = 0.0f, Ac_u = 0.0f, Bc_u = 0.0f;
    __device__ __forceinline__ Arrays(const Geom& G, const StepBufs& B)
        : pb((typename IO::off_t)G.plane * 4u),
          fin(array_io<IO, false>(B, B.fin, FQ * (uint64_t)pb)),
          fout(array_io<IO, true>(B, B.fout, FQ * (uint64_t)pb)),
          gin(array_io<IO, false>(B, B.gin, 5 * (uint64_t)pb)),
          gout(array_io<IO, true>(B, B.gout, 5 * (uint64_t)pb)),
          flin(array_io<IO, false>(B, B.flin, pb)), flout(array_io<IO, true>(B, B.flout, pb)),
          uv(array_io<IO, true>(B, B.ux, 2 * (uint64_t)pb)),  // ux plane, then uy plane (u^{k+1})
          uvin(array_io<IO, false>(B, B.uin ? B.uin : B.ux, 2 * (uint64_t)pb)),  // u^k
          stat(array_io<IO, false>(B, B.eps, 3 * (uint64_t)pb))  // eps, Ac, Bc planes
    {
    }
};

// A node between its first load batch and the rest of its step.
template <class IO>
struct Node {
    typename IO::off_t o, o1, o2, o3, o4;
    int xm, xp, ym, yp;
    float flk, eps, g[5];
    float q[4], uk[2];  // wall nodes: own g+_1..4 and u^k (first load batch)
    int x, y;
};

// Byte offsets of node (x, y) and of its axis sources x - e_i, and the
// wrapped neighbour indices, without branches: periodic axes wrap; a source
// behind a wall is pointed at the node itself (always in bounds) and its
// value is replaced later, so every pull is an unconditional load.  WALLED:
// compiled for a lattice with walls on every side (no periodic axis), whose
// neighbours are the node's offset plus or minus one column or row.
template <class IO, bool WALLED = false>
__device__ __forceinline__ void node_geometry(const Geom& G, int x, int y, Node<IO>& n)
{
    using off_t = typename IO::off_t;
    n.x = x;
    n.y = y;
    const bool xlo = x == 0, xhi = x == G.nx - 1, ylo = y == 0, yhi = y == G.ny - 1;
    if constexpr (WALLED) {
        const off_t row = (off_t)G.pitch * 4u;
        const off_t o = ((off_t)y * (off_t)G.pitch + (off_t)x) * 4u;
        n.o = o;
        n.o1 = xlo ? o : o - 4u;
        n.o3 = xhi ? o : o + 4u;
        n.o2 = ylo ? o : o - row;
        n.o4 = yhi ? o : o + row;
        n.xm = x - 1;
        n.xp = x + 1;
        n.ym = y - 1;
        n.yp = y + 1;
        return;
    }
    const bool wxm = xlo & !G.per_x, wxp = xhi & !G.per_x;
    const bool wym = ylo & !G.per_y, wyp = yhi & !G.per_y;
    const int xm = xlo ? G.nx - 1 : x - 1, xp = xhi ? 0 : x + 1;
    const int ym = ylo ? G.ny - 1 : y - 1, yp = yhi ? 0 : y + 1;
    const off_t pitch = (off_t)G.pitch;
    const off_t r0 = (off_t)y * pitch;
    const off_t o = (r0 + (off_t)x) * 4u;
    n.o = o;
    n.o1 = wxm ? o : (r0 + (off_t)xm) * 4u;
    n.o3 = wxp ? o : (r0 + (off_t)xp) * 4u;
    n.o2 = wym ? o : ((off_t)ym * pitch + (off_t)x) * 4u;
    n.o4 = wyp ? o : ((off_t)yp * pitch + (off_t)x) * 4u;
    n.xm = xm;
    n.xp = xp;
    n.ym = ym;
    n.yp = yp;
}

// First load batch of node (x, y): f_l^k, porosity and the five g pulls
// (every node needs them, liquid or solid); a wall node also loads its own
// g+_1..4 and u^k for the extrapolation at the wall, in the same batch.
template <class IO, bool FLOW, bool USTAT = false, bool WALLED = false>
__device__ __forceinline__ void node_load(const Geom& G, const Arrays<IO>& A, int x, int y,
                                          Node<IO>& n)
{
    using off_t = typename IO::off_t;
    node_geometry<IO, WALLED>(G, x, y, n);
    const off_t pb = A.pb, o = n.o;
    n.flk = A.flin.ld(o, 0);
    n.eps = USTAT ? A.eps_u : A.stat.ld(o, 0);
    n.g[0] = A.gin.ld(o, 0);
    n.g[1] = A.gin.ld(n.o1, pb);
    n.g[2] = A.gin.ld(n.o2, 2 * pb);
    n.g[3] = A.gin.ld(n.o3, 3 * pb);
    n.g[4] = A.gin.ld(n.o4, 4 * pb);
    const bool wall = (((x == 0) | (x == G.nx - 1)) & !G.per_x) | (((y == 0) | (y == G.ny - 1)) & !G.per_y);
    if (wall) {
        n.q[0] = A.gin.ld(o, pb);
        n.q[1] = A.gin.ld(o, 2 * pb);
        n.q[2] = A.gin.ld(o, 3 * pb);
        n.q[3] = A.gin.ld(o, 4 * pb);
        if (FLOW) {
            n.uk[0] = A.uvin.ld(o, 0);  // stale where the node is solid: masked later
            n.uk[1] = A.uvin.ld(o, pb);
        }
    }
}

// Thermal models of the node functions: the default readings, the literal
// variants of sigma (Eq. 7) and k_e (Eq. 8), and the last pass of a step
// with the latent source at the pre-stream site (R2, with f_l^{k+1} from a
// global iteration that ran before).
enum { TM_DEFAULT = 0, TM_VARIANT = 1, TM_R2 = 2 };

// Wall sources of g (Eq. 36 with non-equilibrium extrapolation) from the
// start-of-step values of a wall node; sigma(f_l^k) = sg0 + f_l^k dsg.
template <class IO, bool FLOW>
__device__ __forceinline__ void node_wall_g(const Geom& G, const Phys& P, Node<IO>& n, float sg0,
                                            float dsg)
{
    const bool wxm = (n.x == 0) & !G.per_x, wxp = (n.x == G.nx - 1) & !G.per_x;
    const bool wym = (n.y == 0) & !G.per_y, wyp = (n.y == G.ny - 1) & !G.per_y;
    if (wxm | wxp | wym | wyp) {
        const float flk = n.flk;
        float (&g)[5] = n.g;
        const bool liqk = FLOW && flk > 0.0f;
        const float uxk = liqk ? n.uk[0] : 0.0f, uyk = liqk ? n.uk[1] : 0.0f;
        const float q1 = n.q[0], q2 = n.q[1], q3 = n.q[2], q4 = n.q[3];
        const float Tk = g[0] + ((q1 + q3) + (q2 + q4));
        const float cu = frcp((sg0 + flk * dsg) * P.csT2);
        const float wTk = P.w5_1 * Tk;
        if (wxm) g[1] = P.w5_1 * (G.wall_T[0] ? G.T_wall[0] : Tk) + q1 - wTk * (1.0f + uxk * cu);
        if (wym) g[2] = P.w5_1 * (G.wall_T[2] ? G.T_wall[2] : Tk) + q2 - wTk * (1.0f + uyk * cu);
        if (wxp) g[3] = P.w5_1 * (G.wall_T[1] ? G.T_wall[1] : Tk) + q3 - wTk * (1.0f - uxk * cu);
        if (wyp) g[4] = P.w5_1 * (G.wall_T[3] ? G.T_wall[3] : Tk) + q4 - wTk * (1.0f - uyk * cu);
    }
}

// S~_0 dt of Eq. (38) at a node of porosity eps whose f_l goes from fk to f1.
template <bool VAR>
__device__ __forceinline__ float latent_S0(const Phys& P, float eps, float fk, float f1)
{
    float s0, ds;
    node_sigma<VAR>(P, eps, s0, ds);
    return -(eps * P.inv_St) * (f1 - fk) * frcp(s0 + f1 * ds);
}

// Thermal part of the step before the flow: wall sources of g, then the
// enthalpy update and the latent source added to g.  Gives T^{k+1},
// f_l^{k+1} and 1/sigma(f_l^{k+1}).
//   R1 (TM_DEFAULT, TM_VARIANT): iterated enthalpy update at the receiving
//     node (Eqs. 38, 40-42), its source w~_i S~_0 added to every g_i.
//   TM_R2: f_l^{k+1} of every node is given (B.r2f); each pulled g_i
//     receives w~_i S~_0 of its pre-stream site x - e_i (Eq. 30; the node
//     itself for i = 0 and behind a wall).
template <class IO, bool FLOW, bool COUNT, int TM = TM_DEFAULT, bool UT = false>
__device__ __forceinline__ void node_enthalpy(const Geom& G, const Phys& P, const StepBufs& B,
                                              const Arrays<IO>& A, Node<IO>& n, float& T1,
                                              float& fl1, float& isig1)
{
    constexpr bool VAR = TM != TM_DEFAULT;
    const float flk = n.flk, eps = n.eps;
    float (&g)[5] = n.g;
    float sg0, dsg;  // sigma(f_l) = sg0 + f_l dsg at this node
    node_sigma<VAR>(P, eps, sg0, dsg);
    node_wall_g<IO, FLOW>(G, P, n, sg0, dsg);

    if constexpr (TM == TM_R2) {
        using off_t = typename IO::off_t;
        const IO f1v(B.r2f, (uint64_t)A.pb);
        const off_t src[4] = {n.o1, n.o2, n.o3, n.o4};
        float f1s[4], fks[4], es[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            f1s[i] = f1v.ld(src[i], 0);
            fks[i] = A.flin.ld(src[i], 0);
            es[i] = A.stat.ld(src[i], 0);
        }
        fl1 = f1v.ld(n.o, 0);
        g[0] += P.w5_0 * latent_S0<true>(P, eps, flk, fl1);
#pragma unroll
        for (int i = 0; i < 4; ++i) g[i + 1] += P.w5_1 * latent_S0<true>(P, es[i], fks[i], f1s[i]);
        T1 = g[0] + ((g[1] + g[3]) + (g[2] + g[4]));
        isig1 = frcp(sg0 + fl1 * dsg);
        if (COUNT) {
            const size_t ci = (size_t)n.y * G.pitch + n.x;
            B.it_sum[ci] += B.r2_its;
            if (B.r2_its > B.it_max[ci]) B.it_max[ci] = B.r2_its;
        }
        return;
    }

    // ---- iterated enthalpy update at the receiving node; the wavefront
    // loops until every lane has converged.
    const float Tstar = g[0] + ((g[1] + g[3]) + (g[2] + g[4]));
    const float alat = eps * P.inv_St;  // phi L_a / c_p
    float f = flk;
    int it = 0;
    if (VAR && P.sig_mode) {
        // Eq. (7) sigma of this node; Eq. (40) with the mixture c_p and
        // Eq. (41) with En_s = c_ps T_s
        const float dcp = 1.0f - P.cps;
        for (;;) {
            ++it;
            const float T = Tstar - alat * (f - flk) * frcp(sg0 + f * dsg);
            const float En = (P.cps + f * dcp) * T + f * P.inv_St;
            const float fn = fminf(fmaxf((En - P.Es) * P.inv_den_c, 0.0f), 1.0f);
            const bool done = fabsf(fn - f) <= P.fl_tol || it >= P.fl_maxit;
            f = fn;
            if (done) break;
        }
    } else if (UT || P.dsig == 0.0f) {
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
    fl1 = f;
    isig1 = (VAR && P.sig_mode) ? frcp(sg0 + fl1 * dsg)
                                : (UT || P.dsig == 0.0f) ? P.isig_s : frcp(P.sig_s + fl1 * P.dsig);
    const float dT = -alat * (fl1 - flk) * isig1;  // S~_0 (Eq. 38)
    T1 = Tstar + dT;
    g[0] += P.w5_0 * dT;
    g[1] += P.w5_1 * dT;
    g[2] += P.w5_1 * dT;
    g[3] += P.w5_1 * dT;
    g[4] += P.w5_1 * dT;
    if (COUNT) {
        const size_t ci = (size_t)n.y * G.pitch + n.x;
        B.it_sum[ci] += it;
        if (it > B.it_max[ci]) B.it_max[ci] = it;
    }
}

// Pull sources of the flow populations at a node: bit i set when the source
// of direction i lies behind a wall (x-, y-, x+, y+ and the four diagonals).
struct FlowWalls {
    bool w[9];
    __device__ __forceinline__ FlowWalls(const Geom& G, int x, int y)
    {
        const bool wxm = (x == 0) & !G.per_x, wxp = (x == G.nx - 1) & !G.per_x;
        const bool wym = (y == 0) & !G.per_y, wyp = (y == G.ny - 1) & !G.per_y;
        w[0] = false;
        w[1] = wxm;
        w[2] = wym;
        w[3] = wxp;
        w[4] = wyp;
        w[5] = wxm | wym;
        w[6] = wxp | wym;
        w[7] = wxp | wyp;
        w[8] = wxm | wyp;
    }
};

// Pre-collision deviations of a node that was liquid at the start of the
// step (Sec. 4): pulled populations d_i = f+_i(x - e_i) where the source is
// a liquid node; a wall or solid source gives f_i^eq(rho, 0) + f+_i(x) -
// f_i^eq(rho, u^k; varphi^k), rho cancelling.  v: neighbour f_l (0-7, the
// sources of directions 1-8), pulls (8-16), own f+_1..8 (17-24), u^k (25-26).
__device__ __forceinline__ void flow_gather_liquid(const float (&v)[27], const FlowWalls& W,
                                                   float eps, float flk, float (&d)[9])
{
#pragma unroll
    for (int i = 0; i < 9; ++i) d[i] = v[8 + i];
    float own[9];  // this node's own f+_i(x), for extrapolated directions
    own[0] = 0.0f;
#pragma unroll
    for (int i = 1; i < 9; ++i) own[i] = v[16 + i];
    const float uxk = v[25], uyk = v[26];
    // bit i set: the source of direction i is a liquid node
    unsigned liq = 0u;
#pragma unroll
    for (int i = 1; i < 9; ++i) liq |= (unsigned)(!W.w[i] & (v[i - 1] > 0.0f)) << i;
    // a wall or solid source: computed for every direction and selected, so
    // the loads are used on every path and stay in one batch
    const float iph = frcp(eps * flk);
    const float uu = 1.5f * (uxk * uxk + uyk * uyk) * iph;
    const float eu[9] = {0.0f, uxk, uyk, -uxk, -uyk, uxk + uyk, uyk - uxk, -uxk - uyk, uxk - uyk};
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const float e = eu[i];
        const float nee = own[i] - w9(i) * (3.0f * e + 4.5f * e * e * iph - uu);
        d[i] = (liq & (1u << i)) ? d[i] : nee;
    }
}

// A node that melted in this step restarts at rest at the mean start-of-step
// density of its liquid lattice neighbours (rho0 if none): nf, nr are the
// neighbours' f_l and rho - 1 (sources of directions 1-8).
__device__ __forceinline__ void flow_gather_restart(const float (&nf)[8], const float (&nr)[8],
                                                    const FlowWalls& W, float (&d)[9])
{
    float rsum = 0.0f;
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (!W.w[k + 1] && nf[k] > 0.0f) {
            rsum += nr[k];
            ++cnt;
        }
    }
    const float drho = cnt ? rsum * frcp((float)cnt) : 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i) d[i] = w9(i) * drho;
}

// rho - 1 of post-collision deviations, summed in population order.
__device__ __forceinline__ float rho_dev(const float (&d)[9])
{
    float r = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i) r += d[i];
    return r;
}

// Flow part of a node with f_l^{k+1} > 0 (Sec. 4), up to its post-collision
// populations: pull f_i(x) = f+_i(x - e_i) from liquid sources; a wall or
// solid source gives the extrapolation of flow_gather_liquid; a node that
// melted in this step restarts at rest (flow_gather_restart).  Then the
// velocity closure and the MRT collision with forcing.  Every load of the
// node is issued in one batch; values are selected afterwards, so no load
// waits behind a data-dependent branch.  The node's drag coefficients are
// handed back for a second step of the same node.
template <class IO, bool USTAT, bool WALLED = false>
__device__ __forceinline__ void node_flow_core(const Geom& G, const Phys& P, const Arrays<IO>& A,
                                               int x, int y, float flk, float fl1, float T1,
                                               float eps, float (&d)[9], float& ux, float& uy,
                                               typename IO::off_t& o_out, float& Ac_out,
                                               float& Bc_out)
{
    using off_t = typename IO::off_t;
    const off_t pb = A.pb;
    const IO &fin = A.fin, &flin = A.flin;
    Node<IO> n;
    node_geometry<IO, WALLED>(G, x, y, n);
    const off_t o = n.o, o1 = n.o1, o2 = n.o2, o3 = n.o3, o4 = n.o4;
    const FlowWalls W(G, x, y);
    off_t o5, o6, o7, o8;
    if constexpr (WALLED) {
        const off_t row = (off_t)G.pitch * 4u;
        o5 = W.w[5] ? o : o - row - 4u;
        o6 = W.w[6] ? o : o - row + 4u;
        o7 = W.w[7] ? o : o + row + 4u;
        o8 = W.w[8] ? o : o + row - 4u;
    } else {
        const off_t pitch = (off_t)G.pitch;
        const off_t rm = (off_t)n.ym * pitch, rp = (off_t)n.yp * pitch;
        o5 = W.w[5] ? o : (rm + (off_t)n.xm) * 4u;
        o6 = W.w[6] ? o : (rm + (off_t)n.xp) * 4u;
        o7 = W.w[7] ? o : (rp + (off_t)n.xp) * 4u;
        o8 = W.w[8] ? o : (rp + (off_t)n.xm) * 4u;
    }
    const float Ac = USTAT ? A.Ac_u : A.stat.ld(o, pb);
    const float Bc = USTAT ? A.Bc_u : A.stat.ld(o, 2 * pb);
    o_out = o;
    Ac_out = Ac;
    Bc_out = Bc;

    if (flk > 0.0f) {
        float v[27];  // neighbour f_l (0-7), pulls (8-16), own f+_1..8 (17-24), u^k
        v[0] = flin.ld(o1, 0);
        v[1] = flin.ld(o2, 0);
        v[2] = flin.ld(o3, 0);
        v[3] = flin.ld(o4, 0);
        v[4] = flin.ld(o5, 0);
        v[5] = flin.ld(o6, 0);
        v[6] = flin.ld(o7, 0);
        v[7] = flin.ld(o8, 0);
        v[8] = fin.ld(o, 0);
        v[9] = fin.ld(o1, pb);
        v[10] = fin.ld(o2, 2 * pb);
        v[11] = fin.ld(o3, 3 * pb);
        v[12] = fin.ld(o4, 4 * pb);
        v[13] = fin.ld(o5, 5 * pb);
        v[14] = fin.ld(o6, 6 * pb);
        v[15] = fin.ld(o7, 7 * pb);
        v[16] = fin.ld(o8, 8 * pb);
#pragma unroll
        for (int i = 1; i < 9; ++i) v[16 + i] = fin.ld(o, (off_t)i * pb);
        v[25] = A.uvin.ld(o, 0);
        v[26] = A.uvin.ld(o, pb);
        pin_loads(v);
        flow_gather_liquid(v, W, eps, flk, d);
    } else {
        // their f_l and stored rho - 1 in one batch
        const off_t on[8] = {o1, o2, o3, o4, o5, o6, o7, o8};
        float nf[8], nr[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            nf[k] = flin.ld(on[k], 0);
            nr[k] = fin.ld(on[k], 9 * pb);
        }
        pin_loads(nf);
        pin_loads(nr);
        flow_gather_restart(nf, nr, W, d);
    }
    flow_collide(d, fl1, eps, Ac, Bc, T1, P, ux, uy);
}

// The flow part of a node with its stores: f+, rho - 1 and u^{k+1}.
template <class IO, bool USTAT>
__device__ __forceinline__ void node_flow(const Geom& G, const Phys& P, const Arrays<IO>& A,
                                          int x, int y, float flk, float fl1, float T1,
                                          float eps, float& ux, float& uy)
{
    using off_t = typename IO::off_t;
    const off_t pb = A.pb;
    float d[9], Ac, Bc;
    off_t o;
    node_flow_core<IO, USTAT>(G, P, A, x, y, flk, fl1, T1, eps, d, ux, uy, o, Ac, Bc);
#pragma unroll
    for (int i = 0; i < 9; ++i) A.fout.st(o, (off_t)i * pb, d[i]);
    A.fout.st(o, 9 * pb, rho_dev(d));
    A.uv.st(o, 0, ux);
    A.uv.st(o, pb, uy);
}

// D2Q5 MRT collision (Eqs. 35, 37) and the stores of g+ and f_l^{k+1}.
template <class IO, int TM = TM_DEFAULT>
__device__ __forceinline__ void node_thermal(const Phys& P, const Arrays<IO>& A, Node<IO>& n,
                                             float fl1, float isig1, float T1, float ux, float uy)
{
    using off_t = typename IO::off_t;
    thermal_collide<TM != TM_DEFAULT>(n.g, fl1, isig1, T1, ux, uy, n.eps, P);
#pragma unroll
    for (int i = 0; i < 5; ++i) A.gout.st(n.o, (off_t)i * A.pb, n.g[i]);
    A.flout.st(n.o, 0, fl1);
}

// The rest of the step of one node, without handing work to other lanes.
template <class IO, bool FLOW, bool COUNT, bool USTAT = false, int TM = TM_DEFAULT>
__device__ __forceinline__ void node_finish(const Geom& G, const Phys& P, const StepBufs& B,
                                            const Arrays<IO>& A, Node<IO>& n)
{
    float T1, fl1, isig1, ux = 0.0f, uy = 0.0f;
    node_enthalpy<IO, FLOW, COUNT, TM>(G, P, B, A, n, T1, fl1, isig1);
    if (FLOW && fl1 > 0.0f) node_flow<IO, USTAT>(G, P, A, n.x, n.y, n.flk, fl1, T1, n.eps, ux, uy);
    node_thermal<IO, TM>(P, A, n, fl1, isig1, T1, ux, uy);
}

// ---------------------------------------------------------------------------
// Block step with the flow work gathered onto the lowest lanes.
//
// Only nodes with f_l^{k+1} > 0 solve the flow, and a wavefront that holds a
// single such node would otherwise execute the whole flow part.  After the
// thermal part, every such node leaves its inputs in LDS and the k-th of
// them (in lane order) is handed to lane k of the block, so the flow part
// runs on ceil(count / 64) wavefronts; the velocities come back through
// LDS for the thermal collision.  The arithmetic of each node is unchanged.
// ---------------------------------------------------------------------------
template <int NT>
struct FlowStage {
    static constexpr int NW = NT / 64;
    unsigned long long mask[2][NW];  // per tile parity: lanes with a flow node
    int x[NT], y[NT];
    float flk[NT], fl1[NT], T1[NT], eps[NT];
    float ux[NT], uy[NT];
};

// Position of the j-th set bit of m (j < popcount(m)).
__device__ __forceinline__ int nth_set_bit(unsigned long long m, int j)
{
    int pos = 0;
#pragma unroll
    for (int s = 32; s > 0; s >>= 1) {
        const int c = __popcll(m & ((1ull << s) - 1ull));
        if (j >= c) {
            j -= c;
            m >>= s;
            pos += s;
        }
    }
    return pos;
}

// One node per lane of a 64 x (NT/64) block; every lane of the block must
// call this (valid = false for lanes outside the lattice).  `parity`
// alternates between consecutive tiles of a block that reuses S.
template <class IO, bool FLOW, bool COUNT, bool USTAT, int NT, int TM = TM_DEFAULT>
__device__ __forceinline__ void block_step(const Geom& G, const Phys& P, const StepBufs& B,
                                           const Arrays<IO>& A, int x, int y, bool valid,
                                           FlowStage<NT>& S, int parity)
{
    constexpr int NW = NT / 64;
    const int lane = (int)threadIdx.x, w = (int)threadIdx.y;
    const int tid = w * 64 + lane;
    Node<IO> n;
    float T1 = 0.0f, fl1 = 0.0f, isig1 = 0.0f, ux = 0.0f, uy = 0.0f;
    // issue the first load batch at raised wave priority, so that waves
    // still computing do not delay the memory requests of new ones.  The
    // priority belongs to the wavefront; it is lowered right after the loads
    // inside the lane condition (placed outside, the compiler also lowers it
    // on the masked-off path before the loads).  A wavefront with no valid
    // lane (past the last tile) keeps the raised priority; it only meets the
    // block's barriers.
    __builtin_amdgcn_s_setprio(2);
    if (valid) {
        node_load<IO, FLOW, USTAT>(G, A, x, y, n);
        __builtin_amdgcn_s_setprio(0);
        node_enthalpy<IO, FLOW, COUNT, TM>(G, P, B, A, n, T1, fl1, isig1);
    }
    if (FLOW) {
        const bool act = valid && fl1 > 0.0f;
        const unsigned long long m = __ballot(act);
        if (act) {
            S.x[tid] = x;
            S.y[tid] = y;
            S.flk[tid] = n.flk;
            S.fl1[tid] = fl1;
            S.T1[tid] = T1;
            S.eps[tid] = n.eps;
        }
        if (lane == 0) S.mask[parity][w] = m;
        __syncthreads();
        int total = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) total += __popcll(S.mask[parity][k]);
        total = __builtin_amdgcn_readfirstlane(total);  // the same in every lane
        if (total > 0) {
            if (tid < total) {
                int j = tid, owner = 0;
#pragma unroll
                for (int k = 0; k < NW; ++k) {
                    const unsigned long long mk = S.mask[parity][k];
                    const int c = __popcll(mk);
                    if (j >= 0 && j < c) owner = k * 64 + nth_set_bit(mk, j);
                    j -= c;
                }
                float wx, wy;
                node_flow<IO, USTAT>(G, P, A, S.x[owner], S.y[owner], S.flk[owner],
                                     S.fl1[owner], S.T1[owner], S.eps[owner], wx, wy);
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
    if (valid) node_thermal<IO, TM>(P, A, n, fl1, isig1, T1, ux, uy);
}

}  // namespace dmrtk
