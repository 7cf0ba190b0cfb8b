// Discrete adjoint of the fused time step of the double-MRT lattice Boltzmann
// phase-change model (Liu & He, arXiv:1503.08406): reverse-mode derivatives
// of a misfit of the final T and f_l fields with respect to the per-node
// porosity and the drag coefficients Ac, Bc (from which the host forms the
// gradients with respect to log K and porosity).
//
// Treatment of the non-smooth parts of the step: the enthalpy update is
// differentiated at its converged fixed point (on the mushy branch
// 0 < f_l < 1, f_l = (T* + a f_l^k - T_s) / (T_l - T_s + a) with
// a = phi / (sigma St); zero derivative where f_l is clamped); the flow mask
// and the liquid/solid classification of pull sources are held fixed; |v|
// has the subgradient 0 at v = 0.  Requires uniform sigma and tau_T.
//
// One reversed step k+1 -> k is one launch of k_adj_step per node x: it
// first completes the adjoint of x's state at k+1 by gathering, from the
// local adjoints the previous launch wrote, x's own terms and the adjoints
// of the pulls its downstream neighbours x + e_i made from it; then it
// recomputes x's step k from the stored state k (and f_l^{k+1}), back-
// propagates through the thermal collision, the flow closure and
// collision, the latent source and enthalpy update and the wall/interface
// extrapolations, and writes the local adjoints of step k (the adjoints of
// its pulled inputs and of its own state) for the next launch.
#include <type_traits>

#include "dmrt_device.h"

namespace dmrtk {
namespace {

// D2Q9 velocity components in the order of Eq. (15).
__device__ __forceinline__ int ex9(int i) { return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0); }
__device__ __forceinline__ int ey9(int i) { return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0); }

// Reverse of flow_collide: recomputes its intermediates from the pre-
// collision deviations d (same arithmetic) and back-propagates the adjoints
// Ld (of the nine post-collision deviations), Lux, Luy.  Returns the
// adjoints of d (in Ld) and accumulates those of fl1, eps, Ac, Bc and T1.
__device__ __forceinline__ void flow_collide_adj(const float (&d)[9], float fl1, float eps,
                                                 float Ac, float Bc, float T1, const Phys& P,
                                                 float (&Ld)[9], float Lux, float Luy,
                                                 float& Lfl1, float& Leps, float& LAc,
                                                 float& LBc, float& LT1)
{
    // ---- forward (as flow_collide)
    const float dx13 = d[1] - d[3], dy24 = d[2] - d[4];
    const float a58 = d[5] - d[7], b68 = d[6] - d[8];
    const float jx = dx13 + (a58 - b68);
    const float jy = dy24 + (a58 + b68);
    const float phi = eps * fl1;
    const float tb = P.gbeta * (T1 - P.T0);
    const float vy = jy + 0.5f * phi * tb;
    const float vx = jx;
    const float w2 = fl1 * fl1, om = 1.0f - phi;
    const float l0 = 0.5f * (w2 + 0.5f * Ac * om * om);
    const float l1 = 0.5f * Bc * om;
    const float vm = fsqrt(vx * vx + vy * vy);
    const float R = fsqrt(l0 * l0 + l1 * w2 * vm);
    const float den = l0 + R;
    const float iden = den > 0.0f ? frcp(den) : 0.0f;
    const float sc = w2 * iden;
    const float ux = vx * sc, uy = vy * sc;
    const float Fx = 2.0f * (ux - jx), Fy = 2.0f * (uy - jy);
    const float iphi = frcp(phi);
    const float uxi = ux * iphi, uyi = uy * iphi;

    // ---- reverse of the moment update and M^-1
    const float L0 = Ld[0], L1 = Ld[1], L2 = Ld[2], L3 = Ld[3], L4 = Ld[4];
    const float L5 = Ld[5], L6 = Ld[6], L7 = Ld[7], L8 = Ld[8];
    float La = 4.0f * L0, Lb = -4.0f * L0;
    const float Lca = -(L1 + L2 + L3 + L4);
    const float LX1 = L3 - L1, LY1 = L4 - L2;
    const float LPq = -L1 + L2 - L3 + L4;
    const float Lcd = -(L5 + L6 + L7 + L8);
    const float LX2 = -L5 + L6 + L7 - L8;
    const float LY2 = -L5 - L6 + L7 + L8;
    const float LQq = -L5 + L6 - L7 + L8;
    La += -Lca + 2.0f * Lcd;
    Lb += -2.0f * Lca + Lcd;
    const float LD1 = La * (1.0f / 36.0f), LD2 = Lb * (1.0f / 36.0f);
    float LFx = -(LX1 + LX2) * (1.0f / 6.0f);
    float LFy = -(LY1 + LY2) * (1.0f / 6.0f);
    const float LD4 = -LX1 * (1.0f / 6.0f) + LX2 * (1.0f / 12.0f);
    const float LD6 = -LY1 * (1.0f / 6.0f) + LY2 * (1.0f / 12.0f);
    const float LD7 = 0.25f * LPq, LD8 = 0.25f * LQq;
    // D1..D8
    float Lm1 = P.s_e * LD1, Lm2 = P.s_eps * LD2;
    float Lrho = 2.0f * P.s_e * LD1 - P.s_eps * LD2;
    float Lq = -P.s_e * LD1 + P.s_eps * LD2;
    float LS1 = -(1.0f - 0.5f * P.s_e) * LD1 + (1.0f - 0.5f * P.s_eps) * LD2;
    const float Lm4 = P.s_q * LD4, Lm6 = P.s_q * LD6;
    float Lux_ = Lux + P.s_q * LD4, Luy_ = Luy + P.s_q * LD6;
    LFx += (1.0f - 0.5f * P.s_q) * LD4;
    LFy += (1.0f - 0.5f * P.s_q) * LD6;
    const float Lm7 = P.s_nu * LD7, Lm8 = P.s_nu * LD8;
    float LPxx = -P.s_nu * LD7, LPyy = P.s_nu * LD7, LPxy = -P.s_nu * LD8;
    const float LS7 = -(1.0f - 0.5f * P.s_nu) * LD7, LS8 = -(1.0f - 0.5f * P.s_nu) * LD8;
    LPxx += 3.0f * Lq;
    LPyy += 3.0f * Lq;
    // S1, S7, S8
    float Luxi = 6.0f * Fx * LS1 + 2.0f * Fx * LS7 + Fy * LS8;
    float Luyi = 6.0f * Fy * LS1 - 2.0f * Fy * LS7 + Fx * LS8;
    LFx += 6.0f * uxi * LS1 + 2.0f * uxi * LS7 + uyi * LS8;
    LFy += 6.0f * uyi * LS1 - 2.0f * uyi * LS7 + uxi * LS8;
    // products ux*uxi, uy*uyi, ux*uyi
    Lux_ += uxi * LPxx + uyi * LPxy;
    Luxi += ux * LPxx;
    Luy_ += uyi * LPyy;
    Luyi += uy * LPyy + ux * LPxy;
    // uxi = ux iphi, uyi = uy iphi, iphi = 1/phi
    Lux_ += iphi * Luxi;
    Luy_ += iphi * Luyi;
    float Lphi = -(iphi * iphi) * (ux * Luxi + uy * Luyi);
    // F = 2 (u - j)
    Lux_ += 2.0f * LFx;
    Luy_ += 2.0f * LFy;
    float Ljx = -2.0f * LFx, Ljy = -2.0f * LFy;
    // u = v sc
    float Lvx = sc * Lux_, Lvy = sc * Luy_;
    const float Lsc = vx * Lux_ + vy * Luy_;
    // sc = w2 / den
    float Lw2 = iden * Lsc;
    const float Lden = -sc * iden * Lsc;
    // den = l0 + R, R = sqrt(l0^2 + l1 w2 vm)
    float Ll0 = Lden;
    const float LR2 = R > 0.0f ? 0.5f * frcp(R) * Lden : 0.0f;
    Ll0 += 2.0f * l0 * LR2;
    const float Ll1 = w2 * vm * LR2;
    Lw2 += l1 * vm * LR2;
    const float Lvm = l1 * w2 * LR2;
    if (vm > 0.0f) {  // subgradient 0 at v = 0
        const float ivm = frcp(vm);
        Lvx += vx * ivm * Lvm;
        Lvy += vy * ivm * Lvm;
    }
    // l1 = Bc om / 2, l0 = (w2 + Ac om^2 / 2) / 2
    LBc += 0.5f * om * Ll1;
    float Lom = 0.5f * Bc * Ll1 + 0.5f * Ac * om * Ll0;
    LAc += 0.25f * om * om * Ll0;
    Lw2 += 0.5f * Ll0;
    Lphi -= Lom;
    // vy = jy + phi tb / 2, vx = jx
    Ljy += Lvy;
    Ljx += Lvx;
    Lphi += 0.5f * tb * Lvy;
    LT1 += 0.5f * phi * P.gbeta * Lvy;
    // w2 = fl1^2, phi = eps fl1
    Lfl1 += 2.0f * fl1 * Lw2 + eps * Lphi;
    Leps += fl1 * Lphi;
    // moments and sums back to d
    float Lsa = Lrho, Lsd = Lrho;
    Ld[0] = L0 + Lrho - 4.0f * Lm1 + 4.0f * Lm2;
    Lsd += 2.0f * Lm1 + Lm2;
    Lsa += -Lm1 - 2.0f * Lm2;
    const float La58 = Lm4 + Lm6 + Ljx + Ljy;
    const float Lb68 = -Lm4 + Lm6 - Ljx + Ljy;
    const float Ldx13 = -2.0f * Lm4 + Ljx;
    const float Ldy24 = -2.0f * Lm6 + Ljy;
    Ld[1] = L1 + Lsa + Ldx13 + Lm7;
    Ld[2] = L2 + Lsa + Ldy24 - Lm7;
    Ld[3] = L3 + Lsa - Ldx13 + Lm7;
    Ld[4] = L4 + Lsa - Ldy24 - Lm7;
    Ld[5] = L5 + Lsd + La58 + Lm8;
    Ld[6] = L6 + Lsd + Lb68 - Lm8;
    Ld[7] = L7 + Lsd - La58 + Lm8;
    Ld[8] = L8 + Lsd - Lb68 - Lm8;
}

// Adjoint of the state at step k+1 of node (x, y), gathered from the local
// adjoints of step k+1 (la: written by the launch for step k+1): the node's
// own terms plus the adjoints of the pulls its downstream neighbours y + e_i
// made from it.  flA = f_l^{k+1} of the node (already loaded), flB =
// f_l^{k+2}: the flow part exists only
// where the node was liquid at k+1, and a node's flow local adjoints only
// where it was liquid at k+2.  L: d+ (0..8), rho - 1 (9), g+ (10..14),
// f_l (15), u (16, 17).
// An array of the reversed step.  O32: every element index of the launch
// is below 2^30, and an access adds a 32-bit byte offset to the array's
// base (the load takes the base from scalar registers); else 64-bit
// indices.
template <class T, bool O32>
struct AdjArr {
    T* p;
    __device__ __forceinline__ T& operator[](size_t i) const
    {
        if constexpr (O32) {
            using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
            return *reinterpret_cast<T*>(reinterpret_cast<C*>(p) + ((uint32_t)i << 2));
        } else {
            return p[i];
        }
    }
};

// Receivers y + e_i of node (x, y) (rc) and whether each exists (ok).
__device__ __forceinline__ void gather_receivers(const Geom& G, int x, int y, bool (&ok)[9],
                                                 size_t (&rc)[9])
{
    const size_t p = (size_t)G.pitch;
    const size_t c = (size_t)y * p + (size_t)x;
    const bool hx = x + 1 < G.nx || G.per_x, lx = x > 0 || G.per_x;
    const bool hy = y + 1 < G.ny || G.per_y, ly = y > 0 || G.per_y;
    const size_t xp = x + 1 < G.nx ? x + 1 : 0, xm = x > 0 ? x - 1 : G.nx - 1;
    const size_t yp = y + 1 < G.ny ? y + 1 : 0, ym = y > 0 ? y - 1 : G.ny - 1;
    ok[0] = false;
    rc[0] = c;
    ok[1] = hx;
    rc[1] = y * p + xp;
    ok[2] = hy;
    rc[2] = yp * p + x;
    ok[3] = lx;
    rc[3] = y * p + xm;
    ok[4] = ly;
    rc[4] = ym * p + x;
    ok[5] = hx & hy;
    rc[5] = yp * p + xp;
    ok[6] = lx & hy;
    rc[6] = yp * p + xm;
    ok[7] = lx & ly;
    rc[7] = ym * p + xm;
    ok[8] = hx & ly;
    rc[8] = ym * p + xp;
}

// The thermal terms of gather_state, loaded with the node's first batch:
// own g terms (0..4), own f_l (5), the receivers' g pulls (6..9; loaded from
// in-lattice addresses even where a receiver is absent).
template <bool O32>
__device__ __forceinline__ void gather_thermal_loads(const Geom& G, AdjArr<const float, O32> la,
                                                     int x, int y, float (&t)[10])
{
    const size_t pl = (size_t)G.plane;
    const size_t c = (size_t)y * (size_t)G.pitch + (size_t)x;
    bool ok[9];
    size_t rc[9];
    gather_receivers(G, x, y, ok, rc);
#pragma unroll
    for (int i = 0; i < 5; ++i) t[i] = la[(15 + i) * pl + c];
    t[5] = la[29 * pl + c];
#pragma unroll
    for (int i = 1; i < 5; ++i) t[5 + i] = la[i * pl + rc[i]];
}

template <bool FLOW, bool O32>
__device__ __forceinline__ void gather_state(const Geom& G, AdjArr<const float, O32> la,
                                             float flA, AdjArr<const float, O32> flB, int x,
                                             int y, const float (&t)[10], float (&L)[ADJ_LS])
{
    const size_t pl = (size_t)G.plane;
    const size_t c = (size_t)y * (size_t)G.pitch + (size_t)x;
    bool ok[9];
    size_t rc[9];  // receivers y + e_i
    gather_receivers(G, x, y, ok, rc);
    L[10] = t[0];
#pragma unroll
    for (int i = 1; i < 5; ++i) L[10 + i] = t[i] + (ok[i] ? t[5 + i] : 0.0f);
    L[15] = t[5];
#pragma unroll
    for (int i = 0; i < 10; ++i) L[i] = 0.0f;
    L[16] = L[17] = 0.0f;
    if (FLOW && flA > 0.0f) {
        // every load in one batch (stale values of absent terms are loaded
        // from in-lattice addresses and selected away)
        float v[38];  // own d+ (0..8), receivers: f_l (9..16), pulls (17..24), restart (25..32), u (33, 34), own f_l (35)
#pragma unroll
        for (int i = 0; i < 9; ++i) v[i] = la[(20 + i) * pl + c];
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            v[8 + i] = flB[rc[i]];
            v[16 + i] = la[(5 + i) * pl + rc[i]];
            v[24 + i] = la[14 * pl + rc[i]];
        }
        v[33] = la[30 * pl + c];
        v[34] = la[31 * pl + c];
        v[35] = flB[c];
        v[36] = v[37] = 0.0f;
        pin_loads(v);
        const bool own1 = v[35] > 0.0f;
        L[0] = own1 ? v[0] : 0.0f;
        float Lr = 0.0f;
#pragma unroll
        for (int i = 1; i < 9; ++i) {
            const bool rec = ok[i] && v[8 + i] > 0.0f;
            L[i] = (own1 ? v[i] : 0.0f) + (rec ? v[16 + i] : 0.0f);
            Lr += rec ? v[24 + i] : 0.0f;
        }
        L[9] = Lr;
        L[16] = v[33];
        L[17] = v[34];
    }
}

// One reversed step k+1 -> k for one node: the adjoint of its state at
// k+1 (the terminal adjoint when FIRST, else gathered from the local
// adjoints of step k+1), then the local adjoint of its step k.
template <bool FLOW, bool FIRST, bool O32>
__global__ __launch_bounds__(TX * TY) void k_adj_step(Geom G, Phys P, AdjBufs B)
{
    int x, y;
    if (!tile_coords_rotated<TY>(G, x, y)) return;
    using CA = AdjArr<const float, O32>;
    const CA aF0{B.f0}, aG0{B.g0}, aFL0{B.fl0}, aU0{B.u0}, aFL1{B.fl1}, aEPS{B.eps}, aAC{B.Ac},
        aBC{B.Bc}, aFL2{B.fl2}, aLS{B.ls}, aLAP{B.la_prev};
    const AdjArr<float, O32> aLA{B.la}, aGA{B.ga};
    const size_t pl = (size_t)G.plane;
    const size_t p = (size_t)G.pitch;
    const size_t c = (size_t)y * p + (size_t)x;
    const bool xlo = x == 0, xhi = x == G.nx - 1, ylo = y == 0, yhi = y == G.ny - 1;
    const bool wxm = xlo & !G.per_x, wxp = xhi & !G.per_x;
    const bool wym = ylo & !G.per_y, wyp = yhi & !G.per_y;
    const size_t xm = xlo ? G.nx - 1 : x - 1, xp = xhi ? 0 : x + 1;
    const size_t ym = ylo ? G.ny - 1 : y - 1, yp = yhi ? 0 : y + 1;
    bool wn[9];
    size_t src[9];  // node x - e_i (x itself behind a wall)
    wn[0] = false;
    src[0] = c;
    wn[1] = wxm;
    src[1] = y * p + xm;
    wn[2] = wym;
    src[2] = ym * p + x;
    wn[3] = wxp;
    src[3] = y * p + xp;
    wn[4] = wyp;
    src[4] = yp * p + x;
    wn[5] = wxm | wym;
    src[5] = ym * p + xm;
    wn[6] = wxp | wym;
    src[6] = ym * p + xp;
    wn[7] = wxp | wyp;
    src[7] = yp * p + xp;
    wn[8] = wxm | wyp;
    src[8] = yp * p + xm;
#pragma unroll
    for (int i = 1; i < 9; ++i)
        if (wn[i]) src[i] = c;
    const bool wall = wxm | wxp | wym | wyp;

    // ---- first load batch: every value whose address is known now (the
    // flow values follow in a second batch where the node is liquid)
    const float flk = aFL0[c], fl1 = aFL1[c];
    float t[10];  // thermal terms of the state adjoint (gather_state)
    float Ls[ADJ_LS];
    if (FIRST) {
#pragma unroll
        for (int i = 0; i < ADJ_LS; ++i) Ls[i] = aLS[i * pl + c];
    } else {
        gather_thermal_loads<O32>(G, aLAP, x, y, t);
    }
    const float eps = aEPS[c], Ac = aAC[c], Bc = aBC[c];
    float q[5], g[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) q[i] = aG0[i * pl + c];
    g[0] = q[0];
#pragma unroll
    for (int i = 1; i < 5; ++i) g[i] = aG0[i * pl + src[i]];
    const float u0x = FLOW ? aU0[c] : 0.0f, u0y = FLOW ? aU0[pl + c] : 0.0f;
    const bool liqk = FLOW && flk > 0.0f;
    const bool liq1 = FLOW && fl1 > 0.0f;

    // ---- forward recomputation: pulled g with wall extrapolation
    const float uxk = liqk ? u0x : 0.0f, uyk = liqk ? u0y : 0.0f;
    float Tk = 0.0f, cu = 0.0f;
    if (wall) {
        Tk = q[0] + ((q[1] + q[3]) + (q[2] + q[4]));
        cu = frcp((P.sig_s + flk * P.dsig) * P.csT2);
        const float wTk = P.w5_1 * Tk;
        if (wxm) g[1] = P.w5_1 * (G.wall_T[0] ? G.T_wall[0] : Tk) + q[1] - wTk * (1.0f + uxk * cu);
        if (wym) g[2] = P.w5_1 * (G.wall_T[2] ? G.T_wall[2] : Tk) + q[2] - wTk * (1.0f + uyk * cu);
        if (wxp) g[3] = P.w5_1 * (G.wall_T[1] ? G.T_wall[1] : Tk) + q[3] - wTk * (1.0f - uxk * cu);
        if (wyp) g[4] = P.w5_1 * (G.wall_T[3] ? G.T_wall[3] : Tk) + q[4] - wTk * (1.0f - uyk * cu);
    }
    const float Tstar = g[0] + ((g[1] + g[3]) + (g[2] + g[4]));
    const float alat = eps * P.inv_St;
    const float isig1 = P.isig_s;  // uniform sigma
    const float dT = -alat * (fl1 - flk) * isig1;
    const float T1 = Tstar + dT;

    // ---- forward recomputation: pre-collision f of a flow node
    float d[9];
    unsigned liq = 0;
    int cnt = 0;
    float iph = 0.0f;
    const float eu[9] = {0.0f, uxk, uyk, -uxk, -uyk, uxk + uyk, uyk - uxk, -uxk - uyk, uxk - uyk};
    float ux = 0.0f, uy = 0.0f;
    if (liq1) {
        // one batch: neighbour f_l, then the pulls and own values (liquid at
        // k) or the neighbour densities (melted in this step)
        float nf[9];
        nf[0] = 0.0f;
#pragma unroll
        for (int i = 1; i < 9; ++i) nf[i] = aFL0[src[i]];
        if (liqk) {
            float v[17];  // own f+_0..8 (0..8), pulls 1..8 (9..16)
#pragma unroll
            for (int i = 0; i < 9; ++i) v[i] = aF0[i * pl + c];
#pragma unroll
            for (int i = 1; i < 9; ++i) v[8 + i] = aF0[i * pl + src[i]];
            pin_loads(nf);
            pin_loads(v);
#pragma unroll
            for (int i = 1; i < 9; ++i) liq |= (unsigned)(!wn[i] & (nf[i] > 0.0f)) << i;
            d[0] = v[0];
            iph = frcp(eps * flk);
            const float uu = 1.5f * (uxk * uxk + uyk * uyk) * iph;
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                const float e = eu[i];
                const float nee = v[i] - w9(i) * (3.0f * e + 4.5f * e * e * iph - uu);
                d[i] = (liq & (1u << i)) ? v[8 + i] : nee;
            }
        } else {
            float nr[9];
            nr[0] = 0.0f;
#pragma unroll
            for (int k = 1; k < 9; ++k) nr[k] = aF0[9 * pl + src[k]];
            pin_loads(nf);
            pin_loads(nr);
            float rsum = 0.0f;
#pragma unroll
            for (int k = 1; k < 9; ++k)
                if (!wn[k] && nf[k] > 0.0f) {
                    rsum += nr[k];
                    ++cnt;
                }
            const float drho = cnt ? rsum * frcp((float)cnt) : 0.0f;
#pragma unroll
            for (int i = 0; i < 9; ++i) d[i] = w9(i) * drho;
        }
        float dd[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) dd[i] = d[i];
        flow_collide(dd, fl1, eps, Ac, Bc, T1, P, ux, uy);
    }

    // ---- adjoint of the outputs of this node's step (state k+1)
    // the gradient accumulators of a node liquid at k+1 (each is added to by
    // this node only) ride with the flow batch of the gather
    float ga0 = 0.0f, ga1 = 0.0f, ga2 = 0.0f;
    if (liq1) {
        ga0 = aGA[c];
        ga1 = aGA[pl + c];
        ga2 = aGA[2 * pl + c];
    }
    if (!FIRST) gather_state<FLOW, O32>(G, aLAP, fl1, aFL2, x, y, t, Ls);

    // ---- reverse: thermal collision (uniform zeta)
    float Lg[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) Lg[i] = Ls[10 + i];
    float Lfl1 = Ls[15];
    float Leps = 0.0f, LAc = 0.0f, LBc = 0.0f, Lflk = 0.0f;
    const float za = P.zeta_a;
    const float ct = P.conv * T1 * isig1;
    const float LD3 = 0.2f * Lg[0] - 0.05f * ((Lg[1] + Lg[2]) + (Lg[3] + Lg[4]));
    const float LD4 = 0.25f * ((Lg[2] + Lg[4]) - (Lg[1] + Lg[3]));
    const float LD1 = 0.5f * (Lg[3] - Lg[1]), LD2 = 0.5f * (Lg[4] - Lg[2]);
    const float Ln1 = za * LD1, Ln2 = za * LD2, Ln3 = P.zeta_e * LD3, Ln4 = P.zeta_nu * LD4;
    const float Lct = -za * (ux * LD1 + uy * LD2);
    float Lux = -za * ct * LD1, Luy = -za * ct * LD2;
    float LT1 = -P.zeta_e * P.varpi * LD3 + P.conv * isig1 * Lct;
    float Lgl[5];
    Lgl[0] = Lg[0] - 4.0f * Ln3;
    Lgl[1] = Lg[1] + Ln1 + Ln3 + Ln4;
    Lgl[2] = Lg[2] + Ln2 + Ln3 - Ln4;
    Lgl[3] = Lg[3] - Ln1 + Ln3 + Ln4;
    Lgl[4] = Lg[4] - Ln2 + Ln3 - Ln4;

    // ---- reverse: flow part
    float Ld[9];
    float Lrb = 0.0f;
    float Lown_d[9], Luxk = 0.0f, Luyk = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        Ld[i] = 0.0f;
        Lown_d[i] = 0.0f;
    }
    if (liq1) {
        const float Lr = Ls[9];  // rho - 1 stored as the sum of f+
#pragma unroll
        for (int i = 0; i < 9; ++i) Ld[i] = Ls[i] + Lr;
        Lux += Ls[16];
        Luy += Ls[17];
        flow_collide_adj(d, fl1, eps, Ac, Bc, T1, P, Ld, Lux, Luy, Lfl1, Leps, LAc, LBc, LT1);
        if (liqk) {
            Lown_d[0] = Ld[0];
            Ld[0] = 0.0f;
            const float u2 = uxk * uxk + uyk * uyk;
            float Luu = 0.0f, Liph = 0.0f;
#pragma unroll
            for (int i = 1; i < 9; ++i) {
                if (!(liq & (1u << i))) {
                    const float e = eu[i], w = w9(i), L = Ld[i];
                    Lown_d[i] = L;
                    const float Le = -w * (3.0f + 9.0f * e * iph) * L;
                    Liph += -w * 4.5f * e * e * L;
                    Luu += w * L;
                    Luxk += (float)ex9(i) * Le;
                    Luyk += (float)ey9(i) * Le;
                    Ld[i] = 0.0f;  // not a pull
                }
            }
            Liph += 1.5f * u2 * Luu;
            Luxk += 3.0f * uxk * iph * Luu;
            Luyk += 3.0f * uyk * iph * Luu;
            Leps += -iph * iph * flk * Liph;
            Lflk += -iph * iph * eps * Liph;
        } else {
            float s = 0.0f;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                s += w9(i) * Ld[i];
                Ld[i] = 0.0f;
            }
            Lrb = cnt ? s * frcp((float)cnt) : 0.0f;
        }
    }

    // ---- reverse: latent source, T1 = T* + dT, enthalpy fixed point
    float LdT = P.w5_0 * Lgl[0] + P.w5_1 * ((Lgl[1] + Lgl[2]) + (Lgl[3] + Lgl[4]));
    float LTs = LT1;
    LdT += LT1;
    Lfl1 += -alat * isig1 * LdT;
    Lflk += alat * isig1 * LdT;
    Leps += -P.inv_St * isig1 * (fl1 - flk) * LdT;
    if (fl1 > 0.0f && fl1 < 1.0f) {
        const float a = alat * P.isig_s;
        const float dTm = frcp(P.inv_dTm);
        const float ih = frcp(dTm + a);
        LTs += ih * Lfl1;
        Lflk += a * ih * Lfl1;
        Leps += P.inv_St * P.isig_s * (flk - fl1) * ih * Lfl1;
    }
    float Lgp[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) Lgp[i] = Lgl[i] + LTs;

    // ---- reverse: wall extrapolation of g
    float Lown_g[5] = {Lgp[0], 0.0f, 0.0f, 0.0f, 0.0f};
    Lgp[0] = 0.0f;
    if (wall) {
        float LTk = 0.0f;
        const float wc = P.w5_1 * Tk * cu;
        if (wxm) {
            Lown_g[1] += Lgp[1];
            LTk += (G.wall_T[0] ? 0.0f : P.w5_1) * Lgp[1] - P.w5_1 * (1.0f + uxk * cu) * Lgp[1];
            Luxk += -wc * Lgp[1];
            Lgp[1] = 0.0f;
        }
        if (wym) {
            Lown_g[2] += Lgp[2];
            LTk += (G.wall_T[2] ? 0.0f : P.w5_1) * Lgp[2] - P.w5_1 * (1.0f + uyk * cu) * Lgp[2];
            Luyk += -wc * Lgp[2];
            Lgp[2] = 0.0f;
        }
        if (wxp) {
            Lown_g[3] += Lgp[3];
            LTk += (G.wall_T[1] ? 0.0f : P.w5_1) * Lgp[3] - P.w5_1 * (1.0f - uxk * cu) * Lgp[3];
            Luxk += wc * Lgp[3];
            Lgp[3] = 0.0f;
        }
        if (wyp) {
            Lown_g[4] += Lgp[4];
            LTk += (G.wall_T[3] ? 0.0f : P.w5_1) * Lgp[4] - P.w5_1 * (1.0f - uyk * cu) * Lgp[4];
            Luyk += wc * Lgp[4];
            Lgp[4] = 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 5; ++i) Lown_g[i] += LTk;
    }
    if (!liqk) Luxk = Luyk = 0.0f;

    // ---- outputs (a node solid at k+1 reads its porosity accumulator here)
    const bool acc_eps = Leps != 0.0f;
    if (acc_eps && !liq1) ga0 = aGA[c];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        aLA[i * pl + c] = Lgp[i];
        aLA[(15 + i) * pl + c] = Lown_g[i];
    }
    // the flow planes only for a node liquid at k+1 (the gather reads them
    // only there), u^k only for a node liquid at k; a node solid at k+1
    // contributes nothing to Ac, Bc
    if (liq1) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            aLA[(5 + i) * pl + c] = Ld[i];
            aLA[(20 + i) * pl + c] = Lown_d[i];
        }
        aLA[14 * pl + c] = Lrb;
        aGA[pl + c] = ga1 + LAc;
        aGA[2 * pl + c] = ga2 + LBc;
    }
    if (liqk) {  // u^k also enters the wall extrapolation of g
        aLA[30 * pl + c] = Luxk;
        aLA[31 * pl + c] = Luyk;
    }
    aLA[29 * pl + c] = Lflk;
    if (acc_eps) aGA[c] = ga0 + Leps;
}

// Terminal adjoint of a loss of the final fields: T = sum of g+, so every
// g+ plane gets dL/dT; f_l gets dL/df_l (packed inputs, nx*ny; null = 0).
__global__ __launch_bounds__(TX * TY) void k_adj_terminal(Geom G, const float* dT, const float* dfl,
                                                          float* ls)
{
    int x, y;
    if (!tile_coords<TY>(G, x, y)) return;
    const size_t pl = (size_t)G.plane, c = (size_t)y * G.pitch + x, i = (size_t)y * G.nx + x;
    const float t = dT ? dT[i] : 0.0f;
#pragma unroll
    for (int k = 0; k < 5; ++k) ls[(10 + k) * pl + c] = t;
    ls[15 * pl + c] = dfl ? dfl[i] : 0.0f;
}

// Gradients per cell from the accumulated adjoints of porosity (direct
// terms), Ac and Bc: Ac = phi nu / (K (1-phi)^2) and Bc = phi F / (sqrt(K)
// (1-phi)) give dAc/dlog K = -Ac, dBc/dlog K = -Bc/2, dAc/dphi = Ac (1/phi +
// 2/(1-phi)), dBc/dphi = Bc (1/phi + 1/(1-phi) + dlog F/dphi) with
// dlog F/dphi = -3/(2 phi) for the Ergun relation (0 when F was given).
__global__ __launch_bounds__(TX * TY) void k_adj_grads(Geom G, const float* ga, const float* eps,
                                                       const float* Ac, const float* Bc, int ergun,
                                                       float* gk, float* ge)
{
    int x, y;
    if (!tile_coords<TY>(G, x, y)) return;
    const size_t pl = (size_t)G.plane, c = (size_t)y * G.pitch + x, i = (size_t)y * G.nx + x;
    const double ep = eps[c], a = Ac[c], b = Bc[c];
    const double lE = ga[c], lA = ga[pl + c], lB = ga[2 * pl + c];
    gk[i] = (float)(-a * lA - 0.5 * b * lB);
    double g = lE;
    if (ep < 1.0) {
        g += lA * a * (1.0 / ep + 2.0 / (1.0 - ep));
        g += lB * b * (1.0 / ep + 1.0 / (1.0 - ep) - (ergun ? 1.5 / ep : 0.0));
    }
    ge[i] = (float)g;
}

}  // namespace

hipError_t launch_adjoint_terminal(const Geom& G, const float* dT, const float* dfl, float* ls,
                                   hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_terminal, dim3(tile_blocks(G, TY)), dim3(TX, TY), 0, s, G, dT, dfl, ls);
    return hipGetLastError();
}

hipError_t launch_adjoint_grads(const Geom& G, const float* ga, const float* eps, const float* Ac,
                                const float* Bc, bool ergun, float* gk, float* ge, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_grads, dim3(tile_blocks(G, TY)), dim3(TX, TY), 0, s, G, ga, eps, Ac,
                       Bc, (int)ergun, gk, ge);
    return hipGetLastError();
}

hipError_t launch_adjoint_step(const Geom& G, const Phys& P, const AdjBufs& B, bool flow,
                               bool first, hipStream_t s)
{
    const dim3 grd(tile_blocks(G, TY)), blk(TX, TY);
    // 32-bit offsets while the largest array (the local adjoints) indexes
    // below 2^30 elements
    if ((uint64_t)ADJ_LA * (uint64_t)G.plane < (1ull << 30)) {
        if (flow && first)
            hipLaunchKernelGGL((k_adj_step<true, true, true>), grd, blk, 0, s, G, P, B);
        else if (flow)
            hipLaunchKernelGGL((k_adj_step<true, false, true>), grd, blk, 0, s, G, P, B);
        else if (first)
            hipLaunchKernelGGL((k_adj_step<false, true, true>), grd, blk, 0, s, G, P, B);
        else
            hipLaunchKernelGGL((k_adj_step<false, false, true>), grd, blk, 0, s, G, P, B);
        return hipGetLastError();
    }
    if (flow && first)
        hipLaunchKernelGGL((k_adj_step<true, true, false>), grd, blk, 0, s, G, P, B);
    else if (flow)
        hipLaunchKernelGGL((k_adj_step<true, false, false>), grd, blk, 0, s, G, P, B);
    else if (first)
        hipLaunchKernelGGL((k_adj_step<false, true, false>), grd, blk, 0, s, G, P, B);
    else
        hipLaunchKernelGGL((k_adj_step<false, false, false>), grd, blk, 0, s, G, P, B);
    return hipGetLastError();
}

}  // namespace dmrtk
