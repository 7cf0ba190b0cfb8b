// HIP kernels (gfx950) of the double-MRT lattice Boltzmann solver for
// solid-liquid phase change in porous media (Liu & He, arXiv:1503.08406).
//
// State layout in HBM (all float32, planar, x fastest, row pitch a multiple
// of 64 elements so every row starts on a 256-byte boundary):
//   f[2][9][ny][pitch]  post-collision D2Q9 populations stored as deviations
//                       f_i - w_i rho0 (rho0 = 1), double-buffered
//   g[2][5][ny][pitch]  post-collision D2Q5 populations, double-buffered
//   fl[2][ny][pitch]    liquid fraction, double-buffered
//   ux, uy[ny][pitch]   velocity of the last step (read only by the same node
//                       for boundary extrapolation, so single-buffered)
//   eps, Ac, Bc         porosity and the two porous drag coefficients
//
// One step = one launch of k_step: every lane owns one node and pulls its
// incoming populations (Eqs. 21, 36), applies the boundary / interface
// extrapolation, iterates the enthalpy update (Eqs. 38, 40-42), recomputes
// the velocity (Eqs. 26-28) and collides both lattices (Eqs. 20, 35).
#include "dmrt_internal.h"

namespace dmrtk {
namespace {

constexpr float W9_0 = 4.0f / 9.0f, W9_1 = 1.0f / 9.0f, W9_2 = 1.0f / 36.0f;

__device__ __forceinline__ float w9(int i) { return i == 0 ? W9_0 : (i <= 4 ? W9_1 : W9_2); }

// Decode the XCD-aware tile index of this block: consecutive blocks go to
// different dies (round-robin), so block b works on tile (b % 8)*per_xcd + b/8
// and each die sweeps a contiguous band of rows, keeping the pull-stencil
// halo rows in that die's L2.
__device__ __forceinline__ bool tile_coords(const Geom& G, int& x, int& y)
{
    const int b = blockIdx.x;
    const int tile = (b % NXCD) * G.per_xcd + (b / NXCD);
    if (tile >= G.ntiles) return false;
    const int tx = tile % G.tiles_x, ty = tile / G.tiles_x;
    x = tx * TX + threadIdx.x;
    y = ty * TY + threadIdx.y;
    return x < G.nx && y < G.ny;
}

// Velocity closure and D2Q9 MRT collision of one node, on the deviations
// d_i = f_i - w_i.  Implements Eqs. (24)-(28) for u, the total force of
// Eq. (4) through Eq. (25) as F = 2 (u - j) (exact identity), the porous
// drag of Eq. (6) in varphi = phi f_l, and Eq. (20) as f+ = f - M^-1 Delta
// with Delta = Lambda (m - m^eq) - (I - Lambda/2) S (Eqs. 19, 22, 23).
__device__ __forceinline__ void flow_collide(float (&d)[9], float fl1, float eps, float Ac,
                                             float Bc, float T1, const Phys& P, float& ux,
                                             float& uy)
{
    const float rho_d = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
    const float jx = (d[1] - d[3]) + (d[5] - d[6]) - (d[7] - d[8]);
    const float jy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
    const float phi = eps * fl1;
    const float Gy = P.gbeta * (T1 - P.T0);
    const float vx = jx, vy = jy + 0.5f * phi * Gy;  // Eq. (27)
    // Eq. (28) with K_e = K f_l^3 ((1-phi)/(1-varphi))^2 and
    // C_e = F_eps f_l^(-3/2), both multiplied through by f_l^2 so that no
    // term overflows as f_l -> 0.
    const float w2 = fl1 * fl1, om = 1.0f - phi;
    const float l0 = 0.5f * (w2 + 0.5f * Ac * om * om);
    const float l1 = 0.5f * Bc * om;
    const float vm = sqrtf(vx * vx + vy * vy);
    const float den = l0 + sqrtf(l0 * l0 + l1 * w2 * vm);  // Eq. (26) times f_l^2
    const float sc = den > 0.0f ? w2 / den : 0.0f;
    ux = vx * sc;
    uy = vy * sc;
    const float Fx = 2.0f * (ux - jx), Fy = 2.0f * (uy - jy);

    const float iphi = 1.0f / phi;
    const float uu = ux * ux + uy * uy;
    const float sa = (d[1] + d[2]) + (d[3] + d[4]);
    const float sd = (d[5] + d[6]) + (d[7] + d[8]);
    const float m1 = -4.0f * d[0] - sa + 2.0f * sd;
    const float m2 = 4.0f * d[0] - 2.0f * sa + sd;
    const float m4 = -2.0f * (d[1] - d[3]) + ((d[5] - d[6]) - (d[7] - d[8]));
    const float m6 = -2.0f * (d[2] - d[4]) + ((d[5] + d[6]) - (d[7] + d[8]));
    const float m7 = (d[1] - d[2]) + (d[3] - d[4]);
    const float m8 = (d[5] - d[6]) + (d[7] - d[8]);
    // equilibrium moments (Eq. 19) minus their rest values
    const float q = 3.0f * uu * iphi;
    const float e1 = -2.0f * rho_d + q, e2 = rho_d - q;
    const float e7 = (ux * ux - uy * uy) * iphi, e8 = ux * uy * iphi;
    // forcing moments (Eq. 22), rho0 = 1
    const float S1 = 6.0f * (ux * Fx + uy * Fy) * iphi;
    const float S7 = 2.0f * (ux * Fx - uy * Fy) * iphi;
    const float S8 = (ux * Fy + uy * Fx) * iphi;
    const float D1 = P.s_e * (m1 - e1) - (1.0f - 0.5f * P.s_e) * S1;
    const float D2 = P.s_eps * (m2 - e2) + (1.0f - 0.5f * P.s_eps) * S1;
    const float D4 = P.s_q * (m4 + ux) + (1.0f - 0.5f * P.s_q) * Fx;
    const float D6 = P.s_q * (m6 + uy) + (1.0f - 0.5f * P.s_q) * Fy;
    const float D7 = P.s_nu * (m7 - e7) - (1.0f - 0.5f * P.s_nu) * S7;
    const float D8 = P.s_nu * (m8 - e8) - (1.0f - 0.5f * P.s_nu) * S8;
    // conserved moments: Delta_3 = -F_x, Delta_5 = -F_y for any s_3 = s_5
    // M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
    const float a = D1 * (1.0f / 36.0f), b = D2 * (1.0f / 36.0f);
    const float ca = -a - 2.0f * b, cd = 2.0f * a + b;
    const float X1 = (-Fx - D4) * (1.0f / 6.0f), Y1 = (-Fy - D6) * (1.0f / 6.0f);
    const float X2 = -Fx * (1.0f / 6.0f) + D4 * (1.0f / 12.0f);
    const float Y2 = -Fy * (1.0f / 6.0f) + D6 * (1.0f / 12.0f);
    const float Pq = 0.25f * D7, Qq = 0.25f * D8;
    d[0] -= 4.0f * (b - a);
    d[1] -= ca + X1 + Pq;
    d[2] -= ca + Y1 - Pq;
    d[3] -= ca - X1 + Pq;
    d[4] -= ca - Y1 - Pq;
    d[5] -= cd + X2 + Y2 + Qq;
    d[6] -= cd - X2 + Y2 - Qq;
    d[7] -= cd - X2 - Y2 + Qq;
    d[8] -= cd + X2 - Y2 - Qq;
}

// D2Q5 MRT collision (Eqs. 32, 34, 35, 37) with T = T1, relaxation of
// moment 1, 2 from tau_T(f_l) = 1/2 + alpha_e(f_l)/(sigma(f_l) c_sT^2).
__device__ __forceinline__ void thermal_collide(float (&g)[5], float fl1, float sig1, float T1,
                                                float ux, float uy, const Phys& P)
{
    const float n1 = g[1] - g[3], n2 = g[2] - g[4];
    const float n3 = -4.0f * g[0] + ((g[1] + g[2]) + (g[3] + g[4]));
    const float n4 = (g[1] + g[3]) - (g[2] + g[4]);
    float za = P.zeta_a;
    if (!P.zeta_uniform) za = 1.0f / (0.5f + (P.lam_as + fl1 * P.dlam) / (sig1 * P.csT2));
    const float ct = P.conv * T1 / sig1;
    const float D1 = za * (n1 - ct * ux), D2 = za * (n2 - ct * uy);
    const float D3 = P.zeta_e * (n3 - P.varpi * T1), D4 = P.zeta_nu * n4;
    // N^-1 = N^T diag(1/5, 1/2, 1/2, 1/20, 1/4)
    const float c3 = 0.05f * D3, c4 = 0.25f * D4;
    g[0] += 0.2f * D3;
    g[1] -= 0.5f * D1 + c3 + c4;
    g[2] -= 0.5f * D2 + c3 - c4;
    g[3] -= -0.5f * D1 + c3 + c4;
    g[4] -= -0.5f * D2 + c3 - c4;
}

template <bool FLOW, bool COUNT>
__global__ __launch_bounds__(TX * TY) void k_step(Geom G, Phys P, StepBufs B)
{
    int x, y;
    if (!tile_coords(G, x, y)) return;
    const long long pl = G.plane;
    const int r0 = y * G.pitch;
    const int c = r0 + x;

    int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
    bool wxm = false, wxp = false, wym = false, wyp = false;
    if (xm < 0) { if (G.per_x) xm += G.nx; else wxm = true; }
    if (xp >= G.nx) { if (G.per_x) xp -= G.nx; else wxp = true; }
    if (ym < 0) { if (G.per_y) ym += G.ny; else wym = true; }
    if (yp >= G.ny) { if (G.per_y) yp -= G.ny; else wyp = true; }
    const int rm = ym * G.pitch, rp = yp * G.pitch;

    const float flk = B.flin[c];
    const float eps = B.eps[c];
    const bool act0 = flk > 0.0f;

    // ---- pull-stream g (Eq. 36)
    float g[5];
    g[0] = B.gin[c];
    g[1] = wxm ? 0.0f : B.gin[pl + r0 + xm];
    g[2] = wym ? 0.0f : B.gin[2 * pl + rm + x];
    g[3] = wxp ? 0.0f : B.gin[3 * pl + r0 + xp];
    g[4] = wyp ? 0.0f : B.gin[4 * pl + rp + x];
    if (wxm | wxp | wym | wyp) {
        // wall: g_i = g_i^eq(T_w, 0) + g_i^+(x) - g_i^eq(T(x), u(x)), own
        // start-of-step values; adiabatic walls take T_w = T(x).
        const float o1 = B.gin[pl + c], o2 = B.gin[2 * pl + c];
        const float o3 = B.gin[3 * pl + c], o4 = B.gin[4 * pl + c];
        const float Tk = g[0] + ((o1 + o2) + (o3 + o4));
        float uxk = 0.0f, uyk = 0.0f;
        if (FLOW && act0) { uxk = B.ux[c]; uyk = B.uy[c]; }
        const float cu = 1.0f / ((P.sig_s + flk * P.dsig) * P.csT2);
        const float w = P.w5_1;
        if (wxm) { const float Tw = G.wall_T[0] ? G.T_wall[0] : Tk; g[1] = w * Tw + o1 - w * Tk * (1.0f + uxk * cu); }
        if (wym) { const float Tw = G.wall_T[2] ? G.T_wall[2] : Tk; g[2] = w * Tw + o2 - w * Tk * (1.0f + uyk * cu); }
        if (wxp) { const float Tw = G.wall_T[1] ? G.T_wall[1] : Tk; g[3] = w * Tw + o3 - w * Tk * (1.0f - uxk * cu); }
        if (wyp) { const float Tw = G.wall_T[3] ? G.T_wall[3] : Tk; g[4] = w * Tw + o4 - w * Tk * (1.0f - uyk * cu); }
    }

    // ---- iterated enthalpy update (Eqs. 38, 40-42) at the receiving node.
    // The loop runs until every lane of the wavefront has converged.
    const float Tstar = g[0] + ((g[1] + g[2]) + (g[3] + g[4]));
    const float alat = eps * P.inv_St;  // phi L_a / c_p
    float f = flk;
    int it = 0;
    for (;;) {
        ++it;
        const float sig = P.sig_s + f * P.dsig;
        const float T = Tstar - alat * (f - flk) / sig;
        const float En = T + f * P.inv_St;
        const float fn = fminf(fmaxf((En - P.T_s) * P.inv_den, 0.0f), 1.0f);
        const bool done = fabsf(fn - f) <= P.fl_tol || it >= P.fl_maxit;
        f = fn;
        if (done) break;
    }
    const float fl1 = f;
    const float sig1 = P.sig_s + fl1 * P.dsig;
    const float T1 = Tstar - alat * (fl1 - flk) / sig1;
    {   // latent source N^-1 S~ = w~_i S~_0 (Eq. 38)
        const float dT = T1 - Tstar;
        g[0] += P.w5_0 * dT;
        g[1] += P.w5_1 * dT;
        g[2] += P.w5_1 * dT;
        g[3] += P.w5_1 * dT;
        g[4] += P.w5_1 * dT;
    }
    if (COUNT) {
        B.it_sum[c] += it;
        if (it > B.it_max[c]) B.it_max[c] = it;
    }

    // ---- flow: only where f_l > 0 (Sec. 4)
    float ux = 0.0f, uy = 0.0f;
    if (FLOW && fl1 > 0.0f) {
        float d[9];
        if (act0) {
            const bool v1 = !wxm && B.flin[r0 + xm] > 0.0f;
            const bool v2 = !wym && B.flin[rm + x] > 0.0f;
            const bool v3 = !wxp && B.flin[r0 + xp] > 0.0f;
            const bool v4 = !wyp && B.flin[rp + x] > 0.0f;
            const bool v5 = !(wxm | wym) && B.flin[rm + xm] > 0.0f;
            const bool v6 = !(wxp | wym) && B.flin[rm + xp] > 0.0f;
            const bool v7 = !(wxp | wyp) && B.flin[rp + xp] > 0.0f;
            const bool v8 = !(wxm | wyp) && B.flin[rp + xm] > 0.0f;
            d[0] = B.fin[c];
            d[1] = v1 ? B.fin[pl + r0 + xm] : 0.0f;
            d[2] = v2 ? B.fin[2 * pl + rm + x] : 0.0f;
            d[3] = v3 ? B.fin[3 * pl + r0 + xp] : 0.0f;
            d[4] = v4 ? B.fin[4 * pl + rp + x] : 0.0f;
            d[5] = v5 ? B.fin[5 * pl + rm + xm] : 0.0f;
            d[6] = v6 ? B.fin[6 * pl + rm + xp] : 0.0f;
            d[7] = v7 ? B.fin[7 * pl + rp + xp] : 0.0f;
            d[8] = v8 ? B.fin[8 * pl + rp + xm] : 0.0f;
            if (!(v1 && v2 && v3 && v4 && v5 && v6 && v7 && v8)) {
                // wall or solid source: f_i = f_i^eq(rho, 0) + f_i^+(x)
                //   - f_i^eq(rho, u; varphi) with the node's own start-of-step
                // values (Eq. 29; rho cancels).
                const float uxk = B.ux[c], uyk = B.uy[c];
                const float iph = 1.0f / (eps * flk);
                const float uu = 1.5f * (uxk * uxk + uyk * uyk) * iph;
#define DMRT_NEE(I, EU, W) \
    if (!v##I) { const float eu = (EU); d[I] = B.fin[I * pl + c] - (W) * (3.0f * eu + 4.5f * eu * eu * iph - uu); }
                DMRT_NEE(1, uxk, W9_1)
                DMRT_NEE(2, uyk, W9_1)
                DMRT_NEE(3, -uxk, W9_1)
                DMRT_NEE(4, -uyk, W9_1)
                DMRT_NEE(5, uxk + uyk, W9_2)
                DMRT_NEE(6, uyk - uxk, W9_2)
                DMRT_NEE(7, -uxk - uyk, W9_2)
                DMRT_NEE(8, uxk - uyk, W9_2)
#undef DMRT_NEE
            }
        } else {
            // node became liquid in this step: restart at rest, f_i = w_i rho0
#pragma unroll
            for (int i = 0; i < 9; ++i) d[i] = 0.0f;
        }
        flow_collide(d, fl1, eps, B.Ac[c], B.Bc[c], T1, P, ux, uy);
#pragma unroll
        for (int i = 0; i < 9; ++i) B.fout[i * pl + c] = d[i];
        B.ux[c] = ux;
        B.uy[c] = uy;
    }

    thermal_collide(g, fl1, sig1, T1, ux, uy, P);
#pragma unroll
    for (int i = 0; i < 5; ++i) B.gout[i * pl + c] = g[i];
    B.flout[c] = fl1;
}

template <bool FLOW>
__global__ __launch_bounds__(TX * TY) void k_load_state(Geom G, Phys P, const float* f_pre,
                                                        const float* g_pre, const float* fl_pre,
                                                        float* fcur, float* gcur, float* flcur,
                                                        float* uxb, float* uyb, const float* epsb,
                                                        const float* Ac, const float* Bc)
{
    int x, y;
    if (!tile_coords(G, x, y)) return;
    const long long pl = G.plane;
    const long long cp = (long long)G.nx * G.ny;  // plane of the packed input
    const int c = y * G.pitch + x;
    const long long ci = (long long)y * G.nx + x;
    float g[5];
#pragma unroll
    for (int i = 0; i < 5; ++i)
        g[i] = g_pre ? g_pre[i * cp + ci] : (i == 0 ? P.w5_0 : P.w5_1) * P.T_init;
    const float T = g[0] + ((g[1] + g[2]) + (g[3] + g[4]));
    float fl;
    if (fl_pre) {
        fl = fl_pre[ci];
    } else {
        fl = fminf(fmaxf((T - P.T_s) * P.inv_dTm, 0.0f), 1.0f);  // Eq. (42)
    }
    const float eps = epsb[c];
    float ux = 0.0f, uy = 0.0f;
    if (FLOW && fl > 0.0f) {
        float d[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = f_pre ? f_pre[i * cp + ci] - w9(i) : 0.0f;
        flow_collide(d, fl, eps, Ac[c], Bc[c], T, P, ux, uy);
#pragma unroll
        for (int i = 0; i < 9; ++i) fcur[i * pl + c] = d[i];
        uxb[c] = ux;
        uyb[c] = uy;
    }
    const float sig = P.sig_s + fl * P.dsig;
    thermal_collide(g, fl, sig, T, ux, uy, P);
#pragma unroll
    for (int i = 0; i < 5; ++i) gcur[i * pl + c] = g[i];
    flcur[c] = fl;
}

__global__ __launch_bounds__(TX * TY) void k_fields(Geom G, const float* gcur, const float* flcur,
                                                    const float* uxb, const float* uyb, int flow,
                                                    float* out)
{
    int x, y;
    if (!tile_coords(G, x, y)) return;
    const long long pl = G.plane, cp = (long long)G.nx * G.ny;
    const int c = y * G.pitch + x;
    const long long ci = (long long)y * G.nx + x;
    const float T = gcur[c] + ((gcur[pl + c] + gcur[2 * pl + c]) + (gcur[3 * pl + c] + gcur[4 * pl + c]));
    const float fl = flcur[c];
    const bool act = flow && fl > 0.0f;
    out[ci] = T;
    out[cp + ci] = act ? uxb[c] : 0.0f;
    out[2 * cp + ci] = act ? uyb[c] : 0.0f;
    out[3 * cp + ci] = fl;
}

__global__ __launch_bounds__(TX * TY) void k_populations(Geom G, const float* fcur,
                                                         const float* gcur, const float* flcur,
                                                         int flow, float* fpost, float* gpost)
{
    int x, y;
    if (!tile_coords(G, x, y)) return;
    const long long pl = G.plane, cp = (long long)G.nx * G.ny;
    const int c = y * G.pitch + x;
    const long long ci = (long long)y * G.nx + x;
    const bool act = flcur[c] > 0.0f;
    if (fpost) {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            fpost[i * cp + ci] = act ? (flow ? fcur[i * pl + c] : 0.0f) + w9(i) : 0.0f;
    }
    if (gpost) {
#pragma unroll
        for (int i = 0; i < 5; ++i) gpost[i * cp + ci] = gcur[i * pl + c];
    }
}

// Wavefront (64-lane) sum / max, then across the 4 waves of a block.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ __launch_bounds__(TX * TY) void k_diag(Geom G, Phys P, const float* fcur,
                                                  const float* gcur, const float* flcur,
                                                  const float* uxb, const float* uyb,
                                                  const float* epsb, int flow, double* partials)
{
    __shared__ double red[TY][DIAG_SLOTS];
    int x, y;
    double v[DIAG_SLOTS] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (tile_coords(G, x, y)) {
        const long long pl = G.plane;
        const int c = y * G.pitch + x;
        float gs[5];
        for (int i = 0; i < 5; ++i) gs[i] = gcur[i * pl + c];
        const float T = gs[0] + ((gs[1] + gs[2]) + (gs[3] + gs[4]));
        const float fl = flcur[c];
        const float eps = epsb[c];
        int bad = 0;
        for (int i = 0; i < 5; ++i) bad += !isfinite(gs[i]);
        bad += !isfinite(fl);
        double mass = 0.0, um = 0.0;
        if (fl > 0.0f) {
            double r = 1.0;
            if (flow) {
                for (int i = 0; i < 9; ++i) {
                    const float di = fcur[i * pl + c];
                    bad += !isfinite(di);
                    r += (double)di;
                }
                const float ux = uxb[c], uy = uyb[c];
                bad += !isfinite(ux) + !isfinite(uy);
                um = sqrt((double)ux * ux + (double)uy * uy);
            }
            mass = r;
        }
        const double sig = (double)P.sig_s + (double)fl * P.dsig;
        v[0] = mass;
        v[1] = sig * T + (double)eps * fl * P.inv_St;
        v[2] = fl;
        v[3] = T;
        v[4] = um;
        v[5] = fl > 0.0f ? 1.0 : 0.0;
        v[6] = bad;
        v[7] = 0.0;
    }
    const int lane = threadIdx.x, wv = threadIdx.y;
#pragma unroll
    for (int k = 0; k < DIAG_SLOTS; ++k) v[k] = (k == 4) ? wave_max(v[k]) : wave_sum(v[k]);
    if (lane == 0)
        for (int k = 0; k < DIAG_SLOTS; ++k) red[wv][k] = v[k];
    __syncthreads();
    if (wv == 0 && lane < DIAG_SLOTS) {
        double a = red[0][lane];
        for (int w = 1; w < TY; ++w) a = (lane == 4) ? fmax(a, red[w][lane]) : a + red[w][lane];
        partials[(long long)blockIdx.x * DIAG_SLOTS + lane] = a;
    }
}

// Front of each row: first f_l = 1/2 crossing scanned from x = 0, linearly
// interpolated, plus one for the wall offset (0 when the row has none).
__global__ __launch_bounds__(256) void k_front(Geom G, const float* flcur, float* front)
{
    __shared__ int red[4];
    const int row = blockIdx.x;
    const float* r = flcur + (long long)row * G.pitch;
    const bool s0 = r[0] >= 0.5f;
    int first = G.nx;
    for (int i = threadIdx.x; i < G.nx; i += blockDim.x)
        if ((r[i] >= 0.5f) != s0) { first = i; break; }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) first = min(first, __shfl_xor(first, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = first;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = min(m, red[w]);
        float out = 0.0f;
        if (m < G.nx) {
            const float a = r[m - 1], b = r[m];
            out = (float)(m - 1) + (a - 0.5f) / (a - b) + 1.0f;
        }
        front[row] = out;
    }
}

inline dim3 tile_grid(const Geom& G) { return dim3(NXCD * G.per_xcd); }

}  // namespace

hipError_t launch_step(const Geom& G, const Phys& P, const StepBufs& B, bool flow, bool counted,
                       hipStream_t s)
{
    const dim3 blk(TX, TY), grd = tile_grid(G);
    if (flow) {
        if (counted) hipLaunchKernelGGL((k_step<true, true>), grd, blk, 0, s, G, P, B);
        else hipLaunchKernelGGL((k_step<true, false>), grd, blk, 0, s, G, P, B);
    } else {
        if (counted) hipLaunchKernelGGL((k_step<false, true>), grd, blk, 0, s, G, P, B);
        else hipLaunchKernelGGL((k_step<false, false>), grd, blk, 0, s, G, P, B);
    }
    return hipGetLastError();
}

hipError_t launch_load_state(const Geom& G, const Phys& P, const float* f_pre, const float* g_pre,
                             const float* fl_pre, float* fcur, float* gcur, float* flcur,
                             float* ux, float* uy, const float* eps, const float* Ac,
                             const float* Bc, bool flow, hipStream_t s)
{
    const dim3 blk(TX, TY), grd = tile_grid(G);
    if (flow)
        hipLaunchKernelGGL((k_load_state<true>), grd, blk, 0, s, G, P, f_pre, g_pre, fl_pre, fcur,
                           gcur, flcur, ux, uy, eps, Ac, Bc);
    else
        hipLaunchKernelGGL((k_load_state<false>), grd, blk, 0, s, G, P, f_pre, g_pre, fl_pre,
                           fcur, gcur, flcur, ux, uy, eps, Ac, Bc);
    return hipGetLastError();
}

hipError_t launch_fields(const Geom& G, const float* gcur, const float* flcur, const float* ux,
                         const float* uy, bool flow, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_fields, tile_grid(G), dim3(TX, TY), 0, s, G, gcur, flcur, ux, uy,
                       (int)flow, out);
    return hipGetLastError();
}

hipError_t launch_populations(const Geom& G, const float* fcur, const float* gcur,
                              const float* flcur, bool flow, float* fpost, float* gpost,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_populations, tile_grid(G), dim3(TX, TY), 0, s, G, fcur, gcur, flcur,
                       (int)flow, fpost, gpost);
    return hipGetLastError();
}

hipError_t launch_diag(const Geom& G, const Phys& P, const float* fcur, const float* gcur,
                       const float* flcur, const float* ux, const float* uy, const float* eps,
                       bool flow, double* partials, int* nblocks, hipStream_t s)
{
    const dim3 grd = tile_grid(G);
    *nblocks = (int)grd.x;
    hipLaunchKernelGGL(k_diag, grd, dim3(TX, TY), 0, s, G, P, fcur, gcur, flcur, ux, uy, eps,
                       (int)flow, partials);
    return hipGetLastError();
}

hipError_t launch_front(const Geom& G, const float* flcur, float* front, hipStream_t s)
{
    hipLaunchKernelGGL(k_front, dim3(G.ny), dim3(256), 0, s, G, flcur, front);
    return hipGetLastError();
}

}  // namespace dmrtk
