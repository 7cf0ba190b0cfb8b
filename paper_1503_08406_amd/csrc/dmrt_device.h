// Device-side building blocks of the double-MRT lattice Boltzmann kernels
// (Liu & He, arXiv:1503.08406): tile decoding, memory access policies and
// the per-node collision arithmetic shared by the step and state kernels.
#pragma once

#include "dmrt_internal.h"

namespace dmrtk {

constexpr float W9_0 = 4.0f / 9.0f, W9_1 = 1.0f / 9.0f, W9_2 = 1.0f / 36.0f;

__device__ __forceinline__ float w9(int i) { return i == 0 ? W9_0 : (i <= 4 ? W9_1 : W9_2); }

// Hardware reciprocal and square root (1 ulp); the arithmetic of a node does
// not need correctly rounded division.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Tile of this block for a launch of 64 x TYB threads.  Blocks are handed to
// the 8 dies round-robin, so block b takes tile (b % 8)*per_xcd + b/8: each
// die sweeps one contiguous band of rows and the pull-stencil halo rows stay
// in that die's L2.
template <int TYB>
__device__ __forceinline__ bool tile_coords(const Geom& G, int& x, int& y)
{
    const int tiles_x = (G.nx + TX - 1) / TX;
    const int ntiles = tiles_x * ((G.ny + TYB - 1) / TYB);
    const int per_xcd = (ntiles + NXCD - 1) / NXCD;
    const int b = blockIdx.x;
    const int tile = (b % NXCD) * per_xcd + b / NXCD;
    if (tile >= ntiles) return false;
    x = (tile % tiles_x) * TX + (int)threadIdx.x;
    y = (tile / tiles_x) * TYB + (int)threadIdx.y;
    return x < G.nx && y < G.ny;
}

// Origin of this block's tile of 64 x ROWS nodes (same mapping).
template <int ROWS>
__device__ __forceinline__ bool tile_origin(const Geom& G, int& x0, int& y0)
{
    const int tiles_x = (G.nx + TX - 1) / TX;
    const int ntiles = tiles_x * ((G.ny + ROWS - 1) / ROWS);
    const int per_xcd = (ntiles + NXCD - 1) / NXCD;
    const int b = blockIdx.x;
    const int tile = (b % NXCD) * per_xcd + b / NXCD;
    if (tile >= ntiles) return false;
    x0 = (tile % tiles_x) * TX;
    y0 = (tile / tiles_x) * ROWS;
    return true;
}

// Position in a die's tile list of the die's j-th block (of n): the list in
// groups of 32 consecutive tiles, group g rotated by g.  Blocks reach a
// die's CUs in a fixed rotation, so with rows of tiles whose length shares
// a factor of 8 or more with 32 (8 tiles per cavity row, say) the same CUs
// would keep getting the same tile column; the column at the hot wall,
// which holds the liquid and the flow work, then lands on a few CUs.
// Rotating each group spreads it while neighbouring tiles stay within 32
// list places (measured: 64 cavities of 496 x 512, 179 -> 145 us per step;
// a 992-wide lattice, 10.3 -> 9.3 us per step).  Where rows do not share
// the factor (17 or 67 tiles) the rotation cost 3-4 %, so it is used only
// where they do.  A full group rotates without a division (0.4-0.8 %
// faster where the rotation is used).
__device__ __forceinline__ int rotated_tile(int j, int n)
{
    const int g = j >> 5, base = g << 5;
    const int len = min(32, n - base);  // the last group may be shorter
    if (len == 32) return base + (((j & 31) + g) & 31);  // a full group: no division
    return base + ((j & 31) + g % len) % len;
}

// Tile origin of the step kernel from the host-computed tiling constants
// (tiles W wide); RT: each die's tiles in the rotated groups of rotated_tile
// where G.st_rot says so (rows of tiles a multiple of 8 long):
// q = tile / st_tx via q = (hi + ((t - hi) >> 1)) >> (shift - 1), hi =
// mulhi(t, magic) (division by an invariant integer, Granlund & Montgomery).
// Branch-free, so that nothing stands between the kernel-argument loads and
// the first memory batch.
template <int ROWS, int W = TX, bool RT = false>
__device__ __forceinline__ bool step_tile_origin(const Geom& G, int& x0, int& y0)
{
    const uint32_t b = blockIdx.x;
    uint32_t tile = (b & (NXCD - 1)) * (uint32_t)G.st_per_xcd + (b >> 3);
    if (RT && G.st_rot) {
        const int first = (int)(b & (NXCD - 1)) * G.st_per_xcd, j = (int)(b >> 3);
        const int n = min(G.st_per_xcd, G.st_ntiles - first);
        tile = j < n ? (uint32_t)(first + rotated_tile(j, n)) : (uint32_t)G.st_ntiles;
    }
    const uint32_t hi = __umulhi(tile, G.st_magic);
    const uint32_t qd = (hi + ((tile - hi) >> 1)) >> ((uint32_t)(G.st_shift - 1) & 31u);
    const uint32_t q = G.st_shift == 0 ? tile : qd;  // shift 0: one tile per row
    x0 = (int)(tile - q * (uint32_t)G.st_tx) * W;
    y0 = (int)q * ROWS;
    return tile < (uint32_t)G.st_ntiles;
}

// tile_coords with each die's tiles in the rotated groups of rotated_tile
// where a row of tiles is a multiple of 8 long (the discrete adjoint: at
// 512^2 its 8 tiles per row put the hot wall's column, the flow part of the
// reversed step, on 4 of each die's 32 CUs; rotated, 26.5 -> 22.7 ms per
// reversed run of 2000 steps).
template <int TYB>
__device__ __forceinline__ bool tile_coords_rotated(const Geom& G, int& x, int& y)
{
    const int tiles_x = (G.nx + TX - 1) / TX;
    const int ntiles = tiles_x * ((G.ny + TYB - 1) / TYB);
    const int per_xcd = (ntiles + NXCD - 1) / NXCD;
    const int b = blockIdx.x, first = (b % NXCD) * per_xcd, j = b / NXCD;
    const int n = min(per_xcd, ntiles - first);
    if (j >= n) return false;
    const int tile = first + (tiles_x % 8 == 0 ? rotated_tile(j, n) : j);
    x = (tile % tiles_x) * TX + (int)threadIdx.x;
    y = (tile / tiles_x) * TYB + (int)threadIdx.y;
    return x < G.nx && y < G.ny;
}

// Keeps a batch of loads together: the empty statement takes every value as
// a register operand, so each load is issued on every path (none is sunk
// into the branch that uses it) and the batch is waited for once, here.
template <int N>
__device__ __forceinline__ void pin_loads(float (&v)[N])
{
#pragma unroll
    for (int i = 0; i < N; ++i) asm volatile("" : "+v"(v[i]));
}

inline int tile_blocks(const Geom& G, int TYB)
{
    const int tiles_x = (G.nx + TX - 1) / TX;
    const int ntiles = tiles_x * ((G.ny + TYB - 1) / TYB);
    return NXCD * ((ntiles + NXCD - 1) / NXCD);
}

// Cache policy of the state stores: the cache-policy bits of a gfx950
// buffer store (sc0 = 1, nt = 2, sc1 = 16).
//   ST_PLAIN  default write-back through the die's L2;
//   ST_WT     sc0 | sc1, system scope: written through the L2, for state the
//             next step reads back from the Infinity Cache (a working set
//             that fits there);
//   ST_NT     nt, streaming: for state larger than the Infinity Cache.
enum : int { ST_PLAIN = 0, ST_WT = 17, ST_NT = 2 };

// Access to an array of float planes.  BufIOT uses a buffer resource with a
// 32-bit byte offset per node (VGPR) and a 32-bit plane offset (SGPR): one
// instruction per access, range-checked by the hardware; SP is the cache
// policy of its stores.  PtrIO is the 64-bit pointer form for arrays larger
// than 4 GB.
template <int SP>
struct BufIOT {
    using off_t = uint32_t;
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ BufIOT(const float* p, uint64_t nbytes)
        : r(__builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(uint32_t)nbytes, 0x00020000))
    {
    }
    __device__ __forceinline__ float ld(off_t o, off_t plane_off) const
    {
        // the b32 buffer intrinsics move raw 32-bit words: bit-cast, never convert
        // plane offsets are uniform; readfirstlane keeps them in SGPRs (the
        // buffer instruction's soffset) instead of a per-lane waterfall loop
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                             r, o, __builtin_amdgcn_readfirstlane(plane_off), 0));
    }
    __device__ __forceinline__ void st(off_t o, off_t plane_off, float v) const
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, o,
                                              __builtin_amdgcn_readfirstlane(plane_off), SP);
    }
};
using BufIO = BufIOT<ST_PLAIN>;

// WinIOT: the arrays of a step inside one window of fewer than 4 GB
// (StepBufs::win), all through one buffer resource over the window; an
// array is its byte offset in the window, added to the plane offset in the
// instruction's scalar offset.  One resource for all arrays instead of one
// each (four scalar registers apiece) leaves the step kernels' scalar
// values in registers rather than spilled to vector-register lanes.  PAIR:
// two windows, the arrays written in StepBufs::wout.
template <int SP, bool PAIR = false>
struct WinIOT {
    using off_t = uint32_t;
    static constexpr bool in_window = true;
    static constexpr bool pair = PAIR;
    __amdgpu_buffer_rsrc_t r;
    uint32_t a;  // byte offset of the array in the window
    __device__ __forceinline__ WinIOT(const char* win, uint32_t nbytes, const float* p)
        : r(__builtin_amdgcn_make_buffer_rsrc((void*)win, (short)0, (int)nbytes, 0x00020000)),
          a((uint32_t)((const char*)p - win))
    {
    }
    __device__ __forceinline__ float ld(off_t o, off_t plane_off) const
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                             r, o, __builtin_amdgcn_readfirstlane(a + plane_off), 0));
    }
    __device__ __forceinline__ void st(off_t o, off_t plane_off, float v) const
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, o,
                                              __builtin_amdgcn_readfirstlane(a + plane_off), SP);
    }
};

template <int SP>
struct PtrIOT {
    using off_t = uint64_t;
    char* p;
    __device__ __forceinline__ PtrIOT(const float* q, uint64_t) : p((char*)q) {}
    __device__ __forceinline__ float ld(off_t o, off_t plane_off) const
    {
        return *(const float*)(p + plane_off + o);
    }
    __device__ __forceinline__ void st(off_t o, off_t plane_off, float v) const
    {
        float* a = (float*)(p + plane_off + o);
        if constexpr (SP == ST_NT)
            __builtin_nontemporal_store(v, a);
        else
            *a = v;
    }
};
using PtrIO = PtrIOT<ST_PLAIN>;

// Velocity closure and D2Q9 MRT collision of one node, on the deviations
// d_i = f_i - w_i rho0 (rho0 = 1).  Eqs. (24)-(28) give u; the total force
// of Eq. (4) follows from Eq. (25) as F = 2 (u - j) (an exact identity); the
// porous drag of Eq. (6) is taken in varphi = phi f_l; Eq. (20) is applied
// as f+ = f - M^-1 Delta with Delta = Lambda (m - m^eq) - (I - Lambda/2) S
// (Eqs. 19, 22, 23).  Ac = phi nu_l / (K (1-phi)^2), Bc = phi F_eps /
// (sqrt(K) (1-phi)) are the drag coefficients at f_l = 1.
__device__ __forceinline__ void flow_collide(float (&d)[9], float fl1, float eps, float Ac,
                                             float Bc, float T1, const Phys& P, float& ux,
                                             float& uy)
{
    const float sa = (d[1] + d[2]) + (d[3] + d[4]);
    const float sd = (d[5] + d[6]) + (d[7] + d[8]);
    const float rho_d = d[0] + sa + sd;
    const float dx13 = d[1] - d[3], dy24 = d[2] - d[4];
    const float a58 = d[5] - d[7], b68 = d[6] - d[8];  // e_x: a58 - b68, e_y: a58 + b68
    const float jx = dx13 + (a58 - b68);
    const float jy = dy24 + (a58 + b68);
    const float phi = eps * fl1;
    const float vy = jy + 0.5f * phi * (P.gbeta * (T1 - P.T0));  // Eq. (27)
    const float vx = jx;
    // Eq. (28) with K_e = K f_l^3 ((1-phi)/(1-varphi))^2 and
    // C_e = F_eps f_l^(-3/2), multiplied through by f_l^2 so that no term
    // overflows as f_l -> 0.
    const float w2 = fl1 * fl1, om = 1.0f - phi;
    const float l0 = 0.5f * (w2 + 0.5f * Ac * om * om);
    const float l1 = 0.5f * Bc * om;
    const float vm = fsqrt(vx * vx + vy * vy);
    const float den = l0 + fsqrt(l0 * l0 + l1 * w2 * vm);  // Eq. (26) times f_l^2
    const float sc = den > 0.0f ? w2 * frcp(den) : 0.0f;
    ux = vx * sc;
    uy = vy * sc;
    const float Fx = 2.0f * (ux - jx), Fy = 2.0f * (uy - jy);

    const float iphi = frcp(phi);
    const float m1 = 2.0f * sd - sa - 4.0f * d[0];
    const float m2 = sd - 2.0f * sa + 4.0f * d[0];
    const float m4 = (a58 - b68) - 2.0f * dx13;
    const float m6 = (a58 + b68) - 2.0f * dy24;
    const float m7 = (d[1] + d[3]) - (d[2] + d[4]);
    const float m8 = (d[5] + d[7]) - (d[6] + d[8]);
    // equilibrium moments (Eq. 19) minus their rest values, forcing (Eq. 22)
    const float uxi = ux * iphi, uyi = uy * iphi;
    const float q = 3.0f * (ux * uxi + uy * uyi);
    const float S1 = 6.0f * (uxi * Fx + uyi * Fy);
    const float S7 = 2.0f * (uxi * Fx - uyi * Fy);
    const float S8 = uxi * Fy + uyi * Fx;
    const float D1 = P.s_e * (m1 + 2.0f * rho_d - q) - (1.0f - 0.5f * P.s_e) * S1;
    const float D2 = P.s_eps * (m2 - rho_d + q) + (1.0f - 0.5f * P.s_eps) * S1;
    const float D4 = P.s_q * (m4 + ux) + (1.0f - 0.5f * P.s_q) * Fx;
    const float D6 = P.s_q * (m6 + uy) + (1.0f - 0.5f * P.s_q) * Fy;
    const float D7 = P.s_nu * (m7 - (ux * uxi - uy * uyi)) - (1.0f - 0.5f * P.s_nu) * S7;
    const float D8 = P.s_nu * (m8 - ux * uyi) - (1.0f - 0.5f * P.s_nu) * S8;
    // conserved moments: Delta_3 = -F_x, Delta_5 = -F_y for any s_3 = s_5.
    // M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
    const float a = D1 * (1.0f / 36.0f), b = D2 * (1.0f / 36.0f);
    const float ca = -a - 2.0f * b, cd = 2.0f * a + b;
    const float X1 = (-Fx - D4) * (1.0f / 6.0f), Y1 = (-Fy - D6) * (1.0f / 6.0f);
    const float X2 = D4 * (1.0f / 12.0f) - Fx * (1.0f / 6.0f);
    const float Y2 = D6 * (1.0f / 12.0f) - Fy * (1.0f / 6.0f);
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

// Heat-capacity ratio of a node, sigma(f_l) = s0 + f_l ds: the uniform
// pair, or Eq. (7) with the node's porosity (rho_s = rho_l).  VAR = false
// compiles the default model only.
template <bool VAR>
__device__ __forceinline__ void node_sigma(const Phys& P, float eps, float& s0, float& ds)
{
    if (VAR && P.sig_mode) {
        s0 = eps * P.cps + (1.0f - eps) * P.cm;
        ds = eps * (1.0f - P.cps);
    } else {
        s0 = P.sig_s;
        ds = P.dsig;
    }
}

// k_e / k_l of Eq. (8).  With z = k_e^(1/3) the equation is the cubic
// z^3 + p z - k_m = 0, p = phi (k_m - k_p) / k_p^(1/3), k_p = f_l + (1 - f_l)
// k_s; k_e lies between k_m and k_p, and from z = cbrt(max(k_m, k_p)), where
// the cubic is non-negative and convex, Newton's method descends
// monotonically to the largest root.
__device__ __forceinline__ float ke_ratio(const Phys& P, float phi, float fl)
{
    const float kp = fl + (1.0f - fl) * P.ks;
    const float p = phi * (P.km - kp) / cbrtf(kp);
    float z = cbrtf(fmaxf(P.km, kp));
    for (int i = 0; i < 32; ++i) {
        const float dz = ((z * z + p) * z - P.km) / (3.0f * z * z + p);
        z -= dz;
        if (!(fabsf(dz) > 4e-7f * z)) break;  // a few ulps: rounding can keep |dz| at 1-2 ulps
    }
    return z * z * z;
}

// zeta_alpha = 1/tau_T(f_l) with tau_T = 1/2 + alpha_e(f_l)/(sigma c_sT^2);
// alpha_e = lambda alpha(f_l), linear between the phases, or alpha_l k_e /
// k_l (Eq. 8) with the node's porosity eps.  UT: compiled for uniform
// thermal properties (P.zeta_uniform set, sigma_s = sigma_l), which the
// launch has checked.
template <bool VAR, bool UT = false>
__device__ __forceinline__ float zeta_alpha(const Phys& P, float fl, float isig, float eps)
{
    if (UT || P.zeta_uniform) return P.zeta_a;
    if (VAR && P.ke_mode)
        return frcp(0.5f + P.alpha_l * ke_ratio(P, eps, fl) * isig * P.inv_csT2);
    return frcp(0.5f + (P.lam_as + fl * P.dlam) * isig * P.inv_csT2);
}

// D2Q5 MRT collision (Eqs. 32, 34, 35, 37) with temperature T1 and
// 1/sigma = isig at a node of porosity eps.
template <bool VAR, bool UT = false>
__device__ __forceinline__ void thermal_collide(float (&g)[5], float fl1, float isig, float T1,
                                                float ux, float uy, float eps, const Phys& P)
{
    const float n1 = g[1] - g[3], n2 = g[2] - g[4];
    const float s13 = g[1] + g[3], s24 = g[2] + g[4];
    const float n3 = (s13 + s24) - 4.0f * g[0];
    const float n4 = s13 - s24;
    const float za = zeta_alpha<VAR, UT>(P, fl1, isig, eps);
    const float ct = P.conv * T1 * isig;
    const float D1 = za * (n1 - ct * ux), D2 = za * (n2 - ct * uy);
    const float D3 = P.zeta_e * (n3 - P.varpi * T1), D4 = P.zeta_nu * n4;
    // N^-1 = N^T diag(1/5, 1/2, 1/2, 1/20, 1/4)
    const float c3 = 0.05f * D3, c4 = 0.25f * D4;
    const float h1 = 0.5f * D1, h2 = 0.5f * D2;
    g[0] += 0.2f * D3;
    g[1] -= h1 + c3 + c4;
    g[2] -= h2 + c3 - c4;
    g[3] -= c3 + c4 - h1;
    g[4] -= c3 - c4 - h2;
}

}  // namespace dmrtk
