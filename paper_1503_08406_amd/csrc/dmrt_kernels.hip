// HIP kernels (gfx950) of the double-MRT lattice Boltzmann solver for
// solid-liquid phase change in porous media (Liu & He, arXiv:1503.08406).
//
// State layout in HBM (all float32, planar, x fastest, row pitch a multiple
// of 64 elements so every row starts on a 256-byte boundary):
//   f[2][10][ny][pitch] post-collision D2Q9 populations stored as deviations
//                       f_i - w_i rho0 (rho0 = 1) and, in plane 9, rho - 1
//                       of liquid nodes; double-buffered
//   g[2][5][ny][pitch]  post-collision D2Q5 populations, double-buffered
//   fl[2][ny][pitch]    liquid fraction, double-buffered
//   ux, uy[ny][pitch]   velocity of the last step (read only by the same node
//                       for boundary extrapolation, so single-buffered)
//   eps, Ac, Bc         porosity and the two porous drag coefficients
//
// This file holds the auxiliary kernels (state loading, field extraction,
// diagnostics); the time step itself is in dmrt_step.hip.
#include "dmrt_device.h"

#include <algorithm>

namespace dmrtk {
namespace {

template <bool FLOW>
__global__ __launch_bounds__(TX * TY) void k_load_state(Geom G, Phys P, const float* f_pre,
                                                        const float* g_pre, const float* fl_pre,
                                                        float* fcur, float* gcur, float* flcur,
                                                        float* uxb, float* uyb, const float* epsb,
                                                        const float* Acb, const float* Bcb,
                                                        float eps_u, float Ac_u, float Bc_u)
{
    int x, y;
    if (!tile_coords<TY>(G, x, y)) return;
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
    const float eps = epsb ? epsb[c] : eps_u;
    float ux = 0.0f, uy = 0.0f;
    if (FLOW && fl > 0.0f) {
        float d[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) d[i] = f_pre ? f_pre[i * cp + ci] - w9(i) : 0.0f;
        flow_collide(d, fl, eps, Acb ? Acb[c] : Ac_u, Bcb ? Bcb[c] : Bc_u, T, P, ux, uy);
        float r = 0.0f;  // rho - 1, summed in population order
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            fcur[i * pl + c] = d[i];
            r += d[i];
        }
        fcur[9 * pl + c] = r;
        uxb[c] = ux;
        uyb[c] = uy;
    }
    float sg0, dsg;
    node_sigma<true>(P, eps, sg0, dsg);
    thermal_collide<true>(g, fl, frcp(sg0 + fl * dsg), T, ux, uy, eps, P);
#pragma unroll
    for (int i = 0; i < 5; ++i) gcur[i * pl + c] = g[i];
    flcur[c] = fl;
}

// Plain copy of n floats (kept as a kernel so that it can sit in a graph).
__global__ __launch_bounds__(256) void k_copy(float* __restrict__ dst, const float* __restrict__ src,
                                              size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ __launch_bounds__(TX * TY) void k_fields(Geom G, const float* gcur, const float* flcur,
                                                    const float* uxb, const float* uyb, int flow,
                                                    float* out)
{
    int x, y;
    if (!tile_coords<TY>(G, x, y)) return;
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
    if (!tile_coords<TY>(G, x, y)) return;
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
    if (tile_coords<TY>(G, x, y)) {
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
        float sg0, dsg;
        node_sigma<true>(P, eps, sg0, dsg);
        const double sig = (double)sg0 + (double)fl * dsg;
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

// Final reduction of the diagnostics on the device, in the order of the host
// loop of dmrt_diag (block by block, row by row), one lane per result, so
// that both give the same bits.
__global__ __launch_bounds__(64) void k_diag_reduce(const double* part, int nb,
                                                    const float* front, int ny, double* res)
{
    const int k = (int)threadIdx.x;
    if (k < DIAG_SLOTS) {
        double a = 0.0;
        for (int b = 0; b < nb; ++b) {
            const double v = part[(long long)b * DIAG_SLOTS + k];
            a = (k == 4) ? fmax(a, v) : a + v;
        }
        res[k] = a;
    } else if (k == DIAG_SLOTS) {
        double a = 0.0;
        for (int r = 0; r < ny; ++r) a += front[r];
        res[k] = a;
    } else if (k == DIAG_SLOTS + 1) {
        double a = 0.0;
        for (int r = 0; r < ny; ++r) a = fmax(a, (double)front[r]);
        res[k] = a;
    }
}

inline dim3 tile_grid(const Geom& G) { return dim3(tile_blocks(G, TY)); }

}  // namespace

hipError_t launch_load_state(const Geom& G, const Phys& P, const float* f_pre, const float* g_pre,
                             const float* fl_pre, float* fcur, float* gcur, float* flcur,
                             float* ux, float* uy, const float* eps, const float* Ac,
                             const float* Bc, bool flow, hipStream_t s, float eps_u, float Ac_u,
                             float Bc_u)
{
    const dim3 blk(TX, TY), grd = tile_grid(G);
    if (flow)
        hipLaunchKernelGGL((k_load_state<true>), grd, blk, 0, s, G, P, f_pre, g_pre, fl_pre, fcur,
                           gcur, flcur, ux, uy, eps, Ac, Bc, eps_u, Ac_u, Bc_u);
    else
        hipLaunchKernelGGL((k_load_state<false>), grd, blk, 0, s, G, P, f_pre, g_pre, fl_pre,
                           fcur, gcur, flcur, ux, uy, eps, Ac, Bc, eps_u, Ac_u, Bc_u);
    return hipGetLastError();
}

hipError_t launch_copy(float* dst, const float* src, size_t n, hipStream_t s)
{
    const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, dst, src, n);
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

hipError_t launch_diag_reduce(const double* partials, int nblocks, const float* front, int ny,
                              double* res, hipStream_t s)
{
    hipLaunchKernelGGL(k_diag_reduce, dim3(1), dim3(64), 0, s, partials, nblocks, front, ny, res);
    return hipGetLastError();
}

hipError_t launch_front(const Geom& G, const float* flcur, float* front, hipStream_t s)
{
    hipLaunchKernelGGL(k_front, dim3(G.ny), dim3(256), 0, s, G, flcur, front);
    return hipGetLastError();
}

}  // namespace dmrtk
