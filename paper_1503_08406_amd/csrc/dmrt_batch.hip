// Batched step: many independent cavities of uneven size and parameters
// advance together in one persistent launch per time step.  Every cavity
// runs the same per-node step as a single lattice (dmrt_node.h), with its
// own lattice constants and uniform porous fields.
//
// Tiles of all cavities form one list (cavity by cavity, in memory order
// inside a cavity): 64 x rows nodes, and 32 x 2*rows nodes where a
// cavity's last columns are no more than 32 wide.  The list is cut into eight
// contiguous parts of about equal node count, one per die; block b works on
// die b % 8 and strides through that die's part, so a die keeps whole
// cavities (and their halo rows) in its own L2.
//
// Two steps per launch (k_batch_step2): the tiles of dmrt_tile2.h (62 x 6
// nodes and their ring) of every cavity in one list, cut the same way; one
// block per tile.
#include "dmrt_tile2.h"

namespace dmrtk {
namespace {

// The tile list and the cavity table do not change during a launch: they
// are read word by word through the constant address space, so the uniform
// loads become scalar loads and every per-cavity constant stays in scalar
// registers.
template <class T>
__device__ __forceinline__ T load_uniform(const T* p)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized records only");
    using cword = const __attribute__((address_space(4))) uint32_t;
    cword* src = (cword*)p;
    T v;
    uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) dst[i] = src[i];
    return v;
}

// Waves per SIMD of the 64 x 4 tiles: eight (the most), which keeps the
// scalar registers within budget (the rest spill to vector-register lanes);
// measured 3 % faster on the batch of 512 cavities than the seven that the
// scalar registers allow otherwise.
#ifndef DMRT_BATCH_OCC
#define DMRT_BATCH_OCC 8
#endif

template <int TYB, int SP>
__global__ __launch_bounds__(TX * TYB) __attribute__((amdgpu_waves_per_eu(TYB == 4 ? DMRT_BATCH_OCC : 1)))
void k_batch_step(BatchArgs a)
{
    __shared__ FlowStage<TX * TYB> S;
    const int xcd = (int)(blockIdx.x & (NXCD - 1));
    const int local = (int)(blockIdx.x >> 3), nloc = (int)(gridDim.x >> 3);
    const int hi = a.die[xcd + 1];
    int parity = 0;
    for (int t = a.die[xcd] + local; t < hi; t += nloc, parity ^= 1) {
        const int4 tile = load_uniform(a.tiles + t);
        const Cavity C = load_uniform(a.cav + tile.x);
        const Geom& G = C.G;
        const Phys& P = C.P;
        StepBufs B;
        B.fin = a.fin + C.f_off;
        B.fout = a.fout + C.f_off;
        B.gin = a.gin + C.g_off;
        B.gout = a.gout + C.g_off;
        B.flin = a.flin + C.fl_off;
        B.flout = a.flout + C.fl_off;
        B.ux = a.uout + C.u_off;
        B.uy = a.uout + C.u_off + G.plane;
        B.uin = a.uin + C.u_off;
        B.eps = B.Ac = B.Bc = nullptr;
        B.it_sum = B.it_max = nullptr;
        B.r2f = nullptr;
        B.r2_its = 0;
        Arrays<BufIOT<SP>> A(G, B);
        A.eps_u = C.eps;
        A.Ac_u = C.Ac;
        A.Bc_u = C.Bc;
        // a wide tile is 64 x TYB nodes (a wavefront per row); a narrow one
        // 32 x 2*TYB (a wavefront per two rows), for a cavity's last 1-32 columns
        const int lane = (int)threadIdx.x, w = (int)threadIdx.y;
        const bool narrow = tile.w != 0;
        const int x = tile.y + (narrow ? (lane & 31) : lane);
        const int y = tile.z + (narrow ? 2 * w + (lane >> 5) : w);
        block_step<BufIOT<SP>, true, false, true, TX * TYB>(G, P, B, A, x, y, x < G.nx && y < G.ny, S,
                                                      parity);
    }
}

// Waves of a two-step block in a batch: tiles of 62 x 6 nodes, as on a
// single lattice (a narrow last column of a cavity: 30 x 14).  With the
// per-node code of the cavity form the 8-wave blocks hold 48 VGPRs and 88
// SGPRs, four blocks per CU, and measured 3 % faster on the 512-cavity
// workload than 12-wave blocks at two per CU (430 against 444 us per step;
// 457 against 474 with general thermal properties).  Before that form the
// 12-wave blocks were 3 % faster (531 against 548).
#ifndef DMRT_B2_WAVES
#define DMRT_B2_WAVES 8
#endif
#ifndef DMRT_B2_OCC
#define DMRT_B2_OCC 7
#endif
constexpr int B2_WAVES = DMRT_B2_WAVES;

// Two steps of one tile of the list per block: block b works on die b % 8,
// tile a.die[die] + b / 8 of that die's part.  IO: BufIOT, or WinIOT with
// the window pair of the two halves of the state arena, compiled for
// DMRT_B2_OCC waves per SIMD (7 for 8-wave blocks, 6 for 12-wave ones, as
// the LDS allows); the window pair took 94 scalar registers with 15
// spilled (106 with 23 spilled for BufIOT) in the general build and
// measured 4.6 % faster on the batch of 512 cavities; without the bound
// 0.8 %, with a bound of 8 slower.  UT:
// every cavity has the cavity form of tile_step2 (uniform thermal
// properties, walls on every side).
template <class IO, bool UT = false>
__global__ __launch_bounds__(TX * B2_WAVES) __attribute__((amdgpu_waves_per_eu(InWindow<IO>::value ? DMRT_B2_OCC : 1)))
void k_batch_step2(BatchArgs a)
{
    __shared__ float tl[TPLANES * B2_WAVES * TX];
    const int xcd = (int)(blockIdx.x & (NXCD - 1));
    const int lo = a.die[xcd], n = a.die[xcd + 1] - lo;
    const int j = (int)(blockIdx.x >> 3);
    if (j >= n) return;  // the whole block: no barrier is left waiting
    const int t = lo + rotated_tile(j, n);
    const int4 tile = load_uniform(a.tiles + t);
    const Cavity C = load_uniform(a.cav + tile.x);
    StepBufs B;
    B.fin = a.fin + C.f_off;
    B.fout = a.fout + C.f_off;
    B.gin = a.gin + C.g_off;
    B.gout = a.gout + C.g_off;
    B.flin = a.flin + C.fl_off;
    B.flout = a.flout + C.fl_off;
    B.ux = a.uout + C.u_off;
    B.uy = a.uout + C.u_off + C.G.plane;
    B.uin = a.uin + C.u_off;
    B.eps = B.Ac = B.Bc = nullptr;
    B.it_sum = B.it_max = nullptr;
    B.r2f = nullptr;
    B.r2_its = 0;
    B.win = a.win;
    B.wout = a.wout;
    B.win_bytes = B.wout_bytes = a.win_bytes;
    Arrays<IO> A(C.G, B);
    A.eps_u = C.eps;
    A.Ac_u = C.Ac;
    A.Bc_u = C.Bc;
    if (tile.w)  // a narrow last column: rows of 32 lanes
        tile_step2<IO, true, B2_WAVES, true, false, TX / 2, UT>(C.G, C.P, B, A, tile.y, tile.z, tl);
    else
        tile_step2<IO, true, B2_WAVES, true, false, TX, UT>(C.G, C.P, B, A, tile.y, tile.z, tl);
}

// Per-cavity partial counts (blockIdx.y = cavity): liquid nodes (f_l > 0)
// and non-finite values of f_l and g.  Padding columns hold zeros.
__global__ __launch_bounds__(256) void k_batch_count(const Cavity* cav, const float* fl,
                                                     const float* g, long long* partials)
{
    __shared__ long long red[2][4];
    const Cavity& C = cav[blockIdx.y];
    const long long n = C.G.plane, n5 = 5 * C.G.plane;
    const float* flc = fl + C.fl_off;
    const float* gc = g + C.g_off;
    long long liq = 0, bad = 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long long i = i0; i < n; i += stride) {
        const float v = flc[i];
        liq += v > 0.0f;
        bad += !isfinite(v);
    }
    for (long long i = i0; i < n5; i += stride) bad += !isfinite(gc[i]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        liq += __shfl_xor(liq, o, 64);
        bad += __shfl_xor(bad, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = liq;
        red[1][w] = bad;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        long long v = 0;
        for (int k = 0; k < 4; ++k) v += red[threadIdx.x][k];
        partials[2 * ((long long)blockIdx.y * gridDim.x + blockIdx.x) + threadIdx.x] = v;
    }
}

}  // namespace

namespace {
template <int SP>
void launch_batch_sp(const BatchArgs& a, int rows, int blocks, hipStream_t s)
{
    if (rows == 8)
        hipLaunchKernelGGL((k_batch_step<8, SP>), dim3(blocks), dim3(TX, 8), 0, s, a);
    else
        hipLaunchKernelGGL((k_batch_step<4, SP>), dim3(blocks), dim3(TX, 4), 0, s, a);
}
}  // namespace

hipError_t launch_batch_step(const BatchArgs& a, int rows, int blocks, hipStream_t s)
{
    if (a.store == ST_NT)
        launch_batch_sp<ST_NT>(a, rows, blocks, s);
    else if (a.store == ST_WT)
        launch_batch_sp<ST_WT>(a, rows, blocks, s);
    else
        launch_batch_sp<ST_PLAIN>(a, rows, blocks, s);
    return hipGetLastError();
}

namespace {
template <int SP>
void launch_batch2_sp(const BatchArgs& a, int blocks, hipStream_t s)
{
    if (a.win_bytes && a.uniform_thermal)
        hipLaunchKernelGGL((k_batch_step2<WinIOT<SP, true>, true>), dim3(blocks), dim3(TX, B2_WAVES), 0, s, a);
    else if (a.win_bytes)
        hipLaunchKernelGGL((k_batch_step2<WinIOT<SP, true>>), dim3(blocks), dim3(TX, B2_WAVES), 0, s, a);
    else
        hipLaunchKernelGGL((k_batch_step2<BufIOT<SP>>), dim3(blocks), dim3(TX, B2_WAVES), 0, s, a);
}
}  // namespace

hipError_t launch_batch_step2(const BatchArgs& a, int blocks, hipStream_t s)
{
    if (a.store == ST_NT)
        launch_batch2_sp<ST_NT>(a, blocks, s);
    else if (a.store == ST_WT)
        launch_batch2_sp<ST_WT>(a, blocks, s);
    else
        launch_batch2_sp<ST_PLAIN>(a, blocks, s);
    return hipGetLastError();
}

int batch_step2_tile(int* width, int* rows, int* narrow_width, int* narrow_rows)
{
    if (width) *width = T2_W;
    if (rows) *rows = B2_WAVES - 2;
    if (narrow_width) *narrow_width = TX / 2 - 2;
    if (narrow_rows) *narrow_rows = 2 * B2_WAVES - 2;
    return B2_WAVES;
}

int batch_blocks_per_cu(int rows)
{
    int nb = 0;
    hipError_t e = rows == 8
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_step<8, ST_PLAIN>, TX * 8, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch_step<4, ST_PLAIN>, TX * 4, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

hipError_t launch_batch_count(const Cavity* cav, int ncav, const float* fl, const float* g,
                              long long* partials, int nblk, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_count, dim3(nblk, ncav), dim3(256), 0, s, cav, fl, g, partials);
    return hipGetLastError();
}

}  // namespace dmrtk
