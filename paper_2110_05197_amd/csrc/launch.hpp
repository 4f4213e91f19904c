// launch.hpp -- __global__ kernels (solo and batched) around the per-node
// bodies, and the per-instantiation launcher table used by the C ABI.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace mclbm {

// Divergence flag: one vector atomic per wavefront that saw a bad node.
__device__ __forceinline__ void flag_if_bad(unsigned *flag, bool bad)
{
    const unsigned long long b = __ballot(bad);
    if (b != 0ull && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

// ----------------------------- solo kernels --------------------------------
template <class L, int PR, int MODEL>
__global__ __launch_bounds__(kBlock) void k_density(KParams P, const typename Prec<PR>::S *__restrict__ f,
                                                    typename Prec<PR>::F *__restrict__ field, unsigned *flag)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    bool bad = false;
    if (n < P.N) bad = density_body<L, PR, MODEL>(P, f, field, n);
    flag_if_bad(flag, bad);
}

template <class L, int PR>
__global__ __launch_bounds__(kBlock) void k_gradN(KParams P, const typename Prec<PR>::F *__restrict__ field,
                                                  typename Prec<PR>::F *__restrict__ gfield)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n < P.N) gradN_body<L, PR>(P, field, gfield, n);
}

template <class L, int PR, int MODEL, bool REP>
__global__ __launch_bounds__(kBlock) void k_collide(KParams P, const typename Prec<PR>::S *__restrict__ src,
                                                    typename Prec<PR>::S *__restrict__ dst,
                                                    const typename Prec<PR>::F *__restrict__ field,
                                                    const typename Prec<PR>::F *__restrict__ gfield)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n < P.N) collide_body<L, PR, MODEL, REP>(P, src, dst, field, gfield, n);
}

// Stages two fields (a, b) of a box in LDS: columns x0 - RCH .. x0 - RCH +
// BX - 1, rows y0 - RCH .. and planes z - RCH .., [z][y][x], at the wrapped or
// clamped coordinates a stencil read would use.  Each wave stages whole rows:
// lane l holds columns l and, for l < BX - 64, 64 + l; a row's y and z
// (wave-uniform) are wrapped once.  Coordinates past nx - 1 + RCH (ny - 1 +
// RCH) are read by no node of the tile; their slots are left at zero.
template <int BX, int BY, int BZ, int RCH, int THREADS, class FT>
__device__ __forceinline__ void stage_box(const KParams &P, const FT *__restrict__ a, const FT *__restrict__ b,
                                          FT *boxA, FT *boxB, int x0, int y0, int z)
{
    static_assert(BX >= 64 && BX <= 128 && THREADS % 64 == 0, "rows of 64 to 128 columns, whole waves");
    const int nx = P.nx, sxy = P.nx * P.ny;   // N < 2^31: 32-bit offsets
    const int lane = (int)threadIdx.x % 64, wave = (int)threadIdx.x / 64;
    const int gx0 = x0 - RCH + lane, gx1 = x0 - RCH + 64 + lane;
    const bool in0 = gx0 <= P.nx - 1 + RCH, in1 = lane < BX - 64 && gx1 <= P.nx - 1 + RCH;
    const int qx0 = in0 ? stencil_coord(gx0, P.nx, P.bc[0]) : 0;
    const int qx1 = in1 ? stencil_coord(gx1, P.nx, P.bc[0]) : 0;
    for (int row = wave; row < BY * BZ; row += THREADS / 64) {
        const int gy = y0 - RCH + row % BY, gz = z - RCH + row / BY;
        FT a0 = FT(0), b0 = FT(0), a1 = FT(0), b1 = FT(0);
        if (gy <= P.ny - 1 + RCH) {
            const int base = nx * stencil_coord(gy, P.ny, P.bc[1]) + sxy * stencil_coord(gz, P.nz, P.bc[2]);
            if (in0) {
                a0 = a[(unsigned)(base + qx0)];
                b0 = b[(unsigned)(base + qx0)];
            }
            if (in1) {
                a1 = a[(unsigned)(base + qx1)];
                b1 = b[(unsigned)(base + qx1)];
            }
        }
        boxA[row * BX + lane] = a0;
        boxB[row * BX + lane] = b0;
        if (lane < BX - 64) {
            boxA[row * BX + 64 + lane] = a1;
            boxB[row * BX + 64 + lane] = b1;
        }
    }
}

// Waves per SIMD the multirange collide is compiled for.  Left to itself the
// compiler gives FP32 136 registers a lane (three waves); a fourth wave, at
// the cost of a dozen spilled registers, took the 256^3 step from 2.19 to
// 2.06 ms.  Mixed (173 registers, two waves) fits three without spilling;
// FP16 storage takes three and FP64 two, both without spilling.
template <int PR> constexpr int kMrWaves = PR == 1 ? 4 : PR == 0 ? 2 : 3;

// Collide pass of the multirange two-component Shan-Chen step (D3Q19): a
// block takes a kMrTX x kMrTY tile of one plane (blocks ordered x tile, y
// tile, z), first stages in LDS psi_R and psi_B of the tile and two nodes
// around it, then collides its nodes with the multirange sums reading that
// box (the one-node stencil of the cross force reads the field).
template <int PR>
__global__ __launch_bounds__(kMrTX *kMrTY) __attribute__((amdgpu_waves_per_eu(kMrWaves<PR>)))
void k_collide_mr(KParams P, const typename Prec<PR>::S *__restrict__ src, typename Prec<PR>::S *__restrict__ dst,
                  const typename Prec<PR>::F *__restrict__ field)
{
    using FT = typename Prec<PR>::F;
    __shared__ FT psiR[kMrBox], psiB[kMrBox];
    const int tiles_x = (P.nx + kMrTX - 1) / kMrTX, tiles_y = (P.ny + kMrTY - 1) / kMrTY;
    const int b = (int)blockIdx.x;
    const int x0 = (b % tiles_x) * kMrTX, y0 = ((b / tiles_x) % tiles_y) * kMrTY, z = b / (tiles_x * tiles_y);
    stage_box<kMrBX, kMrBY, kMrBZ, 2, kMrTX * kMrTY>(P, field + 2 * P.N, field + 3 * P.N, psiR, psiB, x0, y0, z);
    __syncthreads();
    const int tx = (int)threadIdx.x % kMrTX, ty = (int)threadIdx.x / kMrTX;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= P.nx || y >= P.ny) return;
    const long long n = (long long)x + (long long)P.nx * ((long long)y + (long long)P.ny * z);
    collide_body<D3Q19, PR, SC_MC, true>(P, src, dst, field, nullptr, n, MrStaged<FT>{psiR, psiB, tx, ty});
}

inline long long mr_blocks(const KParams &P)
{
    return (long long)((P.nx + kMrTX - 1) / kMrTX) * ((P.ny + kMrTY - 1) / kMrTY) * P.nz;
}

template <class L, int PR, int MODEL>
__global__ __launch_bounds__(kBlock) void k_outflow(KParams P, typename Prec<PR>::S *__restrict__ dst,
                                                    long long count)
{
    const long long idx = (long long)blockIdx.x * kBlock + threadIdx.x;
    int x, y, z;
    if (idx < count && outflow_face_node(P, idx, x, y, z))
        outflow_body<L, NComp<MODEL>::n>(P, dst, x, y, z);
}

template <class L, int PR, int MODEL>
__global__ __launch_bounds__(kBlock) void k_init(KParams P, const double *__restrict__ rhoR,
                                                 const double *__restrict__ rhoB, const double *__restrict__ u,
                                                 typename Prec<PR>::S *__restrict__ f)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n < P.N) init_body<L, PR, MODEL>(P, rhoR, rhoB, u, f, n);
}

template <class L, int PR, int MODEL>
__global__ __launch_bounds__(kBlock) void k_export(KParams P, const typename Prec<PR>::S *__restrict__ f,
                                                   double *__restrict__ out)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= P.N) return;
    constexpr int K = NComp<MODEL>::n;
    for (int k = 0; k < K; ++k)
        for (int i = 0; i < L::Q; ++i) {
            const long long a = (long long)(k * L::Q + i) * P.N + n;
            out[a] = (double)f[sidx<L, K, typename Prec<PR>::S>(k, i, P.S, n)] + P.shift[k][L::grp[i]];
        }
}

template <class L, int PR, int MODEL>
__global__ __launch_bounds__(kBlock) void k_import(KParams P, const double *__restrict__ in,
                                                   typename Prec<PR>::S *__restrict__ f)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= P.N) return;
    constexpr int K = NComp<MODEL>::n;
    for (int k = 0; k < K; ++k)
        for (int i = 0; i < L::Q; ++i) {
            const long long a = (long long)(k * L::Q + i) * P.N + n;
            f[sidx<L, K, typename Prec<PR>::S>(k, i, P.S, n)] = (typename Prec<PR>::S)(in[a] - P.shift[k][L::grp[i]]);
        }
}

template <class L, int PR, int MODEL>
__global__ __launch_bounds__(kBlock) void k_moments_out(KParams P, const typename Prec<PR>::S *__restrict__ f,
                                                        const typename Prec<PR>::F *__restrict__ field,
                                                        double *rhoR, double *rhoB, double *u)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n >= P.N) return;
    double rR, rB, uu[3], j[3];
    node_state64<L, PR, MODEL>(P, f, field, n, rR, rB, uu, j);
    if (rhoR) rhoR[n] = rR;
    if (rhoB) rhoB[n] = rB;
    if (u) { u[n] = uu[0]; u[P.N + n] = uu[1]; u[2 * P.N + n] = uu[2]; }
}

template <class L, int PR, int MODEL>
__global__ __launch_bounds__(kBlock) void k_obs(KParams P, const typename Prec<PR>::S *__restrict__ f,
                                                const typename Prec<PR>::F *__restrict__ field, EpsTable eps,
                                                double *__restrict__ partials)
{
    double acc[kNAcc];
#pragma unroll
    for (int a = 0; a < kNAcc; ++a) acc[a] = 0.0;
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long n = (long long)blockIdx.x * kBlock + threadIdx.x; n < P.N; n += stride)
        obs_body<L, PR, MODEL>(P, f, field, n, eps, acc);
    block_reduce_store(acc, partials + (long long)blockIdx.x * kNAcc);
}

// ---------------------------- batched kernels ------------------------------
// One grid covers every running simulation of a group; block b belongs to
// the simulation whose [block0, block0 + nblocks) holds b.
struct SimDesc {
    KParams P;
    void *f[2];
    void *field;
    void *gfield;
    unsigned *flag;
    long long block0, nblocks;     // node-parallel grid slice
    long long oblock0, onblocks;   // outflow-face grid slice
    long long ocount;              // outflow face nodes
    long long fblock0, fnblocks;   // one-pass (fused) grid slice; 0 blocks: two-pass
    int ftz;                        // planes per fused column
    long long steps, target;
    int cur, state;
};

// A pointer read from memory is generic (flat) to the compiler; flat loads
// count against the LDS wait counter as well as the vector-memory one, so an
// LDS wait would also wait for every load in flight.  The descriptors' state
// pointers are device memory: convert them to global-address-space pointers.
template <class T>
__device__ __forceinline__ T *global_ptr(const void *p)
{
    return (T *)(__attribute__((address_space(1))) T *)(uintptr_t)p;
}

__device__ __forceinline__ int find_sim(const SimDesc *D, int n, long long b, bool outflow)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const long long s = outflow ? D[mid].oblock0 : D[mid].block0;
        if (s <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <class L, int PR, int MODEL>
__global__ __launch_bounds__(kBlock) void kb_density(SimDesc *D, int nsims)
{
    const int s = find_sim(D, nsims, blockIdx.x, false);
    const SimDesc &d = D[s];
    if (d.state != 0) return;
    const long long n = (blockIdx.x - d.block0) * kBlock + threadIdx.x;
    bool bad = false;
    if (n < d.P.N)
        bad = density_body<L, PR, MODEL>(d.P, global_ptr<const typename Prec<PR>::S>(d.f[d.cur]),
                                         global_ptr<typename Prec<PR>::F>(d.field), n);
    flag_if_bad(global_ptr<unsigned>(d.flag), bad);
}

template <class L, int PR, int MODEL, bool REP>
__device__ __forceinline__ void kb_collide_body(SimDesc *D, int nsims)
{
    const int s = find_sim(D, nsims, blockIdx.x, false);
    const SimDesc &d = D[s];
    if (d.state != 0) return;
    const long long n = (blockIdx.x - d.block0) * kBlock + threadIdx.x;
    if (n < d.P.N)
        collide_body<L, PR, MODEL, REP>(d.P, global_ptr<const typename Prec<PR>::S>(d.f[d.cur]),
                                        global_ptr<typename Prec<PR>::S>(d.f[d.cur ^ 1]),
                                        global_ptr<const typename Prec<PR>::F>(d.field),
                                        global_ptr<const typename Prec<PR>::F>(d.gfield), n);
}

template <class L, int PR, int MODEL, bool REP>
__global__ __launch_bounds__(kBlock) void kb_collide(SimDesc *D, int nsims)
{
    kb_collide_body<L, PR, MODEL, REP>(D, nsims);
}

// The same kernel compiled for three waves per SIMD, for the D3Q19 mixed
// colour-gradient collide: left to itself the compiler gives it 172
// registers a lane (two waves); at three it holds 168 with no spill, and a
// batch of eight 80^3 two-pass lattices stepped in 0.450 instead of 0.483 ms.
// (Caps that make the other collides spill slowed them, up to twofold.)
template <class L, int PR, int MODEL, bool REP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
void kb_collide_w3(SimDesc *D, int nsims)
{
    kb_collide_body<L, PR, MODEL, REP>(D, nsims);
}
template <class L, int PR, int MODEL, bool REP>
constexpr bool kb_collide_three_waves = L::Q == 19 && PR == 2 && MODEL == CG && !REP;

template <class L, int PR>
__global__ __launch_bounds__(kBlock) void kb_gradN(SimDesc *D, int nsims)
{
    const int s = find_sim(D, nsims, blockIdx.x, false);
    const SimDesc &d = D[s];
    if (d.state != 0) return;
    const long long n = (blockIdx.x - d.block0) * kBlock + threadIdx.x;
    if (n < d.P.N)
        gradN_body<L, PR>(d.P, global_ptr<const typename Prec<PR>::F>(d.field),
                          global_ptr<typename Prec<PR>::F>(d.gfield), n);
}

template <class L, int PR, int MODEL>
__global__ __launch_bounds__(kBlock) void kb_outflow(SimDesc *D, int nsims)
{
    const int s = find_sim(D, nsims, blockIdx.x, true);
    const SimDesc &d = D[s];
    if (d.state != 0 || d.ocount == 0) return;
    const long long idx = (blockIdx.x - d.oblock0) * kBlock + threadIdx.x;
    int x, y, z;
    if (idx < d.ocount && outflow_face_node(d.P, idx, x, y, z))
        outflow_body<L, NComp<MODEL>::n>(d.P, global_ptr<typename Prec<PR>::S>(d.f[d.cur ^ 1]), x, y, z);
}

}  // namespace mclbm
