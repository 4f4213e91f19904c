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
__global__ __launch_bounds__(kBlock) void kb_collide(SimDesc *D, int nsims)
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
