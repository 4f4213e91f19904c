// interface.hpp -- phase indicator kernels for the interface observables
// (interpolated interface position along a lattice line, phase area of a
// plane, connected droplets).  The indicator is computed in FP64 from the
// stored populations, as the observables are: rho^N = (rho_R - rho_B)/rho for
// the two-component models, rho - (rho0_R + rho0_B)/2 for SC multiphase; a
// node is inside the red (liquid) phase when it is > 0.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace mclbm {

template <class L, int PR, int MODEL>
__device__ __forceinline__ double node_phase64(const KParams &P, const typename Prec<PR>::S *__restrict__ f,
                                               long long n)
{
    constexpr int K = NComp<MODEL>::n;
    double g[K][L::Q];
    load_node<L, K>(f, P.S, n, g);
    double dr[2], j[3];
    node_moments<L, K>(g, dr, j);
    const double rR = P.rho0[0] + dr[0];
    if constexpr (MODEL == SC_MP) return rR - P.sc_mid;
    const double rB = P.rho0[1] + dr[1];
    return (rR - rB) / (rR + rB);
}

// A strided node set: node(t) = base + (t % len1) * s1 + (t / len1) * s2,
// t < count (a line, a plane, or the whole lattice).
struct NodeSet {
    long long base, s1, s2, len1, count;
    __device__ __forceinline__ long long node(long long t) const { return base + (t % len1) * s1 + (t / len1) * s2; }
};

// Phase indicator of every node of the set.
template <class L, int PR, int MODEL>
__global__ __launch_bounds__(kBlock) void k_phase_sample(KParams P, const typename Prec<PR>::S *__restrict__ f,
                                                         NodeSet S, double *__restrict__ out)
{
    const long long t = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (t < S.count) out[t] = node_phase64<L, PR, MODEL>(P, f, S.node(t));
}

// Per-block partial sums of the red fraction over the set: (1 + rho^N)/2,
// or [rho >= (rho0_R + rho0_B)/2] for SC multiphase.  Fixed assignment of
// nodes to blocks and a fixed reduction order: the sum is reproducible.
template <class L, int PR, int MODEL>
__global__ __launch_bounds__(kBlock) void k_phase_area(KParams P, const typename Prec<PR>::S *__restrict__ f,
                                                       NodeSet S, double *__restrict__ partials)
{
    double a = 0.0;
    for (long long t = (long long)blockIdx.x * kBlock + threadIdx.x; t < S.count; t += (long long)gridDim.x * kBlock) {
        const double ph = node_phase64<L, PR, MODEL>(P, f, S.node(t));
        a += MODEL == SC_MP ? (ph >= 0.0 ? 1.0 : 0.0) : 0.5 * (1.0 + ph);
    }
    __shared__ double part[kBlock / 64];
    a = wave_sum(a);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = part[0];
        for (int w = 1; w < kBlock / 64; ++w) v += part[w];
        partials[blockIdx.x] = v;
    }
}

// Initial component labels: own node index inside the red phase, -1 outside.
template <class L, int PR, int MODEL>
__global__ __launch_bounds__(kBlock) void k_phase_labels(KParams P, const typename Prec<PR>::S *__restrict__ f,
                                                         int *__restrict__ labels)
{
    const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (n < P.N) labels[n] = node_phase64<L, PR, MODEL>(P, f, n) > 0.0 ? (int)n : -1;
}

}  // namespace mclbm
