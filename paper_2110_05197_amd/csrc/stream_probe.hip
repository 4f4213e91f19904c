// stream_probe.hip -- memory-pattern ceilings for the D3Q19 FP32 step.
//
// Times kernels that move exactly the bytes of one step (38 populations read
// and 38 written per node, structure-of-arrays, n^3 nodes) with no stencil and
// no collision, in the access patterns a step can use:
//   copy-float4   : one contiguous stream in, one out (the device's best case)
//   soa-aligned   : every population read and written at its own node
//   soa-push      : read at the node, written to node + c_i (x-shifted
//                   directions write partial cache lines)
//   soa-pull      : read from node - c_i, written at the node
//   soa-push-nta  : push, with non-temporal stores for the c_x = 0 directions
// Nodes are kept one plane and one row away from the array ends, so every
// shifted index stays inside the arrays without a wrap; the first node is on
// a 256-byte boundary.  Prints one JSON line per pattern.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                        \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                \
            std::exit(1);                                                               \
        }                                                                               \
    } while (0)

namespace {

constexpr int Q = 19;
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

enum Pattern { ALIGNED = 0, PUSH = 1, PULL = 2, PUSH_NTA = 3 };

template <int PAT>
__global__ __launch_bounds__(256) void soa(const float *__restrict__ src, float *__restrict__ dst, int nx,
                                           int sxy, long long N, long long lo, long long hi)
{
    const long long n = lo + (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= hi) return;
    float v[2 * Q];
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) {
        const int q = i % Q;
        const long long off = (long long)CX[q] + (long long)nx * CY[q] + (long long)sxy * CZ[q];
        v[i] = src[(long long)i * N + n - (PAT == PULL ? off : 0)];
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) s += v[i];
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) {
        const int q = i % Q;
        const long long off = (long long)CX[q] + (long long)nx * CY[q] + (long long)sxy * CZ[q];
        const bool pushed = PAT == PUSH || PAT == PUSH_NTA;
        float *p = dst + (long long)i * N + n + (pushed ? off : 0);
        const float w = v[i] * 0.999f + s * 1e-6f;
        if (PAT == PUSH_NTA && CX[q] == 0) __builtin_nontemporal_store(w, p);
        else *p = w;
    }
}

__global__ __launch_bounds__(256) void copy4(const float4 *__restrict__ a, float4 *__restrict__ b, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

}  // namespace

int main(int argc, char **argv)
{
    const int nx = argc > 1 ? std::atoi(argv[1]) : 256;
    const int reps = argc > 2 ? std::atoi(argv[2]) : 20;
    if (nx < 8 || nx > 512 || nx % 64 || reps < 1) {
        std::fprintf(stderr, "usage: stream_probe [n (multiple of 64, 64..512)] [repetitions]\n");
        return 2;
    }
    const long long N = (long long)nx * nx * nx, sxy = (long long)nx * nx;
    const long long lo = (sxy + nx + 1 + 63) / 64 * 64, hi = (N - sxy - nx - 1) / 64 * 64;
    const size_t bytes = (size_t)2 * Q * N * sizeof(float);
    float *a = nullptr, *b = nullptr;
    CHECK(hipMalloc(&a, bytes));
    CHECK(hipMalloc(&b, bytes));
    CHECK(hipMemset(a, 0, bytes));
    CHECK(hipMemset(b, 0, bytes));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const double moved = 2.0 * (double)bytes;   // read + write, every node
    auto run = [&](const char *name, auto launch) {
        for (int r = 0; r < 2; ++r) launch(a, b);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e0, 0));
        for (int r = 0; r < reps; ++r) launch((r & 1) ? b : a, (r & 1) ? a : b);
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipGetLastError());
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        ms /= reps;
        std::printf("{\"pattern\": \"%s\", \"n\": %d, \"ms\": %.4f, \"GBps\": %.0f}\n", name, nx, ms,
                    moved / (ms * 1e-3) / 1e9);
        std::fflush(stdout);
    };
    const long long cnt = hi - lo;
    const dim3 g((unsigned)((cnt + 255) / 256)), blk(256);
    const long long n4 = (long long)(bytes / sizeof(float4));
    run("copy-float4", [&](float *x, float *y) {
        hipLaunchKernelGGL(copy4, dim3((unsigned)((n4 + 255) / 256)), blk, 0, 0, (const float4 *)x, (float4 *)y, n4);
    });
    run("soa-aligned", [&](float *x, float *y) {
        hipLaunchKernelGGL(soa<ALIGNED>, g, blk, 0, 0, x, y, nx, (int)sxy, N, lo, hi);
    });
    run("soa-push", [&](float *x, float *y) {
        hipLaunchKernelGGL(soa<PUSH>, g, blk, 0, 0, x, y, nx, (int)sxy, N, lo, hi);
    });
    run("soa-pull", [&](float *x, float *y) {
        hipLaunchKernelGGL(soa<PULL>, g, blk, 0, 0, x, y, nx, (int)sxy, N, lo, hi);
    });
    run("soa-push-nta", [&](float *x, float *y) {
        hipLaunchKernelGGL(soa<PUSH_NTA>, g, blk, 0, 0, x, y, nx, (int)sxy, N, lo, hi);
    });
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    return 0;
}
