// stream_probe.hip -- memory-pattern ceilings for the D3Q19 FP32 step.
//
// Times kernels that move exactly the bytes of one step (38 populations read
// and 38 written per node, structure-of-arrays, n^3 nodes) with no stencil and
// no collision, in the access patterns a step can use:
//   copy-float4      : one contiguous stream in, one out (the device's best case)
//   soa-aligned-xV   : every population read and written at its own node, V
//                      consecutive nodes per lane (dword, dwordx2, dwordx4)
//   soa-push         : read at the node, written to node + c_i (x-shifted
//                      directions write partial cache lines)
//   soa-pull         : read from node - c_i, written at the node
//   soa-push-nta     : push, with non-temporal stores for the c_x = 0 directions
//   aa-odd-inplace   : the odd step of the in-place AA pattern: population i
//                      read from and written back to node + c_i of one array
//   row-push-x4      : a wavefront owns a whole x row (64 lanes x 4 nodes,
//                      n = 256), reads dwordx4 at its nodes and pushes with the
//                      x shift done across lanes (DPP wave rotate), so every
//                      store is a whole aligned row
//   tiled-B-*        : the same patterns on a tiled layout: the nodes split
//                      into chunks of B consecutive nodes, each chunk holding
//                      its 38 populations one after the other (B values each),
//                      so the loads of a row segment fall in one contiguous
//                      38 B-float region instead of 38 separate arrays
//   copy-*           : plain copies of the same bytes that differ in the work
//                      of a lane: one dword (copy-dword), 38 float4 copied
//                      one after the other (copy-loop38), or 38 float4 loaded
//                      before any is stored, from 38 arrays (copy-burst38-soa)
//                      or from one contiguous 38 KB region per wavefront
//                      (copy-burst38-contig)
//   *-ldsK           : the same kernel with K KB of (unused) dynamic LDS per
//                      block, capping the blocks a compute unit holds at once
//   copy-float4-gs   : float4 copy by 2048 blocks looping over the array
//   march-*-TXxTY-cC : the one-pass step's schedule without its stencil and
//                      arithmetic: each block owns a TX x TY column and walks
//                      one of C equal runs of planes (C chunks in z; C sets the
//                      blocks per compute unit), loading plane z+1 while
//                      storing plane z, aligned or pushed (c_x = 0 stores
//                      non-temporal); periodic wrap at the faces.  march-tiled
//                      stores each column's plane contiguously (a tiled layout)
// Population arrays are `stride` = n^3 + pad floats apart (pad from the command
// line, a multiple of 64): with pad = 0 and n a power of two every array
// starts at the same offset modulo a large power of two.  Nodes are kept one
// plane and one row away from the array ends, so every shifted index stays
// inside its array without a wrap; the first node is on a 256-byte boundary.
// Prints one JSON line per pattern.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

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

enum Pattern { ALIGNED = 0, PUSH = 1, PULL = 2, PUSH_NTA = 3, AA_ODD = 4 };

template <int V> struct Vec;
template <> struct Vec<1> { using T = float; };
template <> struct Vec<2> { using T = float2; };
template <> struct Vec<4> { using T = float4; };

__device__ __forceinline__ float scale(float v, float s) { return v * 0.999f + s * 1e-6f; }
__device__ __forceinline__ float2 scale(float2 v, float s) { return make_float2(scale(v.x, s), scale(v.y, s)); }
__device__ __forceinline__ float4 scale(float4 v, float s)
{
    return make_float4(scale(v.x, s), scale(v.y, s), scale(v.z, s), scale(v.w, s));
}
__device__ __forceinline__ float first(float v) { return v; }
__device__ __forceinline__ float first(float2 v) { return v.x; }
__device__ __forceinline__ float first(float4 v) { return v.x; }

// Nodes [lo, hi) in runs of V per lane; shifted patterns only with V = 1.
template <int PAT, int V>
__global__ __launch_bounds__(256) void soa(const float *__restrict__ src, float *__restrict__ dst, int nx,
                                           int sxy, long long S, long long lo, long long hi)
{
    using T = typename Vec<V>::T;
    static_assert(V == 1 || PAT == ALIGNED, "shifted patterns are scalar");
    const long long n = lo + V * ((long long)blockIdx.x * blockDim.x + threadIdx.x);
    if (n + V > hi) return;
    T v[2 * Q];
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) {
        const int q = i % Q;
        const long long off = (long long)CX[q] + (long long)nx * CY[q] + (long long)sxy * CZ[q];
        const long long at = PAT == PULL ? n - off : (PAT == AA_ODD ? n + off : n);
        v[i] = *reinterpret_cast<const T *>(src + (long long)i * S + at);
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) s += first(v[i]);
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) {
        const int q = i % Q;
        const long long off = (long long)CX[q] + (long long)nx * CY[q] + (long long)sxy * CZ[q];
        const bool shifted = PAT == PUSH || PAT == PUSH_NTA || PAT == AA_ODD;
        T *p = reinterpret_cast<T *>(dst + (long long)i * S + n + (shifted ? off : 0));
        const T w = scale(v[i], s);
        if constexpr (PAT == PUSH_NTA) {
            if (CX[q] == 0) __builtin_nontemporal_store(w, p);
            else *p = w;
        } else {
            *p = w;
        }
    }
}

// Lane l receives the value of lane l - 1 (mod 64) / l + 1 (mod 64).
__device__ __forceinline__ float from_left(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x13C, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_right(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x134, 0xF, 0xF, false));
}

// One wavefront per x row of 256 nodes (rows [rlo, rhi)), 4 nodes per lane.
__global__ __launch_bounds__(256) void row_push(const float *__restrict__ src, float *__restrict__ dst, int ny,
                                                long long S, long long rlo, long long rhi)
{
    const long long r = rlo + (long long)blockIdx.x * 4 + threadIdx.x / 64;
    if (r >= rhi) return;   // whole wavefronts leave together
    const int lane = threadIdx.x & 63;
    const long long base = r * 256 + 4 * lane;
    float4 v[2 * Q];
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) v[i] = *reinterpret_cast<const float4 *>(src + (long long)i * S + base);
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) s += v[i].x;
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) {
        const int q = i % Q;
        float4 w = scale(v[i], s);
        if (CX[q] > 0) w = make_float4(from_left(w.w), w.x, w.y, w.z);
        if (CX[q] < 0) w = make_float4(w.y, w.z, w.w, from_right(w.x));
        const long long t = base + 256ll * (CY[q] + (long long)ny * CZ[q]);
        *reinterpret_cast<float4 *>(dst + (long long)i * S + t) = w;
    }
}

// Tiled layout: population i of node n at ((n / B) * 38 + i) * B + n % B.
template <int B>
__device__ __forceinline__ long long tix(int i, long long n)
{
    return ((n / B) * (2 * Q) + i) * B + (n % B);
}

template <int PAT, int B>
__global__ __launch_bounds__(256) void tiled(const float *__restrict__ src, float *__restrict__ dst, int nx,
                                             int sxy, long long lo, long long hi)
{
    const long long n = lo + (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= hi) return;
    float v[2 * Q];
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) {
        const int q = i % Q;
        const long long off = (long long)CX[q] + (long long)nx * CY[q] + (long long)sxy * CZ[q];
        v[i] = src[tix<B>(i, PAT == PULL ? n - off : n)];
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) s += v[i];
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) {
        const int q = i % Q;
        const long long off = (long long)CX[q] + (long long)nx * CY[q] + (long long)sxy * CZ[q];
        dst[tix<B>(i, PAT == PUSH ? n + off : n)] = scale(v[i], s);
    }
}

// Tiled layout with B = 256 = one x row per chunk; one wavefront per row,
// 4 nodes per lane, x shift across lanes (rows [rlo, rhi)).
__global__ __launch_bounds__(256) void tiled_row_push(const float *__restrict__ src, float *__restrict__ dst, int ny,
                                                      long long rlo, long long rhi)
{
    const long long r = rlo + (long long)blockIdx.x * 4 + threadIdx.x / 64;
    if (r >= rhi) return;
    const int lane = threadIdx.x & 63;
    float4 v[2 * Q];
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) v[i] = *reinterpret_cast<const float4 *>(src + (r * (2 * Q) + i) * 256 + 4 * lane);
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) s += v[i].x;
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) {
        const int q = i % Q;
        float4 w = scale(v[i], s);
        if (CX[q] > 0) w = make_float4(from_left(w.w), w.x, w.y, w.z);
        if (CX[q] < 0) w = make_float4(w.y, w.z, w.w, from_right(w.x));
        const long long t = r + CY[q] + (long long)ny * CZ[q];
        *reinterpret_cast<float4 *>(dst + (t * (2 * Q) + i) * 256 + 4 * lane) = w;
    }
}

__global__ __launch_bounds__(256) void copy1(const float *__restrict__ a, float *__restrict__ b, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// n4 float4 in 38 parts of m = n4 / 38; thread t copies element t of each part.
template <bool BURST>
__global__ __launch_bounds__(256) void copy38_soa(const float4 *__restrict__ a, float4 *__restrict__ b, long long m)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    if constexpr (BURST) {
        float4 v[2 * Q];
#pragma unroll
        for (int i = 0; i < 2 * Q; ++i) v[i] = a[i * m + t];
#pragma unroll
        for (int i = 0; i < 2 * Q; ++i) b[i * m + t] = v[i];
    } else {
#pragma unroll 1
        for (int i = 0; i < 2 * Q; ++i) b[i * m + t] = a[i * m + t];
    }
}

// Wavefront w copies the contiguous 38 x 64 float4 region starting at
// 38 * 64 * w: loads all 38 then stores all 38.
__global__ __launch_bounds__(256) void copy38_contig(const float4 *__restrict__ a, float4 *__restrict__ b, long long waves)
{
    const long long w = (long long)blockIdx.x * 4 + threadIdx.x / 64;
    if (w >= waves) return;
    const long long base = w * (2 * Q) * 64 + (threadIdx.x & 63);
    float4 v[2 * Q];
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) v[i] = a[base + 64 * i];
#pragma unroll
    for (int i = 0; i < 2 * Q; ++i) b[base + 64 * i] = v[i];
}

__global__ __launch_bounds__(256) void copy4_gs(const float4 *__restrict__ a, float4 *__restrict__ b, long long n)
{
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

// z-march of a TX x TY column over one of `chunks` equal runs of planes: the
// one-pass step's schedule with its loads and stores only.  TILED stores the
// nodes tile by tile (each TX x TY column's plane one contiguous run of TX*TY
// values per array) instead of row by row.
template <int TX, int TY, bool TILED>
__device__ __forceinline__ unsigned march_index(int x, int y, int z, int n)
{
    if (!TILED) return (unsigned)(x + n * (y + n * z));
    const int tiles_x = n / TX, tiles_y = n / TY;
    return (unsigned)(((z * tiles_y + y / TY) * tiles_x + x / TX) * (TX * TY) + (y % TY) * TX + x % TX);
}

template <int TX, int TY, bool PUSH, bool TILED = false>
__global__ __launch_bounds__(TX *TY) void march(const float *__restrict__ src, float *__restrict__ dst, int n,
                                                long long S, int chunks)
{
    const int tiles_x = n / TX, tiles_y = n / TY;
    const int nb = (int)gridDim.x;
    const int t = nb % 8 ? (int)blockIdx.x : (int)(blockIdx.x % 8) * (nb / 8) + (int)blockIdx.x / 8;
    const int bx = t % tiles_x, by = (t / tiles_x) % tiles_y, bz = t / (tiles_x * tiles_y);
    const int x = bx * TX + (int)threadIdx.x % TX, y = by * TY + (int)threadIdx.x / TX;
    const int z0 = bz * (n / chunks), z1 = z0 + n / chunks;
    float c[2 * Q], d[2 * Q];
    auto ld = [&](int z, float (&v)[2 * Q]) {
        const unsigned o = march_index<TX, TY, TILED>(x, y, z, n);
#pragma unroll
        for (int i = 0; i < 2 * Q; ++i) v[i] = (src + (size_t)i * (size_t)S)[o];
    };
    ld(z0, c);
    for (int z = z0; z < z1; ++z) {
        if (z + 1 < z1) ld(z + 1, d);
        const int xp = x == n - 1 ? 0 : x + 1, xm = x == 0 ? n - 1 : x - 1;
        const int yp = y == n - 1 ? 0 : y + 1, ym = y == 0 ? n - 1 : y - 1;
        const int zp = z == n - 1 ? 0 : z + 1, zm = z == 0 ? n - 1 : z - 1;
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < 2 * Q; ++i) s += c[i];
#pragma unroll
        for (int i = 0; i < 2 * Q; ++i) {
            const int q = i % Q;
            unsigned o;
            if (PUSH) {
                const int tx = CX[q] > 0 ? xp : CX[q] < 0 ? xm : x;
                const int ty = CY[q] > 0 ? yp : CY[q] < 0 ? ym : y;
                const int tz = CZ[q] > 0 ? zp : CZ[q] < 0 ? zm : z;
                o = march_index<TX, TY, TILED>(tx, ty, tz, n);
            } else {
                o = march_index<TX, TY, TILED>(x, y, z, n);
            }
            float *p = &(dst + (size_t)i * (size_t)S)[o];
            const float w = scale(c[i], s);
            if (!PUSH || CX[q] == 0) __builtin_nontemporal_store(w, p);
            else *p = w;
        }
#pragma unroll
        for (int i = 0; i < 2 * Q; ++i) c[i] = d[i];
    }
}

// Lane-layout check of the two rotates: out[l] = from_left(l), out[64 + l] = from_right(l).
__global__ __launch_bounds__(64) void rotate_check(float *out)
{
    const float v = (float)threadIdx.x;
    out[threadIdx.x] = from_left(v);
    out[64 + threadIdx.x] = from_right(v);
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
    const long long pad = argc > 3 ? std::atoll(argv[3]) : 0;
    if (nx < 128 || nx > 512 || nx % 128 || reps < 1 || pad < 0 || pad % 64 || pad > (1 << 22)) {
        std::fprintf(stderr, "usage: stream_probe [n (multiple of 128, 128..512)] [repetitions] [pad (multiple of 64)]\n");
        return 2;
    }
    const long long N = (long long)nx * nx * nx, sxy = (long long)nx * nx, S = N + pad;
    const long long lo = (sxy + nx + 1 + 63) / 64 * 64, hi = (N - sxy - nx - 1) / 64 * 64;
    const size_t bytes = (size_t)2 * Q * S * sizeof(float);
    float *a = nullptr, *b = nullptr;
    CHECK(hipMalloc(&a, bytes));
    CHECK(hipMalloc(&b, bytes));
    CHECK(hipMemset(a, 0, bytes));
    CHECK(hipMemset(b, 0, bytes));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    {
        float *o = nullptr;
        CHECK(hipMalloc(&o, 128 * sizeof(float)));
        hipLaunchKernelGGL(rotate_check, dim3(1), dim3(64), 0, 0, o);
        CHECK(hipGetLastError());
        std::vector<float> h(128);
        CHECK(hipMemcpy(h.data(), o, 128 * sizeof(float), hipMemcpyDeviceToHost));
        CHECK(hipFree(o));
        bool ok = true;
        for (int l = 0; l < 64; ++l)
            ok = ok && h[l] == (float)((l + 63) % 64) && h[64 + l] == (float)((l + 1) % 64);
        std::printf("{\"rotate_check\": %s}\n", ok ? "true" : "false");
        std::fflush(stdout);
        if (!ok) return 1;
    }
    // bytes of one step: 38 reads + 38 writes per node of the whole box
    const double moved = 2.0 * 2.0 * Q * (double)N * sizeof(float);
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
        std::printf("{\"pattern\": \"%s\", \"n\": %d, \"pad\": %lld, \"ms\": %.4f, \"GBps\": %.0f, \"frac\": %.3f}\n",
                    name, nx, pad, ms, moved / (ms * 1e-3) / 1e9, moved / (ms * 1e-3) / 8e12);
        std::fflush(stdout);
    };
    const long long cnt = hi - lo;
    const dim3 blk(256);
    auto grid = [&](int v) { return dim3((unsigned)((cnt / v + 255) / 256)); };
    const long long n4 = (long long)(2 * Q * N / 4);
    run("copy-float4", [&](float *x, float *y) {
        hipLaunchKernelGGL(copy4, dim3((unsigned)((n4 + 255) / 256)), blk, 0, 0, (const float4 *)x, (float4 *)y, n4);
    });
    run("copy-dword", [&](float *x, float *y) {
        hipLaunchKernelGGL(copy1, dim3((unsigned)((4 * n4 + 255) / 256)), blk, 0, 0, x, y, 4 * n4);
    });
    {
        const long long m = n4 / (2 * Q);
        run("copy-loop38", [&](float *x, float *y) {
            hipLaunchKernelGGL(copy38_soa<false>, dim3((unsigned)((m + 255) / 256)), blk, 0, 0, (const float4 *)x,
                               (float4 *)y, m);
        });
        run("copy-burst38-soa", [&](float *x, float *y) {
            hipLaunchKernelGGL(copy38_soa<true>, dim3((unsigned)((m + 255) / 256)), blk, 0, 0, (const float4 *)x,
                               (float4 *)y, m);
        });
        const long long waves = n4 / (2 * Q * 64);
        run("copy-burst38-contig", [&](float *x, float *y) {
            hipLaunchKernelGGL(copy38_contig, dim3((unsigned)((waves + 3) / 4)), blk, 0, 0, (const float4 *)x,
                               (float4 *)y, waves);
        });
    }
    run("copy-float4-gs", [&](float *x, float *y) {
        hipLaunchKernelGGL(copy4_gs, dim3(2048), blk, 0, 0, (const float4 *)x, (float4 *)y, n4);
    });
    for (int kb : {40, 80, 160}) {
        const int lds = kb * 1024;
        char name[64];
        CHECK(hipFuncSetAttribute((const void *)soa<ALIGNED, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
        CHECK(hipFuncSetAttribute((const void *)copy38_contig, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
        CHECK(hipFuncSetAttribute((const void *)tiled<PUSH, 64>, hipFuncAttributeMaxDynamicSharedMemorySize, lds));
        std::snprintf(name, sizeof name, "soa-aligned-x1-lds%d", kb);
        run(name, [&](float *x, float *y) {
            hipLaunchKernelGGL((soa<ALIGNED, 1>), grid(1), blk, lds, 0, x, y, nx, (int)sxy, S, lo, hi);
        });
        std::snprintf(name, sizeof name, "tiled-64-push-lds%d", kb);
        run(name, [&](float *x, float *y) {
            hipLaunchKernelGGL((tiled<PUSH, 64>), grid(1), blk, lds, 0, x, y, nx, (int)sxy, lo, hi);
        });
        const long long waves = n4 / (2 * Q * 64);
        std::snprintf(name, sizeof name, "copy-burst38-contig-lds%d", kb);
        run(name, [&](float *x, float *y) {
            hipLaunchKernelGGL(copy38_contig, dim3((unsigned)((waves + 3) / 4)), blk, lds, 0, (const float4 *)x,
                               (float4 *)y, waves);
        });
    }
    run("soa-aligned-x1", [&](float *x, float *y) {
        hipLaunchKernelGGL((soa<ALIGNED, 1>), grid(1), blk, 0, 0, x, y, nx, (int)sxy, S, lo, hi);
    });
    run("soa-aligned-x2", [&](float *x, float *y) {
        hipLaunchKernelGGL((soa<ALIGNED, 2>), grid(2), blk, 0, 0, x, y, nx, (int)sxy, S, lo, hi);
    });
    run("soa-aligned-x4", [&](float *x, float *y) {
        hipLaunchKernelGGL((soa<ALIGNED, 4>), grid(4), blk, 0, 0, x, y, nx, (int)sxy, S, lo, hi);
    });
    run("soa-push", [&](float *x, float *y) {
        hipLaunchKernelGGL((soa<PUSH, 1>), grid(1), blk, 0, 0, x, y, nx, (int)sxy, S, lo, hi);
    });
    run("soa-pull", [&](float *x, float *y) {
        hipLaunchKernelGGL((soa<PULL, 1>), grid(1), blk, 0, 0, x, y, nx, (int)sxy, S, lo, hi);
    });
    run("soa-push-nta", [&](float *x, float *y) {
        hipLaunchKernelGGL((soa<PUSH_NTA, 1>), grid(1), blk, 0, 0, x, y, nx, (int)sxy, S, lo, hi);
    });
    run("aa-odd-inplace", [&](float *x, float *) {
        hipLaunchKernelGGL((soa<AA_ODD, 1>), grid(1), blk, 0, 0, x, x, nx, (int)sxy, S, lo, hi);
    });
    if (nx == 256) {
        const long long rlo = nx + 1, rhi = N / nx - nx - 1;
        run("row-push-x4", [&](float *x, float *y) {
            hipLaunchKernelGGL(row_push, dim3((unsigned)((rhi - rlo + 3) / 4)), blk, 0, 0, x, y, nx, S, rlo, rhi);
        });
    }
    run("tiled-64-aligned", [&](float *x, float *y) {
        hipLaunchKernelGGL((tiled<ALIGNED, 64>), grid(1), blk, 0, 0, x, y, nx, (int)sxy, lo, hi);
    });
    run("tiled-64-push", [&](float *x, float *y) {
        hipLaunchKernelGGL((tiled<PUSH, 64>), grid(1), blk, 0, 0, x, y, nx, (int)sxy, lo, hi);
    });
    run("tiled-64-pull", [&](float *x, float *y) {
        hipLaunchKernelGGL((tiled<PULL, 64>), grid(1), blk, 0, 0, x, y, nx, (int)sxy, lo, hi);
    });
    run("tiled-256-aligned", [&](float *x, float *y) {
        hipLaunchKernelGGL((tiled<ALIGNED, 256>), grid(1), blk, 0, 0, x, y, nx, (int)sxy, lo, hi);
    });
    run("tiled-256-push", [&](float *x, float *y) {
        hipLaunchKernelGGL((tiled<PUSH, 256>), grid(1), blk, 0, 0, x, y, nx, (int)sxy, lo, hi);
    });
    if (nx == 256) {
        const long long rlo = nx + 1, rhi = N / nx - nx - 1;
        run("tiled-256-row-push-x4", [&](float *x, float *y) {
            hipLaunchKernelGGL(tiled_row_push, dim3((unsigned)((rhi - rlo + 3) / 4)), blk, 0, 0, x, y, nx, rlo, rhi);
        });
    }
    {
        const dim3 b512(512);
        auto mgrid = [&](int tx, int ty, int ch) { return dim3((unsigned)((nx / tx) * (nx / ty) * ch)); };
        char name[64];
        for (int ch : {2, 4, 8}) {
            std::snprintf(name, sizeof name, "march-aligned-64x8-c%d", ch);
            run(name, [&](float *x, float *y) {
                hipLaunchKernelGGL((march<64, 8, false>), mgrid(64, 8, ch), b512, 0, 0, x, y, nx, S, ch);
            });
            std::snprintf(name, sizeof name, "march-push-64x8-c%d", ch);
            run(name, [&](float *x, float *y) {
                hipLaunchKernelGGL((march<64, 8, true>), mgrid(64, 8, ch), b512, 0, 0, x, y, nx, S, ch);
            });
            std::snprintf(name, sizeof name, "march-tiled-aligned-64x8-c%d", ch);
            run(name, [&](float *x, float *y) {
                hipLaunchKernelGGL((march<64, 8, false, true>), mgrid(64, 8, ch), b512, 0, 0, x, y, nx, S, ch);
            });
            std::snprintf(name, sizeof name, "march-tiled-push-64x8-c%d", ch);
            run(name, [&](float *x, float *y) {
                hipLaunchKernelGGL((march<64, 8, true, true>), mgrid(64, 8, ch), b512, 0, 0, x, y, nx, S, ch);
            });
            std::snprintf(name, sizeof name, "march-aligned-128x4-c%d", ch);
            run(name, [&](float *x, float *y) {
                hipLaunchKernelGGL((march<128, 4, false>), mgrid(128, 4, ch), b512, 0, 0, x, y, nx, S, ch);
            });
            std::snprintf(name, sizeof name, "march-push-128x4-c%d", ch);
            run(name, [&](float *x, float *y) {
                hipLaunchKernelGGL((march<128, 4, true>), mgrid(128, 4, ch), b512, 0, 0, x, y, nx, S, ch);
            });
        }
        for (int ch : {32, 64, 128}) {   // short runs of planes: 8, 4, 2 at n = 256
            if (nx % ch) continue;
            std::snprintf(name, sizeof name, "march-aligned-64x8-c%d", ch);
            run(name, [&](float *x, float *y) {
                hipLaunchKernelGGL((march<64, 8, false>), mgrid(64, 8, ch), b512, 0, 0, x, y, nx, S, ch);
            });
            std::snprintf(name, sizeof name, "march-push-64x8-c%d", ch);
            run(name, [&](float *x, float *y) {
                hipLaunchKernelGGL((march<64, 8, true>), mgrid(64, 8, ch), b512, 0, 0, x, y, nx, S, ch);
            });
        }
        if (nx % 256 == 0) {
            run("march-aligned-256x2-c2", [&](float *x, float *y) {
                hipLaunchKernelGGL((march<256, 2, false>), mgrid(256, 2, 2), b512, 0, 0, x, y, nx, S, 2);
            });
            run("march-push-256x2-c2", [&](float *x, float *y) {
                hipLaunchKernelGGL((march<256, 2, true>), mgrid(256, 2, 2), b512, 0, 0, x, y, nx, S, 2);
            });
        }
    }
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    return 0;
}
