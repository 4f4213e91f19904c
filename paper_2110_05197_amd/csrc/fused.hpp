// fused.hpp -- one-pass step: each block owns a TX x TY column of nodes and
// marches it through a chunk of TZ planes (D3Q19), or a row of TX nodes
// through a chunk of rows (D2Q9, the box seen as nx x 1 x ny).  The stencil
// inputs (colour-gradient densities / pseudopotential) of a plane are
// computed from its populations as they are loaded (two planes ahead of the
// collision), for the tile and a one-node halo ring, into a four-plane LDS
// ring; a tile node's populations wait one iteration in the thread's LDS slot
// and are collided from registers.  Only the halo ring's populations are read
// twice (by this block and by its neighbour), so HBM traffic stays near one
// read and one write of every population per step; no density field is
// written.  The solo and the batched kernels share the column body.
//
// ny % TY == 0; any nx (the last column in x is masked when TX does not
// divide it) and any nz.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "launch.hpp"

namespace mclbm {

// Stencil-field values of one node from its populations (the same values the
// density-field pass stores).
template <int MODEL, int NF, class C, class M, class FT>
__device__ __forceinline__ void field_values(const HP<C, M> &H, const M (&dr)[2], FT (&v)[NF])
{
    if constexpr (MODEL == CG) {
        v[0] = (FT)dr[0];
        v[1] = (FT)dr[1];
        v[2] = (FT)colour_field(H, dr[0], dr[1]);
    } else if constexpr (MODEL == SC_MP) {
        v[0] = (FT)pseudo_potential(H, H.rho0[0] + dr[0]);
    } else {
        v[0] = (FT)dr[0];
        v[1] = (FT)dr[1];
    }
}

// Block index -> tile, keeping runs of consecutive tiles on one XCD (blocks
// are dealt round-robin to the 8 XCDs, each with its own L2).
__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    if (nblocks % 8) return b;
    return (b % 8) * (nblocks / 8) + b / 8;
}

// Whether a lattice has velocities along y (D2Q9Z has none: its tile rows
// need no halo rows).
template <class L>
constexpr bool uses_y()
{
    for (int i = 0; i < L::Q; ++i)
        if (L::cy[i] != 0) return true;
    return false;
}
template <class L, int TY>
constexpr int ring_rows() { return uses_y<L>() ? TY + 2 : TY; }

template <class L, int MODEL, int TX, int TY, class FT>
constexpr int fused_ring_bytes()
{
    return (4 * NField<MODEL>::n * (TX + 2) * ring_rows<L, TY>() * (int)sizeof(FT) + 15) / 16 * 16;
}
template <int PR, int MODEL, int TX, int TY, class L = D3Q19>
constexpr int fused_lds_bytes()
{
    return fused_ring_bytes<L, MODEL, TX, TY, typename Prec<PR>::F>()
           + NComp<MODEL>::n * L::Q * TX * TY * (int)sizeof(typename Prec<PR>::C);
}

// One block's work: the TX x TY column at (x0, y0), planes [z0, z1).  An
// EDGE column is the last one in x when TX does not divide nx: its first
// w = nx - x0 threads hold nodes, the others only take part in the barriers,
// and its +x halo is the column at x0 + w.  L is the lattice of the
// arithmetic, LA the one that places neighbours: both D3Q19, or D2Q9 and
// D2Q9Z for a 2-D box seen as nx x 1 x ny (TY = 1, halo columns only), so
// that a 2-D node's arithmetic is the two-pass kernels', operation for
// operation.  CONS: whether the collision keeps each colour's node mass
// (kConsNever / kConsAsked / kConsAlways, see cg_collide): the batched
// kernels ask each simulation, the solo launches choose a kernel.
template <int PR, int MODEL, int TX, int TY, bool PERIODIC, bool EDGE = false, class L = D3Q19, class LA = L,
          int CONS = kConsShared<PR>>
__device__ __forceinline__ void fused_column(const KParams &P, const typename Prec<PR>::S *__restrict__ src,
                                             typename Prec<PR>::S *__restrict__ dst, unsigned *flag, int x0, int y0,
                                             int z0, int z1, unsigned char *smem)
{
    using C = typename Prec<PR>::C;
    using M = typename Prec<PR>::M;
    using FT = typename Prec<PR>::F;
    constexpr int Q = L::Q;
    constexpr int K = NComp<MODEL>::n;
    constexpr int NF = NField<MODEL>::n;
    static_assert(LA::Q == L::Q, "one velocity set");
    constexpr bool YH = uses_y<LA>();   // halo rows y0-1 and y0+TY
    constexpr int RY = YH ? 1 : 0;      // ring row of tile row 0
    constexpr int HX = TX + 2, HY = ring_rows<LA, TY>(), PL = HX * HY, NT = TX * TY, NH = PL - NT;
    static_assert(NH <= NT, "halo ring larger than the block");
    // Dynamic LDS: a four-plane ring of stencil values (planes z-1, z, z+1
    // are read while plane z+2 is written), then each thread's private slot
    // holding the populations of plane z+1 (laid out [population][thread] so
    // that a wavefront's accesses are contiguous).
    FT (*lds)[NF][PL] = reinterpret_cast<FT (*)[NF][PL]>(smem);
    C *pop = reinterpret_cast<C *>(smem + fused_ring_bytes<LA, MODEL, TX, TY, FT>());

    const long long SW = P.S;
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const HP<C, M> H = make_hp<C, M>(P);
    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int x = x0 + lx, y = y0 + ly;
    const int my_slot = (ly + RY) * HX + (lx + 1);
    const int w = EDGE ? min(TX, nx - x0) : TX;   // nodes per row of this column
    const bool act = !EDGE || lx < w;

    // halo ring node of this thread: rows y0-1 and y0+TY (when the lattice
    // has y velocities), then columns x0-1 and x0+w
    constexpr int NR = YH ? 2 * HX : 0;
    int hx = 0, hy = 0;
    if (YH && tid < HX) { hx = tid - 1; hy = -1; }
    else if (YH && tid < NR) { hx = tid - HX - 1; hy = TY; }
    else if (tid < NR + TY) { hx = -1; hy = tid - NR; }
    else { hx = w; hy = tid - NR - TY; }
    const bool has_h = tid < NH && hx <= w;
    const int h_slot = (hy + RY) * HX + (hx + 1);
    const int hgx = stencil_coord(x0 + hx, nx, P.bc[0]);
    const int hgy = stencil_coord(y0 + hy, ny, P.bc[1]);
    const long long n_xy = (long long)x + (long long)nx * y;
    const long long h_xy = (long long)hgx + (long long)nx * hgy;
    const long long sxy = (long long)nx * ny;
    auto ring = [&](int p) { return (p - z0 + 1) & 3; };

    bool bad = false;
    // stencil values of one node of plane p from its populations
    auto put = [&](int p, int slot, const C (&gv)[K][Q], M (&drv)[2], M (&jv)[3], bool interior) {
        node_moments<L, K>(gv, drv, jv);
        FT v[NF];
        field_values<MODEL, NF>(H, drv, v);
#pragma unroll
        for (int a = 0; a < NF; ++a) lds[ring(p)][a][slot] = v[a];
        if (interior && p >= z0 && p < z1) {
            const M r = H.rho0[0] + drv[0] + (K == 2 ? H.rho0[1] + drv[1] : M(0));
            bad = bad || node_bad(r, jv[0] + jv[1] + jv[2]);
        }
    };
    auto zoff = [&](int p) { return sxy * stencil_coord(p, nz, P.bc[2]); };

    C c[K][Q];                  // populations of plane z (plane z+1's wait in LDS)
    M drc[2], jc[3], drn[2], jn[3];
    {
        // prologue: stencil values of planes z0-1, z0, z0+1; populations of z0, z0+1
        C tmp[K][Q];
        M d2[2], j2[3];
        if (act) {
            load_node<L, K>(src, SW, n_xy + zoff(z0 - 1), tmp);
            put(z0 - 1, my_slot, tmp, d2, j2, true);
            load_node<L, K>(src, SW, n_xy + zoff(z0), c);
            put(z0, my_slot, c, drc, jc, true);
            load_node<L, K>(src, SW, n_xy + zoff(z0 + 1), tmp);
            put(z0 + 1, my_slot, tmp, drn, jn, true);
#pragma unroll
            for (int k = 0; k < K; ++k)
#pragma unroll
                for (int i = 0; i < Q; ++i) pop[(k * Q + i) * NT + tid] = tmp[k][i];
        }
        if (has_h)
            for (int p = z0 - 1; p <= z0 + 1; ++p) {
                load_node<L, K>(src, SW, h_xy + zoff(p), tmp);
                put(p, h_slot, tmp, d2, j2, false);
            }
    }
    __syncthreads();

    for (int z = z0; z < z1; ++z) {
        // 1. issue the loads of plane z+2 (consumed after the collision).  The
        // 2-D row kernel issues them at raised wave priority, so that they
        // leave before the SIMD's other waves take the issue slots for their
        // arithmetic: 4096^2 FP32 0.489 -> 0.480 ms.  The D3Q19 column
        // kernel ran 2 % slower with it (1.115 -> 1.134-1.151 ms at 256^3),
        // and raised priority around the stores cost 1.5 % in a timing copy.
        constexpr bool prio = !YH;
        const bool ahead = z + 2 <= z1;
        RawNode<L, K, typename Prec<PR>::S, C> dr_, hr_;
        if constexpr (prio) __builtin_amdgcn_s_setprio(3);
        if (ahead) {
            if (act) dr_.load(src, SW, n_xy + zoff(z + 2));
            if (has_h) hr_.load(src, SW, h_xy + zoff(z + 2));
        }
        if constexpr (prio) __builtin_amdgcn_s_setprio(0);

        // 2. collide plane z with the stencil values of planes z-1, z, z+1
        if (act) {
            C v[NF][Q];
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int s = ring(z + LA::cz[i]);
                const int o = my_slot + LA::cy[i] * HX + LA::cx[i];
#pragma unroll
                for (int a = 0; a < NF; ++a) v[a][i] = (C)lds[s][a][o];
            }
#pragma unroll
            for (int a = 0; a < NF; ++a) v[a][0] = C(0);

            if constexpr (MODEL == CG) {
                C gR[3], gB[3], gN[3];
                stencil_sum<L>(v[0], gR);
                stencil_sum<L>(v[1], gB);
                stencil_sum<L>(v[NF - 1], gN);
#pragma unroll
                for (int dd = 0; dd < 3; ++dd) { gR[dd] *= C(3); gB[dd] *= C(3); gN[dd] *= C(3); }
                const C F0[3] = {C(0), C(0), C(0)};
                cg_collide<L, C, M, false, CONS>(H, c, drc, jc, gR, gB, gN, F0);
            } else if constexpr (MODEL == SC_MP) {
                C s3[3];
                stencil_sum<L>(v[0], s3);
                const C psi = (C)lds[ring(z)][0][my_slot];
                const M rho = H.rho0[0] + drc[0];
                const M irho = rcp(rho);
                C F[3], u[3];
#pragma unroll
                for (int dd = 0; dd < 3; ++dd) {
                    F[dd] = -H.G * psi * s3[dd];
                    u[dd] = (C)((jc[dd] + M(0.5) * (M)F[dd]) * irho);
                }
                sc_collide_component<L, C, M>(c[0], H.om[0], drc[0], rho, u, F, H.rho0[0], H.corrM[0], H.shiftM[0]);
            } else {
                C sR[3], sB[3];
                stencil_sum<L>(v[0], sR);
                stencil_sum<L>(v[NF - 1], sB);
                const M rR = H.rho0[0] + drc[0], rB = H.rho0[1] + drc[1];
                const M ir = rcp(rR + rB);
                C FR[3], FB[3], u[3];
#pragma unroll
                for (int dd = 0; dd < 3; ++dd) {
                    FR[dd] = -H.xpref * (C)rR * sB[dd];
                    FB[dd] = -H.xpref * (C)rB * sR[dd];
                    u[dd] = (C)((jc[dd] + M(0.5) * ((M)FR[dd] + (M)FB[dd])) * ir);
                }
                sc_collide_component<L, C, M>(c[0], H.om[0], drc[0], rR, u, FR, H.rho0[0], H.corrM[0], H.shiftM[0]);
                sc_collide_component<L, C, M>(c[K - 1], H.om[1], drc[1], rB, u, FB, H.rho0[1], H.corrM[1], H.shiftM[1]);
            }
            const long long n = n_xy + sxy * z;
            // populations that stay on their x (cx = 0) land on whole cache
            // lines and are never read again in this step: stream them past
            // the cache; the x-shifted ones share lines with the neighbouring
            // tile's stores and go through L2
            if constexpr (PERIODIC) push_store_periodic<LA, K, typename Prec<PR>::S, C, true>(P, dst, x, y, z, n, c);
            else push_store_general<LA, K, typename Prec<PR>::S, C, true>(P, dst, x, y, z, n, c);
        }

        // 3. stencil values of plane z+2
        M drd[2], jd[3];
        C d[K][Q];
        dr_.get(d);
        if (ahead) {
            if (act) put(z + 2, my_slot, d, drd, jd, true);
            if (has_h) {
                C hh[K][Q];
                hr_.get(hh);
                M dh[2], jh[3];
                put(z + 2, h_slot, hh, dh, jh, false);
            }
        }
        // 4. rotate through this thread's LDS slot: z+1 -> z, z+2 -> z+1
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                C *sl = &pop[(k * Q + i) * NT + tid];
                c[k][i] = *sl;
                *sl = d[k][i];
            }
        __syncthreads();  // plane z+2 complete; plane z-1's slot is free
        drc[0] = drn[0]; drc[1] = drn[1];
        jc[0] = jn[0]; jc[1] = jn[1]; jc[2] = jn[2];
        drn[0] = drd[0]; drn[1] = drd[1];
        jn[0] = jd[0]; jn[1] = jd[1]; jn[2] = jd[2];
    }
    const unsigned long long any = __ballot(bad);
    if (any != 0ull && (tid & 63) == 0) atomicOr(flag, 1u);
}

// RAGGED: TX does not divide nx, and the last column in x is an edge column.
template <int PR, int MODEL, int TX, int TY, bool PERIODIC, bool RAGGED, class L = D3Q19, class LA = L,
          bool CONS = false>
__global__ __launch_bounds__(TX *TY) void k_fused(KParams P, const typename Prec<PR>::S *__restrict__ src,
                                                  typename Prec<PR>::S *__restrict__ dst, unsigned *flag, int TZ,
                                                  int tiles_x, int tiles_y)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int bx = t % tiles_x, by = (t / tiles_x) % tiles_y, bz = t / (tiles_x * tiles_y);
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ, z1 = min(z0 + TZ, P.nz);
    constexpr int cons = CONS ? kConsAlways : kConsNever;
    if constexpr (RAGGED) {
        if (bx == tiles_x - 1) {
            fused_column<PR, MODEL, TX, TY, PERIODIC, true, L, LA, cons>(P, src, dst, flag, x0, y0, z0, z1, smem);
            return;
        }
    }
    fused_column<PR, MODEL, TX, TY, PERIODIC, false, L, LA, cons>(P, src, dst, flag, x0, y0, z0, z1, smem);
}

// Batched one-pass step: the blocks of all eligible simulations of a group
// (D3Q19, ny a multiple of the column height) in one launch per kind; a
// block finds its simulation in the descriptor array (one-pass block ranges),
// skips it unless it is running and of the launch's kind (all faces periodic
// or not; nx a multiple of 64 or not; 96-wide columns or not), and processes
// one column of that simulation.  EDGE launches take the simulations whose nx
// is not a multiple of 64 and run every column through the masked column body
// (the last column in x holds nx mod 64 nodes; a full column computes the same
// as unmasked); WIDE launches take those on 96 x 4 columns.
// The per-node arithmetic is the solo kernels', so a batched simulation
// evolves bitwise as it would alone.  Columns: 64-wide rows (at 16
// or 32 nodes the rows of the x-shifted pushes split cache lines between
// neighbouring blocks and the step runs at half speed), 8 rows (4 in FP64 and
// in mixed precision, whose FP64 sums need the registers).  One kernel per
// kind keeps a single column body per kernel: with two inlined the
// mixed-precision kernel needed 270 registers (one wave per SIMD) and ran no
// faster than the batched two-pass kernels.
constexpr int kBatchTX = 64;
constexpr int batch_ty(int precision) { return precision == 0 || precision == 2 ? 4 : 8; }
// As in the solo kernel, a simulation whose nx 96 divides and 64 does not
// takes 96 x 4 columns (kernels of their own, WIDE): no lane idles where a
// 64-wide split would leave half of its last column empty.  Not FP64, nor the
// mixed-precision colour gradient: a six-wave block allows 256 registers a
// lane, and their batched columns (which ask each simulation whether to keep
// colour mass) need more (FP64 about 400; mixed 40 spilled).
constexpr int kBatchWideTX = 96, kBatchWideTY = 4;
constexpr bool batch_wide_kernel(int precision, int model)
{
    return precision != 0 && !(precision == 2 && model == CG);
}
constexpr bool batch_wide(int precision, int model, int nx, int ny)
{
    return batch_wide_kernel(precision, model) && nx % kBatchWideTX == 0 && nx % kBatchTX != 0
           && ny % kBatchWideTY == 0;
}
constexpr int batch_tile_tx(int precision, int model, int nx, int ny)
{
    return batch_wide(precision, model, nx, ny) ? kBatchWideTX : kBatchTX;
}
constexpr int batch_tile_ty(int precision, int model, int nx, int ny)
{
    return batch_wide(precision, model, nx, ny) ? kBatchWideTY : batch_ty(precision);
}
// which kernels a group launches: all-periodic sims and others, each with nx
// a multiple of 64 or not (EDGE), or on 96 x 4 columns (WIDE)
constexpr int kFusedPeriodic = 1, kFusedBounded = 2, kFusedPeriodicEdge = 4, kFusedBoundedEdge = 8;
constexpr int kFusedPeriodicWide = 16, kFusedBoundedWide = 32;
constexpr int fused_kind(bool periodic, bool edge, bool wide)
{
    return wide ? (periodic ? kFusedPeriodicWide : kFusedBoundedWide)
           : edge ? (periodic ? kFusedPeriodicEdge : kFusedBoundedEdge) : (periodic ? kFusedPeriodic : kFusedBounded);
}

__device__ __forceinline__ int find_sim_fused(const SimDesc *D, int n, long long b)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (D[mid].fblock0 <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

constexpr int kb_tx(bool wide) { return wide ? kBatchWideTX : kBatchTX; }
constexpr int kb_ty(int precision, bool wide) { return wide ? kBatchWideTY : batch_ty(precision); }

template <int PR, int MODEL, bool PERIODIC, bool EDGE, bool WIDE = false>
__global__ __launch_bounds__(kb_tx(WIDE) * kb_ty(PR, WIDE)) void kb_fused(SimDesc *D, int nsims)
{
    static_assert(!(WIDE && EDGE) && !(WIDE && !batch_wide_kernel(PR, MODEL)), "96-wide columns: full columns");
    constexpr int TX = kb_tx(WIDE), TY = kb_ty(PR, WIDE);
    extern __shared__ __align__(16) unsigned char smem[];
    const int s = find_sim_fused(D, nsims, blockIdx.x);
    const SimDesc &d = D[s];
    if (d.state != 0) return;
    if ((d.P.bc[0] == 0 && d.P.bc[1] == 0 && d.P.bc[2] == 0) != PERIODIC) return;
    if (batch_wide(PR, MODEL, d.P.nx, d.P.ny) != WIDE) return;
    if (!WIDE && (d.P.nx % kBatchTX != 0) != EDGE) return;
    const long long b = blockIdx.x - d.fblock0;
    const int tiles_x = (d.P.nx + TX - 1) / TX, tiles_y = d.P.ny / TY;
    const int bx = (int)(b % tiles_x), by = (int)((b / tiles_x) % tiles_y), bz = (int)(b / ((long long)tiles_x * tiles_y));
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * d.ftz, z1 = min(z0 + d.ftz, d.P.nz);
    using S = typename Prec<PR>::S;
    const S *src = global_ptr<const S>(d.f[d.cur]);
    S *dst = global_ptr<S>(d.f[d.cur ^ 1]);
    unsigned *flag = global_ptr<unsigned>(d.flag);
    fused_column<PR, MODEL, TX, TY, PERIODIC, EDGE>(d.P, src, dst, flag, x0, y0, z0, z1, smem);
}

// Planes per column of the batched simulations of a group.  A column
// advances one plane at a time and starts with three planes of loads, and
// the blocks run in rounds of `resident` (the blocks the chip holds at
// once), so the time of a step goes as rounds * (planes per chunk + 3).  The
// chunk length is searched for the least such cost (ties: fewer blocks);
// each simulation then balances its chunks over its nz.
inline int batch_fused_tz(int nz, int group_tz)
{
    const int chunks = (nz + group_tz - 1) / group_tz;
    return (nz + chunks - 1) / chunks;
}

// cols[s], nz[s]: columns per plane and planes of the group's one-pass sims
inline int batch_group_tz(const long long *cols, const int *nz, int n, long long resident)
{
    int best = 1;
    long long best_cost = -1, best_blocks = 0;
    for (int tz = 1; tz <= 64; ++tz) {
        long long blocks = 0;
        int longest = 0;
        for (int s = 0; s < n; ++s) {
            const int t = batch_fused_tz(nz[s], tz);
            blocks += cols[s] * ((nz[s] + t - 1) / t);
            longest = std::max(longest, t);
        }
        const long long rounds = (blocks + resident - 1) / std::max<long long>(1, resident);
        const long long cost = rounds * (longest + 3);
        if (best_cost < 0 || cost < best_cost || (cost == best_cost && blocks < best_blocks)) {
            best = tz;
            best_cost = cost;
            best_blocks = blocks;
        }
    }
    return best;
}

// Blocks of kb_fused<PR, MODEL, ...> the device holds at once (the smallest
// over the kinds).
template <int PR, int MODEL>
long long batch_fused_resident()
{
    constexpr int lds = fused_lds_bytes<PR, MODEL, kBatchTX, batch_ty(PR)>();
    int dev = 0, cus = 0, per_cu = 1 << 30;
    if (hipGetDevice(&dev) != hipSuccess
        || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 256;
    const void *fns[4] = {(const void *)kb_fused<PR, MODEL, true, false>, (const void *)kb_fused<PR, MODEL, false, false>,
                          (const void *)kb_fused<PR, MODEL, true, true>, (const void *)kb_fused<PR, MODEL, false, true>};
    for (const void *fn : fns) {
        int b = 0;
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, kBatchTX * batch_ty(PR), lds) != hipSuccess)
            return 256;
        per_cu = std::min(per_cu, b);
    }
    if constexpr (batch_wide_kernel(PR, MODEL)) {
        constexpr int lds_w = fused_lds_bytes<PR, MODEL, kBatchWideTX, kBatchWideTY>();
        const void *wide[2] = {(const void *)kb_fused<PR, MODEL, true, false, true>,
                               (const void *)kb_fused<PR, MODEL, false, false, true>};
        for (const void *fn : wide) {
            int b = 0;
            (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_w);
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, kBatchWideTX * kBatchWideTY, lds_w) != hipSuccess)
                return 256;
            per_cu = std::min(per_cu, b);
        }
    }
    return (long long)std::max(1, per_cu) * std::max(1, cus);
}

// kinds: the fused_kind() bits of the simulations present.  Every launch
// covers the group's whole one-pass block range; a block whose simulation is
// of another kind returns at once.
template <int PR, int MODEL>
void launch_batch_fused(SimDesc *D, int n, long long fblocks, int kinds, hipStream_t s)
{
    constexpr int lds = fused_lds_bytes<PR, MODEL, kBatchTX, batch_ty(PR)>();
    const void *fns[4] = {(const void *)kb_fused<PR, MODEL, true, false>, (const void *)kb_fused<PR, MODEL, false, false>,
                          (const void *)kb_fused<PR, MODEL, true, true>, (const void *)kb_fused<PR, MODEL, false, true>};
    static bool attr_set = false;
    if (!attr_set) {
        for (const void *fn : fns) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        attr_set = true;
    }
    const dim3 grid((unsigned)fblocks), block(kBatchTX * batch_ty(PR));
    if (kinds & kFusedPeriodic) hipLaunchKernelGGL((kb_fused<PR, MODEL, true, false>), grid, block, lds, s, D, n);
    if (kinds & kFusedBounded) hipLaunchKernelGGL((kb_fused<PR, MODEL, false, false>), grid, block, lds, s, D, n);
    if (kinds & kFusedPeriodicEdge) hipLaunchKernelGGL((kb_fused<PR, MODEL, true, true>), grid, block, lds, s, D, n);
    if (kinds & kFusedBoundedEdge) hipLaunchKernelGGL((kb_fused<PR, MODEL, false, true>), grid, block, lds, s, D, n);
    if constexpr (batch_wide_kernel(PR, MODEL)) {
        constexpr int lds_w = fused_lds_bytes<PR, MODEL, kBatchWideTX, kBatchWideTY>();
        static bool attr_w = false;
        if (!attr_w) {
            (void)hipFuncSetAttribute((const void *)kb_fused<PR, MODEL, true, false, true>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds_w);
            (void)hipFuncSetAttribute((const void *)kb_fused<PR, MODEL, false, false, true>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds_w);
            attr_w = true;
        }
        const dim3 block_w(kBatchWideTX * kBatchWideTY);
        if (kinds & kFusedPeriodicWide)
            hipLaunchKernelGGL((kb_fused<PR, MODEL, true, false, true>), grid, block_w, lds_w, s, D, n);
        if (kinds & kFusedBoundedWide)
            hipLaunchKernelGGL((kb_fused<PR, MODEL, false, false, true>), grid, block_w, lds_w, s, D, n);
    }
}

struct FusedShape {
    int tx, ty, tz;
    bool ragged;   // the last column in x is an edge column
};

// Tile choice: 64-wide rows (narrower rows split the x-shifted pushes' cache
// lines between blocks), the last column masked when 64 does not divide nx;
// TY = 8 when ny allows, else 4; TZ planes per block.  FP64 (wide) tiles are
// 4 rows: half the threads, so that each wave may hold its double-precision
// planes in up to 512 registers and the LDS slot of plane z+1 stays at the
// FP32 size.  Where 96 divides nx and 64 does not (nx = 96, 288, ...), the
// columns are 96 x 4 instead (six waves, no lane idle), in place of 64-wide
// columns whose last one would leave a third of its lanes or more idle.
inline bool fused_shape(const KParams &P, FusedShape &sh, bool wide = false)
{
    sh.tx = 64;
    sh.ragged = P.nx % 64 != 0;
    if (!wide && P.nx % 96 == 0 && P.nx % 64 != 0 && P.ny % 4 == 0) {
        sh.tx = 96;
        sh.ty = 4;
        sh.ragged = false;
    } else if (!wide && P.ny % 8 == 0) sh.ty = 8;
    else if (P.ny % 4 == 0) sh.ty = 4;
    else return false;
    // z-chunk: at most one block per compute unit (256 on MI355X) -- more
    // resident blocks per XCD overflow its L2 and the halo re-reads miss,
    // and a grid just above 256 blocks runs a second, nearly empty round
    const long long txy = (long long)((P.nx + sh.tx - 1) / sh.tx) * (P.ny / sh.ty);
    const long long tiles_z = std::max<long long>(1, 256 / txy);
    sh.tz = (int)((P.nz + tiles_z - 1) / tiles_z);
    return true;
}

template <int PR, int MODEL, int TX, int TY, bool RAGGED, bool CONS>
void launch_fused_kernel(const KParams &P, const void *src, void *dst, unsigned *flag, int tz, hipStream_t s)
{
    const int tiles_x = (P.nx + TX - 1) / TX, tiles_y = P.ny / TY, tiles_z = (P.nz + tz - 1) / tz;
    const dim3 grid(tiles_x * tiles_y * tiles_z), block(TX * TY);
    using S = typename Prec<PR>::S;
    constexpr int lds = fused_lds_bytes<PR, MODEL, TX, TY>();
    static bool attr_set = false;   // raise the dynamic-LDS limit once per process
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_fused<PR, MODEL, TX, TY, true, RAGGED, D3Q19, D3Q19, CONS>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        (void)hipFuncSetAttribute((const void *)k_fused<PR, MODEL, TX, TY, false, RAGGED, D3Q19, D3Q19, CONS>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        attr_set = true;
    }
    if (P.bc[0] == 0 && P.bc[1] == 0 && P.bc[2] == 0)
        hipLaunchKernelGGL((k_fused<PR, MODEL, TX, TY, true, RAGGED, D3Q19, D3Q19, CONS>), grid, block, lds, s, P,
                           (const S *)src, (S *)dst, flag, tz, tiles_x, tiles_y);
    else
        hipLaunchKernelGGL((k_fused<PR, MODEL, TX, TY, false, RAGGED, D3Q19, D3Q19, CONS>), grid, block, lds, s, P,
                           (const S *)src, (S *)dst, flag, tz, tiles_x, tiles_y);
}

// The mass-keeping collision has kernels of its own, so that the default
// step carries none of it.
template <int PR, int MODEL, int TX, int TY, bool RAGGED>
void launch_fused_shape(const KParams &P, const void *src, void *dst, unsigned *flag, int tz, hipStream_t s)
{
    if constexpr (kConserveRest<PR> && MODEL == CG) {
        if (P.conserve) {
            launch_fused_kernel<PR, MODEL, TX, TY, RAGGED, true>(P, src, dst, flag, tz, s);
            return;
        }
    }
    launch_fused_kernel<PR, MODEL, TX, TY, RAGGED, false>(P, src, dst, flag, tz, s);
}

template <int PR, int MODEL>
void launch_fused(const KParams &P, const void *src, void *dst, unsigned *flag, hipStream_t s)
{
    FusedShape sh;
    fused_shape(P, sh, PR == 0);  // checked at create time
    if constexpr (PR != 0) {
        if (sh.tx == 96) {
            launch_fused_shape<PR, MODEL, 96, 4, false>(P, src, dst, flag, sh.tz, s);
            return;
        }
    }
    if (sh.ty == 4) {
        if (sh.ragged) launch_fused_shape<PR, MODEL, 64, 4, true>(P, src, dst, flag, sh.tz, s);
        else launch_fused_shape<PR, MODEL, 64, 4, false>(P, src, dst, flag, sh.tz, s);
    } else if constexpr (PR != 0) {
        if (sh.ragged) launch_fused_shape<PR, MODEL, 64, 8, true>(P, src, dst, flag, sh.tz, s);
        else launch_fused_shape<PR, MODEL, 64, 8, false>(P, src, dst, flag, sh.tz, s);
    }
}

// D2Q9 one-pass step: the 2-D box as nx x 1 x ny (neighbours placed by
// D2Q9Z, arithmetic in D2Q9), rows of
// 256 nodes marching along y, the last row segment masked when 256 does not
// divide nx.  Chunks of at least 8 rows, about two blocks per compute unit.
constexpr int k2dTX = 256;

inline KParams as_marching_2d(const KParams &P)
{
    KParams Q = P;
    Q.ny = 1;
    Q.nz = P.ny;
    Q.bc[1] = 0;
    Q.bc[2] = P.bc[1];
    return Q;
}

// Row segments and rows per block of the 2-D launch (Q: the box as
// nx x 1 x ny).
inline void fused2d_rows(const KParams &Q, int &tiles_x, int &tz)
{
    tiles_x = (Q.nx + k2dTX - 1) / k2dTX;
    const int tiles_z = std::max(1, std::min(512 / tiles_x, Q.nz / 8));
    tz = (Q.nz + tiles_z - 1) / tiles_z;
}

template <int PR, int MODEL, bool RAGGED, bool CONS>
void launch_fused2d_shape(const KParams &Q, const void *src, void *dst, unsigned *flag, hipStream_t s)
{
    int tiles_x = 0, tz = 0;
    fused2d_rows(Q, tiles_x, tz);
    const dim3 grid(tiles_x * ((Q.nz + tz - 1) / tz)), block(k2dTX);
    using S = typename Prec<PR>::S;
    constexpr int lds = fused_lds_bytes<PR, MODEL, k2dTX, 1, D2Q9Z>();
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute((const void *)k_fused<PR, MODEL, k2dTX, 1, true, RAGGED, D2Q9, D2Q9Z, CONS>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        (void)hipFuncSetAttribute((const void *)k_fused<PR, MODEL, k2dTX, 1, false, RAGGED, D2Q9, D2Q9Z, CONS>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        attr_set = true;
    }
    if (Q.bc[0] == 0 && Q.bc[2] == 0)
        hipLaunchKernelGGL((k_fused<PR, MODEL, k2dTX, 1, true, RAGGED, D2Q9, D2Q9Z, CONS>), grid, block, lds, s, Q,
                           (const S *)src, (S *)dst, flag, tz, tiles_x, 1);
    else
        hipLaunchKernelGGL((k_fused<PR, MODEL, k2dTX, 1, false, RAGGED, D2Q9, D2Q9Z, CONS>), grid, block, lds, s, Q,
                           (const S *)src, (S *)dst, flag, tz, tiles_x, 1);
}

template <int PR, int MODEL>
void launch_fused2d(const KParams &P, const void *src, void *dst, unsigned *flag, hipStream_t s)
{
    const KParams Q = as_marching_2d(P);
    if constexpr (kConserveRest<PR> && MODEL == CG) {
        if (P.conserve) {
            if (Q.nx % k2dTX) launch_fused2d_shape<PR, MODEL, true, true>(Q, src, dst, flag, s);
            else launch_fused2d_shape<PR, MODEL, false, true>(Q, src, dst, flag, s);
            return;
        }
    }
    if (Q.nx % k2dTX) launch_fused2d_shape<PR, MODEL, true, false>(Q, src, dst, flag, s);
    else launch_fused2d_shape<PR, MODEL, false, false>(Q, src, dst, flag, s);
}

}  // namespace mclbm
