// kernels.hpp -- node-parallel kernels of the step (density-field pass,
// collide + push-stream pass, outflow completion), initialisation,
// export/import and the observable reductions.  Each kernel body is a
// __device__ function of (parameters, buffers, node) so that the solo
// kernels and the batched kernels run the very same arithmetic.
#pragma once

#include <type_traits>
#include <utility>

#include <hip/hip_runtime.h>

#include "node.hpp"

namespace mclbm {

constexpr int kBlock = 256;

// Observable accumulators (FP64):
//   0 mass_R  1 mass_B  2..4 momentum  5 E_kin  6 max|u|  7 red volume
//   8 diverged (max)  9 + 4m + {0 sum_in, 1 n_in, 2 sum_out, 3 n_out}, m = 0..9
constexpr int kNAcc = 9 + 40;
constexpr int kRedBlocks = 1024;

struct EpsTable { double e[10]; };


// ---------------------------------------------------------------------------
// Loads and stores of one node's populations.
// ---------------------------------------------------------------------------
// Memory access with an optional non-temporal hint (streamed data that this
// step will not read again through the cache).
template <bool NT, class T> __device__ __forceinline__ T ld(const T *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, class T> __device__ __forceinline__ void st(T *p, T v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Storage order.  Two-colour FP16 storage keeps both colours of a population
// in one 32-bit word, [i][n][k], so that a node moves 19 dwords each way as in
// FP32 (2-byte accesses would halve the payload of every memory instruction);
// every other storage is [k][i][n].
using Half2 = _Float16 __attribute__((ext_vector_type(2)));
template <int K, class S> constexpr bool kPairs = K == 2 && std::is_same<S, _Float16>::value;

// SW: storage words from one population array to the next (KParams::S).
template <class L, int K, class S>
__device__ __forceinline__ size_t sidx(int k, int i, size_t SW, size_t n)
{
    if constexpr (kPairs<K, S>) return 2 * ((size_t)i * SW + n) + (size_t)k;
    else return (size_t)(k * L::Q + i) * SW + n;
}

// Populations of node n; SW is the array stride KParams::S.
template <class L, int K, class S, class C, bool NT = false>
__device__ __forceinline__ void load_node(const S *__restrict__ f, long long SW, long long n,
                                          C (&g)[K][L::Q])
{
    const unsigned o = (unsigned)n;   // N < 2^31: per-lane 32-bit offset, uniform base
    if constexpr (kPairs<K, S>) {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const Half2 v = ld<NT>(&(reinterpret_cast<const Half2 *>(f) + (size_t)i * (size_t)SW)[o]);
            g[0][i] = (C)v.x;
            g[1][i] = (C)v.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int i = 0; i < L::Q; ++i) g[k][i] = (C)ld<NT>(&(f + (size_t)(k * L::Q + i) * (size_t)SW)[o]);
    }
}

// A node's populations held as loaded, for software prefetching: the load is
// issued early and the conversion to the arithmetic type waits until the
// values are used (converting on arrival would wait for the load at once).
template <class L, int K, class S, class C, bool PAIRS = kPairs<K, S>>
struct RawNode {
    C v[K][L::Q];
    __device__ __forceinline__ void load(const S *__restrict__ f, long long SW, long long n)
    {
        load_node<L, K>(f, SW, n, v);
    }
    __device__ __forceinline__ void get(C (&g)[K][L::Q]) const
    {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int i = 0; i < L::Q; ++i) g[k][i] = v[k][i];
    }
};
template <class L, int K, class S, class C>
struct RawNode<L, K, S, C, true> {
    Half2 v[L::Q];
    __device__ __forceinline__ void load(const S *__restrict__ f, long long SW, long long n)
    {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) v[i] = (reinterpret_cast<const Half2 *>(f) + (size_t)i * (size_t)SW)[(unsigned)n];
    }
    __device__ __forceinline__ void get(C (&g)[K][L::Q]) const
    {
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            g[0][i] = (C)v[i].x;
            g[1][i] = (C)v[i].y;
        }
    }
};

// Population i of every colour of g stored into slot j of node t.
template <class L, int K, class S, class C, bool NT>
__device__ __forceinline__ void store_pop(S *__restrict__ dst, size_t SW, unsigned t, int j, int i,
                                          const C (&g)[K][L::Q])
{
    if constexpr (kPairs<K, S>) {
        Half2 v;
        v.x = (S)g[0][i];
        v.y = (S)g[1][i];
        st<NT>(&(reinterpret_cast<Half2 *>(dst) + (size_t)j * SW)[t], v);
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) st<NT>(&(dst + (size_t)(k * L::Q + j) * SW)[t], (S)g[k][i]);
    }
}

// Streaming as a push from node (x, y, z): population i goes to x + c_i
// (periodic wrap), bounces back into the opposite direction at the same node
// when x + c_i is behind a wall, and leaves when it is behind an outflow face
// only (the outflow completion supplies the entering populations afterwards).
// NTA: store the populations with c_x = 0 (whose targets keep the row's cache
// line alignment) with the non-temporal hint.
template <class L, int K, class S, class C, bool NTA = false>
__device__ __forceinline__ void push_store_general(const KParams &P, S *__restrict__ dst, int x, int y, int z,
                                                   long long n, const C (&g)[K][L::Q])
{
    const size_t SW = (size_t)P.S;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        int kind = 0;
        const int tx = push_coord(x + L::cx[i], P.nx, P.bc[0], kind);
        const int ty = push_coord(y + L::cy[i], P.ny, P.bc[1], kind);
        const int tz = push_coord(z + L::cz[i], P.nz, P.bc[2], kind);
        const int o = i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1);
        if (kind & 1) {
            store_pop<L, K, S, C, false>(dst, SW, (unsigned)n, o, i, g);
        } else if (kind == 0) {
            const unsigned t = (unsigned)tx + (unsigned)P.nx * ((unsigned)ty + (unsigned)P.ny * (unsigned)tz);
            if (NTA && L::cx[i] == 0) store_pop<L, K, S, C, true>(dst, SW, t, i, i, g);
            else store_pop<L, K, S, C, false>(dst, SW, t, i, i, g);
        }
    }
}

// All-periodic push: the target of direction i is n + c_i . (1, nx, nx ny)
// with a wrap correction on the faces, selected at compile time per i.
template <class L, int K, class S, class C, bool NTA = false>
__device__ __forceinline__ void push_store_periodic(const KParams &P, S *__restrict__ dst, int x, int y, int z,
                                                    long long n, const C (&g)[K][L::Q])
{
    const size_t N = (size_t)P.N, SW = (size_t)P.S;
    const int nx = P.nx, sxy = P.nx * P.ny;
    const int dxp = x == P.nx - 1 ? 1 - nx : 1, dxm = x == 0 ? nx - 1 : -1;
    const int dyp = y == P.ny - 1 ? nx - sxy : nx, dym = y == 0 ? sxy - nx : -nx;
    const int dzp = z == P.nz - 1 ? sxy - (int)N : sxy, dzm = z == 0 ? (int)N - sxy : -sxy;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        int d = 0;
        if (L::cx[i]) d += L::cx[i] > 0 ? dxp : dxm;
        if (L::cy[i]) d += L::cy[i] > 0 ? dyp : dym;
        if (L::cz[i]) d += L::cz[i] > 0 ? dzp : dzm;
        const unsigned t = (unsigned)((int)n + d);
        if (NTA && L::cx[i] == 0) store_pop<L, K, S, C, true>(dst, SW, t, i, i, g);
        else store_pop<L, K, S, C, false>(dst, SW, t, i, i, g);
    }
}

template <class L, int K, class S, class C>
__device__ __forceinline__ void push_store(const KParams &P, S *__restrict__ dst, int x, int y, int z,
                                           long long n, const C (&g)[K][L::Q])
{
    if (P.bc[0] == 0 && P.bc[1] == 0 && P.bc[2] == 0) push_store_periodic<L, K>(P, dst, x, y, z, n, g);
    else push_store_general<L, K>(P, dst, x, y, z, n, g);
}

// ---------------------------------------------------------------------------
// Density-field pass: per node the stencil inputs of the next collision.
//   CG: drho_R, drho_B, rho^N;  SC_MP: psi(rho);  SC_MC: drho_R, drho_B.
// Returns whether the node is diverged (non-finite or rho <= 0).
// ---------------------------------------------------------------------------
template <class L, int PR, int MODEL>
__device__ __forceinline__ bool density_body(const KParams &P, const typename Prec<PR>::S *__restrict__ f,
                                             typename Prec<PR>::F *__restrict__ field, long long n)
{
    using C = typename Prec<PR>::C;
    using M = typename Prec<PR>::M;
    using FT = typename Prec<PR>::F;
    constexpr int K = NComp<MODEL>::n;
    C g[K][L::Q];
    load_node<L, K>(f, P.S, n, g);
    M dr[2], j[3];
    node_moments<L, K>(g, dr, j);
    const HP<C, M> H = make_hp<C, M>(P);
    const M r = H.rho0[0] + dr[0] + (K == 2 ? H.rho0[1] + dr[1] : M(0));
    if constexpr (MODEL == CG) {
        field[n] = (FT)dr[0];
        field[P.N + n] = (FT)dr[1];
        field[2 * P.N + n] = (FT)colour_field(H, dr[0], dr[1]);
    } else if constexpr (MODEL == SC_MP) {
        field[n] = (FT)pseudo_potential(H, H.rho0[0] + dr[0]);
    } else {
        field[n] = (FT)dr[0];
        field[P.N + n] = (FT)dr[1];
        if (P.multirange) {
            field[2 * P.N + n] = (FT)pseudo_potential(H, H.rho0[0] + dr[0]);
            field[3 * P.N + n] = (FT)pseudo_potential(H, H.rho0[1] + dr[1]);
        }
    }
    return node_bad(r, j[0] + j[1] + j[2]);
}

// Multirange forces of the two-component Shan-Chen model added to FR, FB
// (Eqs. doublebeltattractiveforce, doublebeltrepulsionforce):
//   F^a_s = -G^a_s psi_s(x) sum_{belt 1} w_i psi_s(x + c_i) c_i,
//   F^r_s = -G^r_s psi_s(x) sum_{belts 1, 2} p_i psi_s(x + c_i) c_i,
// from the psi fields of the density pass (field + 2N red, + 3N blue), the
// sums taken over the pairs (c, -c) of the belt table in table order.  The
// neighbourhood reaches two nodes along each axis, so the wrapped (periodic)
// or clamped coordinates of x-2..x+2, y-2..y+2, z-2..z+2 are formed once per
// node and each neighbour's index is two additions.  The table is known at
// compile time, so a pair adds only to the components where c is non-zero,
// and to the attraction sums only on belt 1 (w = 0 beyond it).  Only the
// kernels of multirange simulations carry it (the extended-force
// instantiation of the two-component model).

template <int B, class T, class FT>
__device__ __forceinline__ void belt_pair(const FT *__restrict__ psR, const FT *__restrict__ psB, const int (&ox)[5],
                                          const int (&oy)[5], const int (&oz)[5], T (&aR)[3], T (&aB)[3],
                                          T (&rR)[3], T (&rB)[3])
{
    constexpr int cx = Belts::tab.c[B][0], cy = Belts::tab.c[B][1], cz = Belts::tab.c[B][2];
    static_assert(cx >= -2 && cx <= 2 && cy >= -2 && cy <= 2 && cz >= -2 && cz <= 2, "two-node reach");
    constexpr bool belt1 = Belts::tab.w[B] != 0.0;
    const unsigned mp = (unsigned)(ox[2 + cx] + oy[2 + cy] + oz[2 + cz]);
    const unsigned mm = (unsigned)(ox[2 - cx] + oy[2 - cy] + oz[2 - cz]);
    const T dR = (T)psR[mp] - (T)psR[mm];
    const T dB = (T)psB[mp] - (T)psB[mm];
    const T qR = T(Belts::tab.p[B]) * dR, qB = T(Belts::tab.p[B]) * dB;
    const T wR = belt1 ? T(Belts::tab.w[B]) * dR : T(0), wB = belt1 ? T(Belts::tab.w[B]) * dB : T(0);
    auto add = [&](int d, T c) {
        rR[d] += qR * c;
        rB[d] += qB * c;
        if constexpr (belt1) {
            aR[d] += wR * c;
            aB[d] += wB * c;
        }
    };
    if constexpr (cx != 0) add(0, T(cx));
    if constexpr (cy != 0) add(1, T(cy));
    if constexpr (cz != 0) add(2, T(cz));
}

template <class T, class FT, int... B>
__device__ __forceinline__ void belt_sums(std::integer_sequence<int, B...>, const FT *__restrict__ psR,
                                          const FT *__restrict__ psB, const int (&ox)[5], const int (&oy)[5],
                                          const int (&oz)[5], T (&aR)[3], T (&aB)[3], T (&rR)[3], T (&rB)[3])
{
    (belt_pair<B, T>(psR, psB, ox, oy, oz, aR, aB, rR, rB), ...);
}

// The forces from the belt sums and psi at the node.
template <class T, class FT>
__device__ __forceinline__ void multirange_forces(const KParams &P, const FT *__restrict__ psR,
                                                  const FT *__restrict__ psB, const int (&ox)[5], const int (&oy)[5],
                                                  const int (&oz)[5], T (&FR)[3], T (&FB)[3])
{
    T aR[3] = {T(0), T(0), T(0)}, aB[3] = {T(0), T(0), T(0)};
    T rR[3] = {T(0), T(0), T(0)}, rB[3] = {T(0), T(0), T(0)};
    belt_sums<T>(std::make_integer_sequence<int, Belts::n>(), psR, psB, ox, oy, oz, aR, aB, rR, rB);
    const unsigned c = (unsigned)(ox[2] + oy[2] + oz[2]);
    const T pR = (T)psR[c], pB = (T)psB[c];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        FR[d] += -(T)P.Ga[0] * pR * aR[d] - (T)P.Gr[0] * pR * rR[d];
        FB[d] += -(T)P.Ga[1] * pB * aB[d] - (T)P.Gr[1] * pB * rB[d];
    }
}

// psi read from the field in global memory, any thread layout.
template <class T, class FT>
__device__ __forceinline__ void add_multirange(const KParams &P, const FT *__restrict__ field, int x, int y, int z,
                                               T (&FR)[3], T (&FB)[3])
{
    const int nx = P.nx, sxy = P.nx * P.ny;   // N < 2^31: 32-bit offsets
    int ox[5], oy[5], oz[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        ox[k] = stencil_coord(x + k - 2, P.nx, P.bc[0]);
        oy[k] = nx * stencil_coord(y + k - 2, P.ny, P.bc[1]);
        oz[k] = sxy * stencil_coord(z + k - 2, P.nz, P.bc[2]);
    }
    multirange_forces<T>(P, field + 2 * P.N, field + 3 * P.N, ox, oy, oz, FR, FB);
}

// psi read from a block's staged box in LDS (k_collide_mr): the box holds the
// block's kMrTX x kMrTY nodes of one plane and two nodes around them, at the
// wrapped or clamped coordinates the field read would use, so the sums see
// the same values in the same order as add_multirange.
constexpr int kMrTX = 64, kMrTY = 4;
constexpr int kMrBX = kMrTX + 4, kMrBY = kMrTY + 4, kMrBZ = 5, kMrBox = kMrBX * kMrBY * kMrBZ;
template <class FT> struct MrStaged {
    const FT *R, *B;   // psi_R, psi_B: [z][y][x] of kMrBZ x kMrBY x kMrBX, two nodes around the tile
    int tx, ty;        // the node's place in the block's tile
};
struct MrGlobal {};    // no staged box: read the field

template <class T, class FT>
__device__ __forceinline__ void add_multirange(const KParams &P, const MrStaged<FT> &s, T (&FR)[3], T (&FB)[3])
{
    int ox[5], oy[5], oz[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        ox[k] = s.tx + k;
        oy[k] = (s.ty + k) * kMrBX;
        oz[k] = k * (kMrBX * kMrBY);
    }
    multirange_forces<T>(P, s.R, s.B, ox, oy, oz, FR, FB);
}

// Gradient field of rho^N (repulsion variant): 3 sum w rho^N(x + c) c.
template <class L, int PR>
__device__ __forceinline__ void gradN_body(const KParams &P, const typename Prec<PR>::F *__restrict__ field,
                                           typename Prec<PR>::F *__restrict__ gfield, long long n)
{
    using C = typename Prec<PR>::C;
    const int x = (int)(n % P.nx), y = (int)((n / P.nx) % P.ny), z = (int)(n / ((long long)P.nx * P.ny));
    C v[L::Q];
    v[0] = C(0);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) v[i] = (C)field[2 * P.N + stencil_node<L>(P, x, y, z, i)];
    C s[3];
    stencil_sum<L>(v, s);
#pragma unroll
    for (int d = 0; d < 3; ++d) gfield[d * P.N + n] = (typename Prec<PR>::F)(C(3) * s[d]);
}

// Repulsion force at (x, y, z) (Eq. repForce; psi_rep = (1 - |rho^N|)^chi;
// applied outward from the extremum of rho^N, as section 2.3 describes).
template <class L, class C, class FT>
__device__ __forceinline__ void repulsion_force(const KParams &P, const FT *__restrict__ field,
                                                const FT *__restrict__ gfield, int x, int y, int z,
                                                long long n, C (&F)[3])
{
    const long long N = P.N;
    C nv[3] = {(C)gfield[n], (C)gfield[N + n], (C)gfield[2 * N + n]};
    {
        const C gn = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
        const C s = gn > (C)P.g_min ? C(1) / gn : C(0);
        nv[0] *= s; nv[1] *= s; nv[2] *= s;
    }
    C acc[3] = {C(0), C(0), C(0)};
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        const long long m = stencil_node<L>(P, x, y, z, i);
        C np[3] = {(C)gfield[m], (C)gfield[N + m], (C)gfield[2 * N + m]};
        const C gp = sqrt(np[0] * np[0] + np[1] * np[1] + np[2] * np[2]);
        const C s = gp > (C)P.g_min ? C(1) / gp : C(0);
        np[0] *= s; np[1] *= s; np[2] *= s;
        const C nc = cdot<L>(i, nv), npc = cdot<L>(i, np);
        if (-(nc * npc) > C(0)) {
            const C il = (C)L::inv_len[L::grp[i]];
#pragma unroll
            for (int d = 0; d < 3; ++d) acc[d] += (nc * nv[d] + npc * np[d]) * il;
        }
    }
    // outward, away from the extremum of rho^N between the interfaces: minus
    // the sum above, which points toward it
    const C rn = (C)field[2 * N + n];
    const C psi = pow(C(1) - fabs(rn), (C)P.chi);
#pragma unroll
    for (int d = 0; d < 3; ++d) F[d] = -(C)P.Pi * psi * acc[d];
}

// ---------------------------------------------------------------------------
// Collide + push-stream of one node, reading stencil inputs from the field.
// REP: with the model's extended force (CG repulsion, SC_MC multirange).
// ---------------------------------------------------------------------------
// MR: where the multirange forces read psi (MrGlobal: the field; MrStaged: a
// box in LDS).
template <class L, int PR, int MODEL, bool REP, class MR = MrGlobal>
__device__ __forceinline__ void collide_body(const KParams &P, const typename Prec<PR>::S *__restrict__ src,
                                             typename Prec<PR>::S *__restrict__ dst,
                                             const typename Prec<PR>::F *__restrict__ field,
                                             const typename Prec<PR>::F *__restrict__ gfield, long long n,
                                             const MR &mr = MR{})
{
    using C = typename Prec<PR>::C;
    using M = typename Prec<PR>::M;
    constexpr int K = NComp<MODEL>::n;
    const long long N = P.N;
    const int x = (int)(n % P.nx), y = (int)((n / P.nx) % P.ny), z = (int)(n / ((long long)P.nx * P.ny));
    const HP<C, M> H = make_hp<C, M>(P);
    C g[K][L::Q];
    load_node<L, K>(src, P.S, n, g);
    M dr[2], j[3];
    node_moments<L, K>(g, dr, j);
    long long nb[L::Q];
#pragma unroll
    for (int i = 1; i < L::Q; ++i) nb[i] = stencil_node<L>(P, x, y, z, i);
    if constexpr (MODEL == CG) {
        C vR[L::Q], vB[L::Q], vN[L::Q];
        vR[0] = vB[0] = vN[0] = C(0);
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            vR[i] = (C)field[nb[i]];
            vB[i] = (C)field[N + nb[i]];
            vN[i] = (C)field[2 * N + nb[i]];
        }
        C gR[3], gB[3], gN[3];
        stencil_sum<L>(vR, gR);
        stencil_sum<L>(vB, gB);
        stencil_sum<L>(vN, gN);
#pragma unroll
        for (int d = 0; d < 3; ++d) { gR[d] *= C(3); gB[d] *= C(3); gN[d] *= C(3); }
        C F[3] = {C(0), C(0), C(0)};
        if constexpr (REP) repulsion_force<L>(P, field, gfield, x, y, z, n, F);
        cg_collide<L, C, M, REP, kConsShared<PR>>(H, g, dr, j, gR, gB, gN, F);
    } else if constexpr (MODEL == SC_MP) {
        C v[L::Q];
        v[0] = C(0);
#pragma unroll
        for (int i = 1; i < L::Q; ++i) v[i] = (C)field[nb[i]];
        C s[3];
        stencil_sum<L>(v, s);
        const C psi = (C)field[n];
        const M rho = H.rho0[0] + dr[0];
        const M irho = rcp(rho);
        C F[3], u[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            F[d] = -H.G * psi * s[d];
            u[d] = (C)((j[d] + M(0.5) * (M)F[d]) * irho);
        }
        sc_collide_component<L, C, M>(g[0], H.om[0], dr[0], rho, u, F, H.rho0[0], H.corrM[0], H.shiftM[0]);
    } else {
        C vR[L::Q], vB[L::Q];
        vR[0] = vB[0] = C(0);
#pragma unroll
        for (int i = 1; i < L::Q; ++i) {
            vR[i] = (C)field[nb[i]];
            vB[i] = (C)field[N + nb[i]];
        }
        C sR[3], sB[3];
        stencil_sum<L>(vR, sR);
        stencil_sum<L>(vB, sB);
        const M rR = H.rho0[0] + dr[0], rB = H.rho0[1] + dr[1];
        const M ir = rcp(rR + rB);
        C FR[3], FB[3], u[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            FR[d] = -H.xpref * (C)rR * sB[d];
            FB[d] = -H.xpref * (C)rB * sR[d];
        }
        if constexpr (REP) {   // extended force: multirange
            if constexpr (std::is_same_v<MR, MrGlobal>) add_multirange<C>(P, field, x, y, z, FR, FB);
            else add_multirange<C>(P, mr, FR, FB);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) u[d] = (C)((j[d] + M(0.5) * ((M)FR[d] + (M)FB[d])) * ir);
        sc_collide_component<L, C, M>(g[0], H.om[0], dr[0], rR, u, FR, H.rho0[0], H.corrM[0], H.shiftM[0]);
        sc_collide_component<L, C, M>(g[1], H.om[1], dr[1], rB, u, FB, H.rho0[1], H.corrM[1], H.shiftM[1]);
    }
    push_store<L, K>(P, dst, x, y, z, n, g);
}

// Outflow completion for one face node: populations that would come from
// outside through outflow faces only are copied from the node one step
// inward (zero normal gradient).  Face nodes are enumerated per axis.
template <class L, int K, class S>
__device__ __forceinline__ void outflow_body(const KParams &P, S *__restrict__ dst, int x, int y, int z)
{
    const long long SW = P.S;
    const long long n = (long long)x + (long long)P.nx * ((long long)y + (long long)P.ny * z);
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        int kind = 0;
        const int sx = push_coord(x - L::cx[i], P.nx, P.bc[0], kind);
        const int sy = push_coord(y - L::cy[i], P.ny, P.bc[1], kind);
        const int sz = push_coord(z - L::cz[i], P.nz, P.bc[2], kind);
        (void)sx; (void)sy; (void)sz;
        if (kind != 2) continue;  // inside, periodic, or bounced at a wall
        int ix = x, iy = y, iz = z;
        if (P.bc[0] == 2 && (x - L::cx[i] < 0 || x - L::cx[i] >= P.nx)) ix += x == 0 ? 1 : -1;
        if (P.bc[1] == 2 && (y - L::cy[i] < 0 || y - L::cy[i] >= P.ny)) iy += y == 0 ? 1 : -1;
        if (P.bc[2] == 2 && (z - L::cz[i] < 0 || z - L::cz[i] >= P.nz)) iz += z == 0 ? 1 : -1;
        const long long m = (long long)ix + (long long)P.nx * ((long long)iy + (long long)P.ny * iz);
#pragma unroll
        for (int k = 0; k < K; ++k) dst[sidx<L, K, S>(k, i, SW, n)] = dst[sidx<L, K, S>(k, i, SW, m)];
    }
}

// Face-node enumeration: idx in [0, count) over the outflow faces of all axes.
__device__ __forceinline__ bool outflow_face_node(const KParams &P, long long idx, int &x, int &y, int &z)
{
    const long long fx = (long long)P.ny * P.nz, fy = (long long)P.nx * P.nz, fz = (long long)P.nx * P.ny;
    if (P.bc[0] == 2) {
        if (idx < 2 * fx) {
            x = idx < fx ? 0 : P.nx - 1;
            const long long r = idx % fx;
            y = (int)(r % P.ny); z = (int)(r / P.ny);
            return true;
        }
        idx -= 2 * fx;
    }
    if (P.bc[1] == 2) {
        if (idx < 2 * fy) {
            y = idx < fy ? 0 : P.ny - 1;
            const long long r = idx % fy;
            x = (int)(r % P.nx); z = (int)(r / P.nx);
            return true;
        }
        idx -= 2 * fy;
    }
    if (P.bc[2] == 2) {
        if (idx < 2 * fz) {
            z = idx < fz ? 0 : P.nz - 1;
            const long long r = idx % fz;
            x = (int)(r % P.nx); y = (int)(r / P.nx);
            return true;
        }
    }
    return false;
}

// ---------------------------------------------------------------------------
// Initialisation to the equilibrium of given FP64 fields.
// ---------------------------------------------------------------------------
template <class L, int PR, int MODEL>
__device__ __forceinline__ void init_body(const KParams &P, const double *__restrict__ rhoR,
                                          const double *__restrict__ rhoB, const double *__restrict__ uin,
                                          typename Prec<PR>::S *__restrict__ f, long long n)
{
    using S = typename Prec<PR>::S;
    const long long N = P.N;
    const int x = (int)(n % P.nx), y = (int)((n / P.nx) % P.ny), z = (int)(n / ((long long)P.nx * P.ny));
    double u[3] = {0.0, 0.0, 0.0};
    if (uin) { u[0] = uin[n]; u[1] = uin[N + n]; u[2] = uin[2 * N + n]; }
    if constexpr (MODEL == CG) {
        double vR[L::Q], vB[L::Q];
        vR[0] = vB[0] = 0.0;
        for (int i = 1; i < L::Q; ++i) {
            const long long m = stencil_node<L>(P, x, y, z, i);
            vR[i] = rhoR[m];
            vB[i] = rhoB[m];
        }
        double gR[3], gB[3];
        stencil_sum<L>(vR, gR);
        stencil_sum<L>(vB, gB);
        for (int d = 0; d < 3; ++d) { gR[d] *= 3.0; gB[d] *= 3.0; }
        const double rR = rhoR[n], rB = rhoB[n], r = rR + rB;
        const double nub = 1.0 / ((rR / r) * P.inv_nu[0] + (rB / r) * P.inv_nu[1]);
        for (int i = 0; i < L::Q; ++i) {
            f[sidx<L, 2, S>(0, i, P.S, n)] = (S)cg_eq_dev<L>(P, 0, i, rR, u, gR, nub);
            f[sidx<L, 2, S>(1, i, P.S, n)] = (S)cg_eq_dev<L>(P, 1, i, rB, u, gB, nub);
        }
    } else if constexpr (MODEL == SC_MP) {
        for (int i = 0; i < L::Q; ++i) f[sidx<L, 1, S>(0, i, P.S, n)] = (S)sc_eq_dev<L>(P, 0, i, rhoR[n], u);
    } else {
        for (int i = 0; i < L::Q; ++i) {
            f[sidx<L, 2, S>(0, i, P.S, n)] = (S)sc_eq_dev<L>(P, 0, i, rhoR[n], u);
            f[sidx<L, 2, S>(1, i, P.S, n)] = (S)sc_eq_dev<L>(P, 1, i, rhoB[n], u);
        }
    }
}

// ---------------------------------------------------------------------------
// Per-node moments in FP64 (rho_R, rho_B, fluid velocity u as documented in
// the C header) and the node's observable contributions.
// ---------------------------------------------------------------------------
template <class L, int PR, int MODEL>
__device__ __forceinline__ bool node_state64(const KParams &P, const typename Prec<PR>::S *__restrict__ f,
                                             const typename Prec<PR>::F *__restrict__ field, long long n,
                                             double &rR, double &rB, double (&u)[3], double (&j)[3])
{
    constexpr int K = NComp<MODEL>::n;
    const long long N = P.N;
    double g[K][L::Q];
    load_node<L, K>(f, P.S, n, g);
    double dr[2];
    node_moments<L, K>(g, dr, j);
    rR = P.rho0[0] + dr[0];
    rB = K == 2 ? P.rho0[1] + dr[1] : 0.0;
    const double r = rR + rB;
    double F[3] = {0.0, 0.0, 0.0};
    if constexpr (MODEL != CG) {
        const int x = (int)(n % P.nx), y = (int)((n / P.nx) % P.ny), z = (int)(n / ((long long)P.nx * P.ny));
        if constexpr (MODEL == SC_MP) {
            double v[L::Q], s[3];
            v[0] = 0.0;
            for (int i = 1; i < L::Q; ++i) v[i] = (double)field[stencil_node<L>(P, x, y, z, i)];
            stencil_sum<L>(v, s);
            for (int d = 0; d < 3; ++d) F[d] = -P.G * (double)field[n] * s[d];
        } else {
            double vR[L::Q], vB[L::Q], sR[3], sB[3];
            vR[0] = vB[0] = 0.0;
            for (int i = 1; i < L::Q; ++i) {
                const long long m = stencil_node<L>(P, x, y, z, i);
                vR[i] = (double)field[m];
                vB[i] = (double)field[N + m];
            }
            stencil_sum<L>(vR, sR);
            stencil_sum<L>(vB, sB);
            for (int d = 0; d < 3; ++d) F[d] = -P.xpref * (rR * sB[d] + rB * sR[d]);
            if (P.multirange) {
                double FR[3] = {0.0, 0.0, 0.0}, FB[3] = {0.0, 0.0, 0.0};
                add_multirange<double>(P, field, x, y, z, FR, FB);
                for (int d = 0; d < 3; ++d) F[d] += FR[d] + FB[d];
            }
        }
    }
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * F[d]) / r;
    return node_bad(r, j[0] + j[1] + j[2]);
}

template <class L, int PR, int MODEL>
__device__ __forceinline__ void obs_body(const KParams &P, const typename Prec<PR>::S *__restrict__ f,
                                         const typename Prec<PR>::F *__restrict__ field, long long n,
                                         const EpsTable &eps, double (&acc)[kNAcc])
{
    double rR, rB, u[3], j[3];
    const bool bad = node_state64<L, PR, MODEL>(P, f, field, n, rR, rB, u, j);
    if (bad) {
        acc[8] = 1.0;
        return;
    }
    const double r = rR + rB;
    acc[0] += rR;
    acc[1] += rB;
    acc[2] += j[0];
    acc[3] += j[1];
    acc[4] += j[2];
    const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    acc[5] += 0.5 * r * u2;
    acc[6] = fmax(acc[6], sqrt(u2));
    if constexpr (MODEL == SC_MP) {
        if (r >= P.sc_mid) { acc[7] += 1.0; acc[9] += r; acc[10] += 1.0; }
        else { acc[11] += r; acc[12] += 1.0; }
    } else {
        const double rN = (rR - rB) / r;
        acc[7] += 0.5 * (1.0 + rN);
#pragma unroll
        for (int m = 0; m < 10; ++m) {
            if (rN >= eps.e[m]) { acc[9 + 4 * m] += rR; acc[10 + 4 * m] += 1.0; }
            if (rN <= -eps.e[m]) { acc[11 + 4 * m] += rB; acc[12 + 4 * m] += 1.0; }
        }
    }
}

// ---------------------------------------------------------------------------
// Wavefront / block reduction of the accumulators (fixed order).
// ---------------------------------------------------------------------------
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

__device__ __forceinline__ void block_reduce_store(double (&acc)[kNAcc], double *__restrict__ out)
{
    __shared__ double part[kBlock / 64][kNAcc];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < kNAcc; ++a) {
        const double v = (a == 6 || a == 8) ? wave_max(acc[a]) : wave_sum(acc[a]);
        if (lane == 0) part[wv][a] = v;
    }
    __syncthreads();
    if (threadIdx.x < kNAcc) {
        const int a = threadIdx.x;
        double v = part[0][a];
        for (int w = 1; w < kBlock / 64; ++w) v = (a == 6 || a == 8) ? fmax(v, part[w][a]) : v + part[w][a];
        out[a] = v;
    }
}

}  // namespace mclbm
