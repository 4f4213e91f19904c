// node.hpp -- per-node arithmetic of one time step, shared by every kernel
// (two-pass, fused z-marching, batched) so that all of them produce the same
// bits for the same node inputs.
//
// Populations are carried as deviations g_i^k = f_i^k - rho_k^0 phi_i^k from
// the rest equilibrium of the component's initial bulk density (phi of
// Eq. phi for the colour-gradient model, w_i for Shan-Chen), in every
// precision.  Densities are carried as deviations too (drho_k = sum_i g_i^k,
// since sum_i phi_i = 1), which keeps gradients and sums of small numbers
// accurate in FP32.
#pragma once

#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace mclbm {

enum Model { CG = 0, SC_MP = 1, SC_MC = 2 };

// Precision paths: storage type S, arithmetic type C, type M of the moment
// sums / recolouring / blue (light-phase) equilibrium, stencil field type F.
template <int P> struct Prec;
template <> struct Prec<0> { using S = double;   using C = double; using M = double; using F = double; };
template <> struct Prec<1> { using S = float;    using C = float;  using M = float;  using F = float; };
template <> struct Prec<2> { using S = float;    using C = float;  using M = double; using F = float; };
template <> struct Prec<3> { using S = _Float16; using C = float;  using M = float;  using F = float; };
// precisions whose colour-gradient collision can keep each colour's node mass
// to one rounding (mclbm_params.conserve_mass), and the mode of the kernels
// shared by simulations that do and do not ask for it
template <int PR> constexpr bool kConserveRest = PR == 1 || PR == 2;
template <int PR> constexpr int kConsShared = kConserveRest<PR> ? 1 : 0;

// Parameters of one simulation as the kernels see them (host-derived).
struct KParams {
    int nx, ny, nz;
    int bc[3];
    long long N;         // nodes
    long long S;         // storage words from one population array to the next (>= N)
    int enhanced;
    int has_outflow;
    int conserve;        // CG, FP32 / mixed storage: keep each colour's node mass to one rounding
    double rho0[2];      // reference densities of the deviation storage
    double phi[2][3];    // CG: phi_i^k per group; SC: w per group
    double shift[2][3];  // storage reference per group; sum_i shift = rho0[k] exactly
    double corr[2][3];   // rho0[k] * phi[k][group] - shift[k][group] (zero unless quantised)
    double inv_nu[2];    // CG: 1/nu_k, nu_k = (tau_k - 1/2)/3
    double halfA;        // CG: A/2
    double beta;         // CG recolouring strength
    double g_min;        // CG: normal threshold
    double om[2];        // SC: 1/tau_s
    double G;            // SC_MP coupling
    double psi_rho0;     // SC_MP reference density
    double xpref;        // SC_MC: G_RB / rho0_X^2
    double Pi, chi;      // CG repulsion
    double sc_mid;       // SC_MP: (rho0_R + rho0_B)/2, the inside/outside threshold
    int multirange;      // SC_MC: multirange forces on (psi_R, psi_B follow the densities in the field)
    double Ga[2], Gr[2]; // SC_MC multirange attraction / repulsion couplings per species
};

// Arithmetic parameters of the collision in the kernel's own types (C for
// the bulk arithmetic, M for sums / recolouring / light phase), built once per
// thread from KParams so that the hot loop holds no FP64 constants.
template <class C, class M>
struct HP {
    M rho0[2];
    M phiM[2][3], corrM[2][3], shiftM[2][3];
    M inv_nu[2];
    M beta;
    C phiC[3], corrC[3], shiftC[3];  // red, in C
    C halfA, g_min;
    C om[2];
    C G, psi_rho0, xpref, Pi, chi;
    C Ga[2], Gr[2];
    int enhanced;
    int conserve;
};

template <class C, class M>
__device__ __forceinline__ HP<C, M> make_hp(const KParams &P)
{
    HP<C, M> H;
    for (int k = 0; k < 2; ++k) {
        H.rho0[k] = (M)P.rho0[k];
        H.inv_nu[k] = (M)P.inv_nu[k];
        H.om[k] = (C)P.om[k];
        H.Ga[k] = (C)P.Ga[k];
        H.Gr[k] = (C)P.Gr[k];
        for (int q = 0; q < 3; ++q) {
            H.phiM[k][q] = (M)P.phi[k][q];
            H.corrM[k][q] = (M)P.corr[k][q];
            H.shiftM[k][q] = (M)P.shift[k][q];
        }
    }
    for (int q = 0; q < 3; ++q) {
        H.phiC[q] = (C)P.phi[0][q];
        H.corrC[q] = (C)P.corr[0][q];
        H.shiftC[q] = (C)P.shift[0][q];
    }
    H.beta = (M)P.beta;
    H.halfA = (C)P.halfA;
    H.g_min = (C)P.g_min;
    H.G = (C)P.G;
    H.psi_rho0 = (C)P.psi_rho0;
    H.xpref = (C)P.xpref;
    H.Pi = (C)P.Pi;
    H.chi = (C)P.chi;
    H.enhanced = P.enhanced;
    H.conserve = P.conserve;
    return H;
}

// Reciprocal: the hardware one (1 ulp) in FP32, exact division in FP64.
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }

// Number of stencil-field arrays per model.
template <int MODEL> struct NField { static constexpr int n = MODEL == CG ? 3 : (MODEL == SC_MP ? 1 : 2); };
template <int MODEL> struct NComp { static constexpr int n = MODEL == SC_MP ? 1 : 2; };

// ---------------------------------------------------------------------------
// Geometry: stencil neighbours (wrap periodic, clamp otherwise) and push
// targets of streaming (wrap periodic; wall -> bounce back; outflow -> leave).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int stencil_coord(int q, int n, int bc)
{
    if (q < 0) return bc == 0 ? q + n : 0;
    if (q >= n) return bc == 0 ? q - n : n - 1;
    return q;
}

// kind: 0 = inside/wrapped, 1 = through a wall, 2 = through an outflow face
__device__ __forceinline__ int push_coord(int q, int n, int bc, int &kind)
{
    if (q >= 0 && q < n) return q;
    if (bc == 0) return q < 0 ? q + n : q - n;
    kind |= bc == 1 ? 1 : 2;
    return q;
}

template <class L>
__device__ __forceinline__ long long stencil_node(const KParams &P, int x, int y, int z, int i)
{
    const int qx = stencil_coord(x + L::cx[i], P.nx, P.bc[0]);
    const int qy = stencil_coord(y + L::cy[i], P.ny, P.bc[1]);
    const int qz = stencil_coord(z + L::cz[i], P.nz, P.bc[2]);
    return (long long)qx + (long long)P.nx * ((long long)qy + (long long)P.ny * qz);
}

// Node read at x + (cx, cy, cz) for offsets up to two nodes (the multirange
// neighbourhood): wrap periodic axes, clamp otherwise.
__device__ __forceinline__ long long stencil_at(const KParams &P, int x, int y, int z, int cx, int cy, int cz)
{
    const int qx = stencil_coord(x + cx, P.nx, P.bc[0]);
    const int qy = stencil_coord(y + cy, P.ny, P.bc[1]);
    const int qz = stencil_coord(z + cz, P.nz, P.bc[2]);
    return (long long)qx + (long long)P.nx * ((long long)qy + (long long)P.ny * qz);
}

// ---------------------------------------------------------------------------
// Moments of one node (ascending i, red then blue).
// ---------------------------------------------------------------------------
template <class L, int K, class C, class M>
__device__ __forceinline__ void node_moments(const C (&g)[K][L::Q], M (&dr)[2], M (&j)[3])
{
    dr[0] = dr[1] = M(0);
    j[0] = j[1] = j[2] = M(0);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int i = 0; i < L::Q; ++i) {
            const M v = (M)g[k][i];
            dr[k] += v;
            if (L::cx[i]) j[0] += L::cx[i] > 0 ? v : -v;
            if (L::cy[i]) j[1] += L::cy[i] > 0 ? v : -v;
            if (L::cz[i]) j[2] += L::cz[i] > 0 ? v : -v;
        }
}

// Colour field rho^N = (rho_R - rho_B) / (rho_R + rho_B).
template <class C, class M>
__device__ __forceinline__ M colour_field(const HP<C, M> &H, M drR, M drB)
{
    return ((H.rho0[0] - H.rho0[1]) + (drR - drB)) / ((H.rho0[0] + H.rho0[1]) + (drR + drB));
}

template <class C, class M>
__device__ __forceinline__ M pseudo_potential(const HP<C, M> &H, M rho)
{
    return (M)H.psi_rho0 * (M(1) - exp(-rho / (M)H.psi_rho0));
}

__device__ __forceinline__ bool node_bad(double r, double jsum)
{
    return !(r > 0.0) || !__builtin_isfinite(r) || !__builtin_isfinite(jsum);
}
__device__ __forceinline__ bool node_bad(float r, float jsum)
{
    return !(r > 0.0f) || !__builtin_isfinite(r) || !__builtin_isfinite(jsum);
}

// ---------------------------------------------------------------------------
// Isotropic stencil sum  s = sum_{i != 0} w_i X(x + c_i) c_i  over opposite
// pairs; the gradient is 3 s (c_s^2 = 1/3).  nb[i] holds X(x + c_i).
// ---------------------------------------------------------------------------
template <class L, class T>
__device__ __forceinline__ void stencil_sum(const T (&nb)[L::Q], T (&s)[3])
{
    s[0] = s[1] = s[2] = T(0);
#pragma unroll
    for (int i = 1; i < L::Q; i += 2) {
        const T d = (T)L::w[L::grp[i]] * (nb[i] - nb[i + 1]);
        if (L::cx[i]) s[0] += L::cx[i] > 0 ? d : -d;
        if (L::cy[i]) s[1] += L::cy[i] > 0 ? d : -d;
        if (L::cz[i]) s[2] += L::cz[i] > 0 ? d : -d;
    }
}

template <class L, class T>
__device__ __forceinline__ T cdot(int i, const T (&v)[3])
{
    T r = T(0);
    if (L::cx[i]) r += L::cx[i] > 0 ? v[0] : -v[0];
    if (L::cy[i]) r += L::cy[i] > 0 ? v[1] : -v[1];
    if (L::cz[i]) r += L::cz[i] > 0 ? v[2] : -v[2];
    return r;
}

// ---------------------------------------------------------------------------
// Rest-equilibrium part of the deviation equilibrium of one component and
// group, rho phi - shift, written so that it is exact at both ends: as
// drho phi + corr where the component is present (drho small), and as
// rho phi - shift where it is absent (rho = 0 gives -shift exactly, so an
// absent component stays exactly absent in FP32 storage).
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T rest_dev(bool present, T dr, T rho, T phi, T corr, T shift)
{
    return present ? dr * phi + corr : rho * phi - shift;
}

// ---------------------------------------------------------------------------
// Colour-gradient collision of one node (section 2.2):
//   Omega^(1): BGK towards the enhanced equilibrium (Eq. equiliCG) with
//              omega_eff of the interface viscosity (Eqs. effRelax, interpVisc);
//   Omega^(2): perturbation, each colour (A/2)|g|[w (c.n)^2 - B] (Eq.
//              perturbationOp, scaled so that Eq. sigmaA holds);
//   Omega^(3): recolouring of the total (Eqs. recoloringOpR/B, cosphi) with
//              f^eq|_{u=0} = sum_k rho_k phi_i^k.
// Optional body force F (repulsion variant): u = (j + F/2)/rho and a Guo
// source split by rho_k/rho.  In deviation form
//   geq_k - shift_k = (rho_k phi_k - shift_k) + rho_k w [3cu + 9/2 cu^2 - 3/2 u^2]
//                     + nubar [psi (u.grad rho_k) + 2 xi (c.u)(c.grad rho_k)]
// and the recolouring as an exchange between the colours,
//   f_R,out = (rho_R/rho) (f*_R + f*_B) + t = f*_R + X + t,
//   X = (rho_R/rho) f*_B - (rho_B/rho) f*_R,   f_B,out = f*_B - X - t,
// which is exactly zero where one colour is absent.
// ---------------------------------------------------------------------------
// CONS (FP32 and mixed storage, whose arithmetic type is the storage type):
// each colour's node mass is kept exactly, up to one rounding: the rest
// population is set last to the input populations' sum minus the other
// outputs, both sums in FP64.  Without it the FP32 roundings of the pairs
// +-t_i of the recolouring (and of the other sums) leave a bias of about 1e-7
// of the colour mass per step at interfaces.  kConsNever: not compiled in;
// kConsAsked: when the simulation asks for it (H.conserve; kernels shared by
// simulations either way); kConsAlways: unconditionally (kernels launched
// only for simulations that ask for it).  Off, the arithmetic is the same as
// without this code.
constexpr int kConsNever = 0, kConsAsked = 1, kConsAlways = 2;
template <class L, class C, class M, bool FORCED, int CONS = kConsNever>
__device__ __forceinline__ void cg_collide(const HP<C, M> &H, C (&g)[2][L::Q], const M (&dr)[2],
                                           const M (&j)[3], const C (&gR)[3], const C (&gB)[3],
                                           const C (&gN)[3], const C (&F)[3])
{
    const bool cons = CONS == kConsAlways || (CONS == kConsAsked && H.conserve);
    double din[2] = {0.0, 0.0};
    if constexpr (CONS != kConsNever) {
        if (cons) {
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int i = 0; i < L::Q; ++i) din[k] += (double)g[k][i];
        }
    }
    const M rR = H.rho0[0] + dr[0];
    const M rB = H.rho0[1] + dr[1];
    const M r = rR + rB;
    const M ir = rcp(r);
    C u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = FORCED ? (C)((j[d] + M(0.5) * (M)F[d]) * ir) : (C)(j[d] * ir);
    const C nub = (C)(r * rcp(rR * H.inv_nu[0] + rB * H.inv_nu[1]));
    const C om = C(2) * rcp(C(6) * nub + C(1));
    const C uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const C enh = H.enhanced ? nub : C(0);
    const C ugR = enh * (u[0] * gR[0] + u[1] * gR[1] + u[2] * gR[2]);
    const M ugB = (M)enh * ((M)u[0] * (M)gB[0] + (M)u[1] * (M)gB[1] + (M)u[2] * (M)gB[2]);
    const C gn = sqrt(gN[0] * gN[0] + gN[1] * gN[1] + gN[2] * gN[2]);
    const bool has_n = gn > H.g_min;
    const C pA = has_n ? H.halfA : C(0);
    const C inv_gn = has_n ? rcp(gn) : C(0);
    const M cR = rR * ir, cB = rB * ir;
    const M tco = has_n ? H.beta * cR * cB * (M)inv_gn : M(0);
    const C rRc = (C)rR;
    const bool presR = rR > M(0.5) * H.rho0[0];
    const bool presB = rB > M(0.5) * H.rho0[1];
    C baseR[3];
    M baseB[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        baseR[q] = rest_dev<C>(presR, (C)dr[0], rRc, H.phiC[q], H.corrC[q], H.shiftC[q]);
        baseB[q] = rest_dev<M>(presB, dr[1], rB, H.phiM[1][q], H.corrM[1][q], H.shiftM[1][q]);
    }
    C uF = C(0), gs = C(0);
    if constexpr (FORCED) {
        uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
        gs = C(1) - C(0.5) * om;
    }

    // rest population (c = 0: no odd terms, xi_0 = 0, cos phi_0 = 0)
    {
        const C w0 = (C)L::w[0];
        const C eqR = baseR[0] + rRc * w0 * (C(-1.5) * uu) + (C)L::psi[0] * ugR;
        const M eqB = baseB[0] + rB * (M)w0 * (M(-1.5) * (M)uu) + (M)L::psi[0] * ugB;
        C sR = g[0][0] + om * (eqR - g[0][0]);
        M sB = (M)g[1][0] + (M)om * (eqB - (M)g[1][0]);
        if constexpr (FORCED) {
            const C S = w0 * gs * (C(-3) * uF);
            sR += (C)cR * S;
            sB += cB * (M)S;
        }
        const C pert = pA * (-(C)L::B[0] * gn);
        sR += pert;
        sB += (M)pert;
        const M X = cR * (sB + H.shiftM[1][0]) - cB * ((M)sR + H.shiftM[0][0]);
        g[0][0] = (C)((M)sR + X);
        g[1][0] = (C)(sB - X);
    }
#pragma unroll
    for (int i = 1; i < L::Q; i += 2) {
        const int q = L::grp[i];
        const C w = (C)L::w[q];
        const C cu = cdot<L>(i, u);
        const C cgR = cdot<L>(i, gR);
        const M cgB = (M)cdot<L>(i, gB);
        const C cgn = cdot<L>(i, gN);
        // equilibrium deviations, split into even and odd parts in c
        const C symR = baseR[q] + rRc * w * (C(4.5) * cu * cu - C(1.5) * uu)
                       + (C)L::psi[q] * ugR + C(2 * L::xi[q]) * enh * cu * cgR;
        const C antR = rRc * w * (C(3) * cu);
        const M cuM = (M)cu;
        const M symB = baseB[q] + rB * (M)w * (M(4.5) * cuM * cuM - M(1.5) * (M)uu)
                       + (M)L::psi[q] * ugB + M(2 * L::xi[q]) * (M)enh * cuM * cgB;
        const M antB = rB * (M)w * (M(3) * cuM);
        C sRp = g[0][i] + om * ((symR + antR) - g[0][i]);
        C sRm = g[0][i + 1] + om * ((symR - antR) - g[0][i + 1]);
        M sBp = (M)g[1][i] + (M)om * ((symB + antB) - (M)g[1][i]);
        M sBm = (M)g[1][i + 1] + (M)om * ((symB - antB) - (M)g[1][i + 1]);
        if constexpr (FORCED) {
            const C cF = cdot<L>(i, F);
            const C Se = w * gs * (C(-3) * uF + C(9) * cu * cF);
            const C So = w * gs * (C(3) * cF);
            sRp += (C)cR * (Se + So);
            sRm += (C)cR * (Se - So);
            sBp += cB * (M)(Se + So);
            sBm += cB * (M)(Se - So);
        }
        const C pert = pA * ((C)L::B[q] * -gn + w * cgn * cgn * inv_gn);
        sRp += pert;
        sRm += pert;
        sBp += (M)pert;
        sBm += (M)pert;
        const M E = rR * H.phiM[0][q] + rB * H.phiM[1][q];
        const M t = tco * (M)L::inv_len[q] * (M)cgn * E;
        const M shR = H.shiftM[0][q], shB = H.shiftM[1][q];
        const M Xp = cR * (sBp + shB) - cB * ((M)sRp + shR);
        const M Xm = cR * (sBm + shB) - cB * ((M)sRm + shR);
        g[0][i] = (C)((M)sRp + Xp + t);
        g[1][i] = (C)(sBp - Xp - t);
        g[0][i + 1] = (C)((M)sRm + Xm - t);
        g[1][i + 1] = (C)(sBm - Xm + t);
    }
    if constexpr (CONS != kConsNever) {
        if (cons) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                double out = 0.0;
#pragma unroll
                for (int i = 1; i < L::Q; ++i) out += (double)g[k][i];
                g[k][0] = (C)(din[k] - out);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Shan-Chen BGK + Guo source of one component (Eqs. collisSC, equiliSC,
// source): relaxation rate om, component density rho = rho0 + dr, common
// velocity u, component force F.
// ---------------------------------------------------------------------------
template <class L, class C, class M>
__device__ __forceinline__ void sc_collide_component(C (&g)[L::Q], C om, M dr, M rho,
                                                     const C (&u)[3], const C (&F)[3], M rho0,
                                                     const M (&corr)[3], const M (&shift)[3])
{
    const C uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const C uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    const C gs = C(1) - C(0.5) * om;
    const C drc = (C)dr, rc = (C)rho;
    const bool pres = rho > M(0.5) * (M)rho0;
    C base[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) base[q] = rest_dev<C>(pres, drc, rc, (C)L::w[q], (C)corr[q], (C)shift[q]);
    {
        const C w0 = (C)L::w[0];
        const C eq = base[0] + rc * w0 * (C(-1.5) * uu);
        g[0] = g[0] + om * (eq - g[0]) + w0 * gs * (C(-3) * uF);
    }
#pragma unroll
    for (int i = 1; i < L::Q; i += 2) {
        const C w = (C)L::w[L::grp[i]];
        const C cu = cdot<L>(i, u);
        const C cF = cdot<L>(i, F);
        const C sym = base[L::grp[i]] + rc * w * (C(4.5) * cu * cu - C(1.5) * uu);
        const C ant = rc * w * (C(3) * cu);
        const C Se = w * gs * (C(-3) * uF + C(9) * cu * cF);
        const C So = w * gs * (C(3) * cF);
        g[i] = g[i] + om * ((sym + ant) - g[i]) + (Se + So);
        g[i + 1] = g[i + 1] + om * ((sym - ant) - g[i + 1]) + (Se - So);
    }
}

// ---------------------------------------------------------------------------
// Equilibrium deviations for initialisation (FP64 throughout).
// ---------------------------------------------------------------------------
template <class L>
__device__ __forceinline__ double cg_eq_dev(const KParams &P, int k, int i, double rho_k,
                                            const double (&u)[3], const double (&grad)[3], double nub)
{
    const int q = L::grp[i];
    double cu = 0.0, ug = 0.0, cg = 0.0, uu = 0.0;
    cu = cdot<L>(i, u);
    cg = cdot<L>(i, grad);
    for (int d = 0; d < 3; ++d) {
        ug += u[d] * grad[d];
        uu += u[d] * u[d];
    }
    double v = (rho_k - P.rho0[k]) * P.phi[k][q] + P.corr[k][q]
               + rho_k * L::w[q] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    if (P.enhanced) v += nub * (L::psi[q] * ug + 2.0 * L::xi[q] * cu * cg);
    return v;
}

template <class L>
__device__ __forceinline__ double sc_eq_dev(const KParams &P, int k, int i, double rho,
                                            const double (&u)[3])
{
    const int q = L::grp[i];
    double cu = cdot<L>(i, u), uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return (rho - P.rho0[k]) * L::w[q] + P.corr[k][q] + rho * L::w[q] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

}  // namespace mclbm
