// ops.hpp -- launcher table: one Ops object per (lattice, precision, model,
// repulsion) instantiation, behind a small virtual interface so that the C
// ABI can dispatch on run-time parameters.
#pragma once

#include <hip/hip_runtime.h>

#include "interface.hpp"
#include "launch.hpp"

namespace mclbm {

struct Ops {
    virtual ~Ops() {}
    virtual bool has_fused() const = 0;
    // blocks of the batched one-pass kernel the device holds at once (0: none)
    virtual long long batch_fused_resident() const = 0;
    // one step: src -> dst (the divergence flag reflects src)
    virtual void step(const KParams &P, const void *src, void *dst, void *field, void *gfield,
                      unsigned *flag, bool fused, hipStream_t s) const = 0;
    virtual void density(const KParams &P, const void *f, void *field, unsigned *flag, hipStream_t s) const = 0;
    virtual void init(const KParams &P, const double *rR, const double *rB, const double *u, void *f,
                      hipStream_t s) const = 0;
    virtual void export_f(const KParams &P, const void *f, double *out, hipStream_t s) const = 0;
    virtual void import_f(const KParams &P, const double *in, void *f, hipStream_t s) const = 0;
    virtual void moments(const KParams &P, const void *f, const void *field, double *rR, double *rB,
                         double *u, hipStream_t s) const = 0;
    virtual void obs(const KParams &P, const void *f, const void *field, const EpsTable &e, double *partials,
                     int nblocks, hipStream_t s) const = 0;
    // batched step over a group of descriptors: `blocks` two-pass blocks,
    // `fblocks` one-pass blocks, `oblocks` outflow blocks
    virtual void batch_step(SimDesc *D, int n, long long blocks, long long fblocks, int fused_kinds, long long oblocks,
                            bool any_outflow, hipStream_t s) const = 0;
    // interface observables: phase indicator of a node set, per-block red
    // fraction partial sums over a node set, initial component labels
    virtual void phase_sample(const KParams &P, const void *f, const NodeSet &ns, double *out,
                              hipStream_t s) const = 0;
    virtual void phase_area(const KParams &P, const void *f, const NodeSet &ns, double *partials, int nblocks,
                            hipStream_t s) const = 0;
    virtual void phase_labels(const KParams &P, const void *f, int *labels, hipStream_t s) const = 0;
};

inline unsigned grid_of(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

inline long long outflow_count(const KParams &P)
{
    long long c = 0;
    if (P.bc[0] == 2) c += 2LL * P.ny * P.nz;
    if (P.bc[1] == 2) c += 2LL * P.nx * P.nz;
    if (P.bc[2] == 2) c += 2LL * P.nx * P.ny;
    return c;
}

// REP: the model's extended force, which reaches beyond the one-node halo of
// the one-pass kernels: the repulsion force of the colour-gradient model
// (normals at the neighbours), the multirange forces of the two-component
// Shan-Chen model (two nodes out).  Its simulations step on the two-pass
// kernels.
// Fused one-pass step (fused.hpp) for D3Q19 and D2Q9 without an extended
// force.
template <class L, int PR, int MODEL, bool REP> constexpr bool fused_available()
{
    return (L::Q == 19 || L::Q == 9) && !REP;
}
// Batched one-pass step (fused.hpp): D3Q19.
template <class L, int PR, int MODEL, bool REP> constexpr bool batch_fused_available()
{
    return fused_available<L, PR, MODEL, REP>() && L::Q == 19;
}
template <int PR, int MODEL>
void launch_fused(const KParams &P, const void *src, void *dst, unsigned *flag, hipStream_t s);
template <int PR, int MODEL>
void launch_fused2d(const KParams &P, const void *src, void *dst, unsigned *flag, hipStream_t s);
template <int PR, int MODEL>
void launch_batch_fused(SimDesc *D, int n, long long fblocks, int kinds, hipStream_t s);
template <int PR, int MODEL>
long long batch_fused_resident();

template <class L, int PR, int MODEL, bool REP>
struct OpsT final : Ops {
    using S = typename Prec<PR>::S;
    using FT = typename Prec<PR>::F;

    bool has_fused() const override { return fused_available<L, PR, MODEL, REP>(); }
    long long batch_fused_resident() const override
    {
        if constexpr (batch_fused_available<L, PR, MODEL, REP>()) return mclbm::batch_fused_resident<PR, MODEL>();
        return 0;
    }

    void step(const KParams &P, const void *src, void *dst, void *field, void *gfield, unsigned *flag,
              bool fused, hipStream_t s) const override
    {
        bool done = false;
        if constexpr (fused_available<L, PR, MODEL, REP>()) {
            if (fused) {
                if constexpr (L::Q == 19) launch_fused<PR, MODEL>(P, src, dst, flag, s);
                else launch_fused2d<PR, MODEL>(P, src, dst, flag, s);
                done = true;
            }
        }
        if (!done) {
            hipLaunchKernelGGL((k_density<L, PR, MODEL>), dim3(grid_of(P.N)), dim3(kBlock), 0, s, P,
                               (const S *)src, (FT *)field, flag);
            if constexpr (REP && MODEL == CG)
                hipLaunchKernelGGL((k_gradN<L, PR>), dim3(grid_of(P.N)), dim3(kBlock), 0, s, P,
                                   (const FT *)field, (FT *)gfield);
            if constexpr (REP && MODEL == SC_MC && L::Q == 19)
                hipLaunchKernelGGL((k_collide_mr<PR>), dim3((unsigned)mr_blocks(P)), dim3(kMrTX * kMrTY), 0, s, P,
                                   (const S *)src, (S *)dst, (const FT *)field);
            else
                hipLaunchKernelGGL((k_collide<L, PR, MODEL, REP>), dim3(grid_of(P.N)), dim3(kBlock), 0, s, P,
                                   (const S *)src, (S *)dst, (const FT *)field, (const FT *)gfield);
        }
        if (P.has_outflow) {
            const long long c = outflow_count(P);
            hipLaunchKernelGGL((k_outflow<L, PR, MODEL>), dim3(grid_of(c)), dim3(kBlock), 0, s, P, (S *)dst, c);
        }
    }
    void density(const KParams &P, const void *f, void *field, unsigned *flag, hipStream_t s) const override
    {
        hipLaunchKernelGGL((k_density<L, PR, MODEL>), dim3(grid_of(P.N)), dim3(kBlock), 0, s, P,
                           (const S *)f, (FT *)field, flag);
    }
    void init(const KParams &P, const double *rR, const double *rB, const double *u, void *f,
              hipStream_t s) const override
    {
        hipLaunchKernelGGL((k_init<L, PR, MODEL>), dim3(grid_of(P.N)), dim3(kBlock), 0, s, P, rR, rB, u, (S *)f);
    }
    void export_f(const KParams &P, const void *f, double *out, hipStream_t s) const override
    {
        hipLaunchKernelGGL((k_export<L, PR, MODEL>), dim3(grid_of(P.N)), dim3(kBlock), 0, s, P, (const S *)f, out);
    }
    void import_f(const KParams &P, const double *in, void *f, hipStream_t s) const override
    {
        hipLaunchKernelGGL((k_import<L, PR, MODEL>), dim3(grid_of(P.N)), dim3(kBlock), 0, s, P, in, (S *)f);
    }
    void moments(const KParams &P, const void *f, const void *field, double *rR, double *rB, double *u,
                 hipStream_t s) const override
    {
        hipLaunchKernelGGL((k_moments_out<L, PR, MODEL>), dim3(grid_of(P.N)), dim3(kBlock), 0, s, P,
                           (const S *)f, (const FT *)field, rR, rB, u);
    }
    void obs(const KParams &P, const void *f, const void *field, const EpsTable &e, double *partials,
             int nblocks, hipStream_t s) const override
    {
        hipLaunchKernelGGL((k_obs<L, PR, MODEL>), dim3(nblocks), dim3(kBlock), 0, s, P, (const S *)f,
                           (const FT *)field, e, partials);
    }
    void phase_sample(const KParams &P, const void *f, const NodeSet &ns, double *out,
                      hipStream_t s) const override
    {
        hipLaunchKernelGGL((k_phase_sample<L, PR, MODEL>), dim3(grid_of(ns.count)), dim3(kBlock), 0, s, P,
                           (const S *)f, ns, out);
    }
    void phase_area(const KParams &P, const void *f, const NodeSet &ns, double *partials, int nblocks,
                    hipStream_t s) const override
    {
        hipLaunchKernelGGL((k_phase_area<L, PR, MODEL>), dim3(nblocks), dim3(kBlock), 0, s, P, (const S *)f, ns,
                           partials);
    }
    void phase_labels(const KParams &P, const void *f, int *labels, hipStream_t s) const override
    {
        hipLaunchKernelGGL((k_phase_labels<L, PR, MODEL>), dim3(grid_of(P.N)), dim3(kBlock), 0, s, P,
                           (const S *)f, labels);
    }
    void batch_step(SimDesc *D, int n, long long blocks, long long fblocks, int fused_kinds, long long oblocks,
                    bool any_outflow, hipStream_t s) const override
    {
        if (blocks > 0) {
            hipLaunchKernelGGL((kb_density<L, PR, MODEL>), dim3((unsigned)blocks), dim3(kBlock), 0, s, D, n);
            if constexpr (REP && MODEL == CG)
                hipLaunchKernelGGL((kb_gradN<L, PR>), dim3((unsigned)blocks), dim3(kBlock), 0, s, D, n);
            if constexpr (kb_collide_three_waves<L, PR, MODEL, REP>)
                hipLaunchKernelGGL((kb_collide_w3<L, PR, MODEL, REP>), dim3((unsigned)blocks), dim3(kBlock), 0, s, D, n);
            else
                hipLaunchKernelGGL((kb_collide<L, PR, MODEL, REP>), dim3((unsigned)blocks), dim3(kBlock), 0, s, D, n);
        }
        if constexpr (batch_fused_available<L, PR, MODEL, REP>()) {
            if (fblocks > 0) launch_batch_fused<PR, MODEL>(D, n, fblocks, fused_kinds, s);
        }
        if (any_outflow && oblocks > 0)
            hipLaunchKernelGGL((kb_outflow<L, PR, MODEL>), dim3((unsigned)oblocks), dim3(kBlock), 0, s, D, n);
    }
};

// Returns the launcher for a combination, or nullptr if not provided.
const Ops *get_ops(int lattice, int precision, int model, bool rep);
const Ops *ops_prec0(int lattice, int model, bool rep);
const Ops *ops_prec1(int lattice, int model, bool rep);
const Ops *ops_prec2(int lattice, int model, bool rep);
const Ops *ops_prec3(int lattice, int model, bool rep);

// Definition of ops_prec<P> for one precision (used by inst_p<P>.hip).
template <class L, int PR>
const Ops *ops_for_model(int model, bool rep)
{
    static const OpsT<L, PR, CG, false> cg;
    static const OpsT<L, PR, CG, true> cgr;
    static const OpsT<L, PR, SC_MP, false> mp;
    static const OpsT<L, PR, SC_MC, false> mc;
    if (model == CG) return rep ? (const Ops *)&cgr : (const Ops *)&cg;
    if (model == SC_MP) return &mp;
    if (model == SC_MC) {
        if constexpr (L::Q == 19) {   // the multirange neighbourhood is three-dimensional
            static const OpsT<L, PR, SC_MC, true> mcm;
            if (rep) return &mcm;
        }
        return rep ? nullptr : &mc;
    }
    return nullptr;
}
template <int PR>
const Ops *ops_for_lattice(int lattice, int model, bool rep)
{
    if (lattice == 0) return ops_for_model<D2Q9, PR>(model, rep);
    if (lattice == 1) return ops_for_model<D3Q19, PR>(model, rep);
    return nullptr;
}

}  // namespace mclbm
