// mclbm.hip -- C ABI (include/mclbm.h) of the two-component lattice
// Boltzmann library: parameter validation, state layout on caller memory,
// dispatch to the kernel instantiations, observables, checkpoints and the
// batched stepping used for sweep serving.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "mclbm.h"
#include "fused.hpp"
#include "ops.hpp"

using namespace mclbm;

namespace {

thread_local std::string g_last_error;

mclbm_status fail(mclbm_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define MCLBM_HIP(expr)                                                                          \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return fail(MCLBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int lattice_Q(int lattice) { return lattice == MCLBM_D2Q9 ? 9 : 19; }
int ncomp_of(int model) { return model == MCLBM_SC_MP ? 1 : 2; }
bool multirange_of(const mclbm_params &p)
{
    return p.Ga_R != 0.0 || p.Ga_B != 0.0 || p.Gr_R != 0.0 || p.Gr_B != 0.0;
}

// The kernels with the model's extended force (Ops REP): the colour-gradient
// repulsion, or the two-component Shan-Chen multirange forces.
bool extended_of(const mclbm_params &p)
{
    return (p.model == MCLBM_CG && p.Pi != 0.0) || multirange_of(p);
}

// stencil-field values per node: CG drho_R, drho_B, rho^N; SC_MP psi; SC_MC
// drho_R, drho_B (+ psi_R, psi_B with the multirange forces)
int nfield_of(const mclbm_params &p)
{
    if (p.model == MCLBM_CG) return 3;
    if (p.model == MCLBM_SC_MP) return 1;
    return multirange_of(p) ? 4 : 2;
}
size_t storage_size(int prec) { return prec == MCLBM_FP64 ? 8 : (prec == MCLBM_FP16 ? 2 : 4); }
size_t field_size(int prec) { return prec == MCLBM_FP64 ? 8 : 4; }
size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct Layout {
    size_t fbytes, field_off, gfield_off, total;
};

// Population arrays: the word one array element holds (two-colour FP16
// storage keeps both colours of a population in one 32-bit word), and how
// many arrays a population buffer holds.
size_t pop_word(const mclbm_params &p)
{
    return (p.precision == MCLBM_FP16 && ncomp_of(p.model) == 2) ? 4 : storage_size(p.precision);
}
size_t pop_arrays(const mclbm_params &p)
{
    return (size_t)lattice_Q(p.lattice) * ((p.precision == MCLBM_FP16 && ncomp_of(p.model) == 2) ? 1 : ncomp_of(p.model));
}

// Words from one population array to the next.  A node reads the same
// offset of every array, so with arrays a power of two apart (a 256^3 FP32
// array is 64 MB) the 38 concurrent streams of a step fall on the same HBM
// banks: measured on MI355X, the one-pass 256^3 FP32 colour-gradient step
// took 1.18 ms with 64 MB between arrays and 1.12 ms with 64 MB + 64 KB +
// 512 B or 64 MB + 256 KB + 256 B (in a timing copy of the step, exactly
// 64 KB or 128 KB extra were slower than none), and a plain sweep reading and
// writing every population at its node rose from 0.67 to 0.74 of the HBM
// peak with 256 KB + 256 B.  Arrays of 8 MB and more therefore start
// 256 KB + 256 B past a 1 MB boundary of the previous one's end; smaller
// ones (which the 256 MB Infinity Cache largely holds) are only rounded to
// 256 B, plus 256 B.
long long pop_stride(const mclbm_params &p)
{
    const size_t w = pop_word(p);
    const size_t N = (size_t)p.nx * p.ny * p.nz;
    size_t b = N * w;
    if (b >= ((size_t)8 << 20)) b = ((b + ((size_t)1 << 20) - 1) & ~(((size_t)1 << 20) - 1)) + ((size_t)256 << 10) + 256;
    else b = align256(b) + 256;
    return (long long)(b / w);
}

Layout layout_of(const mclbm_params &p)
{
    const size_t N = (size_t)p.nx * p.ny * p.nz;
    Layout L;
    L.fbytes = align256(pop_arrays(p) * (size_t)pop_stride(p) * pop_word(p));
    L.field_off = 2 * L.fbytes;
    L.gfield_off = L.field_off + align256((size_t)nfield_of(p) * N * field_size(p.precision));
    const bool rep = p.model == MCLBM_CG && p.Pi != 0.0;
    L.total = L.gfield_off + (rep ? align256(3 * N * field_size(p.precision)) : 0);
    return L;
}

KParams make_kparams(const mclbm_params &p);

bool fused_ok(const mclbm_params &p, const Ops *ops)
{
    FusedShape sh;
    // the multirange forces read two nodes out: the one-node halo ring of the
    // fused kernel does not hold them
    if (!ops || !ops->has_fused() || multirange_of(p)) return false;
    if (p.lattice == MCLBM_D2Q9) return true;   // rows of any length, any ny
    return fused_shape(make_kparams(p), sh, p.precision == MCLBM_FP64);
}

// Automatic kernel choice where both exist: the one-pass kernel, except on
// D2Q9 boxes under 2^19 nodes, whose few short rows leave the one-pass
// kernel latency-bound (512^2: 0.81x, 64^2: 0.33x of the two-pass speed;
// 1000^2: 1.21x, 4096^2: 1.59x).
bool auto_prefers_fused(const mclbm_params &p)
{
    return p.lattice != MCLBM_D2Q9 || (long long)p.nx * p.ny >= (1LL << 19);
}

// The batched one-pass kernel takes 96 x 4 columns where 96 divides nx and
// 64 does not (batch_wide), else 64 x batch_ty columns, the last one in x
// masked when 64 does not divide nx, as long as at least three quarters of
// the columns' lanes hold nodes (measured against the batched two-pass
// kernels, FP32: nx = 112 1.17x, 96 and 48 1.05-1.08x, 144 and 160 1.01-1.06x;
// nx = 80 0.95x, 32 0.92x); a sim whose kernel is pinned to the two-pass path
// keeps it.
// `resident`: the group's Ops::batch_fused_resident() (0: no batched
// one-pass kernel for this lattice, model and precision).
bool batch_fused_ok(const mclbm_params &p, long long resident)
{
    if (resident <= 0 || multirange_of(p) || p.kernel == MCLBM_KERNEL_TWO_PASS) return false;
    if (batch_wide(p.precision, p.model, p.nx, p.ny)) return true;
    const long long lanes = (long long)kBatchTX * ((p.nx + kBatchTX - 1) / kBatchTX);
    return p.ny % batch_ty(p.precision) == 0 && 4LL * p.nx >= 3 * lanes;
}

// Columns per plane of a batched one-pass simulation.
long long batch_fused_columns(const mclbm_params &p)
{
    const int tx = batch_tile_tx(p.precision, p.model, p.nx, p.ny), ty = batch_tile_ty(p.precision, p.model, p.nx, p.ny);
    return (long long)((p.nx + tx - 1) / tx) * (p.ny / ty);
}

mclbm_status validate(const mclbm_params *p)
{
    if (!p) return fail(MCLBM_EINVAL, "params is NULL");
    if (p->abi_version != MCLBM_ABI_VERSION)
        return fail(MCLBM_EINVAL, "abi_version %d, library has %d", p->abi_version, MCLBM_ABI_VERSION);
    if (p->lattice != MCLBM_D2Q9 && p->lattice != MCLBM_D3Q19) return fail(MCLBM_EINVAL, "bad lattice %d", p->lattice);
    if (p->model < 0 || p->model > 2) return fail(MCLBM_EINVAL, "bad model %d", p->model);
    if (p->precision < 0 || p->precision > 3) return fail(MCLBM_EINVAL, "bad precision %d", p->precision);
    if (p->nx < 2 || p->ny < 2) return fail(MCLBM_EINVAL, "nx, ny must be >= 2 (got %d, %d)", p->nx, p->ny);
    if (p->lattice == MCLBM_D2Q9 && p->nz != 1) return fail(MCLBM_EINVAL, "D2Q9 needs nz == 1");
    if (p->lattice == MCLBM_D3Q19 && p->nz < 2) return fail(MCLBM_EINVAL, "D3Q19 needs nz >= 2");
    const long long N = (long long)p->nx * p->ny * p->nz;
    // the step kernels address a node within a population array with a 32-bit
    // offset, and the periodic push's face corrections are ints
    if (N >= (1LL << 31)) return fail(MCLBM_EUNSUPPORTED, "lattices of 2^31 nodes or more are not supported");
    for (int d = 0; d < 3; ++d)
        if (p->bc[d] < 0 || p->bc[d] > 2) return fail(MCLBM_EINVAL, "bad boundary type on axis %d", d);
    if (p->conserve_mass != 0 && p->conserve_mass != 1) return fail(MCLBM_EINVAL, "conserve_mass must be 0 or 1");
    if (p->lattice == MCLBM_D2Q9 && p->bc[2] != MCLBM_PERIODIC) return fail(MCLBM_EINVAL, "D2Q9: bc[2] must be periodic");
    if (!(p->tau_R > 0.5)) return fail(MCLBM_EINVAL, "tau_R must be > 1/2");
    if (p->model != MCLBM_SC_MP && !(p->tau_B > 0.5)) return fail(MCLBM_EINVAL, "tau_B must be > 1/2");
    if (!(p->rho0_R > 0.0)) return fail(MCLBM_EINVAL, "rho0_R must be > 0");
    if (p->model == MCLBM_CG) {
        if (!(p->rho0_B > 0.0) || p->rho0_B > p->rho0_R)
            return fail(MCLBM_EINVAL, "CG needs 0 < rho0_B <= rho0_R (red is the denser fluid)");
        if (!(p->beta >= 0.0 && p->beta <= 1.0)) return fail(MCLBM_EINVAL, "beta must be in [0, 1]");
        if (!(p->alpha_B >= 0.0 && p->alpha_B < 1.0)) return fail(MCLBM_EINVAL, "alpha_B must be in [0, 1)");
        if (!(p->A >= 0.0)) return fail(MCLBM_EINVAL, "A must be >= 0");
        if (!(p->g_min >= 0.0)) return fail(MCLBM_EINVAL, "g_min must be >= 0");
        if (p->Pi != 0.0 && !(p->chi > 0.0)) return fail(MCLBM_EINVAL, "repulsion needs chi > 0");
    } else {
        if (p->Pi != 0.0) return fail(MCLBM_EUNSUPPORTED, "the repulsion force is a colour-gradient variant");
        if (p->model == MCLBM_SC_MP && !(p->psi_rho0 > 0.0)) return fail(MCLBM_EINVAL, "psi_rho0 must be > 0");
        if (p->model == MCLBM_SC_MC && (!(p->rho0_B > 0.0) || !(p->rho0_X > 0.0)))
            return fail(MCLBM_EINVAL, "SC_MC needs rho0_B > 0 and rho0_X > 0");
    }
    if (multirange_of(*p)) {
        if (p->model != MCLBM_SC_MC)
            return fail(MCLBM_EINVAL, "the multirange couplings belong to the two-component Shan-Chen model");
        if (p->lattice != MCLBM_D3Q19)
            return fail(MCLBM_EUNSUPPORTED, "the multirange neighbourhood is three-dimensional (D3Q19 only)");
        if (!(p->psi_rho0 > 0.0)) return fail(MCLBM_EINVAL, "psi_rho0 must be > 0");
        if (!std::isfinite(p->Ga_R) || !std::isfinite(p->Ga_B) || !std::isfinite(p->Gr_R) || !std::isfinite(p->Gr_B))
            return fail(MCLBM_EINVAL, "multirange couplings must be finite");
    }
    if (p->kernel < 0 || p->kernel > 2) return fail(MCLBM_EINVAL, "bad kernel choice %d", p->kernel);
    const Ops *ops = get_ops(p->lattice, p->precision, p->model, extended_of(*p));
    if (!ops) return fail(MCLBM_EUNSUPPORTED, "combination not provided");
    if (p->kernel == MCLBM_KERNEL_FUSED && !fused_ok(*p, ops))
        return fail(MCLBM_EUNSUPPORTED, "no fused kernel for this lattice/model/precision/size");
    return MCLBM_OK;
}

template <class L>
void fill_phi(const mclbm_params &p, KParams &K)
{
    if (p.model == MCLBM_CG) {
        const double aB = p.alpha_B;
        const double aR = 1.0 - (1.0 - aB) * p.rho0_B / p.rho0_R;  // Eq. gamma
        for (int q = 0; q < 3; ++q) {
            K.phi[0][q] = L::phi_a[q] * aR + L::phi_b[q];
            K.phi[1][q] = L::phi_a[q] * aB + L::phi_b[q];
        }
    } else {
        for (int q = 0; q < 3; ++q) K.phi[0][q] = K.phi[1][q] = L::w[q];
    }
}

KParams make_kparams(const mclbm_params &p)
{
    KParams K;
    memset(&K, 0, sizeof K);
    K.nx = p.nx; K.ny = p.ny; K.nz = p.nz;
    for (int d = 0; d < 3; ++d) K.bc[d] = p.bc[d];
    K.N = (long long)p.nx * p.ny * p.nz;
    K.S = pop_stride(p);
    K.enhanced = p.enhanced_eq ? 1 : 0;
    K.conserve = p.model == MCLBM_CG && (p.precision == MCLBM_FP32 || p.precision == MCLBM_MIXED)
                 && p.conserve_mass ? 1 : 0;
    K.has_outflow = (p.bc[0] == MCLBM_OUTFLOW || p.bc[1] == MCLBM_OUTFLOW || p.bc[2] == MCLBM_OUTFLOW) ? 1 : 0;
    K.rho0[0] = p.rho0_R;
    K.rho0[1] = p.model == MCLBM_SC_MP ? 0.0 : p.rho0_B;
    if (p.lattice == MCLBM_D2Q9) fill_phi<D2Q9>(p, K); else fill_phi<D3Q19>(p, K);
    const int Q = lattice_Q(p.lattice);
    const int count[3] = {1, p.lattice == MCLBM_D2Q9 ? 4 : 6, p.lattice == MCLBM_D2Q9 ? 4 : 12};
    (void)Q;
    for (int k = 0; k < 2; ++k) {
        for (int q = 0; q < 3; ++q) K.shift[k][q] = K.rho0[k] * K.phi[k][q];
        if (p.precision != MCLBM_FP64 && K.rho0[k] > 0.0) {
            // Float paths: put the reference on a grid of step 2^(e-22), e =
            // ceil(log2 rho0), so that every shift, every partial sum of
            // shifts and their total are exact in FP32.  "Component absent"
            // (g = -shift) then sums to rho = 0 exactly instead of a rounding
            // residue of the same sign at every node.
            const int e = (int)std::ceil(std::log2(K.rho0[k] * 1.01));
            const double qnt = std::ldexp(1.0, e - 22);
            double tot = 0.0;
            for (int q = 0; q < 3; ++q) {
                K.shift[k][q] = std::nearbyint(K.shift[k][q] / qnt) * qnt;
                tot += count[q] * K.shift[k][q];
            }
            K.rho0[k] = tot;
        }
        for (int q = 0; q < 3; ++q) K.corr[k][q] = K.rho0[k] * K.phi[k][q] - K.shift[k][q];
    }
    K.inv_nu[0] = 3.0 / (p.tau_R - 0.5);
    K.inv_nu[1] = p.model == MCLBM_SC_MP ? K.inv_nu[0] : 3.0 / (p.tau_B - 0.5);
    K.halfA = 0.5 * p.A;
    K.beta = p.beta;
    K.g_min = p.g_min;
    K.om[0] = 1.0 / p.tau_R;
    K.om[1] = p.model == MCLBM_SC_MP ? K.om[0] : 1.0 / p.tau_B;
    K.G = p.G;
    K.psi_rho0 = p.psi_rho0;
    K.xpref = p.model == MCLBM_SC_MC ? p.G_RB / (p.rho0_X * p.rho0_X) : 0.0;
    K.Pi = p.Pi;
    K.chi = p.chi;
    K.sc_mid = 0.5 * (p.rho0_R + p.rho0_B);
    K.multirange = multirange_of(p) ? 1 : 0;
    K.Ga[0] = p.Ga_R;
    K.Ga[1] = p.Ga_B;
    K.Gr[0] = p.Gr_R;
    K.Gr[1] = p.Gr_B;
    return K;
}

EpsTable eps_table()
{
    EpsTable e;
    for (int m = 0; m < 10; ++m) e.e[m] = 1.0 - pow(0.1, m + 1);
    return e;
}

}  // namespace

// ------------------------------------------------------------------------
// Launcher table: each precision's instantiations live in their own
// translation unit (inst_p<P>.hip) so that they compile in parallel.
// ------------------------------------------------------------------------
namespace mclbm {
const Ops *get_ops(int lattice, int precision, int model, bool rep)
{
    switch (precision) {
    case 0: return ops_prec0(lattice, model, rep);
    case 1: return ops_prec1(lattice, model, rep);
    case 2: return ops_prec2(lattice, model, rep);
    case 3: return ops_prec3(lattice, model, rep);
    }
    return nullptr;
}
}  // namespace mclbm

namespace mclbm {

// Final reduction of the per-block partials: one block per accumulator,
// each thread folds a fixed stride of partials, then a fixed LDS tree.
__global__ __launch_bounds__(256) void k_obs_final(const double *__restrict__ partials, int nblocks,
                                                   double *__restrict__ out)
{
    __shared__ double s[256];
    const int a = blockIdx.x;
    const bool is_max = a == 6 || a == 8;
    double v = is_max ? 0.0 : 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        const double w = partials[(long long)b * kNAcc + a];
        v = is_max ? fmax(v, w) : v + w;
    }
    s[threadIdx.x] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] = is_max ? fmax(s[threadIdx.x], s[threadIdx.x + h]) : s[threadIdx.x] + s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[a] = s[0];
}

// Close one batch step: running simulations flip buffers and count the
// step, then stop when diverged (flag seen during the step) or at target.
__global__ void kb_advance(SimDesc *D, int nsims)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsims) return;
    SimDesc &d = D[s];
    if (d.state != 0) return;
    d.cur ^= 1;
    d.steps += 1;
    if (*d.flag) d.state = 2;
    else if (d.steps >= d.target) d.state = 1;
}

// ---------------------------------------------------------------------------
// Interface observables (precision-independent parts).
// ---------------------------------------------------------------------------
// Sign changes of the phase indicator along a sampled line, each placed by
// linear interpolation between its two nodes, in ascending order (one block:
// contiguous chunks of segments per thread, offsets by a prefix sum).
__global__ __launch_bounds__(256) void k_crossings(const double *__restrict__ line, int len, int periodic, int max,
                                                   double *__restrict__ out, int *__restrict__ count)
{
    __shared__ int off[257];
    const int segs = periodic && len > 1 ? len : len - 1;
    const int per = (segs + 255) / 256;
    const int t = threadIdx.x;
    const int s0 = t * per, s1 = min(segs, s0 + per);
    int c = 0;
    for (int s = s0; s < s1; ++s) {
        const double a = line[s], b = line[(s + 1) % len];
        if ((a > 0.0) != (b > 0.0)) ++c;
    }
    off[t + 1] = c;
    if (t == 0) off[0] = 0;
    __syncthreads();
    if (t == 0)
        for (int i = 1; i <= 256; ++i) off[i] += off[i - 1];
    __syncthreads();
    int k = off[t];
    for (int s = s0; s < s1; ++s) {
        const double a = line[s], b = line[(s + 1) % len];
        if ((a > 0.0) != (b > 0.0)) {
            if (k < max) out[k] = s + a / (a - b);
            ++k;
        }
    }
    if (t == 0) *count = off[256];
}

// Sum of per-block partials in a fixed order (one block).
__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ partials, int n,
                                                      double *__restrict__ out)
{
    __shared__ double s[256];
    double v = 0.0;
    for (int b = threadIdx.x; b < n; b += 256) v += partials[b];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

__global__ void k_fill_int(int *__restrict__ a, long long n, int v)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// Connected components of the inside nodes under face adjacency (periodic
// axes wrap), by alternating launches of min-label propagation and pointer
// jumping.  A label is always the index of a node of the same component and
// never increases: every write is an atomic minimum.  A node that lowers its
// label from l to m also lowers node l's label to m, which carries every node
// labelled l along at its next jump; the jump follows labels while they
// decrease (each step lowers the label, so the walk ends).  When neither pass
// changes anything, every node carries the smallest index of its component.
// A label read during an update is an old or a new value, both valid.
__device__ __forceinline__ long long face_neighbour(const KParams &P, int x, int y, int z, int axis, int dir)
{
    int c[3] = {x, y, z};
    const int d[3] = {P.nx, P.ny, P.nz};
    if (d[axis] == 1) return -1;
    c[axis] += dir;
    if (c[axis] < 0 || c[axis] >= d[axis]) {
        if (P.bc[axis] != 0) return -1;
        c[axis] = c[axis] < 0 ? c[axis] + d[axis] : c[axis] - d[axis];
    }
    return (long long)c[0] + (long long)P.nx * ((long long)c[1] + (long long)P.ny * c[2]);
}

__global__ __launch_bounds__(256) void k_ccl_prop(KParams P, int *__restrict__ lab, unsigned *__restrict__ changed)
{
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= P.N) return;
    const int l = lab[n];
    if (l < 0) return;
    const int x = (int)(n % P.nx), y = (int)((n / P.nx) % P.ny), z = (int)(n / ((long long)P.nx * P.ny));
    int m = l;
    for (int a = 0; a < 3; ++a)
        for (int dir = -1; dir <= 1; dir += 2) {
            const long long q = face_neighbour(P, x, y, z, a, dir);
            if (q < 0) continue;
            const int v = lab[q];
            if (v >= 0 && v < m) m = v;
        }
    if (m < l) {
        atomicMin(&lab[n], m);
        atomicMin(&lab[l], m);
        atomicOr(changed, 1u);
    }
}

__global__ __launch_bounds__(256) void k_ccl_jump(long long N, int *__restrict__ lab, unsigned *__restrict__ changed)
{
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int l = lab[n];
    if (l < 0) return;
    int r = l;
    for (;;) {   // r strictly decreases: at most l steps
        const int rr = lab[r];
        if (rr < 0 || rr >= r) break;
        r = rr;
    }
    if (r < l) {
        atomicMin(&lab[n], r);
        atomicOr(changed, 1u);
    }
}

// Component sizes: the lanes of a wave that carry one label add once, with
// their count (consecutive nodes mostly share a label, and the few roots are
// what every atomic would otherwise hit); each round retires at least the
// leading lane's label, so the loop ends within 64 rounds.
__global__ __launch_bounds__(256) void k_ccl_sizes(long long N, const int *__restrict__ lab, int *__restrict__ sizes)
{
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int l = n < N ? lab[n] : -1;
    bool pending = l >= 0;
    for (unsigned long long m = __ballot(pending); m != 0ull; m = __ballot(pending)) {
        const int lead = __ffsll((long long)m) - 1;
        const int L = __shfl(l, lead);
        const bool mine = pending && l == L;
        const unsigned long long same = __ballot(mine);
        if (mine && (int)(threadIdx.x & 63) == lead) atomicAdd(&sizes[L], (int)__popcll(same));
        if (mine) pending = false;
    }
}

// (root, size) pairs of the components, in any order (sorted on the host).
__global__ __launch_bounds__(256) void k_ccl_roots(long long N, const int *__restrict__ lab,
                                                   const int *__restrict__ sizes, int *__restrict__ pairs,
                                                   int *__restrict__ nroots)
{
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N || lab[n] != (int)n) return;
    const int k = atomicAdd(nroots, 1);
    pairs[2 * k] = (int)n;
    pairs[2 * k + 1] = sizes[n];
}

}  // namespace mclbm

struct mclbm_sim {
    mclbm_params prm;
    KParams kp;
    const Ops *ops;
    Layout lay;
    char *base;
    void *f[2];
    void *field;
    void *gfield;
    int cur;
    int64_t step;
    hipStream_t stream;
    int device;
    bool fused;
    bool in_batch;
    unsigned *d_flag;
    double *d_partials;
    double *d_obs;
    double *h_obs;
    unsigned *h_flag;
    double *d_iface;   // interface observables: sampled line and outputs (lazy)
    int *d_lab;        // component labels, sizes, root pairs and count: 4 N + 64 ints (lazy)
};

struct mclbm_batch {
    std::vector<mclbm_sim *> sims;
    std::vector<int> order;          // descriptor slot -> index into sims
    std::vector<int64_t> step0;
    // per descriptor slot: the final state of a sim that reached its target
    // has been scanned for divergence (and was found diverged)
    std::vector<char> final_scanned, final_bad;
    hipStream_t stream;
    SimDesc *d_desc;
    SimDesc *h_desc;
    struct Group {
        const Ops *ops;
        int first, count;
        long long blocks, fblocks, oblocks;
        int fused_kinds;   // fused_kind() bits of its one-pass sims
        bool any_outflow;
    };
    std::vector<Group> groups;
    // groups after the first run on side streams, forked from and joined
    // back to `stream` every step, so that the groups' kernels overlap (in a
    // captured graph: parallel branches)
    std::vector<hipStream_t> side;
    hipEvent_t fork;
    std::vector<hipEvent_t> join;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int graph_k;
};

extern "C" {

mclbm_status mclbm_version(int32_t *major, int32_t *minor)
{
    if (!major || !minor) return fail(MCLBM_EINVAL, "NULL argument");
    *major = MCLBM_VERSION_MAJOR;
    *minor = MCLBM_VERSION_MINOR;
    return MCLBM_OK;
}

const char *mclbm_status_str(mclbm_status s)
{
    switch (s) {
    case MCLBM_OK: return "ok";
    case MCLBM_DIVERGED: return "diverged";
    case MCLBM_EINVAL: return "invalid argument";
    case MCLBM_EUNSUPPORTED: return "unsupported";
    case MCLBM_EDEVICE: return "device error";
    case MCLBM_ENOMEM: return "out of memory";
    }
    return "unknown status";
}

const char *mclbm_last_error(void) { return g_last_error.c_str(); }

mclbm_status mclbm_params_default(mclbm_params *p, int32_t lattice, int32_t model)
{
    if (!p) return fail(MCLBM_EINVAL, "params is NULL");
    memset(p, 0, sizeof *p);
    p->abi_version = MCLBM_ABI_VERSION;
    p->lattice = lattice;
    p->model = model;
    p->precision = MCLBM_FP32;
    p->nx = p->ny = 64;
    p->nz = lattice == MCLBM_D2Q9 ? 1 : 64;
    p->bc[0] = p->bc[1] = p->bc[2] = MCLBM_PERIODIC;
    p->enhanced_eq = 1;
    p->kernel = MCLBM_KERNEL_AUTO;
    p->rho0_R = 1.0;
    p->rho0_B = 1.0;
    p->tau_R = p->tau_B = 1.0;
    p->A = 0.005;
    p->beta = 0.7;
    p->alpha_B = 0.2;
    p->g_min = 1e-8;
    p->G = -5.0;
    p->psi_rho0 = 1.0;
    p->G_RB = 0.9;
    p->rho0_X = 1.0;
    p->Pi = 0.0;
    p->chi = 1.0;
    if (lattice != MCLBM_D2Q9 && lattice != MCLBM_D3Q19) return fail(MCLBM_EINVAL, "bad lattice");
    if (model < 0 || model > 2) return fail(MCLBM_EINVAL, "bad model");
    return MCLBM_OK;
}

static double omega_interface(const mclbm_params *p)
{
    const double nuR = (p->tau_R - 0.5) / 3.0, nuB = (p->tau_B - 0.5) / 3.0;
    const double nu = 1.0 / (0.5 / nuR + 0.5 / nuB);
    return 2.0 / (6.0 * nu + 1.0);
}

mclbm_status mclbm_params_from_sigma(mclbm_params *p, double sigma)
{
    if (!p) return fail(MCLBM_EINVAL, "params is NULL");
    if (p->model != MCLBM_CG) return fail(MCLBM_EINVAL, "sigma is set through A only for CG");
    if (!(p->tau_R > 0.5) || !(p->tau_B > 0.5) || !(sigma >= 0.0)) return fail(MCLBM_EINVAL, "bad tau or sigma");
    p->A = 9.0 * sigma * omega_interface(p) / 4.0;
    return MCLBM_OK;
}

mclbm_status mclbm_sigma_from_params(const mclbm_params *p, double *sigma)
{
    if (!p || !sigma) return fail(MCLBM_EINVAL, "NULL argument");
    if (p->model != MCLBM_CG) return fail(MCLBM_EINVAL, "sigma follows from A only for CG");
    if (!(p->tau_R > 0.5) || !(p->tau_B > 0.5)) return fail(MCLBM_EINVAL, "bad tau");
    *sigma = 4.0 * p->A / (9.0 * omega_interface(p));
    return MCLBM_OK;
}

mclbm_status mclbm_state_bytes(const mclbm_params *p, size_t *bytes)
{
    if (!bytes) return fail(MCLBM_EINVAL, "bytes is NULL");
    mclbm_status s = validate(p);
    if (s) return s;
    *bytes = layout_of(*p).total;
    return MCLBM_OK;
}

mclbm_status mclbm_population_stride(const mclbm_params *p, int64_t *words, int32_t *word_bytes, int32_t *arrays)
{
    if (!words || !word_bytes || !arrays) return fail(MCLBM_EINVAL, "NULL argument");
    mclbm_status s = validate(p);
    if (s) return s;
    *words = pop_stride(*p);
    *word_bytes = (int32_t)pop_word(*p);
    *arrays = (int32_t)pop_arrays(*p);
    return MCLBM_OK;
}

mclbm_status mclbm_bytes_per_update(const mclbm_params *p, double *bytes)
{
    if (!bytes) return fail(MCLBM_EINVAL, "bytes is NULL");
    mclbm_status s = validate(p);
    if (s) return s;
    *bytes = 2.0 * ncomp_of(p->model) * lattice_Q(p->lattice) * (double)storage_size(p->precision);
    return MCLBM_OK;
}

mclbm_status mclbm_create(const mclbm_params *p, void *d_state, size_t bytes, void *stream, mclbm_sim **out)
{
    if (!out) return fail(MCLBM_EINVAL, "out is NULL");
    *out = nullptr;
    mclbm_status s = validate(p);
    if (s) return s;
    if (!d_state) return fail(MCLBM_EINVAL, "d_state is NULL");
    if ((uintptr_t)d_state % 256) return fail(MCLBM_EINVAL, "d_state must be 256-byte aligned");
    const Layout lay = layout_of(*p);
    if (bytes < lay.total) return fail(MCLBM_ENOMEM, "state buffer has %zu bytes, needs %zu", bytes, lay.total);
    mclbm_sim *sim = new (std::nothrow) mclbm_sim();
    if (!sim) return fail(MCLBM_ENOMEM, "host allocation failed");
    sim->prm = *p;
    sim->kp = make_kparams(*p);
    sim->ops = get_ops(p->lattice, p->precision, p->model, extended_of(*p));
    sim->lay = lay;
    sim->base = (char *)d_state;
    sim->f[0] = sim->base;
    sim->f[1] = sim->base + lay.fbytes;
    sim->field = sim->base + lay.field_off;
    sim->gfield = sim->base + lay.gfield_off;
    sim->cur = 0;
    sim->step = 0;
    sim->stream = (hipStream_t)stream;
    sim->fused = p->kernel != MCLBM_KERNEL_TWO_PASS && fused_ok(*p, sim->ops)
                 && (p->kernel == MCLBM_KERNEL_FUSED || auto_prefers_fused(*p));
    sim->in_batch = false;
    hipError_t e = hipGetDevice(&sim->device);
    if (e == hipSuccess) e = hipMalloc((void **)&sim->d_flag, 256);
    if (e == hipSuccess) e = hipMalloc((void **)&sim->d_partials, sizeof(double) * kNAcc * kRedBlocks);
    if (e == hipSuccess) e = hipMalloc((void **)&sim->d_obs, sizeof(double) * kNAcc);
    if (e == hipSuccess) e = hipHostMalloc((void **)&sim->h_obs, sizeof(double) * kNAcc, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void **)&sim->h_flag, sizeof(unsigned), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemsetAsync(sim->d_flag, 0, 256, sim->stream);
    if (e != hipSuccess) {
        mclbm_destroy(sim);
        return fail(MCLBM_EDEVICE, "scratch allocation: %s", hipGetErrorString(e));
    }
    *out = sim;
    return MCLBM_OK;
}

mclbm_status mclbm_destroy(mclbm_sim *sim)
{
    if (!sim) return MCLBM_OK;
    if (sim->stream || sim->d_flag) (void)hipStreamSynchronize(sim->stream);
    if (sim->d_flag) (void)hipFree(sim->d_flag);
    if (sim->d_partials) (void)hipFree(sim->d_partials);
    if (sim->d_obs) (void)hipFree(sim->d_obs);
    if (sim->h_obs) (void)hipHostFree(sim->h_obs);
    if (sim->h_flag) (void)hipHostFree(sim->h_flag);
    if (sim->d_iface) (void)hipFree(sim->d_iface);
    if (sim->d_lab) (void)hipFree(sim->d_lab);
    delete sim;
    return MCLBM_OK;
}

static mclbm_status check_sim(mclbm_sim *sim)
{
    if (!sim) return fail(MCLBM_EINVAL, "sim is NULL");
    if (sim->in_batch) return fail(MCLBM_EINVAL, "sim belongs to a live batch");
    return MCLBM_OK;
}

static mclbm_status launched(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MCLBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return MCLBM_OK;
}

mclbm_status mclbm_init_equilibrium(mclbm_sim *sim, const double *d_rhoR, const double *d_rhoB, const double *d_u)
{
    mclbm_status s = check_sim(sim);
    if (s) return s;
    if (!d_rhoR) return fail(MCLBM_EINVAL, "d_rhoR is NULL");
    if (sim->prm.model != MCLBM_SC_MP && !d_rhoB) return fail(MCLBM_EINVAL, "d_rhoB is NULL");
    sim->cur = 0;
    sim->step = 0;
    MCLBM_HIP(hipMemsetAsync(sim->d_flag, 0, sizeof(unsigned), sim->stream));
    sim->ops->init(sim->kp, d_rhoR, sim->prm.model == MCLBM_SC_MP ? d_rhoR : d_rhoB, d_u, sim->f[0], sim->stream);
    return launched("init");
}

mclbm_status mclbm_kernel_used(const mclbm_sim *sim, int32_t *kernel)
{
    if (!sim || !kernel) return fail(MCLBM_EINVAL, "null argument");
    *kernel = sim->fused ? MCLBM_KERNEL_FUSED : MCLBM_KERNEL_TWO_PASS;
    return MCLBM_OK;
}

mclbm_status mclbm_fused_tile(const mclbm_sim *sim, int32_t *tx, int32_t *ty, int32_t *tz)
{
    if (!sim || !tx || !ty || !tz) return fail(MCLBM_EINVAL, "null argument");
    if (!sim->fused) return fail(MCLBM_EUNSUPPORTED, "the simulation runs the two-pass kernels");
    if (sim->prm.lattice == MCLBM_D2Q9) {
        int tiles_x = 0, rows = 0;
        fused2d_rows(as_marching_2d(sim->kp), tiles_x, rows);
        *tx = k2dTX;
        *ty = 1;
        *tz = rows;
    } else {
        FusedShape sh;
        fused_shape(sim->kp, sh, sim->prm.precision == MCLBM_FP64);
        *tx = sh.tx;
        *ty = sh.ty;
        *tz = sh.tz;
    }
    return MCLBM_OK;
}

mclbm_status mclbm_diverged(mclbm_sim *sim, int32_t *diverged)
{
    if (!sim || !diverged) return fail(MCLBM_EINVAL, "NULL argument");
    // a step flags the state it reads; scan the state the last step wrote
    sim->ops->density(sim->kp, sim->f[sim->cur], sim->field, sim->d_flag, sim->stream);
    mclbm_status s = launched("diverged");
    if (s) return s;
    MCLBM_HIP(hipMemcpyAsync(sim->h_flag, sim->d_flag, sizeof(unsigned), hipMemcpyDeviceToHost, sim->stream));
    MCLBM_HIP(hipStreamSynchronize(sim->stream));
    *diverged = *sim->h_flag ? 1 : 0;
    return MCLBM_OK;
}

mclbm_status mclbm_step(mclbm_sim *sim, int64_t nsteps, int64_t check_every, int64_t *steps_done)
{
    mclbm_status s = check_sim(sim);
    if (s) return s;
    if (nsteps < 0 || check_every < 0) return fail(MCLBM_EINVAL, "negative step count");
    int64_t done = 0;
    for (int64_t t = 0; t < nsteps; ++t) {
        sim->ops->step(sim->kp, sim->f[sim->cur], sim->f[sim->cur ^ 1], sim->field, sim->gfield, sim->d_flag,
                       sim->fused, sim->stream);
        sim->cur ^= 1;
        ++sim->step;
        ++done;
        if (check_every > 0 && (done % check_every == 0 || t + 1 == nsteps)) {
            s = launched("step");
            if (s) { if (steps_done) *steps_done = done; return s; }
            int32_t dv = 0;
            s = mclbm_diverged(sim, &dv);
            if (s) { if (steps_done) *steps_done = done; return s; }
            if (dv) {
                if (steps_done) *steps_done = done;
                return MCLBM_DIVERGED;
            }
        }
    }
    if (steps_done) *steps_done = done;
    return launched("step");
}

mclbm_status mclbm_moments(mclbm_sim *sim, double *d_rhoR, double *d_rhoB, double *d_u)
{
    mclbm_status s = check_sim(sim);
    if (s) return s;
    sim->ops->density(sim->kp, sim->f[sim->cur], sim->field, sim->d_flag, sim->stream);
    sim->ops->moments(sim->kp, sim->f[sim->cur], sim->field, d_rhoR, d_rhoB, d_u, sim->stream);
    return launched("moments");
}

mclbm_status mclbm_observables(mclbm_sim *sim, mclbm_obs *out)
{
    mclbm_status s = check_sim(sim);
    if (s) return s;
    if (!out) return fail(MCLBM_EINVAL, "out is NULL");
    const int nb = (int)std::min<long long>(kRedBlocks, grid_of(sim->kp.N));
    sim->ops->density(sim->kp, sim->f[sim->cur], sim->field, sim->d_flag, sim->stream);
    sim->ops->obs(sim->kp, sim->f[sim->cur], sim->field, eps_table(), sim->d_partials, nb, sim->stream);
    hipLaunchKernelGGL(k_obs_final, dim3(kNAcc), dim3(256), 0, sim->stream, sim->d_partials, nb, sim->d_obs);
    s = launched("observables");
    if (s) return s;
    MCLBM_HIP(hipMemcpyAsync(sim->h_obs, sim->d_obs, sizeof(double) * kNAcc, hipMemcpyDeviceToHost, sim->stream));
    MCLBM_HIP(hipStreamSynchronize(sim->stream));
    const double *a = sim->h_obs;
    memset(out, 0, sizeof *out);
    out->mass_R = a[0];
    out->mass_B = a[1];
    out->mom[0] = a[2];
    out->mom[1] = a[3];
    out->mom[2] = a[4];
    out->ekin = a[5];
    out->umax = a[6];
    out->red_volume = a[7];
    out->diverged = a[8];
    if (sim->prm.model == MCLBM_SC_MP) {
        out->n_in = a[10];
        out->n_out = a[12];
        out->rho_in = a[10] > 0 ? a[9] / a[10] : 0.0;
        out->rho_out = a[12] > 0 ? a[11] / a[12] : 0.0;
    } else {
        const EpsTable e = eps_table();
        for (int m = 9; m >= 0; --m) {
            const double *q = a + 9 + 4 * m;
            if (q[1] > 0 && q[3] > 0) {
                out->n_in = q[1];
                out->n_out = q[3];
                out->rho_in = q[0] / q[1];
                out->rho_out = q[2] / q[3];
                out->eps_used = e.e[m];
                break;
            }
        }
    }
    out->step = sim->step;
    return MCLBM_OK;
}

mclbm_status mclbm_export_f(mclbm_sim *sim, double *d_f)
{
    mclbm_status s = check_sim(sim);
    if (s) return s;
    if (!d_f) return fail(MCLBM_EINVAL, "d_f is NULL");
    sim->ops->export_f(sim->kp, sim->f[sim->cur], d_f, sim->stream);
    return launched("export");
}

mclbm_status mclbm_import_f(mclbm_sim *sim, const double *d_f)
{
    mclbm_status s = check_sim(sim);
    if (s) return s;
    if (!d_f) return fail(MCLBM_EINVAL, "d_f is NULL");
    MCLBM_HIP(hipMemsetAsync(sim->d_flag, 0, sizeof(unsigned), sim->stream));
    sim->ops->import_f(sim->kp, d_f, sim->f[sim->cur], sim->stream);
    return launched("import");
}

mclbm_status mclbm_checkpoint_bytes(const mclbm_sim *sim, size_t *bytes)
{
    if (!sim || !bytes) return fail(MCLBM_EINVAL, "NULL argument");
    *bytes = pop_arrays(sim->prm) * (size_t)sim->kp.S * pop_word(sim->prm);
    return MCLBM_OK;
}

mclbm_status mclbm_checkpoint(mclbm_sim *sim, void *d_dst, int64_t *step)
{
    mclbm_status s = check_sim(sim);
    if (s) return s;
    if (!d_dst) return fail(MCLBM_EINVAL, "d_dst is NULL");
    size_t b = 0;
    mclbm_checkpoint_bytes(sim, &b);
    MCLBM_HIP(hipMemcpyAsync(d_dst, sim->f[sim->cur], b, hipMemcpyDeviceToDevice, sim->stream));
    if (step) *step = sim->step;
    return MCLBM_OK;
}

mclbm_status mclbm_restore(mclbm_sim *sim, const void *d_src, int64_t step)
{
    mclbm_status s = check_sim(sim);
    if (s) return s;
    if (!d_src || step < 0) return fail(MCLBM_EINVAL, "bad argument");
    size_t b = 0;
    mclbm_checkpoint_bytes(sim, &b);
    MCLBM_HIP(hipMemcpyAsync(sim->f[sim->cur], d_src, b, hipMemcpyDeviceToDevice, sim->stream));
    MCLBM_HIP(hipMemsetAsync(sim->d_flag, 0, sizeof(unsigned), sim->stream));
    sim->step = step;
    return MCLBM_OK;
}

// --------------------------------------------------------------------------
// Batches.
// --------------------------------------------------------------------------
static mclbm_status batch_sync_sims(mclbm_batch *b, int32_t *status, int64_t *steps);

mclbm_status mclbm_batch_destroy(mclbm_batch *b)
{
    if (!b) return MCLBM_OK;
    // hand each sim its step count and current buffer, as mclbm_batch_status does
    if (b->d_desc && b->h_desc && !b->order.empty()) (void)batch_sync_sims(b, nullptr, nullptr);
    (void)hipStreamSynchronize(b->stream);
    for (hipStream_t s : b->side) (void)hipStreamSynchronize(s);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (hipStream_t s : b->side) (void)hipStreamDestroy(s);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->h_desc) (void)hipHostFree(b->h_desc);
    for (mclbm_sim *s : b->sims) s->in_batch = false;
    delete b;
    return MCLBM_OK;
}

mclbm_status mclbm_batch_create(mclbm_sim *const *sims, int32_t n, const int64_t *target_steps, void *stream,
                                mclbm_batch **out)
{
    if (!out || !sims || !target_steps || n <= 0) return fail(MCLBM_EINVAL, "bad batch arguments");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!sims[i]) return fail(MCLBM_EINVAL, "sim %d is NULL", i);
        if (sims[i]->in_batch) return fail(MCLBM_EINVAL, "sim %d is already in a batch", i);
        if (target_steps[i] < 0) return fail(MCLBM_EINVAL, "negative target for sim %d", i);
        for (int j = 0; j < i; ++j)
            if (sims[j] == sims[i]) return fail(MCLBM_EINVAL, "sim %d appears twice", i);
    }
    mclbm_batch *b = new (std::nothrow) mclbm_batch();
    if (!b) return fail(MCLBM_ENOMEM, "host allocation failed");
    b->stream = (hipStream_t)stream;
    b->sims.assign(sims, sims + n);
    // group by (lattice, precision, model, repulsion), stable
    std::map<std::tuple<int, int, int, int>, std::vector<int>> groups;
    std::vector<std::tuple<int, int, int, int>> keys;
    for (int i = 0; i < n; ++i) {
        const mclbm_params &p = sims[i]->prm;
        auto key = std::make_tuple(p.lattice, p.precision, p.model, (int)extended_of(p));
        if (!groups.count(key)) keys.push_back(key);
        groups[key].push_back(i);
    }
    hipError_t e = hipMalloc((void **)&b->d_desc, sizeof(SimDesc) * n);
    if (e == hipSuccess) e = hipHostMalloc((void **)&b->h_desc, sizeof(SimDesc) * n, hipHostMallocDefault);
    if (e != hipSuccess) {
        mclbm_batch_destroy(b);
        return fail(MCLBM_EDEVICE, "batch allocation: %s", hipGetErrorString(e));
    }
    int slot = 0;
    for (auto &key : keys) {
        mclbm_batch::Group g;
        g.ops = sims[groups[key][0]]->ops;
        g.first = slot;
        g.count = (int)groups[key].size();
        g.blocks = 0;
        g.fblocks = 0;
        g.fused_kinds = 0;
        g.oblocks = 0;
        g.any_outflow = false;
        const long long resident = g.ops->batch_fused_resident();
        std::vector<long long> fcols;
        std::vector<int> fnz;
        for (int idx : groups[key]) {
            const mclbm_params &q = sims[idx]->prm;
            if (batch_fused_ok(q, resident)) {
                fcols.push_back(batch_fused_columns(q));
                fnz.push_back(q.nz);
            }
        }
        const int group_tz = fcols.empty() ? 1
                             : batch_group_tz(fcols.data(), fnz.data(), (int)fcols.size(), resident);
        for (int idx : groups[key]) {
            mclbm_sim *s = sims[idx];
            (void)hipStreamSynchronize(s->stream);
            SimDesc &d = b->h_desc[slot];
            memset(&d, 0, sizeof d);
            d.P = s->kp;
            d.f[0] = s->f[0];
            d.f[1] = s->f[1];
            d.field = s->field;
            d.gfield = s->gfield;
            d.flag = s->d_flag;
            d.block0 = g.blocks;
            d.fblock0 = g.fblocks;
            if (batch_fused_ok(s->prm, resident)) {
                d.ftz = batch_fused_tz(s->prm.nz, group_tz);
                d.fnblocks = batch_fused_columns(s->prm) * ((s->prm.nz + d.ftz - 1) / d.ftz);
                g.fblocks += d.fnblocks;
                const bool periodic = s->prm.bc[0] == MCLBM_PERIODIC && s->prm.bc[1] == MCLBM_PERIODIC
                                      && s->prm.bc[2] == MCLBM_PERIODIC;
                g.fused_kinds |= fused_kind(periodic, s->prm.nx % kBatchTX != 0,
                                            batch_wide(s->prm.precision, s->prm.model, s->prm.nx, s->prm.ny));
            } else {
                d.nblocks = grid_of(s->kp.N);
                g.blocks += d.nblocks;
            }
            d.ocount = s->kp.has_outflow ? outflow_count(s->kp) : 0;
            d.oblock0 = g.oblocks;
            d.onblocks = grid_of(d.ocount);
            g.oblocks += d.onblocks;
            if (d.ocount) g.any_outflow = true;
            d.steps = 0;
            d.target = target_steps[idx];
            d.cur = s->cur;
            d.state = target_steps[idx] > 0 ? MCLBM_RUNNING : MCLBM_DONE;
            b->order.push_back(idx);
            b->step0.push_back(s->step);
            b->final_scanned.push_back(0);
            b->final_bad.push_back(0);
            ++slot;
        }
        b->groups.push_back(g);
    }
    if (b->groups.size() > 1) {
        e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        for (size_t g = 1; g < b->groups.size() && e == hipSuccess; ++g) {
            hipStream_t s = nullptr;
            hipEvent_t ev = nullptr;
            e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);   // default priority
            if (e == hipSuccess) b->side.push_back(s);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) b->join.push_back(ev);
        }
        if (e != hipSuccess) {
            mclbm_batch_destroy(b);
            return fail(MCLBM_EDEVICE, "batch streams: %s", hipGetErrorString(e));
        }
    }
    for (int i = 0; i < n; ++i) {
        e = hipMemsetAsync(sims[i]->d_flag, 0, sizeof(unsigned), b->stream);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_desc, b->h_desc, sizeof(SimDesc) * n, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        mclbm_batch_destroy(b);
        return fail(MCLBM_EDEVICE, "batch upload: %s", hipGetErrorString(e));
    }
    for (int i = 0; i < n; ++i) sims[i]->in_batch = true;
    *out = b;
    return MCLBM_OK;
}

// One batch step per iteration: fork the side streams from `stream`, each
// group's kernels on its stream, join, then the per-sim advance.  Returns the
// first error of the stream and event calls.
static hipError_t batch_enqueue(mclbm_batch *b, int k)
{
    const int n = (int)b->sims.size();
    const size_t G = b->groups.size();
    hipError_t e = hipSuccess;
    auto keep = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    for (int t = 0; t < k; ++t) {
        if (G > 1) {
            keep(hipEventRecord(b->fork, b->stream));
            for (size_t g = 1; g < G; ++g) keep(hipStreamWaitEvent(b->side[g - 1], b->fork, 0));
        }
        for (size_t g = 0; g < G; ++g) {
            const auto &gr = b->groups[g];
            gr.ops->batch_step(b->d_desc + gr.first, gr.count, gr.blocks, gr.fblocks, gr.fused_kinds, gr.oblocks,
                               gr.any_outflow, g == 0 ? b->stream : b->side[g - 1]);
        }
        for (size_t g = 1; g < G; ++g) {
            keep(hipEventRecord(b->join[g - 1], b->side[g - 1]));
            keep(hipStreamWaitEvent(b->stream, b->join[g - 1], 0));
        }
        hipLaunchKernelGGL(kb_advance, dim3((n + 63) / 64), dim3(64), 0, b->stream, b->d_desc, n);
    }
    return e;
}

mclbm_status mclbm_batch_step(mclbm_batch *b, int32_t ksteps, int32_t use_graph)
{
    if (!b || ksteps < 0) return fail(MCLBM_EINVAL, "bad batch step arguments");
    if (ksteps == 0) return MCLBM_OK;
    if (use_graph && !b->stream) return fail(MCLBM_EINVAL, "graph capture needs a non-null stream");
    if (!use_graph) {
        const hipError_t e = batch_enqueue(b, ksteps);
        if (e != hipSuccess) return fail(MCLBM_EDEVICE, "batch step: %s", hipGetErrorString(e));
        return launched("batch step");
    }
    if (!b->exec || b->graph_k != ksteps) {
        if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
        if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
        MCLBM_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        const hipError_t eq = batch_enqueue(b, ksteps);
        hipError_t e = hipStreamEndCapture(b->stream, &b->graph);
        if (e == hipSuccess) e = eq;
        if (e != hipSuccess) {
            if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
            return fail(MCLBM_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        }
        MCLBM_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_k = ksteps;
    }
    MCLBM_HIP(hipGraphLaunch(b->exec, b->stream));
    return MCLBM_OK;
}

mclbm_status mclbm_batch_kernels(const mclbm_batch *b, int32_t *kernels)
{
    if (!b || !kernels) return fail(MCLBM_EINVAL, "bad batch kernels arguments");
    for (size_t slot = 0; slot < b->order.size(); ++slot)
        kernels[b->order[slot]] = b->h_desc[slot].fnblocks > 0 ? MCLBM_KERNEL_FUSED : MCLBM_KERNEL_TWO_PASS;
    return MCLBM_OK;
}

mclbm_status mclbm_batch_status(mclbm_batch *b, int32_t *status, int64_t *steps)
{
    if (!b) return fail(MCLBM_EINVAL, "batch is NULL");
    return batch_sync_sims(b, status, steps);
}

}  // extern "C"

// Descriptor state back to the sims (current buffer, step count) and to the
// caller.  A step flags the state it reads, so the state the last step of a
// sim that reached its target wrote is scanned here, once: a bad final state
// turns DONE into STOPPED_DIVERGED (and sets the sim's divergence flag).
static mclbm_status batch_sync_sims(mclbm_batch *b, int32_t *status, int64_t *steps)
{
    const int n = (int)b->sims.size();
    MCLBM_HIP(hipMemcpyAsync(b->h_desc, b->d_desc, sizeof(SimDesc) * n, hipMemcpyDeviceToHost, b->stream));
    MCLBM_HIP(hipStreamSynchronize(b->stream));
    std::vector<int> scan;
    for (int slot = 0; slot < n; ++slot) {
        const SimDesc &d = b->h_desc[slot];
        if (d.state == MCLBM_DONE && !b->final_scanned[slot]) {
            mclbm_sim *s = b->sims[b->order[slot]];
            s->ops->density(s->kp, s->f[d.cur], s->field, s->d_flag, b->stream);
            scan.push_back(slot);
        }
    }
    for (int slot : scan) {
        mclbm_sim *s = b->sims[b->order[slot]];
        MCLBM_HIP(hipMemcpyAsync(s->h_flag, s->d_flag, sizeof(unsigned), hipMemcpyDeviceToHost, b->stream));
    }
    if (!scan.empty()) {
        mclbm_status st = launched("batch_status");
        if (st) return st;
        MCLBM_HIP(hipStreamSynchronize(b->stream));
    }
    for (int slot : scan) {
        b->final_scanned[slot] = 1;
        b->final_bad[slot] = *b->sims[b->order[slot]]->h_flag ? 1 : 0;
    }
    for (int slot = 0; slot < n; ++slot) {
        const int idx = b->order[slot];
        const SimDesc &d = b->h_desc[slot];
        mclbm_sim *s = b->sims[idx];
        s->cur = d.cur;
        s->step = b->step0[slot] + d.steps;
        if (status) status[idx] = (d.state == MCLBM_DONE && b->final_bad[slot]) ? MCLBM_STOPPED_DIVERGED : d.state;
        if (steps) steps[idx] = d.steps;
    }
    return MCLBM_OK;
}

// ---------------------------------------------------------------------------
// Interface observables
// ---------------------------------------------------------------------------
static int axis_len(const mclbm_sim *sim, int a) { return a == 0 ? sim->prm.nx : (a == 1 ? sim->prm.ny : sim->prm.nz); }

static mclbm_status iface_buffers(mclbm_sim *sim)
{
    if (sim->d_iface) return MCLBM_OK;
    const int mx = std::max(sim->prm.nx, std::max(sim->prm.ny, sim->prm.nz));
    MCLBM_HIP(hipMalloc((void **)&sim->d_iface, sizeof(double) * (2 * (size_t)mx + 16)));
    return MCLBM_OK;
}

// Arguments of the two interface-crossing calls.
static mclbm_status crossings_args(mclbm_sim *sim, int32_t axis, int32_t c1, int32_t c2, const double *h_pos,
                                   int32_t max, const int32_t *count)
{
    mclbm_status s = check_sim(sim);
    if (s) return s;
    if (axis < 0 || axis > 2) return fail(MCLBM_EINVAL, "axis %d", axis);
    if (!count || max < 0 || (max > 0 && !h_pos)) return fail(MCLBM_EINVAL, "bad output arguments");
    const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
    if (c1 < 0 || c1 >= axis_len(sim, a1) || c2 < 0 || c2 >= axis_len(sim, a2))
        return fail(MCLBM_EINVAL, "line (%d, %d) outside the box", c1, c2);
    return MCLBM_OK;
}

// Crossings along a line (arguments checked), with device scratch `buf` of at
// least 2 * (line length) + 9 doubles: the sampled indicator, the positions
// and the count.
static mclbm_status crossings_on(mclbm_sim *sim, int32_t axis, int32_t c1, int32_t c2, double *h_pos, int32_t max,
                                 int32_t *count, double *buf)
{
    mclbm_status s;
    const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
    const long long nx = sim->prm.nx, sxy = nx * sim->prm.ny;
    const long long stride[3] = {1, nx, sxy};
    const int len = axis_len(sim, axis);
    NodeSet ns;
    ns.base = (long long)c1 * stride[a1] + (long long)c2 * stride[a2];
    ns.s1 = stride[axis];
    ns.s2 = 0;
    ns.len1 = len;
    ns.count = len;
    double *line = buf, *out = buf + len + 8;
    int *d_count = (int *)(buf + 2 * len + 8);
    const int keep = std::min(max, len);
    sim->ops->phase_sample(sim->kp, sim->f[sim->cur], ns, line, sim->stream);
    hipLaunchKernelGGL(k_crossings, dim3(1), dim3(256), 0, sim->stream, line, len,
                       sim->prm.bc[axis] == MCLBM_PERIODIC ? 1 : 0, keep, out, d_count);
    s = launched("interface_crossings");
    if (s) return s;
    int n = 0;
    MCLBM_HIP(hipMemcpyAsync(&n, d_count, sizeof(int), hipMemcpyDeviceToHost, sim->stream));
    MCLBM_HIP(hipStreamSynchronize(sim->stream));
    if (keep > 0 && n > 0)
        MCLBM_HIP(hipMemcpy(h_pos, out, sizeof(double) * (size_t)std::min(n, keep), hipMemcpyDeviceToHost));
    *count = n;
    return MCLBM_OK;
}

mclbm_status mclbm_interface_crossings(mclbm_sim *sim, int32_t axis, int32_t c1, int32_t c2, double *h_pos,
                                       int32_t max, int32_t *count)
{
    mclbm_status s = crossings_args(sim, axis, c1, c2, h_pos, max, count);
    if (s) return s;
    s = iface_buffers(sim);
    if (s) return s;
    return crossings_on(sim, axis, c1, c2, h_pos, max, count, sim->d_iface);
}

// Scratch of the allocation-free crossing call: a line of up to
// kNoAllocLine nodes (sampled indicator, positions, count).  Each device
// holds its own copy for the life of the process; host code reaches it only
// through the address hipGetSymbolAddress returns on that device.
constexpr int kNoAllocLine = 32768;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[2 * kNoAllocLine + 16];

static std::mutex g_scratch_mu;
static double *g_scratch_at[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current (the caller's current device is restored).
static mclbm_status scratch_on(int device, double **ptr)
{
    if (device < 0 || device >= kMaxDevices) return fail(MCLBM_EUNSUPPORTED, "device %d", device);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_at[device]) {
        int cur = 0;
        MCLBM_HIP(hipGetDevice(&cur));
        if (cur != device) MCLBM_HIP(hipSetDevice(device));
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) MCLBM_HIP(hipSetDevice(cur));
        if (e != hipSuccess) return fail(MCLBM_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_at[device] = (double *)p;
    }
    *ptr = g_scratch_at[device];
    return MCLBM_OK;
}

mclbm_status mclbm_interface_crossings_noalloc(mclbm_sim *sim, int32_t axis, int32_t c1, int32_t c2, double *h_pos,
                                               int32_t max, int32_t *count)
{
    mclbm_status s = crossings_args(sim, axis, c1, c2, h_pos, max, count);
    if (s) return s;
    const int len = axis_len(sim, axis);
    if (len > kNoAllocLine)
        return fail(MCLBM_EUNSUPPORTED, "line of %d nodes: the allocation-free call holds at most %d", len,
                    kNoAllocLine);
    double *buf = nullptr;
    s = scratch_on(sim->device, &buf);
    if (s) return s;
    return crossings_on(sim, axis, c1, c2, h_pos, max, count, buf);
}

mclbm_status mclbm_plane_area(mclbm_sim *sim, int32_t axis, int32_t pos, double *area)
{
    mclbm_status s = check_sim(sim);
    if (s) return s;
    if (axis < 0 || axis > 2) return fail(MCLBM_EINVAL, "axis %d", axis);
    if (!area) return fail(MCLBM_EINVAL, "area is NULL");
    if (pos < 0 || pos >= axis_len(sim, axis)) return fail(MCLBM_EINVAL, "plane %d outside the box", pos);
    const long long nx = sim->prm.nx, ny = sim->prm.ny, nz = sim->prm.nz, sxy = nx * ny;
    NodeSet ns;
    if (axis == 0) { ns.base = pos; ns.s1 = nx; ns.len1 = ny; ns.s2 = sxy; ns.count = ny * nz; }
    else if (axis == 1) { ns.base = (long long)pos * nx; ns.s1 = 1; ns.len1 = nx; ns.s2 = sxy; ns.count = nx * nz; }
    else { ns.base = (long long)pos * sxy; ns.s1 = 1; ns.len1 = nx; ns.s2 = nx; ns.count = nx * ny; }
    const int nb = (int)std::min<long long>(kRedBlocks, grid_of(ns.count));
    sim->ops->phase_area(sim->kp, sim->f[sim->cur], ns, sim->d_partials, nb, sim->stream);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, sim->stream, sim->d_partials, nb, sim->d_obs);
    s = launched("plane_area");
    if (s) return s;
    MCLBM_HIP(hipMemcpyAsync(sim->h_obs, sim->d_obs, sizeof(double), hipMemcpyDeviceToHost, sim->stream));
    MCLBM_HIP(hipStreamSynchronize(sim->stream));
    *area = sim->h_obs[0];
    return MCLBM_OK;
}

mclbm_status mclbm_droplets(mclbm_sim *sim, int32_t max, int32_t *count, int64_t *h_sizes)
{
    mclbm_status s = check_sim(sim);
    if (s) return s;
    if (!count || max < 0 || (max > 0 && !h_sizes)) return fail(MCLBM_EINVAL, "bad output arguments");
    const long long N = sim->kp.N;
    if (N >= (1LL << 31) - 2) return fail(MCLBM_EUNSUPPORTED, "labelling needs fewer than 2^31 nodes");
    // labels N, sizes N, (root, size) pairs 2 N (up to one component per
    // node), the component count
    if (!sim->d_lab) MCLBM_HIP(hipMalloc((void **)&sim->d_lab, sizeof(int) * (4 * (size_t)N + 64)));
    int *lab = sim->d_lab, *sizes = lab + N, *pairs = lab + 2 * N, *d_n = lab + 4 * N;
    const unsigned g = (unsigned)((N + 255) / 256);
    sim->ops->phase_labels(sim->kp, sim->f[sim->cur], lab, sim->stream);
    // each check runs four rounds; a round changes something until the
    // labels have converged, and every change lowers some label
    const long long max_checks = N / 4 + 16;
    for (long long it = 0;; ++it) {
        if (it > max_checks) return fail(MCLBM_EDEVICE, "labelling did not converge");
        hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, sim->stream, (int *)sim->d_flag + 1, 1LL, 0);
        for (int r = 0; r < 4; ++r) {
            hipLaunchKernelGGL(k_ccl_prop, dim3(g), dim3(256), 0, sim->stream, sim->kp, lab,
                               (unsigned *)sim->d_flag + 1);
            hipLaunchKernelGGL(k_ccl_jump, dim3(g), dim3(256), 0, sim->stream, N, lab, (unsigned *)sim->d_flag + 1);
        }
        s = launched("droplets");
        if (s) return s;
        MCLBM_HIP(hipMemcpyAsync(sim->h_flag, (unsigned *)sim->d_flag + 1, sizeof(unsigned), hipMemcpyDeviceToHost,
                                 sim->stream));
        MCLBM_HIP(hipStreamSynchronize(sim->stream));
        if (*sim->h_flag == 0) break;
    }
    hipLaunchKernelGGL(k_fill_int, dim3(g), dim3(256), 0, sim->stream, sizes, N, 0);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, sim->stream, d_n, 1LL, 0);
    hipLaunchKernelGGL(k_ccl_sizes, dim3(g), dim3(256), 0, sim->stream, N, (const int *)lab, sizes);
    hipLaunchKernelGGL(k_ccl_roots, dim3(g), dim3(256), 0, sim->stream, N, (const int *)lab, (const int *)sizes,
                       pairs, d_n);
    s = launched("droplets");
    if (s) return s;
    int n = 0;
    MCLBM_HIP(hipMemcpyAsync(&n, d_n, sizeof(int), hipMemcpyDeviceToHost, sim->stream));
    MCLBM_HIP(hipStreamSynchronize(sim->stream));
    std::vector<int> hp(2 * (size_t)n);
    if (n > 0) MCLBM_HIP(hipMemcpy(hp.data(), pairs, sizeof(int) * 2 * (size_t)n, hipMemcpyDeviceToHost));
    std::vector<std::pair<int, int>> comp((size_t)n);
    for (int i = 0; i < n; ++i) comp[(size_t)i] = {-hp[2 * (size_t)i + 1], hp[2 * (size_t)i]};
    std::sort(comp.begin(), comp.end());   // largest first, then by smallest node index
    for (int i = 0; i < std::min(n, (int)max); ++i) h_sizes[i] = -(int64_t)comp[(size_t)i].first;
    *count = n;
    return MCLBM_OK;
}
