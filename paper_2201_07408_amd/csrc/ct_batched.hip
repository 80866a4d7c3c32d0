// Batched BA-GMRES (Sec. II, Eq. 5) over many independent 2D parallel-beam
// problems of uneven sizes, solved together.
//
// One problem alone (a 128 x 128 slice with 90 views is 1.7e4 rays) fills
// a small fraction of the GPU, and its solve is a chain of about ten small
// launches per iteration.  Here every step of the iteration is ONE launch
// over all problems:
//  * the vectors of all problems are concatenated: image segment i starts at
//    a multiple of kBVec (4096) floats and its tail is kept at zero, data
//    segment i at a multiple of 64 floats;
//  * the projector, back-projector and ramp filter map each workgroup to a
//    problem through a prefix sum of per-problem workgroup counts;
//  * a CGS2 sweep gives every 4096-float block of the concatenated basis to
//    one workgroup, which belongs to exactly one problem, and writes its
//    partial sums to column-major [column][block] tables; each problem's
//    scalar step (one workgroup per problem) reduces its own range of
//    blocks in a fixed order;
//  * every problem has its own Hessenberg matrix, rotations, scales and
//    stop flag, so a problem that breaks down stops while the rest go on.
// The whole chain (K iterations) is captured once into a hipGraph and
// replayed; the per-problem tables live in the workspace and are uploaded
// before each replay, so new b / x arrays need no new graph.  The variants
// of the 2D projector (plane loop unrolled by 4 or 8) and back-projector
// (1, 2 or 4 pixels per work-item) are picked per batch shape by timing
// them on the first solve; every variant computes the same floating-point
// operations in the same order, so the choice never changes a result.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "ct_krylov_dev.h"

namespace ct {
namespace {

using namespace kry;

constexpr int kQ = kBVec / 4;   // float4 groups per sweep workgroup
constexpr int kMaxBatch = 65536;

__device__ __forceinline__ int find_problem(const int *__restrict__ pfx, int count, int b) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pfx[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// d[j] = W[vlo + j] . z and ||z||^2 over one 4096-float block
template <int NV>
__global__ __launch_bounds__(256) void k_bmdot(const float *__restrict__ W, size_t ldw, int vlo, int cnt,
                                               const float *__restrict__ z, int nrm, int ncol,
                                               double *__restrict__ partials, size_t pstride,
                                               const int *__restrict__ pfx, int count,
                                               const BSlice *__restrict__ sl) {
    const int vb = blockIdx.x;
    const int s = find_problem(pfx, count, vb);
    if (*sl[s].stop) return;
    double acc[NV], nacc = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    const size_t q0 = (size_t)vb * kQ;
    mdot_groups<NV>(W + (size_t)vlo * ldw, ldw, cnt, z, q0, q0 + kQ, 256, acc, nacc);
    block_partials<NV>(acc, cnt, nacc, nrm != 0, vlo, ncol, partials, pstride, vb);
}

// z' = zs z - sum_j coef[vlo + j] W[vlo + j] over one block, with ||z'||^2
template <int NV>
__global__ __launch_bounds__(256) void k_bmaxpy(const float *__restrict__ W, size_t ldw, int vlo, int cnt,
                                                const float *zin, float *zout, const KState *__restrict__ states,
                                                int use_zs, int nrm, int ncol, double *__restrict__ partials,
                                                size_t pstride, const int *__restrict__ pfx, int count,
                                                const BSlice *__restrict__ sl) {
    const int vb = blockIdx.x;
    const int s = find_problem(pfx, count, vb);
    if (*sl[s].stop) return;
    const KState &st = states[s];
    __shared__ double cf[NV];
    for (int j = threadIdx.x; j < cnt; j += 256) cf[j] = st.coef[vlo + j];
    __syncthreads();
    const double zs = use_zs ? st.misc[M_ZS] : 1.0;
    double nacc = 0.0;
    const size_t q0 = (size_t)vb * kQ;
    maxpy_groups<NV>(W + (size_t)vlo * ldw, ldw, cnt, cf, zs, zin, zout, 1.0f, q0, q0 + kQ, 256, nacc);
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    block_partials<NV>(acc, 0, nacc, nrm != 0, vlo, ncol, partials, pstride, vb);
}

// one workgroup per problem
__global__ __launch_bounds__(256) void k_binit(KState *states, const int *__restrict__ pfx) {
    __shared__ double d[kMaxVec + 2];
    KState st = states[blockIdx.x];
    gmres_init(st, pfx[blockIdx.x + 1] - pfx[blockIdx.x], 0.0, d);
}

__global__ __launch_bounds__(256) void k_bred(KState *states, const int *__restrict__ pfx, int stage, int k,
                                              double tol) {
    __shared__ double d[kMaxVec + 2];
    KState st = states[blockIdx.x];
    if (st.flags[F_STOP]) return;
    const int nblk = pfx[blockIdx.x + 1] - pfx[blockIdx.x];
    if (stage == 1) gmres_red1(st, nblk, k, d);
    else if (stage == 2) gmres_red2(st, nblk, k, d);
    else gmres_red3(st, nblk, k, tol, 0.0, d);
}

__global__ void k_btrsv(KState *states) {
    KState st = states[blockIdx.x];
    gmres_trsv(st);
}

// x_i = sum_{j < k_done} coef_i[j] W[j] on problem i's segment, written to
// the caller's image
__global__ __launch_bounds__(256) void k_bcombine(const float *__restrict__ W, size_t ldw,
                                                  const KState *__restrict__ states, const int *__restrict__ pfx,
                                                  int count, const BSlice *__restrict__ sl) {
    const int vb = blockIdx.x;
    const int s = find_problem(pfx, count, vb);
    const BSlice &S = sl[s];
    const KState &st = states[s];
    __shared__ double cf[kMaxVec + 1];
    const int kd = st.flags[F_KDONE];
    for (int j = threadIdx.x; j < kd; j += blockDim.x) cf[j] = st.coef[j];
    __syncthreads();
    const size_t n = (size_t)S.g.nx * S.g.ny;
    const size_t lo = (size_t)vb * kBVec - S.voff;
    for (int t = threadIdx.x; t < kBVec; t += 256) {
        const size_t i = lo + t;
        if (i >= n) break;
        double a = 0.0;
        for (int j = 0; j < kd; ++j) a += cf[j] * (double)W[(size_t)j * ldw + S.voff + i];
        S.x[i] = (float)a;
    }
}

__global__ void k_bzero_i32(int *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// ------------------------------------------------------------------ host
enum { PFX_PAD = 0, PFX_RAY, PFX_ROW, PFX_VEC, PFX_PIX0 };
constexpr int kNumPfx = PFX_PIX0 + kBBackVariants;

struct Plan {
    int count = 0, K = 0, B = CT_B_UNMATCHED;
    size_t NI = 0, ND = 0, pad_elems = 0, ldw = 0;
    int max_nu = 0;
    std::vector<int> pfx[kNumPfx];   // count + 1 each
    // workspace carve (byte offsets)
    size_t o_tab = 0, tab_bytes = 0, o_flags = 0, o_H = 0, o_vec = 0, o_misc = 0, o_part = 0, o_W = 0, o_z = 0,
           o_q = 0, o_filt = 0, o_pad = 0, total = 0;
    size_t o_sl = 0, o_st = 0, o_pfx = 0;   // inside the table
    int ptot() const { return pfx[PFX_VEC][count]; }
    int total_blocks(int which) const { return pfx[which][count]; }
};

size_t al(size_t v) { return align_up(v); }

int make_plan(const ct_geometry *const *g, int count, const ct_solver_opts &o, Plan &P) {
    P.count = count;
    P.K = o.iters;
    P.B = o.B;
    for (auto &v : P.pfx) v.assign(count + 1, 0);
    P.NI = P.ND = P.pad_elems = 0;
    P.max_nu = 0;
    for (int i = 0; i < count; ++i) {
        const ct_geometry *gi = g[i];
        CT_ARG_CHECK(gi != nullptr, "ct_ba_gmres_batched: NULL geometry");
        if (gi->k.kind != CT_PARALLEL_2D || gi->k.proj != CT_JOSEPH) {
            set_error("ct_ba_gmres_batched: only 2D parallel-beam problems with the Joseph projector are batched");
            return CT_ERR_UNSUPPORTED;
        }
        const GeomK &k = gi->k;
        const size_t n = gi->n_vox, m = gi->n_rays;
        P.NI += (n + kBVec - 1) / kBVec * kBVec;
        P.ND += (m + 63) / 64 * 64;
        P.pad_elems += (size_t)gi->pad.nvx + gi->pad.nvy;
        if (k.nu > P.max_nu) P.max_nu = k.nu;
        P.pfx[PFX_PAD][i + 1] = P.pfx[PFX_PAD][i] + bpad_blocks(k);
        P.pfx[PFX_RAY][i + 1] = P.pfx[PFX_RAY][i] + bray_blocks(k);
        P.pfx[PFX_ROW][i + 1] = P.pfx[PFX_ROW][i] + k.P;
        P.pfx[PFX_VEC][i + 1] = P.pfx[PFX_VEC][i] + (int)((n + kBVec - 1) / kBVec);
        for (int v = 0; v < kBBackVariants; ++v)
            P.pfx[PFX_PIX0 + v][i + 1] = P.pfx[PFX_PIX0 + v][i] + bpix_blocks(k, bback_ppt(v));
        for (int w = 0; w < kNumPfx; ++w)
            if (P.pfx[w][i + 1] < 0 || P.pfx[w][i + 1] > (1 << 30)) {
                set_error("ct_ba_gmres_batched: batch too large");
                return CT_ERR_UNSUPPORTED;
            }
    }
    if ((double)P.pad_elems * 4.0 >= 4294967296.0) {
        set_error("ct_ba_gmres_batched: padded images of the batch exceed 4 GiB");
        return CT_ERR_UNSUPPORTED;
    }
    const int K = P.K, K1 = K + 1, K2 = K + 2;
    P.ldw = P.NI;
    size_t off = 0;
    P.o_sl = 0;
    P.o_st = al(sizeof(BSlice) * count);
    P.o_pfx = P.o_st + al(sizeof(KState) * count);
    P.tab_bytes = P.o_pfx + al(sizeof(int) * (size_t)(count + 1) * kNumPfx);
    P.o_tab = off;
    off += al(P.tab_bytes);
    P.o_flags = off;
    off += al(sizeof(int) * 16 * (size_t)count);
    P.o_H = off;
    off += al(sizeof(double) * (size_t)count * K1 * (K > 0 ? K : 1));
    P.o_vec = off;   // cs, sn, gv, sc, h1, h2, coef, res: K + 2 each
    off += al(sizeof(double) * (size_t)count * K2 * 8);
    P.o_misc = off;
    off += al(sizeof(double) * (size_t)count * 8);
    P.o_part = off;
    off += al(sizeof(double) * (size_t)(K + 3) * P.ptot());
    P.o_W = off;
    off += al(sizeof(float) * P.ldw * (size_t)K1);
    P.o_z = off;
    off += al(sizeof(float) * P.NI);
    P.o_q = off;
    off += al(sizeof(float) * P.ND);
    P.o_filt = off;
    if (P.B == CT_B_RAMP) off += al(sizeof(float) * P.ND);
    P.o_pad = off;
    off += al(sizeof(float) * P.pad_elems);
    P.total = off;
    return CT_OK;
}

struct Dev {   // device pointers of one carved workspace
    BSlice *sl;
    KState *st;
    int *pfx;
    int *flags;
    double *part;
    float *W, *z, *q, *filt, *pad;
    const int *pf(int which, int count) const { return pfx + (size_t)which * (count + 1); }
};

Dev carve(const Plan &P, void *ws) {
    char *b = (char *)ws;
    Dev d;
    d.sl = (BSlice *)(b + P.o_tab + P.o_sl);
    d.st = (KState *)(b + P.o_tab + P.o_st);
    d.pfx = (int *)(b + P.o_tab + P.o_pfx);
    d.flags = (int *)(b + P.o_flags);
    d.part = (double *)(b + P.o_part);
    d.W = (float *)(b + P.o_W);
    d.z = (float *)(b + P.o_z);
    d.q = (float *)(b + P.o_q);
    d.filt = P.B == CT_B_RAMP ? (float *)(b + P.o_filt) : nullptr;
    d.pad = (float *)(b + P.o_pad);
    return d;
}

// Host image of the tables: per-problem slices, scalar states, prefix sums.
std::vector<char> build_tables(const Plan &P, const Dev &d, void *ws, const ct_geometry *const *g,
                               const float *const *bv, float *const *xv) {
    std::vector<char> t(P.tab_bytes, 0);
    BSlice *sl = (BSlice *)(t.data() + P.o_sl);
    KState *st = (KState *)(t.data() + P.o_st);
    int *pf = (int *)(t.data() + P.o_pfx);
    char *b = (char *)ws;
    const int count = P.count, K = P.K, K1 = K + 1, K2 = K + 2;
    size_t voff = 0, roff = 0, poff = 0;
    double *vecs = (double *)(b + P.o_vec);
    for (int i = 0; i < count; ++i) {
        const ct_geometry *gi = g[i];
        BSlice &s = sl[i];
        s.g = gi->k;
        s.L = gi->pad;
        s.ramp = gi->d_ramp;
        s.b = bv[i];
        s.x = xv[i];
        s.voff = voff;
        s.roff = roff;
        s.pvx = (uint32_t)poff;
        s.pvy = (uint32_t)(poff + gi->pad.nvx);
        s.stop = d.flags + 16 * (size_t)i + F_STOP;
        voff += (gi->n_vox + kBVec - 1) / kBVec * kBVec;
        roff += (gi->n_rays + 63) / 64 * 64;
        poff += gi->pad.nvx + gi->pad.nvy;
        KState &k = st[i];
        k.flags = d.flags + 16 * (size_t)i;
        k.H = (double *)(b + P.o_H) + (size_t)i * K1 * (K > 0 ? K : 1);
        double *v = vecs + (size_t)i * K2 * 8;
        k.cs = v;
        k.sn = v + K2;
        k.gv = v + 2 * K2;
        k.sc = v + 3 * K2;
        k.h1 = v + 4 * K2;
        k.h2 = v + 5 * K2;
        k.coef = v + 6 * K2;
        k.res = v + 7 * K2;
        k.misc = (double *)(b + P.o_misc) + (size_t)i * 8;
        k.fscale = nullptr;
        k.partials = d.part + P.pfx[PFX_VEC][i];
        k.pstride = (size_t)P.ptot();
        k.K = K;
    }
    for (int w = 0; w < kNumPfx; ++w)
        std::memcpy(pf + (size_t)w * (count + 1), P.pfx[w].data(), sizeof(int) * (count + 1));
    return t;
}

// ---------------------------------------------------------- the chain
struct Tiles {
    int a = 0, b = 0;
};

int cgs_mdot(const Plan &P, const Dev &d, int vlo, int cnt, const float *z, bool nrm, int ncol, hipStream_t s) {
    const int nb = P.ptot();
    const int *pf = d.pf(PFX_VEC, P.count);
#define CT_BMDOT(NVV) \
    hipLaunchKernelGGL(k_bmdot<NVV>, dim3(nb), dim3(256), 0, s, d.W, P.ldw, vlo, cnt, z, (int)nrm, ncol, d.part, \
                       (size_t)nb, pf, P.count, d.sl)
    if (cnt <= 1) CT_BMDOT(1);
    else if (cnt <= 4) CT_BMDOT(4);
    else if (cnt <= 8) CT_BMDOT(8);
    else CT_BMDOT(16);
#undef CT_BMDOT
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int cgs_maxpy(const Plan &P, const Dev &d, int vlo, int cnt, const float *zin, float *zout, bool use_zs, bool nrm,
              hipStream_t s) {
    const int nb = P.ptot();
    const int *pf = d.pf(PFX_VEC, P.count);
#define CT_BMAXPY(NVV) \
    hipLaunchKernelGGL(k_bmaxpy<NVV>, dim3(nb), dim3(256), 0, s, d.W, P.ldw, vlo, cnt, zin, zout, d.st, (int)use_zs, \
                       (int)nrm, 0, d.part, (size_t)nb, pf, P.count, d.sl)
    if (cnt <= 1) CT_BMAXPY(1);
    else if (cnt <= 4) CT_BMAXPY(4);
    else if (cnt <= 8) CT_BMAXPY(8);
    else CT_BMAXPY(16);
#undef CT_BMAXPY
    CT_LAUNCH_CHECK();
    return CT_OK;
}

constexpr int kChunk = 16;

// the same three CGS2 passes as the single-problem solver (modes 0, 1, 2)
int run_bcgs(int mode, const Plan &P, const Dev &d, int nvec, const float *zin, float *zout, hipStream_t s) {
    ProfScope prof(PROF_CGS, s);
    if (mode == 0) {
        if (nvec == 0) return cgs_mdot(P, d, 0, 0, zin, true, 0, s);
        for (int lo = 0; lo < nvec; lo += kChunk) {
            const int cnt = nvec - lo < kChunk ? nvec - lo : kChunk;
            CT_TRY(cgs_mdot(P, d, lo, cnt, zin, lo == 0, nvec, s));
        }
        return CT_OK;
    }
    if (nvec == 0) return cgs_maxpy(P, d, 0, 0, zin, zout, false, true, s);
    for (int lo = 0; lo < nvec; lo += kChunk) {
        const int cnt = nvec - lo < kChunk ? nvec - lo : kChunk;
        const bool last = lo + cnt >= nvec;
        CT_TRY(cgs_maxpy(P, d, lo, cnt, lo == 0 ? zin : zout, zout, mode == 1 && lo == 0, mode == 2 && last, s));
    }
    if (mode == 1)
        for (int lo = 0; lo < nvec; lo += kChunk) {
            const int cnt = nvec - lo < kChunk ? nvec - lo : kChunk;
            CT_TRY(cgs_mdot(P, d, lo, cnt, zout, false, 0, s));
        }
    return CT_OK;
}

// z = B y for every problem (y == nullptr: the caller's data)
int bapply_B(const Plan &P, const Dev &d, const Tiles &tl, const float *y, float *z, hipStream_t s) {
    const float *src = y;
    if (P.B == CT_B_RAMP) {
        CT_TRY(launch_bramp(d.sl, P.count, d.pf(PFX_ROW, P.count), P.total_blocks(PFX_ROW), P.max_nu, y, d.filt, s));
        src = d.filt;
    }
    return launch_bbackproject2d(d.sl, P.count, d.pf(PFX_PIX0 + tl.b, P.count), P.total_blocks(PFX_PIX0 + tl.b),
                                 tl.b, src, z, s);
}

int bapply_A(const Plan &P, const Dev &d, const Tiles &tl, const float *w, hipStream_t s) {
    CT_TRY(launch_bpad_copy(d.sl, P.count, d.pf(PFX_PAD, P.count), P.total_blocks(PFX_PAD), w, d.pad, s));
    return launch_bproject2d(d.sl, P.count, d.pf(PFX_RAY, P.count), P.total_blocks(PFX_RAY), tl.a, d.pad,
                             P.pad_elems, d.q, s);
}

int grid1(size_t n) {
    size_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : b > 4096 ? 4096 : b);
}

int enqueue_solve(const Plan &P, const Dev &d, const Tiles &tl, double tol, hipStream_t s) {
    const int count = P.count;
    hipLaunchKernelGGL(k_bzero_i32, dim3(grid1(16 * (size_t)count)), dim3(256), 0, s, d.flags, 16 * count);
    CT_LAUNCH_CHECK();
    // segment tails of W[0] and z stay zero from here on; the pad borders too
    CT_TRY(launch_fill(d.W, P.NI, 0.0f, s));
    CT_TRY(launch_fill(d.z, P.NI, 0.0f, s));
    CT_TRY(launch_fill(d.pad, P.pad_elems, 0.0f, s));
    CT_TRY(bapply_B(P, d, tl, nullptr, d.W, s));
    CT_TRY(run_bcgs(2, P, d, 0, d.W, d.W, s));   // ||r0||^2
    const int *pv = d.pf(PFX_VEC, count);
    hipLaunchKernelGGL(k_binit, dim3(count), dim3(256), 0, s, d.st, pv);
    CT_LAUNCH_CHECK();
    for (int k = 0; k < P.K; ++k) {
        float *wk = d.W + (size_t)k * P.ldw;
        float *wn = d.W + (size_t)(k + 1) * P.ldw;
        CT_TRY(bapply_A(P, d, tl, wk, s));
        CT_TRY(bapply_B(P, d, tl, d.q, d.z, s));
        const int nvec = k + 1;
        CT_TRY(run_bcgs(0, P, d, nvec, d.z, nullptr, s));
        hipLaunchKernelGGL(k_bred, dim3(count), dim3(256), 0, s, d.st, pv, 1, k, tol);
        CT_LAUNCH_CHECK();
        CT_TRY(run_bcgs(1, P, d, nvec, d.z, wn, s));
        hipLaunchKernelGGL(k_bred, dim3(count), dim3(256), 0, s, d.st, pv, 2, k, tol);
        CT_LAUNCH_CHECK();
        CT_TRY(run_bcgs(2, P, d, nvec, wn, wn, s));
        hipLaunchKernelGGL(k_bred, dim3(count), dim3(256), 0, s, d.st, pv, 3, k, tol);
        CT_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_btrsv, dim3(count), dim3(64), 0, s, d.st);
    CT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bcombine, dim3(P.ptot()), dim3(256), 0, s, d.W, P.ldw, d.st, pv, count, d.sl);
    CT_LAUNCH_CHECK();
    return CT_OK;
}

// ---------------------------------------------------- configuration
std::mutex g_mu;
int g_use_graph = 1;
int g_force_a = -1, g_force_b = -1;
int g_last_a = -1, g_last_b = -1, g_last_graph = 0;
std::map<std::string, Tiles> g_tuned;

struct GraphEntry {
    std::string key;
    int device = -1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};
GraphEntry g_graph;
std::map<int, hipStream_t> g_cap_streams;

std::string shape_key(const ct_geometry *const *g, int count, int B) {
    std::ostringstream k;
    k << B << ':' << count;
    for (int i = 0; i < count; ++i) {
        const GeomK &q = g[i]->k;
        k << ';' << q.nx << ',' << q.ny << ',' << q.P << ',' << q.nu;
    }
    return k.str();
}

// Time every projector and back-projector variant on this batch (same
// outputs; the solve overwrites them afterwards) and keep the fastest.
int autotune(const Plan &P, const Dev &d, Tiles &tl, hipStream_t s) {
    hipEvent_t ev[2 * (kBProjVariants + kBBackVariants) + 2];
    const int nev = (int)(sizeof(ev) / sizeof(ev[0]));
    for (int i = 0; i < nev; ++i) ev[i] = nullptr;
    int rc = CT_OK;
    auto cleanup = [&]() {
        for (int i = 0; i < nev; ++i)
            if (ev[i]) (void)hipEventDestroy(ev[i]);
    };
    for (int i = 0; i < nev; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) {
            cleanup();
            set_error("ct_ba_gmres_batched: hipEventCreate failed");
            return CT_ERR_HIP;
        }
    hipLaunchKernelGGL(k_bzero_i32, dim3(grid1(16 * (size_t)P.count)), dim3(256), 0, s, d.flags, 16 * P.count);
    if (hipGetLastError() != hipSuccess) {
        cleanup();
        set_error("ct_ba_gmres_batched: kernel launch failed");
        return CT_ERR_HIP;
    }
    if ((rc = launch_fill(d.pad, P.pad_elems, 0.0f, s)) != CT_OK) { cleanup(); return rc; }
    if ((rc = launch_fill(d.W, P.NI, 0.0f, s)) != CT_OK) { cleanup(); return rc; }
    int e = 0;
    for (int v = 0; v < kBBackVariants && rc == CT_OK; ++v) {
        rc = launch_bbackproject2d(d.sl, P.count, d.pf(PFX_PIX0 + v, P.count), P.total_blocks(PFX_PIX0 + v), v,
                                   nullptr, d.W, s);   // warm-up
        if (rc == CT_OK && hipEventRecord(ev[e], s) != hipSuccess) rc = CT_ERR_HIP;
        for (int r = 0; r < 2 && rc == CT_OK; ++r)
            rc = launch_bbackproject2d(d.sl, P.count, d.pf(PFX_PIX0 + v, P.count), P.total_blocks(PFX_PIX0 + v), v,
                                       nullptr, d.W, s);
        if (rc == CT_OK && hipEventRecord(ev[e + 1], s) != hipSuccess) rc = CT_ERR_HIP;
        e += 2;
    }
    if (rc == CT_OK)
        rc = launch_bpad_copy(d.sl, P.count, d.pf(PFX_PAD, P.count), P.total_blocks(PFX_PAD), d.W, d.pad, s);
    for (int v = 0; v < kBProjVariants && rc == CT_OK; ++v) {
        rc = launch_bproject2d(d.sl, P.count, d.pf(PFX_RAY, P.count), P.total_blocks(PFX_RAY), v, d.pad,
                               P.pad_elems, d.q, s);
        if (rc == CT_OK && hipEventRecord(ev[e], s) != hipSuccess) rc = CT_ERR_HIP;
        for (int r = 0; r < 2 && rc == CT_OK; ++r)
            rc = launch_bproject2d(d.sl, P.count, d.pf(PFX_RAY, P.count), P.total_blocks(PFX_RAY), v, d.pad,
                                   P.pad_elems, d.q, s);
        if (rc == CT_OK && hipEventRecord(ev[e + 1], s) != hipSuccess) rc = CT_ERR_HIP;
        e += 2;
    }
    if (rc == CT_OK && hipEventSynchronize(ev[e - 1]) != hipSuccess) rc = CT_ERR_HIP;
    if (rc != CT_OK) {
        cleanup();
        if (rc == CT_ERR_HIP) set_error("ct_ba_gmres_batched: autotuning failed");
        return rc;
    }
    float best_b = 1e30f, best_a = 1e30f;
    e = 0;
    for (int v = 0; v < kBBackVariants; ++v, e += 2) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, ev[e], ev[e + 1]);
        if (ms < best_b) { best_b = ms; tl.b = v; }
    }
    for (int v = 0; v < kBProjVariants; ++v, e += 2) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, ev[e], ev[e + 1]);
        if (ms < best_a) { best_a = ms; tl.a = v; }
    }
    cleanup();
    return CT_OK;
}

hipStream_t capture_stream(int dev) {
    auto it = g_cap_streams.find(dev);
    if (it != g_cap_streams.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    g_cap_streams[dev] = s;
    return s;
}

void drop_graph() {
    if (g_graph.exec) (void)hipGraphExecDestroy(g_graph.exec);
    if (g_graph.graph) (void)hipGraphDestroy(g_graph.graph);
    g_graph = GraphEntry{};
}

// Capture the solve on a private stream into a graph (or reuse the cached
// one for the same batch shape, workspace and options).
int graph_for(const std::string &key, int dev, const Plan &P, const Dev &d, const Tiles &tl, double tol,
              hipGraphExec_t &exec) {
    if (g_graph.exec && g_graph.key == key && g_graph.device == dev) {
        exec = g_graph.exec;
        return CT_OK;
    }
    drop_graph();
    hipStream_t cs = capture_stream(dev);
    if (!cs) {
        set_error("ct_ba_gmres_batched: cannot create the capture stream");
        return CT_ERR_HIP;
    }
    CT_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    ProfScope::suppress(true);
    const int rc = enqueue_solve(P, d, tl, tol, cs);
    ProfScope::suppress(false);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (rc != CT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ec != hipSuccess || !graph) {
        set_error(std::string("ct_ba_gmres_batched: graph capture failed: ") + hipGetErrorString(ec));
        if (graph) (void)hipGraphDestroy(graph);
        return CT_ERR_HIP;
    }
    hipGraphExec_t ge = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(graph);
        set_error(std::string("ct_ba_gmres_batched: graph instantiation failed: ") + hipGetErrorString(ei));
        return CT_ERR_HIP;
    }
    g_graph.key = key;
    g_graph.device = dev;
    g_graph.graph = graph;
    g_graph.exec = ge;
    exec = ge;
    return CT_OK;
}

int check_batched(const ct_geometry *const *g, int count, const ct_solver_opts *o) {
    CT_ARG_CHECK(o != nullptr, "ct_ba_gmres_batched: NULL options");
    CT_ARG_CHECK(count >= 0 && count <= kMaxBatch, "ct_ba_gmres_batched: count out of range");
    CT_ARG_CHECK(count == 0 || g != nullptr, "ct_ba_gmres_batched: NULL geometry array");
    CT_ARG_CHECK(o->iters >= 0, "ct_ba_gmres_batched: iters must be >= 0");
    if (o->iters + 1 > kMaxVec) {
        set_error("ct_ba_gmres_batched: GMRES supports at most 56 iterations");
        return CT_ERR_UNSUPPORTED;
    }
    CT_ARG_CHECK(o->B == CT_B_UNMATCHED || o->B == CT_B_RAMP || o->B == CT_B_AT, "ct_ba_gmres_batched: unknown B");
    if (o->B == CT_B_AT) {
        set_error("ct_ba_gmres_batched: B = A^T is not batched (use ct_ba_gmres per problem)");
        return CT_ERR_UNSUPPORTED;
    }
    CT_ARG_CHECK(o->sino_dtype == CT_F32 || o->sino_dtype == CT_F16, "ct_ba_gmres_batched: bad sino_dtype");
    if (o->sino_dtype != CT_F32) {
        set_error("ct_ba_gmres_batched: FP16 data storage is not batched");
        return CT_ERR_UNSUPPORTED;
    }
    CT_ARG_CHECK(o->basis_dtype == CT_F32 || o->basis_dtype == CT_F16, "ct_ba_gmres_batched: bad basis_dtype");
    if (o->basis_dtype != CT_F32) {
        set_error("ct_ba_gmres_batched: FP16 basis storage is not batched");
        return CT_ERR_UNSUPPORTED;
    }
    CT_ARG_CHECK(o->breakdown_tol >= 0.0 && std::isfinite(o->breakdown_tol), "ct_ba_gmres_batched: bad breakdown_tol");
    return CT_OK;
}

}  // namespace
}  // namespace ct

using namespace ct;

extern "C" int ct_ba_gmres_batched_workspace_bytes(const ct_geometry *const *g, int count,
                                                   const ct_solver_opts *opts, size_t *bytes) {
    clear_error();
    CT_ARG_CHECK(bytes != nullptr, "ct_ba_gmres_batched_workspace_bytes: NULL bytes");
    CT_TRY(check_batched(g, count, opts));
    if (count == 0) {
        *bytes = 0;
        return CT_OK;
    }
    Plan P;
    CT_TRY(make_plan(g, count, *opts, P));
    *bytes = P.total;
    return CT_OK;
}

extern "C" int ct_ba_gmres_batched(const ct_geometry *const *g, int count, const float *const *b, float *const *x,
                                   const ct_solver_opts *opts, void *ws, size_t ws_bytes, double *res_hist,
                                   int *iters_done, void *stream) {
    clear_error();
    CT_TRY(check_batched(g, count, opts));
    if (count == 0) return CT_OK;
    CT_ARG_CHECK(b && x, "ct_ba_gmres_batched: NULL b or x array");
    for (int i = 0; i < count; ++i) CT_ARG_CHECK(b[i] && x[i], "ct_ba_gmres_batched: NULL b[i] or x[i]");
    Plan P;
    CT_TRY(make_plan(g, count, *opts, P));
    CT_ARG_CHECK(ws != nullptr && ws_bytes >= P.total, "ct_ba_gmres_batched: workspace too small");
    int dev = -1;
    CT_HIP_CHECK(hipGetDevice(&dev));
    for (int i = 0; i < count; ++i)
        CT_ARG_CHECK(g[i]->device == dev, "ct_ba_gmres_batched: geometry created on another device");
    hipStream_t s = (hipStream_t)stream;
    const double tol = opts->breakdown_tol > 0.0 ? opts->breakdown_tol : 64.0 * 5.9604644775390625e-08;
    Dev d = carve(P, ws);

    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<char> tab = build_tables(P, d, ws, g, b, x);
    CT_HIP_CHECK(hipMemcpyAsync((char *)ws + P.o_tab, tab.data(), tab.size(), hipMemcpyHostToDevice, s));

    const std::string shape = shape_key(g, count, opts->B);
    Tiles tl;
    if (g_force_a >= 0 && g_force_b >= 0) {
        tl.a = g_force_a;
        tl.b = g_force_b;
    } else {
        auto it = g_tuned.find(shape);
        if (it == g_tuned.end()) {
            CT_TRY(autotune(P, d, tl, s));
            g_tuned[shape] = tl;
        } else {
            tl = it->second;
        }
        if (g_force_a >= 0) tl.a = g_force_a;
        if (g_force_b >= 0) tl.b = g_force_b;
    }
    g_last_a = tl.a;
    g_last_b = tl.b;
    g_last_graph = g_use_graph;

    if (g_use_graph) {
        std::ostringstream key;
        // tol is baked into the captured kernel arguments: key on its exact bits
        uint64_t tol_bits;
        std::memcpy(&tol_bits, &tol, sizeof(tol_bits));
        key << shape << '|' << ws << '|' << P.K << '|' << std::hex << tol_bits << std::dec << '|' << tl.a
            << ',' << tl.b;
        hipGraphExec_t exec = nullptr;
        CT_TRY(graph_for(key.str(), dev, P, d, tl, tol, exec));
        CT_HIP_CHECK(hipGraphLaunch(exec, s));
    } else {
        CT_TRY(enqueue_solve(P, d, tl, tol, s));
    }

    // per-problem flags and residual histories back to the host
    const int K = P.K, K2 = K + 2;
    std::vector<int> flags(16 * (size_t)count);
    std::vector<double> vecs((size_t)count * K2 * 8);
    CT_HIP_CHECK(hipMemcpyAsync(flags.data(), d.flags, sizeof(int) * flags.size(), hipMemcpyDeviceToHost, s));
    CT_HIP_CHECK(hipMemcpyAsync(vecs.data(), (char *)ws + P.o_vec, sizeof(double) * vecs.size(),
                                hipMemcpyDeviceToHost, s));
    CT_HIP_CHECK(hipStreamSynchronize(s));
    int bad = -1;
    for (int i = 0; i < count; ++i) {
        const int kd = flags[16 * (size_t)i + F_KDONE];
        if (iters_done) iters_done[i] = kd;
        if (res_hist) {
            const double *res = vecs.data() + (size_t)i * K2 * 8 + 7 * (size_t)K2;
            for (int j = 0; j <= K; ++j) res_hist[(size_t)i * (K + 1) + j] = j <= kd ? res[j] : NAN;
        }
        if (flags[16 * (size_t)i + F_STATUS] != CT_OK && bad < 0) bad = i;
    }
    if (bad >= 0) {
        set_error("ct_ba_gmres_batched: non-finite value encountered in problem " + std::to_string(bad));
        return CT_ERR_NUMERIC;
    }
    return CT_OK;
}

extern "C" int ct_batched_config(int use_graph, int a_variant, int b_variant) {
    clear_error();
    CT_ARG_CHECK(a_variant >= -1 && a_variant < kBProjVariants, "ct_batched_config: bad projector variant");
    CT_ARG_CHECK(b_variant >= -1 && b_variant < kBBackVariants, "ct_batched_config: bad back-projector variant");
    std::lock_guard<std::mutex> lk(g_mu);
    g_use_graph = use_graph != 0;
    g_force_a = a_variant;
    g_force_b = b_variant;
    return CT_OK;
}

extern "C" int ct_batched_last_config(int *use_graph, int *a_variant, int *b_variant) {
    clear_error();
    CT_ARG_CHECK(use_graph && a_variant && b_variant, "ct_batched_last_config: NULL argument");
    std::lock_guard<std::mutex> lk(g_mu);
    *use_graph = g_last_graph;
    *a_variant = g_last_a;
    *b_variant = g_last_b;
    return CT_OK;
}
