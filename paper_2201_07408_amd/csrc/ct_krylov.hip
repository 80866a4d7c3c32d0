// Krylov solvers of the ABBA method on gfx950: BA-GMRES (Eq. 5), AB-GMRES
// (Eq. 4) and CGLS (Eq. 2), with the orthonormalisation and least-squares
// update of Sec. II (x0 = 0, first basis vector the normalised right-hand
// side, one new basis vector and one small least-squares solve per step).
//
// Device-resident design: the host enqueues every step of every iteration
// on the caller's stream without waiting; all scalars (dot products, norms,
// the Hessenberg matrix, the Givens rotations, the triangular solve) live in
// FP64 in the workspace, and a device flag stops the remaining kernels after
// a breakdown.  The basis is FP32 and stored "raw": basis vector j is
// sc[j] * W[j], so no kernel has to rescale a whole vector.
//
// Orthonormalisation is classical Gram-Schmidt applied twice (CGS2):
//   pass 1: d1 = W^T z, ||z||^2                 (one sweep over W)
//   pass 2: z1 = z - W h1,  d2 = W^T z1          (one fused sweep; with more
//           than one chunk of basis vectors, the earlier chunks are read a
//           second time for their dots)
//   pass 3: z2 = z1 - W h2, ||z2||^2             (one sweep)
// Each sweep streams chunks of up to 16 basis vectors with 16-byte loads
// and accumulates in FP64.  Per-block partial sums go to a column-major
// [column][block] table that a one-workgroup kernel reduces in a fixed order
// (deterministic, no float atomics) before running the scalar step.
#include <cmath>
#include <cstring>
#include <type_traits>

#include "ct_krylov_dev.h"

namespace ct {
namespace {

using namespace kry;

constexpr int kTile = 256;       // float4 groups per block per grid-stride step

// -------------------------------------------------------- sweep kernels
// CGS2 runs as streaming passes over chunks of at most NV basis vectors:
//   k_mdot:  partial d[j] = W[j] . z for the chunk (columns vlo + j), and
//            optionally ||z||^2 (column ncol);
//   k_maxpy: z' = zs z - sum_j coef[j] W[j] for the chunk, in place or to a
//            new array, optionally with ||z'||^2 (column ncol).
// Work-items stride over 16-byte groups of four elements (the last partial
// group goes element by element), every basis vector of the chunk is read
// once per pass with 16-byte loads, and all sums accumulate in FP64.
template <int NV, typename WT, bool NT>
__global__ __launch_bounds__(256) void k_mdot(const WT *__restrict__ W, size_t ldw, int vlo, int cnt,
                                              const float *__restrict__ z, size_t n, int nrm, int ncol,
                                              double *__restrict__ partials, const int *__restrict__ stop) {
    if (stop && *stop) return;
    double acc[NV], nacc = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    const WT *Wc = W + (size_t)vlo * ldw;
    constexpr int GE = Group<WT>::n;   // elements per group
    const size_t n4 = n / GE;
    mdot_groups<NV, WT, NT>(Wc, ldw, cnt, z, (size_t)blockIdx.x * 256, n4, (size_t)gridDim.x * 256, acc, nacc);
    if (blockIdx.x == 0 && threadIdx.x == 0)   // tail of fewer than four elements
        for (size_t i = n4 * GE; i < n; ++i) {
            const double zd = z[i];
            nacc += zd * zd;
#pragma unroll
            for (int j = 0; j < NV; ++j)
                if (j < cnt) acc[j] += (double)ld_elem(Wc + (size_t)j * ldw, i) * zd;
        }
    block_partials<NV>(acc, cnt, nacc, nrm != 0, vlo, ncol, partials, kMaxBlk, blockIdx.x);
}

// OT = __half stores the result as FP16 of oscale[0] * z' (the last pass of
// an FP16-basis CGS2 step writing the new basis vector).
template <int NV, typename WT, typename OT, bool NT>
__global__ __launch_bounds__(256) void k_maxpy(const WT *__restrict__ W, size_t ldw, int vlo, int cnt,
                                               const float *zin, OT *zout, size_t n,
                                               const double *__restrict__ coef, const double *__restrict__ zscale,
                                               const double *__restrict__ oscale, int nrm, int ncol,
                                               double *__restrict__ partials, const int *__restrict__ stop) {
    if (stop && *stop) return;
    __shared__ double cf[NV];
    for (int j = threadIdx.x; j < cnt; j += 256) cf[j] = coef[vlo + j];
    __syncthreads();
    const double zs = zscale ? *zscale : 1.0;
    const float os = oscale ? (float)*oscale : 1.0f;
    double nacc = 0.0;
    const WT *Wc = W + (size_t)vlo * ldw;
    constexpr int GE = Group<WT>::n;   // elements per group
    const size_t n4 = n / GE;
    maxpy_groups<NV, WT, OT, NT>(Wc, ldw, cnt, cf, zs, zin, zout, os, (size_t)blockIdx.x * 256, n4, (size_t)gridDim.x * 256,
                     nacc);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (size_t i = n4 * GE; i < n; ++i) {
            double u = zs * (double)zin[i];
            for (int j = 0; j < cnt; ++j) u -= cf[j] * (double)ld_elem(Wc + (size_t)j * ldw, i);
            const float o = (float)u;
            st_elem(zout, i, o, os);
            nacc += (double)o * o;
        }
    double acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    block_partials<NV>(acc, 0, nacc, nrm != 0, vlo, ncol, partials, kMaxBlk, blockIdx.x);
}

// z' = zs z - sum_j coef[j] W[j] and partial d[j] = W[j] . z' for one chunk
// in a single sweep (the second pass of CGS2 for the chunk that completes
// z'; the dots of earlier chunks need the finished z' and take k_mdot).
// With an FP16 basis it also sums ||z'||^2 into column ncol.  It holds a
// chunk's basis groups in registers, so fewer of its blocks are resident
// than of the other sweeps; it may run on fewer blocks than the nslot
// partial slots the reductions read, and the slots past its grid get zeros.
template <int NV, typename WT, bool NT>
__global__ __launch_bounds__(256) void k_maxpy_dot(const WT *__restrict__ W, size_t ldw, int vlo, int cnt,
                                                   const float *zin, float *zout, size_t n,
                                                   const double *__restrict__ coef,
                                                   const double *__restrict__ zscale, int ncol,
                                                   double *__restrict__ partials, int nslot,
                                                   const int *__restrict__ stop) {
    constexpr bool kNrm = std::is_same<WT, __half>::value;
    if (stop && *stop) return;
    __shared__ double cf[NV];
    for (int j = threadIdx.x; j < cnt; j += 256) cf[j] = coef[vlo + j];
    __syncthreads();
    const double zs = zscale ? *zscale : 1.0;
    double acc[NV], nacc = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.0;
    const WT *Wc = W + (size_t)vlo * ldw;
    constexpr int GE = Group<WT>::n;   // elements per group
    const size_t n4 = n / GE;
    maxpy_dot_groups<NV, WT, NT>(Wc, ldw, cnt, cf, zs, zin, zout, (size_t)blockIdx.x * 256, n4, (size_t)gridDim.x * 256,
                         acc, nacc);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (size_t i = n4 * GE; i < n; ++i) {
            double u = zs * (double)zin[i];
            for (int j = 0; j < cnt; ++j) u -= cf[j] * (double)ld_elem(Wc + (size_t)j * ldw, i);
            const float o = (float)u;
            zout[i] = o;
            nacc += (double)o * o;
#pragma unroll
            for (int j = 0; j < NV; ++j)
                if (j < cnt) acc[j] += (double)ld_elem(Wc + (size_t)j * ldw, i) * (double)o;
        }
    block_partials<NV>(acc, cnt, nacc, kNrm, vlo, ncol, partials, kMaxBlk, blockIdx.x);
    for (int slot = gridDim.x + blockIdx.x; slot < nslot; slot += gridDim.x) {
        for (int j = threadIdx.x; j < cnt; j += 256) partials[(size_t)(vlo + j) * kMaxBlk + slot] = 0.0;
        if (kNrm && threadIdx.x == 0) partials[(size_t)ncol * kMaxBlk + slot] = 0.0;
    }
}

__global__ void k_gmres_init(KState st, int nblk, double qscale_c, double blen) {
    __shared__ double d[1];
    gmres_init(st, nblk, qscale_c, d, blen);
}

__global__ void k_gmres_red1(KState st, int nblk, int k) {
    extern __shared__ double d[];
    if (st.flags[F_STOP]) return;
    gmres_red1(st, nblk, k, d);
}

__global__ void k_gmres_red2(KState st, int nblk, int k, double blen) {
    extern __shared__ double d[];
    if (st.flags[F_STOP]) return;
    gmres_red2(st, nblk, k, d, blen);
}

__global__ void k_gmres_red3(KState st, int nblk, int k, double tol, double qscale_c) {
    __shared__ double d[1];
    if (st.flags[F_STOP]) return;
    gmres_red3(st, nblk, k, tol, qscale_c, d);
}

__global__ void k_gmres_trsv(KState st) { gmres_trsv(st); }

// out = sum_{j < k_done} coef[j] W[j] (or out + that sum), FP64 accumulation
template <typename WT>
__global__ __launch_bounds__(256) void k_combine(const WT *__restrict__ W, size_t ldw, size_t n,
                                                 KState st, float *__restrict__ out, int accumulate) {
    __shared__ double cf[kMaxVec + 1];
    const int kd = st.flags[F_KDONE];
    for (int j = threadIdx.x; j < kd; j += blockDim.x) cf[j] = st.coef[j];
    __syncthreads();
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        double a = accumulate ? (double)out[i] : 0.0;
        for (int j = 0; j < kd; ++j) a += cf[j] * (double)ld_elem(W + (size_t)j * ldw, i);
        out[i] = (float)a;
    }
}

// ----------------------------------------------------- monitoring
// Per-iteration curves of BA-GMRES without extra applications of A: the
// projections q_j = A W[j] are kept (Q), and after step k the coefficients
// c of the current iterate x_{k+1} = sum_j c_j W[j] give
//   ||b - A x_{k+1}|| = ||b - sum_j c_j Q[j]||  and  x_{k+1} - x_ref.
// Each kernel runs only if step k completed (k_done == k + 1, status OK).
__device__ __forceinline__ bool mon_active(const KState &st, int k) {
    return st.flags[F_KDONE] == k + 1 && st.flags[F_STATUS] == CT_OK;
}

// c = R^-1 g for the first k+1 columns, scaled to the raw basis
__global__ void k_mon_coef(KState st, int k, double *__restrict__ cd) {
    if (threadIdx.x != 0 || !mon_active(st, k)) return;
    const int kd = k + 1, K1 = st.K + 1;
    for (int i = kd - 1; i >= 0; --i) {
        double sum = st.gv[i];
        for (int j = i + 1; j < kd; ++j) sum -= st.H[(size_t)j * K1 + i] * cd[j];
        cd[i] = sum / st.H[(size_t)i * K1 + i];
    }
    for (int i = 0; i < kd; ++i) cd[i] *= st.sc[i];
}

// block partials of sum_i (base_i - sum_{j<=k} c_j V[j][i])^2 (FP64)
__global__ __launch_bounds__(256) void k_mon_resid(const float *__restrict__ base, const float *__restrict__ V,
                                                   size_t ldv, size_t n, int k, KState st,
                                                   const double *__restrict__ cd, double *__restrict__ partials) {
    if (!mon_active(st, k)) return;
    __shared__ double cf[kMaxVec];
    __shared__ double red[4];
    const int kd = k + 1;
    for (int j = threadIdx.x; j < kd; j += 256) cf[j] = cd[j];
    __syncthreads();
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        double r = base ? (double)base[i] : 0.0;
        for (int j = 0; j < kd; ++j) r -= cf[j] * (double)V[(size_t)j * ldv + i];
        acc += r * r;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// The same sums with four consecutive elements per work-item: 16-byte
// loads of every vector, four vectors' loads in flight, and per element the
// same order of FP64 operations (base, then the terms j = 0, 1, ...).  base
// (if any) and V 16-byte aligned, ldv a multiple of four.
__global__ __launch_bounds__(256) void k_mon_resid4(const float *__restrict__ base, const float *__restrict__ V,
                                                    size_t ldv, size_t n, int k, KState st,
                                                    const double *__restrict__ cd, double *__restrict__ partials) {
    if (!mon_active(st, k)) return;
    __shared__ double cf[kMaxVec];
    __shared__ double red[4];
    const int kd = k + 1;
    for (int j = threadIdx.x; j < kd; j += 256) cf[j] = cd[j];
    __syncthreads();
    double acc = 0.0;
    const size_t n4 = n / 4;
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n4; q += (size_t)gridDim.x * 256) {
        double r[4] = {0.0, 0.0, 0.0, 0.0};
        if (base) {
            const float4 bb = reinterpret_cast<const float4 *>(base)[q];
            r[0] = bb.x; r[1] = bb.y; r[2] = bb.z; r[3] = bb.w;
        }
        int j = 0;
        for (; j + 4 <= kd; j += 4) {
            float4 v[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) v[t] = reinterpret_cast<const float4 *>(V + (size_t)(j + t) * ldv)[q];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double c = cf[j + t];
                r[0] -= c * (double)v[t].x; r[1] -= c * (double)v[t].y;
                r[2] -= c * (double)v[t].z; r[3] -= c * (double)v[t].w;
            }
        }
        for (; j < kd; ++j) {
            const float4 v = reinterpret_cast<const float4 *>(V + (size_t)j * ldv)[q];
            const double c = cf[j];
            r[0] -= c * (double)v.x; r[1] -= c * (double)v.y;
            r[2] -= c * (double)v.z; r[3] -= c * (double)v.w;
        }
        acc += (r[0] * r[0] + r[1] * r[1]) + (r[2] * r[2] + r[3] * r[3]);
    }
    if (blockIdx.x == 0 && (size_t)threadIdx.x < n - 4 * n4) {   // the last n mod 4 elements
        const size_t i = 4 * n4 + threadIdx.x;
        double r = base ? (double)base[i] : 0.0;
        for (int j = 0; j < kd; ++j) r -= cf[j] * (double)V[(size_t)j * ldv + i];
        acc += r * r;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out[k+1] = sqrt(sum / div)
__global__ void k_mon_store(const double *__restrict__ partials, int nblk, int k, KState st, double div,
                            double *__restrict__ out) {
    __shared__ double d[1];
    if (!mon_active(st, k)) return;
    reduce_partials(partials, kMaxBlk, nblk, 1, d);
    __syncthreads();
    if (threadIdx.x == 0) out[k + 1] = sqrt(d[0] / div);
}

// r = b - q
__global__ __launch_bounds__(256) void k_residual(const float *__restrict__ b, const float *__restrict__ q,
                                                  float *__restrict__ r, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        r[i] = b[i] - q[i];
}

// ------------------------------------------------------------- CGLS
__global__ __launch_bounds__(256) void k_sumsq(const float *__restrict__ v, size_t n,
                                               double *__restrict__ partials,
                                               const int *__restrict__ stop) {
    if (stop && *stop) return;
    double a = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        a += (double)v[i] * (double)v[i];
    a = wave_sum(a);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void k_zero_i32(int *p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

__global__ void k_copy(const float *__restrict__ a, float *__restrict__ b, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// stage 0: res[0] = ||b||;  stage 1: gamma = ||s||^2 (start)
__global__ void k_cgls_start(KState st, int nblk, int stage) {
    __shared__ double d[1];
    reduce_partials(st.partials, st.pstride, nblk, 1, d);
    __syncthreads();
    if (threadIdx.x != 0) return;
    if (stage == 0) {
        st.flags[F_KDONE] = 0;
        st.flags[F_STOP] = 0;
        st.flags[F_STATUS] = CT_OK;
        st.res[0] = sqrt(d[0]);
        if (!isfinite(st.res[0])) {
            st.flags[F_STOP] = 1;
            st.flags[F_STATUS] = CT_ERR_NUMERIC;
        }
    } else {
        st.misc[M_GAMMA] = d[0];
        if (!(d[0] > 0.0)) st.flags[F_STOP] = 1;
        if (!isfinite(d[0])) st.flags[F_STATUS] = CT_ERR_NUMERIC;
    }
}

// alpha = gamma / ||q||^2
__global__ void k_cgls_alpha(KState st, int nblk) {
    __shared__ double d[1];
    if (st.flags[F_STOP]) return;
    reduce_partials(st.partials, st.pstride, nblk, 1, d);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double a = st.misc[M_GAMMA] / d[0];
    if (!(d[0] > 0.0) || !isfinite(a)) {
        st.flags[F_STOP] = 1;
        if (!isfinite(d[0])) st.flags[F_STATUS] = CT_ERR_NUMERIC;
        return;
    }
    st.misc[M_AB] = a;
}

// x += alpha p (n), r -= alpha q (m)
__global__ __launch_bounds__(256) void k_cgls_xr(float *__restrict__ x, const float *__restrict__ p, size_t n,
                                                 float *__restrict__ r, const float *__restrict__ q, size_t m,
                                                 KState st) {
    if (st.flags[F_STOP]) return;
    const double a = st.misc[M_AB];
    const size_t tot = n + m;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (size_t)gridDim.x * blockDim.x) {
        if (i < n) x[i] = (float)((double)x[i] + a * (double)p[i]);
        else {
            const size_t k = i - n;
            r[k] = (float)((double)r[k] - a * (double)q[k]);
        }
    }
}

// residual history after the r update (partials of ||r||^2)
__global__ void k_cgls_res(KState st, int nblk, int k) {
    __shared__ double d[1];
    if (st.flags[F_STOP]) return;
    reduce_partials(st.partials, st.pstride, nblk, 1, d);
    __syncthreads();
    if (threadIdx.x != 0) return;
    st.res[k + 1] = sqrt(d[0]);
    st.flags[F_KDONE] = k + 1;
}

// beta = gamma'/gamma, gamma = gamma'
__global__ void k_cgls_beta(KState st, int nblk) {
    __shared__ double d[1];
    if (st.flags[F_STOP]) return;
    reduce_partials(st.partials, st.pstride, nblk, 1, d);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double gnew = d[0];
    if (!isfinite(gnew)) {
        st.flags[F_STOP] = 1;
        st.flags[F_STATUS] = CT_ERR_NUMERIC;
        return;
    }
    st.misc[M_AB] = gnew / st.misc[M_GAMMA];
    st.misc[M_GAMMA] = gnew;
    if (gnew == 0.0) st.misc[M_AB] = 0.0;
}

// p = s + beta p
__global__ __launch_bounds__(256) void k_cgls_p(float *__restrict__ p, const float *__restrict__ s, size_t n,
                                                KState st) {
    if (st.flags[F_STOP]) return;
    const double b = st.misc[M_AB];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = (float)((double)s[i] + b * (double)p[i]);
}

}  // namespace

// ===================================================================== host
namespace {

int sweep_blocks(size_t n) {
    size_t t = (n + kTile - 1) / kTile;
    return (int)(t < (size_t)kMaxBlk ? (t == 0 ? 1 : t) : (size_t)kMaxBlk);
}

int grid_1d(size_t n) {
    size_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    return (int)b;
}

struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *p) : base((char *)p) {}
    template <typename T> T *take(size_t count) {
        T *p = base ? (T *)(base + off) : nullptr;
        off += align_up(count * sizeof(T));
        return p;
    }
};

struct GmresBufs {
    void *W = nullptr;      // (K+1) basis vectors of length len, stride ldw (FP32, or FP16 if w16)
    size_t ldw = 0, len = 0;
    bool w16 = false;
    float *wf(int j) const { return (float *)W + (size_t)j * ldw; }
    __half *wh(int j) const { return (__half *)W + (size_t)j * ldw; }
    OpScratch opA;          // padded copies
    void *q = nullptr;      // projections (BA) / image (AB)
    void *filt = nullptr;   // ramp-filtered data
    float *z = nullptr;     // raw new vector
    KState st{};
    // monitoring (BA-GMRES only)
    float *Q = nullptr;     // K projections A W[j], stride ldq
    size_t ldq = 0;
    double *mon_c = nullptr, *mon_data = nullptr, *mon_img = nullptr, *mon_part = nullptr;
};

// Carve (or size, when ws == nullptr) the GMRES workspace.
size_t carve_gmres(const ct_geometry *g, int solver, const ct_solver_opts &o, void *ws, GmresBufs &b,
                   bool monitor = false) {
    Carver c(ws);
    const int K = o.iters;
    const bool ba = solver == CT_SOLVER_BA;
    b.len = ba ? g->n_vox : g->n_rays;
    b.ldw = align_up(b.len, 64);
    b.w16 = o.basis_dtype == CT_F16;
    b.W = b.w16 ? (void *)c.take<__half>(b.ldw * (size_t)(K + 1)) : (void *)c.take<float>(b.ldw * (size_t)(K + 1));
    b.opA.vx = c.take<float>(g->pad.nvx);
    b.opA.vy = c.take<float>(g->pad.nvy);
    const size_t es = o.sino_dtype == CT_F16 ? 2 : 4;
    // filtered data (B_un F) or the step-weighted data of the cone-beam A^T
    const bool filt = o.B == CT_B_RAMP || (o.B == CT_B_AT && g->k.kind == CT_CONE_CIRCULAR_3D);
    if (ba) {
        b.q = c.take<char>(g->n_rays * es);
        // the first back-projection filters the FP32 data whatever the storage
        if (filt) b.filt = c.take<char>(g->n_rays * 4);
        b.z = c.take<float>(g->n_vox);
    } else {
        b.q = c.take<float>(g->n_vox);               // u = B w
        if (filt) b.filt = c.take<float>(g->n_rays);
        b.z = c.take<float>(g->n_rays);
    }
    b.opA.filt = b.filt;
    KState &s = b.st;
    s.K = K;
    s.pstride = kMaxBlk;
    s.flags = c.take<int>(16);
    s.H = c.take<double>((size_t)(K + 1) * (K > 0 ? K : 1));
    s.cs = c.take<double>(K + 1);
    s.sn = c.take<double>(K + 1);
    s.gv = c.take<double>(K + 2);
    s.sc = c.take<double>(K + 2);
    s.h1 = c.take<double>(K + 2);
    s.h2 = c.take<double>(K + 2);
    s.coef = c.take<double>(K + 2);
    s.res = c.take<double>(K + 2);
    s.misc = c.take<double>(8);
    s.fscale = c.take<float>(4);
    s.partials = c.take<double>((size_t)kMaxBlk * (K + 3));
    if (monitor) {
        b.ldq = align_up(g->n_rays, 64);
        b.Q = c.take<float>(b.ldq * (size_t)(K > 0 ? K : 1));
        b.mon_c = c.take<double>(K + 2);
        b.mon_data = c.take<double>(K + 2);
        b.mon_img = c.take<double>(K + 2);
        b.mon_part = c.take<double>(kMaxBlk);
    }
    return c.off;
}

constexpr int kCgsChunk = 16;   // basis vectors per streaming pass (register budget)

// Whether the basis vectors 0 .. nvec-1 exceed the 256 MB last-level cache:
// then a sweep's loads of them are non-temporal (measured at 256^3: sweeps
// 0.795 -> 0.777 ms per iteration; where the basis fits, as for 2D slices,
// the ordinary loads keep it cached between the passes).
static bool basis_beyond_llc(const GmresBufs &b, int nvec) {
    return (double)nvec * (double)b.len * (b.w16 ? 2.0 : 4.0) > 256.0 * 1024 * 1024;
}

static int launch_mdot(const GmresBufs &b, int vlo, int cnt, const float *z, bool nrm, int ncol, hipStream_t s) {
    ProfScope prof(PROF_CGS, s);
    const int nblk = sweep_blocks(b.len / 4 + 1);
    const int *stop = b.st.flags + F_STOP;
    const bool nt = basis_beyond_llc(b, vlo + cnt);
#define CT_MDOT(NVV, WT, WP) \
    do { \
        if (nt) hipLaunchKernelGGL((k_mdot<NVV, WT, true>), dim3(nblk), dim3(256), 0, s, WP, b.ldw, vlo, cnt, z, \
                                   b.len, (int)nrm, ncol, b.st.partials, stop); \
        else hipLaunchKernelGGL((k_mdot<NVV, WT, false>), dim3(nblk), dim3(256), 0, s, WP, b.ldw, vlo, cnt, z, \
                                b.len, (int)nrm, ncol, b.st.partials, stop); \
    } while (0)
#define CT_MDOT_NV(WT, WP) \
    if (cnt <= 1) CT_MDOT(1, WT, WP); \
    else if (cnt <= 4) CT_MDOT(4, WT, WP); \
    else if (cnt <= 8) CT_MDOT(8, WT, WP); \
    else CT_MDOT(16, WT, WP);
    if (b.w16) { CT_MDOT_NV(__half, b.wh(0)) } else { CT_MDOT_NV(float, b.wf(0)) }
#undef CT_MDOT_NV
#undef CT_MDOT
    CT_LAUNCH_CHECK();
    return CT_OK;
}

// zout16 != nullptr: store the result as FP16 (scale st.misc[M_BT]) there
// instead of zout.
static int launch_maxpy(const GmresBufs &b, int vlo, int cnt, const float *zin, float *zout, const double *coef,
                        const double *zscale, bool nrm, int ncol, hipStream_t s, __half *zout16 = nullptr) {
    ProfScope prof(PROF_CGS, s);
    const int nblk = sweep_blocks(b.len / 4 + 1);
    const int *stop = b.st.flags + F_STOP;
    const double *os = b.st.misc + M_BT;
    const bool nt = basis_beyond_llc(b, vlo + cnt);
#define CT_MAXPY(NVV, WT, OT, WP, ZO) \
    do { \
        if (nt) hipLaunchKernelGGL((k_maxpy<NVV, WT, OT, true>), dim3(nblk), dim3(256), 0, s, WP, b.ldw, vlo, cnt, \
                                   zin, ZO, b.len, coef, zscale, os, (int)nrm, ncol, b.st.partials, stop); \
        else hipLaunchKernelGGL((k_maxpy<NVV, WT, OT, false>), dim3(nblk), dim3(256), 0, s, WP, b.ldw, vlo, cnt, \
                                zin, ZO, b.len, coef, zscale, os, (int)nrm, ncol, b.st.partials, stop); \
    } while (0)
#define CT_MAXPY_NV(WT, OT, WP, ZO) \
    if (cnt <= 1) CT_MAXPY(1, WT, OT, WP, ZO); \
    else if (cnt <= 4) CT_MAXPY(4, WT, OT, WP, ZO); \
    else if (cnt <= 8) CT_MAXPY(8, WT, OT, WP, ZO); \
    else CT_MAXPY(16, WT, OT, WP, ZO);
    if (!b.w16) { CT_MAXPY_NV(float, float, b.wf(0), zout) }
    else if (zout16) { CT_MAXPY_NV(__half, __half, b.wh(0), zout16) }
    else { CT_MAXPY_NV(__half, float, b.wh(0), zout) }
#undef CT_MAXPY_NV
#undef CT_MAXPY
    CT_LAUNCH_CHECK();
    return CT_OK;
}

// Blocks of `kern` (256 threads) resident on the current device at once.
template <typename Kern>
static int resident_blocks(Kern kern) {
    int dev = 0, per_cu = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

static int launch_maxpy_dot(const GmresBufs &b, int vlo, int cnt, const float *zin, float *zout, const double *coef,
                            const double *zscale, int ncol, hipStream_t s) {
    ProfScope prof(PROF_CGS, s);
    const int nblk = sweep_blocks(b.len / 4 + 1);
    const int *stop = b.st.flags + F_STOP;
    const bool nt = basis_beyond_llc(b, vlo + cnt);
    // one round of resident blocks where the sweep's grid would take a
    // second, partly filled one (16 FP32 basis vectors: 768 of 1024 blocks
    // resident on 256 CUs, 276 -> 212 us at 256^3)
#define CT_MAXPY_DOT_K(NVV, WT, NTV, WP) \
    do { \
        const int res = resident_blocks(k_maxpy_dot<NVV, WT, NTV>); \
        const int nb = res > 0 && res < nblk ? res : nblk; \
        hipLaunchKernelGGL((k_maxpy_dot<NVV, WT, NTV>), dim3(nb), dim3(256), 0, s, WP, b.ldw, vlo, cnt, zin, zout, \
                           b.len, coef, zscale, ncol, b.st.partials, nblk, stop); \
    } while (0)
#define CT_MAXPY_DOT(NVV, WT, WP) \
    do { \
        if (nt) CT_MAXPY_DOT_K(NVV, WT, true, WP); \
        else CT_MAXPY_DOT_K(NVV, WT, false, WP); \
    } while (0)
#define CT_MAXPY_DOT_NV(WT, WP) \
    if (cnt <= 1) CT_MAXPY_DOT(1, WT, WP); \
    else if (cnt <= 4) CT_MAXPY_DOT(4, WT, WP); \
    else if (cnt <= 8) CT_MAXPY_DOT(8, WT, WP); \
    else CT_MAXPY_DOT(16, WT, WP);
    if (b.w16) { CT_MAXPY_DOT_NV(__half, b.wh(0)) } else { CT_MAXPY_DOT_NV(float, b.wf(0)) }
#undef CT_MAXPY_DOT_NV
#undef CT_MAXPY_DOT
#undef CT_MAXPY_DOT_K
    CT_LAUNCH_CHECK();
    return CT_OK;
}

// Partial sums for every block of a pass land in the same columns, so every
// pass over a vector range uses the same number of blocks (sweep_blocks of
// len/4 + 1) and the reduction kernels read that many.
//   mode 0: d[j] = W[j].z (j < nvec) and ||z||^2 in column nvec
//   mode 1: z1 = zs z - sum coef W (to zout), then d[j] = W[j].z1 (FP16
//           basis: and ||z1||^2 in column nvec)
//   mode 2: z2 = z - sum coef W (to zout) and ||z2||^2 in column 0; with
//           zout16 the last chunk stores FP16 of st.misc[M_BT] * z2 there
int run_cgs(int mode, const GmresBufs &b, int nvec, const float *zin, float *zout, const double *coef,
            const double *zscale, hipStream_t s, __half *zout16 = nullptr) {
    if (mode == 0) {
        if (nvec == 0) return launch_mdot(b, 0, 0, zin, true, 0, s);
        for (int lo = 0; lo < nvec; lo += kCgsChunk) {
            const int cnt = nvec - lo < kCgsChunk ? nvec - lo : kCgsChunk;
            CT_TRY(launch_mdot(b, lo, cnt, zin, lo == 0, nvec, s));
        }
        return CT_OK;
    }
    if (nvec == 0) return launch_maxpy(b, 0, 0, zin, zout, coef, nullptr, true, 0, s);
    for (int lo = 0; lo < nvec; lo += kCgsChunk) {
        const int cnt = nvec - lo < kCgsChunk ? nvec - lo : kCgsChunk;
        const bool last = lo + cnt >= nvec;
        const float *src = lo == 0 ? zin : zout;
        const double *zsc = lo == 0 ? zscale : nullptr;
        if (mode == 1 && last) {
            // the chunk that completes z1 also takes its own dots
            CT_TRY(launch_maxpy_dot(b, lo, cnt, src, zout, coef, zsc, nvec, s));
        } else {
            CT_TRY(launch_maxpy(b, lo, cnt, src, zout, coef, zsc, mode == 2 && last, 0, s,
                                mode == 2 && last ? zout16 : nullptr));
        }
    }
    if (mode == 1)
        for (int lo = 0; lo + kCgsChunk < nvec; lo += kCgsChunk)   // every chunk but the last
            CT_TRY(launch_mdot(b, lo, kCgsChunk, zout, false, 0, s));
    return CT_OK;
}

int check_solver_args(const ct_geometry *g, int solver, const ct_solver_opts *o, const float *b, float *x,
                      void *ws, size_t ws_bytes, size_t &need) {
    CT_ARG_CHECK(g && o, "solver: NULL geometry or options");
    CT_ARG_CHECK(o->iters >= 0, "solver: iters must be >= 0");
    if (solver != CT_SOLVER_CGLS && o->iters + 1 > kMaxVec) {
        set_error("solver: GMRES supports at most 56 iterations");
        return CT_ERR_UNSUPPORTED;
    }
    CT_ARG_CHECK(o->B == CT_B_UNMATCHED || o->B == CT_B_RAMP || o->B == CT_B_AT, "solver: unknown B");
    CT_ARG_CHECK(o->sino_dtype == CT_F32 || o->sino_dtype == CT_F16, "solver: bad sino_dtype");
    CT_ARG_CHECK(o->breakdown_tol >= 0.0 && std::isfinite(o->breakdown_tol), "solver: bad breakdown_tol");
    CT_ARG_CHECK(b && x, "solver: NULL b or x");
    if (solver != CT_SOLVER_BA && o->sino_dtype == CT_F16) {
        set_error("solver: FP16 data storage is implemented for BA-GMRES only");
        return CT_ERR_UNSUPPORTED;
    }
    if (o->sino_dtype == CT_F16 && o->B == CT_B_AT) {
        set_error("solver: FP16 data storage is not implemented with B = A^T");
        return CT_ERR_UNSUPPORTED;
    }
    CT_ARG_CHECK(o->basis_dtype == CT_F32 || o->basis_dtype == CT_F16, "solver: bad basis_dtype");
    if (o->basis_dtype == CT_F16) {
        if (solver != CT_SOLVER_BA) {
            set_error("solver: FP16 basis storage is implemented for BA-GMRES only");
            return CT_ERR_UNSUPPORTED;
        }
        if (g->k.proj == CT_SIDDON && g->k.kind != CT_CONE_CIRCULAR_3D) {
            set_error("solver: FP16 basis storage is not implemented with the 2D line-intersection projector");
            return CT_ERR_UNSUPPORTED;
        }
    }
    if (o->B == CT_B_RAMP && g->k.nu * 16 > 64 * 1024) {
        set_error("solver: detector rows longer than 4096 are not supported by the ramp filter");
        return CT_ERR_UNSUPPORTED;
    }
    CT_ARG_CHECK(ws != nullptr && ws_bytes >= need, "solver: workspace too small");
    return CT_OK;
}

size_t carve_cgls(const ct_geometry *g, const ct_solver_opts &o, void *ws, float **r, float **q, float **sv,
                  float **p, OpScratch &op, KState &st) {
    Carver c(ws);
    *r = c.take<float>(g->n_rays);
    *q = c.take<float>(g->n_rays);
    *sv = c.take<float>(g->n_vox);
    *p = c.take<float>(g->n_vox);
    op.vx = c.take<float>(g->pad.nvx);
    op.vy = c.take<float>(g->pad.nvy);
    op.filt = o.B == CT_B_RAMP || (o.B == CT_B_AT && g->k.kind == CT_CONE_CIRCULAR_3D) ? c.take<float>(g->n_rays)
                                                                                     : nullptr;
    st.K = o.iters;
    st.pstride = kMaxBlk;
    st.flags = c.take<int>(16);
    st.res = c.take<double>(o.iters + 2);
    st.misc = c.take<double>(8);
    st.partials = c.take<double>((size_t)kMaxBlk * 4);
    st.H = st.cs = st.sn = st.gv = st.sc = st.h1 = st.h2 = st.coef = nullptr;
    st.fscale = nullptr;
    return c.off;
}

int finish(KState &st, int K, double *res_hist, int *iters_done, hipStream_t s) {
    int flags[3];
    std::vector<double> res(K + 1, 0.0);
    CT_HIP_CHECK(hipMemcpyAsync(flags, st.flags, sizeof(flags), hipMemcpyDeviceToHost, s));
    CT_HIP_CHECK(hipMemcpyAsync(res.data(), st.res, sizeof(double) * (K + 1), hipMemcpyDeviceToHost, s));
    CT_HIP_CHECK(hipStreamSynchronize(s));
    const int kd = flags[F_KDONE];
    if (iters_done) *iters_done = kd;
    if (res_hist) {
        for (int i = 0; i <= K; ++i) res_hist[i] = i <= kd ? res[i] : NAN;
    }
    if (flags[F_STATUS] != CT_OK) {
        set_error("solver: non-finite value encountered");
        return CT_ERR_NUMERIC;
    }
    return CT_OK;
}

// scale constant so that A applied to a unit-norm vector stores O(1) values
double fp16_scale_const(const ct_geometry *g) {
    const int nmax = g->k.nx > g->k.ny ? g->k.nx : g->k.ny;
    return std::sqrt((double)g->n_vox) / ((double)nmax * g->k.vox);
}

// Host side of the monitored solve: the curves to return (either may be
// NULL) and the reference image (device, may be NULL).
struct MonitorOut {
    const float *x_ref;
    double *data_res;
    double *img_rmse;
};

// b_i - sum c_j V[j]_i over n elements -> out[k+1] (divided by div inside the root)
static int mon_curve(const GmresBufs &bf, const float *base, const float *V, size_t ldv, size_t n, int k,
                     double div, double *out, hipStream_t s) {
    const bool vec = ((uintptr_t)base & 15) == 0 && ((uintptr_t)V & 15) == 0 && ldv % 4 == 0;
    const int ng = grid_1d(vec ? n / 4 + 1 : n);
    const int nblk = ng < kMaxBlk ? ng : kMaxBlk;
    if (vec)
        hipLaunchKernelGGL(k_mon_resid4, dim3(nblk), dim3(256), 0, s, base, V, ldv, n, k, bf.st, bf.mon_c,
                           bf.mon_part);
    else
        hipLaunchKernelGGL(k_mon_resid, dim3(nblk), dim3(256), 0, s, base, V, ldv, n, k, bf.st, bf.mon_c,
                           bf.mon_part);
    CT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mon_store, dim3(1), dim3(64), 0, s, bf.mon_part, nblk, k, bf.st, div, out);
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int gmres_impl(const ct_geometry *g, int solver, const float *b, float *x, const ct_solver_opts *o, void *ws,
               size_t ws_bytes, double *res_hist, int *iters_done, hipStream_t s,
               const MonitorOut *mon = nullptr, bool accumulate = false) {
    GmresBufs bf;
    size_t need = carve_gmres(g, solver, *o, nullptr, bf, mon != nullptr);
    CT_TRY(check_solver_args(g, solver, o, b, x, ws, ws_bytes, need));
    carve_gmres(g, solver, *o, ws, bf, mon != nullptr);
    const int K = o->iters;
    const double tol = o->breakdown_tol > 0.0 ? o->breakdown_tol : 64.0 * 5.9604644775390625e-08;
    const bool ba = solver == CT_SOLVER_BA;
    const bool f16 = o->sino_dtype == CT_F16;
    const int dt = f16 ? CT_F16 : CT_F32;
    const double qc = f16 ? fp16_scale_const(g) : 0.0;
    KState &st = bf.st;
    const int *stop = st.flags + F_STOP;
    const int nblk = sweep_blocks(bf.len / 4 + 1);
    OpScratch &op = bf.opA;
    // flags must start clear: the init kernel writes them, but the sweep that
    // precedes it reads the stop flag (a kernel, not a memset, so the chain
    // stays capturable)
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, st.flags, 16);
    CT_LAUNCH_CHECK();
    CT_TRY(launch_pad_zero(g, op.vx, op.vy, s));

    // FP16 basis: vectors of this length are stored scaled (gmres_red2)
    const double blen = bf.w16 ? (double)bf.len : 0.0;
    if (!bf.w16) {
        // r0 = B b (BA) or b (AB), stored raw as W[0]
        if (ba) CT_TRY(apply_B(g, o->B, b, CT_F32, bf.wf(0), op, nullptr, nullptr, s));
        else {
            hipLaunchKernelGGL(k_copy, dim3(grid_1d(bf.len)), dim3(256), 0, s, b, bf.wf(0), bf.len);
            CT_LAUNCH_CHECK();
        }
        CT_TRY(run_cgs(2, bf, 0, bf.wf(0), bf.wf(0), st.coef, nullptr, s));   // ||r0||^2 (no update)
        hipLaunchKernelGGL(k_gmres_init, dim3(1), dim3(256), 0, s, st, nblk, qc, 0.0);
        CT_LAUNCH_CHECK();
    } else {
        // r0 = B b in FP32, its norm, then W[0] = FP16 of t0 r0 (BA only)
        CT_TRY(apply_B(g, o->B, b, CT_F32, bf.z, op, nullptr, nullptr, s));
        CT_TRY(run_cgs(0, bf, 0, bf.z, nullptr, nullptr, nullptr, s));
        hipLaunchKernelGGL(k_gmres_init, dim3(1), dim3(256), 0, s, st, nblk, qc, blen);
        CT_LAUNCH_CHECK();
        CT_TRY(launch_maxpy(bf, 0, 0, bf.z, nullptr, nullptr, nullptr, false, 0, s, bf.wh(0)));
    }
    if (mon) {   // x_0 = 0: ||b|| and RMS(x_ref)
        CT_TRY(mon_curve(bf, b, bf.Q, bf.ldq, g->n_rays, -1, 1.0, bf.mon_data, s));
        if (mon->x_ref) CT_TRY(mon_curve(bf, mon->x_ref, bf.wf(0), bf.ldw, g->n_vox, -1, (double)g->n_vox, bf.mon_img, s));
    }

    const float *oscale = f16 ? st.fscale : nullptr;
    const float *iscale = f16 ? st.fscale + 1 : nullptr;
    for (int k = 0; k < K; ++k) {
        float *wk = bf.w16 ? nullptr : bf.wf(k);
        // FP32 basis: CGS2 builds the new vector in its basis slot; FP16:
        // in z, and its last pass stores the FP16 vector
        float *wn = bf.w16 ? bf.z : bf.wf(k + 1);
        const bool pad_ready = o->B != CT_B_AT;
        if (ba) {
            void *qk = mon ? (void *)(bf.Q + (size_t)k * bf.ldq) : bf.q;
            if (bf.w16) CT_TRY(apply_A(g, bf.wh(k), qk, dt, op, pad_ready, oscale, stop, s, CT_F16));
            else CT_TRY(apply_A(g, wk, qk, dt, op, pad_ready, oscale, stop, s));
            CT_TRY(apply_B(g, o->B, qk, dt, bf.z, op, iscale, stop, s));
        } else {
            CT_TRY(apply_B(g, o->B, wk, CT_F32, (float *)bf.q, op, nullptr, stop, s));
            CT_TRY(apply_A(g, (const float *)bf.q, bf.z, CT_F32, op, pad_ready, nullptr, stop, s));
        }
        const int nvec = k + 1;
        CT_TRY(run_cgs(0, bf, nvec, bf.z, nullptr, nullptr, nullptr, s));
        // one wavefront per column of block partials, sixteen wavefronts: the
        // column sums are latency-bound loops, and each column's order of
        // summation does not depend on the number of wavefronts
        hipLaunchKernelGGL(k_gmres_red1, dim3(1), dim3(1024), sizeof(double) * (nvec + 1), s, st, nblk, k);
        CT_LAUNCH_CHECK();
        CT_TRY(run_cgs(1, bf, nvec, bf.z, wn, st.coef, st.misc + M_ZS, s));
        hipLaunchKernelGGL(k_gmres_red2, dim3(1), dim3(1024), sizeof(double) * (nvec + 1), s, st, nblk, k, blen);
        CT_LAUNCH_CHECK();
        CT_TRY(run_cgs(2, bf, nvec, wn, wn, st.coef, nullptr, s, bf.w16 ? bf.wh(k + 1) : nullptr));
        hipLaunchKernelGGL(k_gmres_red3, dim3(1), dim3(64), 0, s, st, nblk, k, tol, qc);
        CT_LAUNCH_CHECK();
        if (mon) {
            hipLaunchKernelGGL(k_mon_coef, dim3(1), dim3(64), 0, s, st, k, bf.mon_c);
            CT_LAUNCH_CHECK();
            CT_TRY(mon_curve(bf, b, bf.Q, bf.ldq, g->n_rays, k, 1.0, bf.mon_data, s));
            if (mon->x_ref)
                CT_TRY(mon_curve(bf, mon->x_ref, bf.wf(0), bf.ldw, g->n_vox, k, (double)g->n_vox, bf.mon_img, s));
        }
    }
    hipLaunchKernelGGL(k_gmres_trsv, dim3(1), dim3(64), 0, s, st);
    CT_LAUNCH_CHECK();
    if (ba) {
        if (bf.w16)
            hipLaunchKernelGGL(k_combine<__half>, dim3(grid_1d(bf.len)), dim3(256), 0, s, bf.wh(0), bf.ldw, bf.len,
                               st, x, (int)accumulate);
        else
            hipLaunchKernelGGL(k_combine<float>, dim3(grid_1d(bf.len)), dim3(256), 0, s, bf.wf(0), bf.ldw, bf.len,
                               st, x, (int)accumulate);
        CT_LAUNCH_CHECK();
    } else {
        // x = B (W c): combine in data space, then back-project
        hipLaunchKernelGGL(k_combine<float>, dim3(grid_1d(bf.len)), dim3(256), 0, s, bf.wf(0), bf.ldw, bf.len, st,
                           bf.z, 0);
        CT_LAUNCH_CHECK();
        CT_TRY(apply_B(g, o->B, bf.z, CT_F32, x, op, nullptr, nullptr, s));
    }
    if (mon) {
        std::vector<double> dr(K + 1), im(K + 1);
        CT_HIP_CHECK(hipMemcpyAsync(dr.data(), bf.mon_data, sizeof(double) * (K + 1), hipMemcpyDeviceToHost, s));
        CT_HIP_CHECK(hipMemcpyAsync(im.data(), bf.mon_img, sizeof(double) * (K + 1), hipMemcpyDeviceToHost, s));
        int kd = 0;
        CT_HIP_CHECK(hipMemcpyAsync(&kd, st.flags + F_KDONE, sizeof(int), hipMemcpyDeviceToHost, s));
        CT_HIP_CHECK(hipStreamSynchronize(s));
        for (int i = 0; i <= K; ++i) {
            if (mon->data_res) mon->data_res[i] = i <= kd ? dr[i] : NAN;
            if (mon->img_rmse) mon->img_rmse[i] = (i <= kd && mon->x_ref) ? im[i] : NAN;
        }
    }
    return finish(st, K, res_hist, iters_done, s);
}

int cgls_impl(const ct_geometry *g, const float *b, float *x, const ct_solver_opts *o, void *ws, size_t ws_bytes,
              double *res_hist, int *iters_done, hipStream_t s) {
    float *r, *q, *sv, *p;
    OpScratch op;
    KState st;
    size_t need = carve_cgls(g, *o, nullptr, &r, &q, &sv, &p, op, st);
    CT_TRY(check_solver_args(g, CT_SOLVER_CGLS, o, b, x, ws, ws_bytes, need));
    carve_cgls(g, *o, ws, &r, &q, &sv, &p, op, st);
    const size_t n = g->n_vox, m = g->n_rays;
    const int *stop = st.flags + F_STOP;
    const int nb_n = sweep_blocks(n), nb_m = sweep_blocks(m);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, st.flags, 16);
    CT_LAUNCH_CHECK();
    CT_TRY(launch_fill(x, n, 0.0f, s));
    CT_TRY(launch_pad_zero(g, op.vx, op.vy, s));
    hipLaunchKernelGGL(k_copy, dim3(grid_1d(m)), dim3(256), 0, s, b, r, m);
    CT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sumsq, dim3(nb_m), dim3(256), 0, s, r, m, st.partials, nullptr);
    CT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cgls_start, dim3(1), dim3(256), 0, s, st, nb_m, 0);
    CT_LAUNCH_CHECK();
    CT_TRY(apply_B(g, o->B, r, CT_F32, sv, op, nullptr, stop, s));
    hipLaunchKernelGGL(k_sumsq, dim3(nb_n), dim3(256), 0, s, sv, n, st.partials, stop);
    CT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cgls_start, dim3(1), dim3(256), 0, s, st, nb_n, 1);
    CT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_copy, dim3(grid_1d(n)), dim3(256), 0, s, sv, p, n);
    CT_LAUNCH_CHECK();
    const bool pad_ready = o->B != CT_B_AT;
    for (int k = 0; k < o->iters; ++k) {
        CT_TRY(apply_A(g, p, q, CT_F32, op, pad_ready, nullptr, stop, s));
        hipLaunchKernelGGL(k_sumsq, dim3(nb_m), dim3(256), 0, s, q, m, st.partials, stop);
        CT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_cgls_alpha, dim3(1), dim3(256), 0, s, st, nb_m);
        CT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_cgls_xr, dim3(grid_1d(n + m)), dim3(256), 0, s, x, p, n, r, q, m, st);
        CT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sumsq, dim3(nb_m), dim3(256), 0, s, r, m, st.partials, stop);
        CT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_cgls_res, dim3(1), dim3(256), 0, s, st, nb_m, k);
        CT_LAUNCH_CHECK();
        CT_TRY(apply_B(g, o->B, r, CT_F32, sv, op, nullptr, stop, s));
        hipLaunchKernelGGL(k_sumsq, dim3(nb_n), dim3(256), 0, s, sv, n, st.partials, stop);
        CT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_cgls_beta, dim3(1), dim3(256), 0, s, st, nb_n);
        CT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_cgls_p, dim3(grid_1d(n)), dim3(256), 0, s, p, sv, n, st);
        CT_LAUNCH_CHECK();
    }
    return finish(st, o->iters, res_hist, iters_done, s);
}

// ------------------------------------------------------ restarted BA-GMRES
// Workspace of the restarted solver: the GMRES workspace for m iterations,
// then the data residual, the projection of the current x and the padded
// copies used to form it.
struct RestartBufs {
    size_t gm_bytes = 0;
    float *r = nullptr, *q = nullptr;
    OpScratch op;
};

size_t carve_restart(const ct_geometry *g, const ct_solver_opts &o, void *ws, RestartBufs &rb) {
    GmresBufs bf;
    rb.gm_bytes = align_up(carve_gmres(g, CT_SOLVER_BA, o, nullptr, bf));
    Carver c(ws ? (char *)ws + rb.gm_bytes : nullptr);
    rb.r = c.take<float>(g->n_rays);
    rb.q = c.take<float>(g->n_rays);
    rb.op.vx = c.take<float>(g->pad.nvx);
    rb.op.vy = c.take<float>(g->pad.nvy);
    if (!ws) rb.r = rb.q = rb.op.vx = rb.op.vy = nullptr;
    return rb.gm_bytes + c.off;
}

}  // namespace
}  // namespace ct

using namespace ct;

extern "C" int ct_solver_workspace_bytes(const ct_geometry *g, int solver, const ct_solver_opts *opts,
                                         size_t *bytes) {
    clear_error();
    CT_ARG_CHECK(g && opts && bytes, "ct_solver_workspace_bytes: NULL argument");
    CT_ARG_CHECK(opts->iters >= 0, "ct_solver_workspace_bytes: iters out of range");
    if (solver != CT_SOLVER_CGLS && opts->iters + 1 > kMaxVec) {
        set_error("ct_solver_workspace_bytes: GMRES supports at most 56 iterations");
        return CT_ERR_UNSUPPORTED;
    }
    if (solver == CT_SOLVER_BA || solver == CT_SOLVER_AB || solver == CT_SOLVER_BA_MONITOR) {
        GmresBufs bf;
        *bytes = carve_gmres(g, solver == CT_SOLVER_AB ? CT_SOLVER_AB : CT_SOLVER_BA, *opts, nullptr, bf,
                             solver == CT_SOLVER_BA_MONITOR);
    } else if (solver == CT_SOLVER_BA_RESTARTED) {
        RestartBufs rb;
        *bytes = carve_restart(g, *opts, nullptr, rb);
    } else if (solver == CT_SOLVER_CGLS) {
        float *r, *q, *sv, *p;
        OpScratch op;
        KState st;
        *bytes = carve_cgls(g, *opts, nullptr, &r, &q, &sv, &p, op, st);
    } else {
        set_error("ct_solver_workspace_bytes: unknown solver");
        return CT_ERR_ARG;
    }
    return CT_OK;
}

extern "C" int ct_ba_gmres(const ct_geometry *g, const float *b, float *x, const ct_solver_opts *opts, void *ws,
                           size_t ws_bytes, double *res_hist, int *iters_done, void *stream) {
    clear_error();
    return gmres_impl(g, CT_SOLVER_BA, b, x, opts, ws, ws_bytes, res_hist, iters_done, (hipStream_t)stream);
}

extern "C" int ct_ab_gmres(const ct_geometry *g, const float *b, float *x, const ct_solver_opts *opts, void *ws,
                           size_t ws_bytes, double *res_hist, int *iters_done, void *stream) {
    clear_error();
    return gmres_impl(g, CT_SOLVER_AB, b, x, opts, ws, ws_bytes, res_hist, iters_done, (hipStream_t)stream);
}

extern "C" int ct_cgls(const ct_geometry *g, const float *b, float *x, const ct_solver_opts *opts, void *ws,
                       size_t ws_bytes, double *res_hist, int *iters_done, void *stream) {
    clear_error();
    return cgls_impl(g, b, x, opts, ws, ws_bytes, res_hist, iters_done, (hipStream_t)stream);
}

extern "C" int ct_ba_gmres_monitor(const ct_geometry *g, const float *b, float *x, const float *x_ref,
                                   const ct_solver_opts *opts, void *ws, size_t ws_bytes, double *res_hist,
                                   double *data_res, double *img_rmse, int *iters_done, void *stream) {
    clear_error();
    CT_ARG_CHECK(opts != nullptr, "ct_ba_gmres_monitor: NULL options");
    if (opts->sino_dtype != CT_F32) {
        set_error("ct_ba_gmres_monitor: the kept projections are FP32 (sino_dtype must be CT_F32)");
        return CT_ERR_UNSUPPORTED;
    }
    if (opts->basis_dtype != CT_F32) {
        set_error("ct_ba_gmres_monitor: the monitored solve keeps an FP32 basis (basis_dtype must be CT_F32)");
        return CT_ERR_UNSUPPORTED;
    }
    MonitorOut mon{x_ref, data_res, img_rmse};
    return gmres_impl(g, CT_SOLVER_BA, b, x, opts, ws, ws_bytes, res_hist, iters_done, (hipStream_t)stream, &mon);
}

extern "C" int ct_ba_gmres_restarted(const ct_geometry *g, const float *b, float *x, const ct_solver_opts *opts,
                                     int cycles, void *ws, size_t ws_bytes, double *res_hist, int *iters_done,
                                     void *stream) {
    clear_error();
    CT_ARG_CHECK(g && opts, "ct_ba_gmres_restarted: NULL geometry or options");
    CT_ARG_CHECK(cycles >= 1, "ct_ba_gmres_restarted: cycles must be >= 1");
    CT_ARG_CHECK(b && x, "ct_ba_gmres_restarted: NULL b or x");
    RestartBufs rb;
    const size_t need = carve_restart(g, *opts, nullptr, rb);
    CT_ARG_CHECK(ws != nullptr && ws_bytes >= need, "ct_ba_gmres_restarted: workspace too small");
    carve_restart(g, *opts, ws, rb);
    hipStream_t s = (hipStream_t)stream;
    const int m = opts->iters;
    int total = 0;
    for (int c = 0; c < cycles; ++c) {
        const float *rhs = b;
        if (c > 0) {
            // data residual of the current iterate: r = b - A x
            CT_TRY(apply_A(g, x, rb.q, CT_F32, rb.op, c > 1, nullptr, nullptr, s));
            hipLaunchKernelGGL(k_residual, dim3(grid_1d(g->n_rays)), dim3(256), 0, s, b, rb.q, rb.r, g->n_rays);
            CT_LAUNCH_CHECK();
            rhs = rb.r;
        }
        int done = 0;
        CT_TRY(gmres_impl(g, CT_SOLVER_BA, rhs, x, opts, ws, rb.gm_bytes, res_hist ? res_hist + (size_t)c * (m + 1) : nullptr,
                          &done, s, nullptr, c > 0));
        total += done;
    }
    if (iters_done) *iters_done = total;
    return CT_OK;
}
