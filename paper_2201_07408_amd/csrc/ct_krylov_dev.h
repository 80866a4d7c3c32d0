// Device-side pieces of the GMRES solvers shared by the single-problem and
// the batched translation units: the scalar state, the FP64 reductions and
// the bodies of the small steps of the Arnoldi process (Sec. II: x0 = 0, the
// normalised right-hand side as first basis vector, one orthonormalised
// vector and one Givens-updated least-squares problem per step).
#pragma once

#include "ct_common.h"

namespace ct {
namespace kry {

constexpr int kMaxBlk = 1024;    // column stride of the single-problem partial sums
constexpr int kMaxVec = 57;      // basis vectors (K+1) supported

// Device scalar state carved from the workspace (one per problem).
struct KState {
    int *flags;        // [0] k_done, [1] stop, [2] status
    double *H;         // (K+1) x K, column-major, rotated in place
    double *cs, *sn;   // K rotations
    double *gv;        // K+1 right-hand side of the small problem
    double *sc;        // K+2 basis scale factors (basis j = sc[j] W[j])
    double *h1, *h2;   // K+1 CGS coefficients
    double *coef;      // K+1 coefficients applied by the next sweep
    double *res;       // K+1 residual history
    double *misc;      // [0] scale of the raw z, [1] ||z|| before CGS, [2] CGLS gamma, [3] alpha/beta,
                       // [4] power-of-two scale of the next FP16-stored basis vector (1 for FP32)
    float *fscale;     // [0] A output scale, [1] B input scale (FP16 storage)
    double *partials;  // [column][block]
    size_t pstride;    // column stride of partials (elements)
    int K;
};

enum { F_KDONE = 0, F_STOP = 1, F_STATUS = 2 };
enum { M_ZS = 0, M_ZN0 = 1, M_GAMMA = 2, M_AB = 3, M_BT = 4 };

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Reduce per-thread sums of a 256-thread block to one value per column and
// store it at partials[column * cstride + slot]: a fixed shuffle tree per
// wavefront, then a fixed-order sum over the four wavefronts.
template <int NV>
__device__ __forceinline__ void block_partials(double (&acc)[NV], int cnt, double nacc, bool nrm, int vlo, int ncol,
                                               double *__restrict__ partials, size_t cstride, size_t slot) {
    __shared__ double red[4][NV + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int j = 0; j < NV; ++j)
        if (j < cnt) {
            const double v = wave_sum(acc[j]);
            if (lane == 0) red[wave][j] = v;
        }
    if (nrm) {
        const double v = wave_sum(nacc);
        if (lane == 0) red[wave][NV] = v;
    }
    __syncthreads();
    for (int j = tid; j < cnt; j += 256)
        partials[(size_t)(vlo + j) * cstride + slot] = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
    if (nrm && tid == 0)
        partials[(size_t)ncol * cstride + slot] = (red[0][NV] + red[1][NV]) + (red[2][NV] + red[3][NV]);
}

// Basis vectors are stored as FP32 or as FP16 (values scaled by a power of
// two, see gmres_red2).  A group is the elements one 16-byte load of the
// basis holds: four FP32 or eight FP16 values (kGroup<WT>).
template <typename WT> struct Group;
template <> struct Group<float> { static constexpr int n = 4; };
template <> struct Group<__half> { static constexpr int n = 8; };

// NT: a non-temporal load, for sweeps whose basis vectors exceed the
// last-level cache (each is read once per pass and would only evict what
// the next pass could reuse)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <bool NT = false>
__device__ __forceinline__ void ld_group(const float *p, size_t q, float (&v)[4]) {
    f32x4 t;
    if constexpr (NT) t = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p) + q);
    else t = reinterpret_cast<const f32x4 *>(p)[q];
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
template <bool NT = false>
__device__ __forceinline__ void ld_group(const __half *p, size_t q, float (&v)[8]) {
    u32x4 r;
    if constexpr (NT) r = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p) + q);
    else r = reinterpret_cast<const u32x4 *>(p)[q];
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float2 f = __half22float2(__builtin_bit_cast(__half2, w[k]));
        v[2 * k] = f.x; v[2 * k + 1] = f.y;
    }
}
// z (always FP32) for group q of GE elements
template <int GE>
__device__ __forceinline__ void ld_z(const float *p, size_t q, float (&v)[GE]) {
#pragma unroll
    for (int k = 0; k < GE / 4; ++k) {
        const float4 t = reinterpret_cast<const float4 *>(p)[q * (GE / 4) + k];
        v[4 * k] = t.x; v[4 * k + 1] = t.y; v[4 * k + 2] = t.z; v[4 * k + 3] = t.w;
    }
}
template <int GE>
__device__ __forceinline__ void st_z(float *p, size_t q, const float (&v)[GE]) {
#pragma unroll
    for (int k = 0; k < GE / 4; ++k)
        reinterpret_cast<float4 *>(p)[q * (GE / 4) + k] = make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
}
// Store a group: FP32 as is; FP16 as round-to-nearest of scale * v (the
// scale is a power of two, so the product is exact in FP32).
__device__ __forceinline__ void st_group(float *p, size_t q, const float (&v)[4], float) { st_z<4>(p, q, v); }
__device__ __forceinline__ void st_group(__half *p, size_t q, const float (&v)[8], float scale) {
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w[k] = __builtin_bit_cast(uint32_t, __floats2half2_rn(scale * v[2 * k], scale * v[2 * k + 1]));
    reinterpret_cast<uint4 *>(p)[q] = make_uint4(w[0], w[1], w[2], w[3]);
}
// FP32 output of an FP16-basis sweep (a partial z of several chunks)
__device__ __forceinline__ void st_group(float *p, size_t q, const float (&v)[8], float) { st_z<8>(p, q, v); }
__device__ __forceinline__ float ld_elem(const float *p, size_t i) { return p[i]; }
__device__ __forceinline__ float ld_elem(const __half *p, size_t i) { return __half2float(p[i]); }
__device__ __forceinline__ void st_elem(float *p, size_t i, float v, float) { p[i] = v; }
__device__ __forceinline__ void st_elem(__half *p, size_t i, float v, float scale) { p[i] = __float2half_rn(scale * v); }

// Multi-dot over groups q0 + tid, q0 + tid + qstep, ... < q1 (groups of
// Group<WT>::n elements): acc[j] += W[vlo+j] . z, nacc += z . z, all in
// FP64 (products of FP32 values are exact in FP64).
template <int NV, typename WT, bool NT = false>
__device__ __forceinline__ void mdot_groups(const WT *__restrict__ Wc, size_t ldw, int cnt,
                                            const float *__restrict__ z, size_t q0, size_t q1, size_t qstep,
                                            double (&acc)[NV], double &nacc) {
    constexpr int GE = Group<WT>::n;
    for (size_t q = q0 + threadIdx.x; q < q1; q += qstep) {
        float zf[GE];
        ld_z<GE>(z, q, zf);
        double zd[GE], zz = 0.0;
#pragma unroll
        for (int e = 0; e < GE; ++e) { zd[e] = zf[e]; zz += zd[e] * zd[e]; }
        nacc += zz;
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (j < cnt) {
                float w[GE];
                ld_group<NT>(Wc + (size_t)j * ldw, q, w);
                double d = 0.0;
#pragma unroll
                for (int e = 0; e < GE; ++e) d += (double)w[e] * zd[e];
                acc[j] += d;
            }
    }
}

// Multi-axpy over groups: z' = zs z - sum_j cf[j] W[vlo+j] (FP64), rounded
// to FP32; nacc += z' . z' (of the FP32 values); stored as OT (FP16 output:
// oscale * z').
template <int NV, typename WT, typename OT, bool NT = false>
__device__ __forceinline__ void maxpy_groups(const WT *__restrict__ Wc, size_t ldw, int cnt, const double *cf,
                                             double zs, const float *zin, OT *zout, float oscale, size_t q0,
                                             size_t q1, size_t qstep, double &nacc) {
    constexpr int GE = Group<WT>::n;
    for (size_t q = q0 + threadIdx.x; q < q1; q += qstep) {
        float zf[GE];
        ld_z<GE>(zin, q, zf);
        double u[GE];
#pragma unroll
        for (int e = 0; e < GE; ++e) u[e] = zs * (double)zf[e];
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (j < cnt) {
                float w[GE];
                ld_group<NT>(Wc + (size_t)j * ldw, q, w);
                const double c = cf[j];
#pragma unroll
                for (int e = 0; e < GE; ++e) u[e] -= c * (double)w[e];
            }
        float o[GE];
        double oo = 0.0;
#pragma unroll
        for (int e = 0; e < GE; ++e) { o[e] = (float)u[e]; oo += (double)o[e] * o[e]; }
        nacc += oo;
        st_group(zout, q, o, oscale);
    }
}

// Fused multi-axpy and multi-dot over groups: z' = zs z - sum_j cf[j]
// W[vlo+j] (FP64, rounded to FP32 and stored), then acc[j] += W[vlo+j] . z'
// with the same W values still in registers, so the chunk of basis vectors
// is read once for both; nacc += z' . z'.
template <int NV, typename WT, bool NT = false>
__device__ __forceinline__ void maxpy_dot_groups(const WT *__restrict__ Wc, size_t ldw, int cnt, const double *cf,
                                                 double zs, const float *zin, float *zout, size_t q0, size_t q1,
                                                 size_t qstep, double (&acc)[NV], double &nacc) {
    constexpr int GE = Group<WT>::n;
    for (size_t q = q0 + threadIdx.x; q < q1; q += qstep) {
        float zf[GE];
        ld_z<GE>(zin, q, zf);
        double u[GE];
#pragma unroll
        for (int e = 0; e < GE; ++e) u[e] = zs * (double)zf[e];
        float w[NV][GE];
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (j < cnt) {
                ld_group<NT>(Wc + (size_t)j * ldw, q, w[j]);
                const double c = cf[j];
#pragma unroll
                for (int e = 0; e < GE; ++e) u[e] -= c * (double)w[j][e];
            }
        float o[GE];
        double od[GE], oo = 0.0;
#pragma unroll
        for (int e = 0; e < GE; ++e) { o[e] = (float)u[e]; od[e] = o[e]; oo += od[e] * od[e]; }
        nacc += oo;
        st_z<GE>(zout, q, o);
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (j < cnt) {
                double d = 0.0;
#pragma unroll
                for (int e = 0; e < GE; ++e) d += (double)w[j][e] * od[e];
                acc[j] += d;
            }
    }
}

// out[j] = sum over b < nblk of partials[j * cstride + b], j < count.  One
// wavefront per column, lanes stride the blocks, a fixed shuffle tree
// finishes: the order never changes, so the result is reproducible.
__device__ inline void reduce_partials(const double *__restrict__ partials, size_t cstride, int nblk, int count,
                                       double *out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int j = wave; j < count; j += nw) {
        const double *col = partials + (size_t)j * cstride;
        double s = 0.0;
        for (int b = lane; b < nblk; b += 64) s += col[b];
        s = wave_sum(s);
        if (lane == 0) out[j] = s;
    }
}

__device__ __forceinline__ float pow2_scale(double target) {
    // nearest power of two to target (exact scaling for FP16 storage)
    if (!(target > 0.0) || !isfinite(target)) return 1.0f;
    const double e = rint(log2(target));
    return (float)exp2(fmin(fmax(e, -60.0), 60.0));
}

// ----------------------------------------------------- step bodies
// Each body is run by one workgroup (a multiple of 64 threads); `d` is
// workgroup-shared scratch of at least K+2 doubles.

// Power of two t with t * norm in (sqrt(len) / 2, sqrt(len)]: the stored
// values of an FP16 basis vector t * v then have an RMS near 1, and no value
// can exceed sqrt(len) (< 2^15 for every supported length).  t stays within
// 2^+-120 so that it is an FP32 number (the rule holds for every norm of an
// FP32 vector above 2^-100).
__device__ __forceinline__ double basis_pow2(double norm, double len) {
    if (!(norm > 0.0) || !isfinite(norm)) return 1.0;
    const double e = floor(log2(sqrt(len) / norm));
    return exp2(fmin(fmax(e, -120.0), 120.0));
}

// beta = ||r0|| from the partials; first basis vector's scale.  blen > 0:
// the basis is stored in FP16 (vectors of length blen) and W[0] will hold
// t0 r0, so its scale is 1 / (t0 beta).
__device__ inline void gmres_init(KState &st, int nblk, double qscale_c, double *d, double blen = 0.0) {
    reduce_partials(st.partials, st.pstride, nblk, 1, d);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double beta = sqrt(d[0]);
    st.flags[F_KDONE] = 0;
    st.flags[F_STATUS] = CT_OK;
    st.res[0] = beta;
    st.misc[M_BT] = 1.0;
    if (!isfinite(beta)) {
        st.flags[F_STOP] = 1;
        st.flags[F_STATUS] = CT_ERR_NUMERIC;
        return;
    }
    if (beta == 0.0) {
        st.flags[F_STOP] = 1;
        return;
    }
    st.flags[F_STOP] = 0;
    const double t0 = blen > 0.0 ? basis_pow2(beta, blen) : 1.0;
    st.misc[M_BT] = t0;
    st.sc[0] = 1.0 / (beta * t0);
    st.gv[0] = beta;
    if (st.fscale) {
        const float qs = pow2_scale(st.sc[0] * qscale_c);
        st.fscale[0] = qs;
        st.fscale[1] = 1.0f / qs;
    }
}

// After pass 1 at step k: h1 = V_k^T z, coefficients for pass 2.  The raw
// new vector is B A W[k] (any FP16 storage scale already divided out by the
// back-projector), so the true vector is sc[k] * raw.
__device__ inline void gmres_red1(KState &st, int nblk, int k, double *d) {
    const int nvec = k + 1;
    reduce_partials(st.partials, st.pstride, nblk, nvec + 1, d);
    __syncthreads();
    const double s = st.sc[k];
    for (int j = threadIdx.x; j < nvec; j += blockDim.x) {
        const double h = st.sc[j] * s * d[j];
        st.h1[j] = h;
        st.coef[j] = h * st.sc[j];
    }
    if (threadIdx.x == 0) {
        st.misc[M_ZS] = s;
        st.misc[M_ZN0] = s * sqrt(d[nvec]);
    }
}

// After pass 2: h2 = V_k^T z1, coefficients for pass 3.  blen > 0 (FP16
// basis): the pass also summed ||z1||^2 (column nvec), from which the scale
// of the vector that pass 3 stores is chosen (||z2|| differs from ||z1|| by
// the second-pass correction only).
__device__ inline void gmres_red2(KState &st, int nblk, int k, double *d, double blen = 0.0) {
    const int nvec = k + 1;
    reduce_partials(st.partials, st.pstride, nblk, blen > 0.0 ? nvec + 1 : nvec, d);
    __syncthreads();
    for (int j = threadIdx.x; j < nvec; j += blockDim.x) {
        const double h = st.sc[j] * d[j];
        st.h2[j] = h;
        st.coef[j] = h * st.sc[j];
    }
    if (blen > 0.0 && threadIdx.x == 0) st.misc[M_BT] = basis_pow2(sqrt(d[nvec]), blen);
}

// After pass 3: new column of H, Givens rotations, residual, breakdown test.
__device__ inline void gmres_red3(KState &st, int nblk, int k, double tol, double qscale_c, double *d) {
    reduce_partials(st.partials, st.pstride, nblk, 1, d);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int K1 = st.K + 1;
    double *col = st.H + (size_t)k * K1;
    const double hn = sqrt(d[0]);
    for (int i = 0; i <= k; ++i) col[i] = st.h1[i] + st.h2[i];
    col[k + 1] = hn;
    for (int i = 0; i < k; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = st.cs[i] * a + st.sn[i] * b;
        col[i + 1] = -st.sn[i] * a + st.cs[i] * b;
    }
    const double rho = hypot(col[k], col[k + 1]);
    const double c = col[k] / rho, s = col[k + 1] / rho;
    st.cs[k] = c;
    st.sn[k] = s;
    col[k] = rho;
    col[k + 1] = 0.0;
    st.gv[k + 1] = -s * st.gv[k];
    st.gv[k] = c * st.gv[k];
    st.res[k + 1] = fabs(st.gv[k + 1]);
    st.flags[F_KDONE] = k + 1;
    if (!isfinite(rho) || !isfinite(st.gv[k]) || !isfinite(hn) || rho == 0.0) {
        st.flags[F_STOP] = 1;
        st.flags[F_STATUS] = CT_ERR_NUMERIC;
        return;
    }
    if (hn <= tol * st.misc[M_ZN0]) {   // (happy) breakdown
        st.flags[F_STOP] = 1;
        return;
    }
    st.sc[k + 1] = 1.0 / (hn * st.misc[M_BT]);   // W[k+1] holds t z2 (t = 1 for FP32)
    if (st.fscale) {
        const float qs = pow2_scale(st.sc[k + 1] * qscale_c);
        st.fscale[0] = qs;
        st.fscale[1] = 1.0f / qs;
    }
}

// y = R^-1 g (back substitution); coef[j] = y[j] * sc[j]
__device__ inline void gmres_trsv(KState &st) {
    if (threadIdx.x != 0) return;
    const int kd = st.flags[F_KDONE];
    const int K1 = st.K + 1;
    for (int i = kd - 1; i >= 0; --i) {
        double s = st.gv[i];
        for (int j = i + 1; j < kd; ++j) s -= st.H[(size_t)j * K1 + i] * st.coef[j];
        st.coef[i] = s / st.H[(size_t)i * K1 + i];
    }
    for (int i = 0; i < kd; ++i) st.coef[i] *= st.sc[i];
}

}  // namespace kry
}  // namespace ct
