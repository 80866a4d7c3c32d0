// CT operators of the ABBA method on gfx950: Joseph forward projector A
// (and the line-intersection model), its exact transpose A^T, the
// voxel-driven back-projector B_un and the Ram-Lak ramp filter F (Sec. III
// of the paper names A, B_un, F and B_FBP = B_un F; the discretisations are
// the ones stated in ct.h).
//
// The projectors are gathers, not dense contractions, so they run on the
// vector units; only F, two Toeplitz products per row, runs on MFMA.
//  * A is ray-driven.  In 3D a workgroup is a 16 x 16 tile of one view's
//    detector: per chunk of four sampling planes the patch of the volume its
//    rays cross is staged in LDS with 16-byte loads from a zero-padded,
//    axis-permuted copy, and each ray interpolates its samples from there.
//    Per-ray set-up (direction, dominant axis, plane range) is FP64; the
//    plane loop is FP32 with FMA-from-index positions and FP64 accumulation
//    of groups of four samples.  In 2D one work-item walks one ray.
//  * A^T is gathered per voxel (each voxel sums the weighted values of the
//    rays whose samples touch it, in a fixed order), so its results do not
//    depend on scheduling: in 3D from LDS-staged footprints of the
//    step-weighted data, in 2D per pixel from a tent on the detector.
//  * B_un is voxel-driven: a workgroup owns 16 x 16 columns and a chunk of
//    z, stages each view's detector footprint in LDS, and interpolates there.
//  * F: per detector row, the even and odd outputs are two dense Toeplitz
//    products of the odd-lag taps (v_mfma_f32_16x16x4f32).
#include <type_traits>
#include <cmath>
#include <map>
#include <mutex>
#include <utility>

#include "ct_common.h"

namespace ct {

namespace {

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, size_t elems) {
    // gfx9 raw buffer: stride 0, num_records in bytes, range-checked.
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0,
                                             (int)(uint32_t)(elems * 4u), 0x00020000);
}


// two adjacent floats (4-byte alignment is enough for buffer loads on gfx9)
__device__ __forceinline__ float2 ld2(__amdgpu_buffer_rsrc_t r, uint32_t elem) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)(elem * 4u), 0, 0);
    return make_float2(__builtin_bit_cast(float, (uint32_t)v[0]), __builtin_bit_cast(float, (uint32_t)v[1]));
}

__device__ __forceinline__ float ld1(__amdgpu_buffer_rsrc_t r, uint32_t elem) {
    return __builtin_bit_cast(float, (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, (int)(elem * 4u), 0, 0));
}

__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(__half v) { return __half2float(v); }
template <typename T> __device__ __forceinline__ T from_f(float v);
template <> __device__ __forceinline__ float from_f<float>(float v) { return v; }
template <> __device__ __forceinline__ __half from_f<__half>(float v) { return __float2half_rn(v); }
// four consecutive elements as floats, from a 16-byte (FP32) or 8-byte
// (FP16) aligned address
template <typename InT>
__device__ __forceinline__ float4 ld4f(const InT *p);
template <> __device__ __forceinline__ float4 ld4f<float>(const float *p) {
    return *reinterpret_cast<const float4 *>(p);
}
template <> __device__ __forceinline__ float4 ld4f<__half>(const __half *p) {
    const uint2 h = *reinterpret_cast<const uint2 *>(p);
    const float2 lo = __half22float2(__builtin_bit_cast(__half2, h.x));
    const float2 hi = __half22float2(__builtin_bit_cast(__half2, h.y));
    return make_float4(lo.x, lo.y, hi.x, hi.y);
}

// ------------------------------------------------------------- padding
// Zero only the border cells of both padded copies.
__global__ void k_pad_zero(float *__restrict__ vx, float *__restrict__ vy, int nx, int ny,
                           int nz, PadLayout L) {
    // cells per plane: full border rows + the side strips of each interior row
    const size_t per_x = (size_t)2 * L.pz * L.rx + (size_t)nz * (L.rx - ny);
    const size_t per_y = (size_t)2 * L.pz * L.ry + (size_t)nz * (L.ry - nx);
    const size_t tot_x = per_x * nx, tot = tot_x + per_y * ny;
    size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; t < tot; t += stride) {
        const bool isx = t < tot_x;
        const size_t tt = isx ? t : t - tot_x;
        const size_t per = isx ? per_x : per_y;
        const uint32_t R = isx ? L.rx : L.ry, S = isx ? L.sx : L.sy;
        const int nb = isx ? ny : nx;
        const size_t plane = tt / per;
        const size_t q = tt % per;
        uint32_t row, col;
        const size_t full = (size_t)2 * L.pz * R;
        if (q < full) {
            row = (uint32_t)(q / R);
            col = (uint32_t)(q % R);
            if (row >= (uint32_t)L.pz) row += nz;
        } else {
            // kPad cells on the left, R - nb - kPad on the right of each interior row
            const uint32_t side = R - (uint32_t)nb;
            const size_t q2 = q - full;
            row = (uint32_t)(L.pz + q2 / side);
            const uint32_t c = (uint32_t)(q2 % side);
            col = c < (uint32_t)kPad ? c : (uint32_t)nb + c;
        }
        float *dst = isx ? vx : vy;
        dst[plane * S + (size_t)row * R + col] = 0.0f;
    }
}

// x[z][y][x] -> Vx[x][z+pz][y+kPad] and Vy[y][z+pz][x+kPad] (interior only)
// for the 32 x 32 tile at (x0, y0) of slice z; 256 work-items as 32 x 8.
template <typename InT>
__device__ __forceinline__ void pad_tile(const InT *__restrict__ x, float *__restrict__ vx,
                                         float *__restrict__ vy, int nx, int ny, const PadLayout &L, int x0,
                                         int y0, int z) {
    __shared__ float tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const size_t zoff = (size_t)z * ny * nx;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int yy = y0 + ty + 8 * r, xx = x0 + tx;
        if (yy < ny && xx < nx) {
            const float v = (float)x[zoff + (size_t)yy * nx + xx];
            tile[ty + 8 * r][tx] = v;
            vy[(size_t)yy * L.sy + (size_t)(z + L.pz) * L.ry + xx + kPad] = v;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int xx = x0 + ty + 8 * r, yy = y0 + tx;
        if (yy < ny && xx < nx)
            vx[(size_t)xx * L.sx + (size_t)(z + L.pz) * L.rx + yy + kPad] = tile[tx][ty + 8 * r];
    }
}

template <typename InT>
__global__ __launch_bounds__(256) void k_pad_copy(const InT *__restrict__ x, float *__restrict__ vx,
                                                  float *__restrict__ vy, int nx, int ny, PadLayout L,
                                                  const int *__restrict__ stop) {
    if (stop && *stop) return;
    pad_tile(x, vx, vy, nx, ny, L, blockIdx.x * 32, blockIdx.y * 32, blockIdx.z);
}

// ------------------------------------------------------------ Joseph ray
// FP64 set-up of one ray: dominant axis, in-plane slopes and offsets
// (padding folded in), inclusive plane range, and the step weight.
struct RaySetup {
    int ax;            // 0: planes x = const, 1: planes y = const
    int j0, j1;        // inclusive plane range (empty if j0 > j1)
    float fb0, gb;     // in-plane padded coordinate f_b(j) = fb0 + j gb
    float fc0, gc;     // z padded coordinate (3D)
    float step;        // vox * |r| / |r_a|
};

// In-plane direction of the cone-beam ray through detector column au at
// view (c, s) = (cos, sin): the projector's dominant-axis decision and the
// voxel-driven transpose both take it from here, so they agree bit for bit.
__device__ __forceinline__ void cone_ray_xy(const GeomK &g, double c, double s, int au, double &rx, double &ry) {
    const double u = (au - 0.5 * (g.nu - 1)) * g.du;
    rx = -g.sdd * c - u * s;
    ry = -g.sdd * s + u * c;
}

// Clip [jlo, jhi] to the planes where f(j) = f0 + j g lies in (-1, N), the
// support of the interpolation along one in-plane axis.
__device__ __forceinline__ void clip_planes(double f0, double gg, int N, double &jlo, double &jhi) {
    if (gg == 0.0) {
        if (!(f0 > -1.0 && f0 < (double)N)) { jlo = 1.0; jhi = 0.0; }
        return;
    }
    const double t1 = (-1.0 - f0) / gg, t2 = ((double)N - f0) / gg;
    jlo = fmax(jlo, floor(fmin(t1, t2)) + 1.0);
    jhi = fmin(jhi, ceil(fmax(t1, t2)) - 1.0);
}

// The part of a ray's set-up that depends on its detector column only: the
// dominant axis, the in-plane coordinate along the other axis, the plane
// range that coordinate allows, 1 / r_a and r_x^2 + r_y^2 (parallel beam:
// the bin).  On the circular orbit every row of a column shares it.
__device__ __forceinline__ RayCol ray_column(const GeomK &g, int p, int au, bool cone) {
    const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
    double ox, oy, rx, ry;
    if (cone) {
        ox = g.sod * c;
        oy = g.sod * s;
        cone_ray_xy(g, c, s, au, rx, ry);
    } else {
        const double sa = (au - 0.5 * (g.nu - 1)) * g.du;
        ox = sa * c;
        oy = sa * s;
        rx = -s;
        ry = c;
    }
    RayCol Q;
    Q.ax = cone ? (fabs(rx) >= fabs(ry) ? 0 : 1) : g.axis[p];
    const double ra = Q.ax == 0 ? rx : ry, rb = Q.ax == 0 ? ry : rx;
    const double oa = Q.ax == 0 ? ox : oy, ob = Q.ax == 0 ? oy : ox;
    const int Na = Q.ax == 0 ? g.nx : g.ny, Nb = Q.ax == 0 ? g.ny : g.nx;
    const double inv_vox = 1.0 / g.vox;
    Q.inv_ra = 1.0 / ra;
    Q.base = -0.5 * (Na - 1) - oa * inv_vox;   // plane j at j + base (voxel units from o)
    const double gb = rb * Q.inv_ra;
    const double fb0 = ob * inv_vox + 0.5 * (Nb - 1) + gb * Q.base;
    double jlo = 0.0, jhi = (double)(Na - 1);
    clip_planes(fb0, gb, Nb, jlo, jhi);
    Q.jlo = jlo;
    Q.jhi = jhi;
    Q.fb0 = (float)(fb0 + kPad);
    Q.gb = (float)gb;
    Q.sxy = rx * rx + ry * ry;
    return Q;
}

// The rest of the set-up for detector row av (cone beam: the z slope and
// offset, the plane range they allow, and the step weight).
__device__ __forceinline__ RaySetup ray_finish(const GeomK &g, const PadLayout &L, const RayCol &Q, int av, bool cone) {
    RaySetup R;
    R.ax = Q.ax;
    double jlo = Q.jlo, jhi = Q.jhi;
    double gc = 0.0, fc0 = 0.0, rz = 0.0;
    if (cone) {
        rz = (av - 0.5 * (g.nv - 1)) * g.dv;
        gc = rz * Q.inv_ra;
        fc0 = 0.5 * (g.nz - 1) + gc * Q.base;   // source at z = 0
        clip_planes(fc0, gc, g.nz, jlo, jhi);
    }
    if (!(jlo <= jhi)) { jlo = 1.0; jhi = 0.0; }
    R.j0 = (int)jlo;
    R.j1 = (int)jhi;
    R.fb0 = Q.fb0;
    R.gb = Q.gb;
    R.fc0 = (float)(fc0 + L.pz);
    R.gc = (float)gc;
    R.step = (float)(g.vox * sqrt(Q.sxy + rz * rz) * fabs(Q.inv_ra));
    return R;
}

template <bool CONE>
__device__ __forceinline__ RaySetup ray_setup(const GeomK &g, const PadLayout &L, int p, int av, int au) {
    return ray_finish(g, L, ray_column(g, p, au, CONE), av, CONE);
}

// The per-(view, column) part of the cone-beam ray set-up, tabulated once
// at geometry creation by the same code the kernels would run.
__global__ void k_ray_columns(GeomK g, RayCol *__restrict__ T) {
    const int au = blockIdx.x * blockDim.x + threadIdx.x, p = blockIdx.y;
    if (au >= g.nu) return;
    T[(size_t)p * g.nu + au] = ray_column(g, p, au, true);
}

// Direct (cache-gather) evaluation of the samples of one ray on planes
// [ja, jb], read straight from the padded copy.  `vol` holds Vx at element 0
// and Vy at element `offy`; one buffer resource covers both so that the
// descriptor stays wave-uniform while the copy (and strides) are chosen per
// ray.  The plane loop is unrolled by four so that eight (3D) or four (2D)
// loads are in flight before the first interpolation; each group of four
// samples is summed in FP32 and added to an FP64 accumulator (FP32
// accumulation over hundreds of samples costs more accuracy than the sample
// positions do).
template <bool CONE>
__device__ __forceinline__ double direct_samples(const RaySetup &R, __amdgpu_buffer_rsrc_t rs, uint32_t base,
                                                 uint32_t S, uint32_t Rw, int ja, int jb) {
    double acc = 0.0;
    int j = ja;
    for (; j + 3 <= jb; j += 4) {
        uint32_t off[4];
        float wb[4], wc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float fj = (float)(j + u);
            const float fb = fmaf(fj, R.gb, R.fb0);
            const float ibf = floorf(fb);
            wb[u] = fb - ibf;
            off[u] = base + __umul24((uint32_t)(j + u), S) + (uint32_t)(int)ibf;
            if (CONE) {
                const float fc = fmaf(fj, R.gc, R.fc0);
                const float icf = floorf(fc);
                wc[u] = fc - icf;
                off[u] += __umul24((uint32_t)(int)icf, Rw);
            }
        }
        float2 lo[4], hi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            lo[u] = ld2(rs, off[u]);
            if (CONE) hi[u] = ld2(rs, off[u] + Rw);
        }
        float grp = 0.0f;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float t0 = fmaf(wb[u], lo[u].y - lo[u].x, lo[u].x);
            if (CONE) {
                const float t1 = fmaf(wb[u], hi[u].y - hi[u].x, hi[u].x);
                grp += fmaf(wc[u], t1 - t0, t0);
            } else {
                grp += t0;
            }
        }
        acc += (double)grp;
    }
    for (; j <= jb; ++j) {
        const float fj = (float)j;
        const float fb = fmaf(fj, R.gb, R.fb0);
        const float ibf = floorf(fb);
        const float wb = fb - ibf;
        uint32_t off = base + __umul24((uint32_t)j, S) + (uint32_t)(int)ibf;
        if (CONE) {
            const float fc = fmaf(fj, R.gc, R.fc0);
            const float icf = floorf(fc);
            const float wc = fc - icf;
            off += __umul24((uint32_t)(int)icf, Rw);
            const float2 a = ld2(rs, off), b = ld2(rs, off + Rw);
            const float t0 = fmaf(wb, a.y - a.x, a.x);
            const float t1 = fmaf(wb, b.y - b.x, b.x);
            acc += (double)fmaf(wc, t1 - t0, t0);
        } else {
            const float2 a = ld2(rs, off);
            acc += (double)fmaf(wb, a.y - a.x, a.x);
        }
    }
    return acc;
}

template <typename OutT>
__device__ __forceinline__ void store_ray(const GeomK &g, OutT *y, int p, int av, int au, double acc,
                                          float step, const float *out_scale) {
    float val = (float)(acc * (double)step);
    if (out_scale) val *= *out_scale;
    y[((size_t)p * g.nv + av) * g.nu + au] = from_f<OutT>(val);
}

// Direct projector: one work-item per ray (2D, and 3D fallback).
template <bool CONE, typename OutT>
__global__ __launch_bounds__(256) void k_project(GeomK g, PadLayout L, const float *__restrict__ vol,
                                                 uint32_t offy, OutT *__restrict__ y,
                                                 const float *__restrict__ out_scale,
                                                 const int *__restrict__ stop) {
    if (stop && *stop) return;
    const int au = blockIdx.x * blockDim.x + threadIdx.x;
    const int av = blockIdx.y * blockDim.y + threadIdx.y;
    const int p = blockIdx.z;
    if (au >= g.nu || av >= g.nv) return;
    const RaySetup R = ray_setup<CONE>(g, L, p, av, au);
    const bool isx = R.ax == 0;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(vol, (size_t)offy + L.nvy);
    const double acc = direct_samples<CONE>(R, rs, isx ? 0u : offy, isx ? L.sx : L.sy, isx ? L.rx : L.ry,
                                            R.j0, R.j1);
    store_ray(g, y, p, av, au, acc, R.step, out_scale);
}

// Line-intersection (Siddon) weights of one ray on the slabs of the dominant
// axis.  Slab j spans plane coordinate j -+ 1/2 and advances the ray by
// R.step in length; with the in-plane coordinates shifted by 1/2 (b' = b +
// 1/2, c' = c + 1/2) a voxel index is floor(b').  Where |gb|, |gc| <= 1 the
// ray crosses at most one b boundary and one c boundary inside a slab, at
// slab fractions s_b and s_c, so the slab splits into three segments (some
// of length 0): [0, s1] in voxel (b'_lo, c'_lo), [s1, s2] in the voxel that
// the first crossing leads to, [s2, 1] in (b'_hi, c'_hi), with s1 =
// min(s_b, s_c), s2 = max(s_b, s_c).  The ray sum is R.step times the
// fraction-weighted voxel values.
struct SlabSeg {
    int b0, c0, b1, c1, bm, cm;   // first, last and middle voxel indices
    float s1, s2;
};
__device__ __forceinline__ SlabSeg slab_segments(float blo, float bhi, float clo, float chi, float igb, float igc) {
    SlabSeg q;
    q.b0 = (int)floorf(blo); q.b1 = (int)floorf(bhi);
    q.c0 = (int)floorf(clo); q.c1 = (int)floorf(chi);
    const float sb = q.b0 == q.b1 ? 1.0f : ((float)max(q.b0, q.b1) - blo) * igb;
    const float sc = q.c0 == q.c1 ? 1.0f : ((float)max(q.c0, q.c1) - clo) * igc;
    q.s1 = fminf(sb, sc);
    q.s2 = fmaxf(sb, sc);
    const bool bfirst = sb < sc;
    q.bm = bfirst ? q.b1 : q.b0;
    q.cm = bfirst ? q.c0 : q.c1;
    return q;
}

// Slabs [ja, jb] of one ray read straight from the padded copy (tiles or
// chunks that are not staged).
__device__ __forceinline__ double slab_sums_direct(const RaySetup &R, float igb, float igc,
                                                   __amdgpu_buffer_rsrc_t rs, uint32_t base, uint32_t S,
                                                   uint32_t Rw, int ja, int jb) {
    double acc = 0.0;
    for (int j = ja; j <= jb; ++j) {
        const float fl = (float)j - 0.5f, fh = (float)j + 0.5f;
        const SlabSeg q = slab_segments(fmaf(fl, R.gb, R.fb0) + 0.5f, fmaf(fh, R.gb, R.fb0) + 0.5f,
                                        fmaf(fl, R.gc, R.fc0) + 0.5f, fmaf(fh, R.gc, R.fc0) + 0.5f, igb, igc);
        const uint32_t pj = base + __umul24((uint32_t)j, S);
        const float x0 = ld1(rs, pj + __umul24((uint32_t)q.c0, Rw) + (uint32_t)q.b0);
        const float xm = ld1(rs, pj + __umul24((uint32_t)q.cm, Rw) + (uint32_t)q.bm);
        const float x1 = ld1(rs, pj + __umul24((uint32_t)q.c1, Rw) + (uint32_t)q.b1);
        acc += (double)fmaf(q.s1, x0, fmaf(q.s2 - q.s1, xm, (1.0f - q.s2) * x1));
    }
    return acc;
}

// ---------------------------------------------------- staged 3D projector
// A workgroup is a 16 (u) x 16 (v) tile of one view's detector.  At a given
// plane its 256 rays sample a compact patch of about 18 x 18 voxels, and
// each voxel feeds about three of the tile's samples, so the patch is staged
// in LDS once and the taps are read from there.  For each chunk of kPC
// planes the patch (the union box of the chunk's planes) is copied with
// 16-byte loads; the box comes from the tile's four corner rays: at a fixed
// plane the in-plane position is monotone in u and in v, and it is linear in
// the plane index, so the corners at the chunk's first and last planes bound
// every ray of the tile.  The next chunk's loads are issued into registers
// before the current chunk is interpolated.  The kernel is bound by VALU
// issue, so the per-chunk decisions (skip, unmasked, masked) are taken on
// the scalar unit from per-wavefront plane ranges that lane shuffles reduce
// once per ray (no LDS atomics, which serialise across the 64 lanes), and
// the LDS footprint is kept small (one buffer, rows sized to the boxes that
// occur, boxes packed in one word) to keep more workgroups resident.  Tiles
// whose rays do not share a dominant axis, and chunks whose box does not
// fit, take the direct path.
constexpr int kTU = 16, kTV = 16;     // rays per workgroup
constexpr int kPC = 4;                // planes per staged chunk
constexpr int kSR = 24, kSC = 48;     // staged rows / row stride per plane; 48 = 16 (mod 32 banks)
constexpr int kNQ = 8;                // staged 16-byte columns per row (32 floats)
constexpr int kStage = kSR * kNQ;     // work-items that stage (one cell per plane each)
static_assert(kStage <= kTU * kTV && kNQ * 4 <= kSC, "staging layout");
constexpr int kMaxChunks = 512;       // planes up to 2048 (longer: direct path)
constexpr int kWaves = kTU * kTV / 64;

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// Workgroup order: the hardware deals workgroups to the eight XCDs in turn,
// so the flat index is remapped such that each XCD receives a contiguous
// range of logical work, ordered [view group][tile][view in group].  The
// workgroups resident on one XCD then project the same tiles for
// neighbouring views, whose footprints overlap, and the XCD's L2 serves the
// overlap.  vgrp views form a group (the launch picks it, see
// launch_staged).  Returns false for the padding workgroups of the last XCD.
//
// A negative vgrp selects the band order for volumes beyond the last-level
// cache: groups of -vgrp views, ordered [tile row][view group][tile column]
// [view in group], dealt to the XCDs in runs of one group's tile row (run r
// to XCD r mod 8).  All XCDs then work on the same band of detector rows,
// whose rays cross one slab of the volume, for eight neighbouring view
// groups at a time, so the slab stays in the last-level cache while every
// view passes it; within an XCD the L2 sharing of the same tile across a
// group's views is as before.
__device__ __forceinline__ bool xcd_tile(int ntu, int ntv, int P, int vgrp, int &tu, int &tv, int &p) {
    if (vgrp < 0) {
        const int G = -vgrp, ngrp = (P + G - 1) / G, run = ntu * G;
        const int nlog = ntv * ngrp * run;
        const int b = blockIdx.x, i = b >> 3;
        const int lg = ((i / run) * 8 + (b & 7)) * run + i % run;
        if (lg >= nlog) return false;
        tu = (lg / G) % ntu;
        tv = lg / (run * ngrp);
        p = ((lg / run) % ngrp) * G + lg % G;
        return p < P;
    }
    const int ntiles = ntu * ntv;
    const int ngrp = (P + vgrp - 1) / vgrp;
    const int nlog = ngrp * ntiles * vgrp;
    const int per = (nlog + 7) / 8;
    const int b = blockIdx.x;
    const int lg = (b & 7) * per + (b >> 3);
    if ((b >> 3) >= per || lg >= nlog) return false;
    const int vv = lg % vgrp;
    const int t = (lg / vgrp) % ntiles;
    const int grp = lg / (vgrp * ntiles);
    p = grp * vgrp + vv;
    tu = t % ntu;
    tv = t / ntu;
    return p < P;
}

// Tile columns per view: the detector's, plus one for the column offset.
__host__ __device__ __forceinline__ int staged_tile_cols(int nu) { return (nu + kTU - 1) / kTU + 1; }

// SID: the line-intersection model instead of Joseph's (same tiles, boxes
// and staging; per plane a slab of three segments instead of a bilinear
// sample).  Geometries admit no ray steeper than one voxel per plane in z
// (ct_geometry_create rejects cone angles that allow z-dominant rays), as
// the slab decomposition requires.
// Eight workgroups per CU (LDS 20,480 bytes): the register budget is held
// to 64 (two registers of the rare per-chunk direct path go to scratch).
template <typename OutT, bool SID>
__global__ __launch_bounds__(256, 8) void k_project_staged(GeomK g, PadLayout L, const float *__restrict__ vol,
                                                        uint32_t offy, OutT *__restrict__ y,
                                                        const float *__restrict__ out_scale,
                                                        const int *__restrict__ stop, int vgrp) {
    if (stop && *stop) return;
    int tu, tv, p;
    if (!xcd_tile(staged_tile_cols(g.nu), (g.nv + kTV - 1) / kTV, g.P, vgrp, tu, tv, p)) return;
    // the view's tile columns start vshift columns left of the detector
    const int au0 = tu * kTU - g.vshift[p], av0 = tv * kTV;
    if (au0 + kTU <= 0 || au0 >= g.nu) return;   // no column of the detector
    {
        // no ray of the tile meets the volume: zeros, without the ray set-up
        const int4 rc = g.vrect[p];
        if (au0 + kTU - 1 < rc.x || au0 > rc.y || av0 + kTV - 1 < rc.z || av0 > rc.w) {
            const int au = au0 + (int)threadIdx.x, av = av0 + (int)threadIdx.y;
            if (au >= 0 && au < g.nu && av < g.nv) y[((size_t)p * g.nv + av) * g.nu + au] = from_f<OutT>(0.0f);
            return;
        }
    }
    __shared__ float4 tile4[kPC * kSR * kSC / 4];
    // box words: (b0 + 1) << 19 | (cells - 1) << 16 | c0 << 6 | rows; 0: direct
    __shared__ uint32_t s_box[kMaxChunks];
    // The corner rays and the per-wavefront plane ranges are read only
    // before the first chunk is staged (a barrier lies between), so they
    // share the tile's space: 20,480 bytes of LDS in all, eight workgroups
    // per CU.
    float(*s_corner)[4] = reinterpret_cast<float(*)[4]>(tile4);
    int(*s_wj)[5] = reinterpret_cast<int(*)[5]>(tile4 + 4);   // per wavefront: min j0, max j1 (non-empty rays),
                                                               // max j0, min j1, axes
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kTU + tx, wv = tid >> 6;
    const int au = au0 + tx, av = av0 + ty;
    const bool active = au >= 0 && au < g.nu && av < g.nv;
    // Lanes outside the detector repeat the ray of the tile's nearest
    // detector pixel: their samples are valid (inside the tile's boxes) and
    // are not stored, so no lane needs a separate inactive path.
    const RaySetup R = ray_finish(g, L, g.rcol[(size_t)p * g.nu + min(max(au, 0), g.nu - 1)], min(av, g.nv - 1), true);
    {
        const bool ne = R.j0 <= R.j1;
        const int a = wave_min(ne ? R.j0 : 0x7fffffff), b = wave_max(ne ? R.j1 : -1);
        const int c = wave_max(R.j0), d = wave_min(R.j1);
        const int e = wave_max(1 << R.ax) | wave_min(1 << R.ax);
        if ((tid & 63) == 0) { s_wj[wv][0] = a; s_wj[wv][1] = b; s_wj[wv][2] = c; s_wj[wv][3] = d; s_wj[wv][4] = e; }
    }
    if (active) {
        // corner rays of the (possibly partial) tile
        const int ufirst = max(-au0, 0), ulast = min(au0 + kTU, g.nu) - 1 - au0, vlast = min(av0 + kTV, g.nv) - 1 - av0;
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx)
                if ((cx ? tx == ulast : tx == ufirst) && (cy ? ty == vlast : ty == 0)) {
                    s_corner[cy * 2 + cx][0] = R.fb0;
                    s_corner[cy * 2 + cx][1] = R.gb;
                    s_corner[cy * 2 + cx][2] = R.fc0;
                    s_corner[cy * 2 + cx][3] = R.gc;
                }
    }
    __syncthreads();
    int axes = 0, jlo = 0x7fffffff, jhi = -1;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        jlo = min(jlo, s_wj[w][0]);
        jhi = max(jhi, s_wj[w][1]);
        axes |= s_wj[w][4];
    }
    // wavefront-uniform plane ranges: the union of the lanes' ranges (skip
    // test) and their intersection (all lanes sample every plane of a chunk;
    // a ray that misses the volume leaves it empty)
    const int wlo = __builtin_amdgcn_readfirstlane(s_wj[wv][0]), whi = __builtin_amdgcn_readfirstlane(s_wj[wv][1]);
    const int wilo = __builtin_amdgcn_readfirstlane(s_wj[wv][2]), wihi = __builtin_amdgcn_readfirstlane(s_wj[wv][3]);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(vol, (size_t)offy + L.nvy);
    const int nch = jhi >= jlo ? (jhi - jlo) / kPC + 1 : 0;
    // per-ray reciprocal slopes of the line-intersection slabs
    const float igb = SID ? 1.0f / R.gb : 0.0f, igc = SID ? 1.0f / R.gc : 0.0f;
    if (axes == 3 || nch > kMaxChunks) {   // mixed dominant axes: direct path
        if (active) {
            const bool isx = R.ax == 0;
            const uint32_t bs = isx ? 0u : offy, Ss = isx ? L.sx : L.sy, Rs = isx ? L.rx : L.ry;
            const double acc = SID ? slab_sums_direct(R, igb, igc, rs, bs, Ss, Rs, R.j0, R.j1)
                                   : direct_samples<true>(R, rs, bs, Ss, Rs, R.j0, R.j1);
            store_ray(g, y, p, av, au, acc, R.step, out_scale);
        }
        return;
    }
    const bool isx = axes != 2;
    const uint32_t S = isx ? L.sx : L.sy, Rw = isx ? L.rx : L.ry, base = isx ? 0u : offy;
    const int nrows = g.nz + 2 * L.pz;
    // box of every chunk
    for (int c = tid; c < nch; c += kTU * kTV) {
        const int ja = jlo + c * kPC, jb = min(ja + kPC - 1, jhi);
        float bmin = 3.0e38f, bmax = -3.0e38f, cmin = 3.0e38f, cmax = -3.0e38f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const float fj = (float)(e ? jb : ja);
                const float fb = fmaf(fj, s_corner[k][1], s_corner[k][0]);
                const float fc = fmaf(fj, s_corner[k][3], s_corner[k][2]);
                bmin = fminf(bmin, fb); bmax = fmaxf(bmax, fb);
                cmin = fminf(cmin, fc); cmax = fmaxf(cmax, fc);
            }
        }
        // one cell of margin on each side absorbs rounding; clamp to the copy
        const int b0 = max((int)floorf(bmin) - 1, 0) & ~3;
        const int b1 = min((int)floorf(bmax) + 2, (int)Rw - 1);
        const int c0 = max((int)floorf(cmin) - 1, 0);
        const int c1 = min((int)floorf(cmax) + 2, nrows - 1);
        const int nr = c1 - c0 + 1;
        // only the 16-byte cells that cover the box are staged
        const int ncl = (b1 - b0) / 4 + 1;
        const bool fits = nr <= kSR && b1 - b0 < 4 * kNQ && c0 < 1024 && b0 < 8191;
        s_box[c] = fits ? ((uint32_t)(b0 + 1) << 19) | ((uint32_t)(ncl - 1) << 16) | ((uint32_t)c0 << 6) | (uint32_t)nr
                        : 0u;
    }
    // Staging: work-item t < kStage owns 16-byte column t % kNQ of box row
    // t / kNQ in every plane of a chunk, so its element offset within the
    // box is fixed; per chunk it issues one load and one LDS store per plane
    // (rows outside the box skip both).  All kPC planes are staged, also
    // past the last plane of the volume: such planes feed only masked
    // samples, and the range-checked buffer loads stay inside the copies or
    // return zero.
    const bool stager = tid < kStage;
    const int r_t = tid / kNQ, c4_t = tid % kNQ;
    // byte offset of the work-item's cell within a box (the box origin and
    // plane offsets are wavefront-uniform and added on the scalar unit)
    const uint32_t toffb = 4u * (__umul24((uint32_t)r_t, Rw) + 4u * (uint32_t)c4_t);
    float4 pre[kPC];
    // chunk c's loads into registers; bx is its box word (0: not staged)
    auto fetch = [&](int c, uint32_t bx) {
        if (bx == 0u) return;
        const int b0 = (int)(bx >> 19) - 1, c0 = (int)((bx >> 6) & 1023u), nr = (int)(bx & 63u);
        const int ncl = (int)((bx >> 16) & 7u) + 1;
        const int ja = jlo + c * kPC;
        if (stager && r_t < nr && c4_t < ncl) {
            const uint32_t e0b = 4u * (base + __umul24((uint32_t)ja, S) + __umul24((uint32_t)c0, Rw) + (uint32_t)b0);
#pragma unroll
            for (int pl = 0; pl < kPC; ++pl) {
                const auto w = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(toffb + (e0b + 4u * pl * S)), 0, 0);
                pre[pl] = make_float4(__builtin_bit_cast(float, (uint32_t)w[0]), __builtin_bit_cast(float, (uint32_t)w[1]),
                                      __builtin_bit_cast(float, (uint32_t)w[2]), __builtin_bit_cast(float, (uint32_t)w[3]));
            }
        }
    };
    const float *tile = (const float *)tile4;
    __syncthreads();   // boxes visible
    // the box word of the next chunk, read once (prefetch, then use)
    uint32_t bx_next = nch > 0 ? __builtin_amdgcn_readfirstlane(s_box[0]) : 0u;
    if (nch > 0) fetch(0, bx_next);
    double acc = 0.0;
    // row slope plus the tile's plane stride in rows: plane pl of a chunk
    // sits kSR rows below plane pl - 1
    const float gcs = R.gc + (float)kSR;
    for (int c = 0; c < nch; ++c) {
        const int ja = jlo + c * kPC;
        const uint32_t bx = bx_next;
        const int b0 = (int)(bx >> 19) - 1, c0 = (int)((bx >> 6) & 1023u);
        if (bx != 0u) {
            const int nr = (int)(bx & 63u), ncl = (int)((bx >> 16) & 7u) + 1;
            __syncthreads();   // previous chunk's readers are done with the tile
            if (stager && r_t < nr && c4_t < ncl) {
#pragma unroll
                for (int pl = 0; pl < kPC; ++pl) tile4[(pl * kSR + r_t) * (kSC / 4) + c4_t] = pre[pl];
            }
            __syncthreads();
        }
        if (c + 1 < nch) {
            bx_next = __builtin_amdgcn_readfirstlane(s_box[c + 1]);
            fetch(c + 1, bx_next);
        }
        if (ja + kPC - 1 < wlo || ja > whi) continue;   // no lane of this wavefront samples the chunk
        const int jb = min(ja + kPC - 1, R.j1), jf = max(ja, R.j0);
        if (bx == 0u) {    // box too large: direct loads for this chunk
            if (jf <= jb)
                acc += SID ? slab_sums_direct(R, igb, igc, rs, base, S, Rw, jf, jb)
                           : direct_samples<true>(R, rs, base, S, Rw, jf, jb);
            continue;
        }
        // Box-relative coordinates at the chunk's first plane.  Subtracting
        // the integer box origin is exact, and the box keeps one cell of
        // margin, so inside the lane's plane range the coordinates are >= 0
        // and truncation is floor.
        const float fb0c = fmaf((float)ja, R.gb, R.fb0) - (float)b0;
        const float fc0c = fmaf((float)ja, R.gc, R.fc0) - (float)c0;
        float grp;
        if (SID) {
            // slab boundaries k = 0..kPC at plane coordinates ja + k - 1/2,
            // shifted by 1/2 so that floor gives the voxel; unmasked where
            // every lane samples every plane, else indices clamped into the
            // tile and slabs outside a lane's range dropped
            const bool all = wilo <= ja && wihi >= ja + kPC - 1;
            float bq[kPC + 1], cq[kPC + 1];
#pragma unroll
            for (int k = 0; k <= kPC; ++k) {
                bq[k] = fmaf((float)k - 0.5f, R.gb, fb0c) + 0.5f;
                cq[k] = fmaf((float)k - 0.5f, R.gc, fc0c) + 0.5f;
            }
            grp = 0.0f;
#pragma unroll
            for (int pl = 0; pl < kPC; ++pl) {
                SlabSeg q = slab_segments(bq[pl], bq[pl + 1], cq[pl], cq[pl + 1], igb, igc);
                if (!all) {
                    q.b0 = min(max(q.b0, 0), kSC - 1); q.b1 = min(max(q.b1, 0), kSC - 1); q.bm = min(max(q.bm, 0), kSC - 1);
                    q.c0 = min(max(q.c0, 0), kSR - 1); q.c1 = min(max(q.c1, 0), kSR - 1); q.cm = min(max(q.cm, 0), kSR - 1);
                }
                const float *t = tile + pl * kSR * kSC;
                const float x0 = t[q.c0 * kSC + q.b0], xm = t[q.cm * kSC + q.bm], x1 = t[q.c1 * kSC + q.b1];
                const float v = fmaf(q.s1, x0, fmaf(q.s2 - q.s1, xm, (1.0f - q.s2) * x1));
                const int j = ja + pl;
                grp += (all || (j >= jf && j <= jb)) ? v : 0.0f;
            }
        } else if (wilo <= ja && wihi >= ja + kPC - 1) {
            // every lane samples all planes of the chunk: no masks
            grp = 0.0f;
#pragma unroll
            for (int pl = 0; pl < kPC; ++pl) {
                const float fb = pl ? fmaf((float)pl, R.gb, fb0c) : fb0c;
                const float fc = pl ? fmaf((float)pl, gcs, fc0c) : fc0c;
                const float wb = __builtin_amdgcn_fractf(fb), wc = __builtin_amdgcn_fractf(fc);
                const float *t = tile + __umul24((uint32_t)(int)fc, (uint32_t)kSC) + (uint32_t)(int)fb;
                const float t00 = t[0], t01 = t[1], t10 = t[kSC], t11 = t[kSC + 1];
                const float a0 = fmaf(wb, t01 - t00, t00);
                const float a1 = fmaf(wb, t11 - t10, t10);
                const float v = fmaf(wc, a1 - a0, a0);
                grp = pl ? grp + v : v;
            }
        } else {
            grp = 0.0f;
            // boundary chunk: planes outside a lane's range are dropped; their
            // coordinates may leave the box, so the tap indices are clamped
            // into the tile
#pragma unroll
            for (int pl = 0; pl < kPC; ++pl) {
                const int j = ja + pl;
                const float fb = pl ? fmaf((float)pl, R.gb, fb0c) : fb0c;
                const float fc = pl ? fmaf((float)pl, R.gc, fc0c) : fc0c;
                const float wb = __builtin_amdgcn_fractf(fb), wc = __builtin_amdgcn_fractf(fc);
                const uint32_t ib = (uint32_t)min(max((int)fb, 0), kSC - 2);
                const uint32_t ic = (uint32_t)min(max((int)fc, 0), kSR - 2);
                const float *t = tile + pl * kSR * kSC + __umul24(ic, (uint32_t)kSC) + ib;
                const float t00 = t[0], t01 = t[1], t10 = t[kSC], t11 = t[kSC + 1];
                const float a0 = fmaf(wb, t01 - t00, t00);
                const float a1 = fmaf(wb, t11 - t10, t10);
                const float v = fmaf(wc, a1 - a0, a0);
                grp += (j >= jf && j <= jb) ? v : 0.0f;
            }
        }
        acc += (double)grp;
    }
    if (active) store_ray(g, y, p, av, au, acc, R.step, out_scale);
}

constexpr int kZC = 16;   // z voxels per work-item in the voxel-driven cone kernels
// per-view classification word (vdom): bit 0 / 1 as in GeomK, then
constexpr int kVdomX0 = 4;          // column 0 is x-dominant
constexpr int kVdomOneSwitch = 8;   // the axis changes at most once across the detector,
constexpr int kVdomSwitchShift = 8; // at the column stored from this bit up (0: never)

// Per (view, column) ray table of a cone geometry (ColT), from the same
// direction helper as the projector, so the dominant axis matches bit for
// bit.
__global__ void k_col_table(GeomK g, ColT *__restrict__ T) {
    const int au = blockIdx.x * blockDim.x + threadIdx.x, p = blockIdx.y;
    if (au >= g.nu) return;
    const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
    double rx, ry;
    cone_ray_xy(g, c, s, au, rx, ry);
    const bool xdom = fabs(rx) >= fabs(ry);
    const double ra = xdom ? rx : ry, rb = xdom ? ry : rx;
    ColT e;
    e.t = rb / ra;
    e.ar = (float)(g.dv / (ra * g.vox));
    e.is = (float)((xdom ? 1.0 : -1.0) * g.vox / fabs(ra));
    e.sxy = (float)(rx * rx + ry * ry);
    e.pad = 0.0f;
    T[(size_t)p * g.nu + au] = e;
}

// Per view: which dominant axes occur among its columns, and the column
// offset of the projector's ray tiles that puts a tile edge at the first
// column whose dominant axis differs from column 0's (the table's axis is
// the projector's own decision), so that no tile mixes the two axes where
// the axis changes once across the detector.  vdom also records column 0's
// axis and, where the axis changes at most once, that column (kVdom*).
__global__ void k_view_dom(GeomK g, const ColT *__restrict__ T, int *__restrict__ vdom, int *__restrict__ vshift) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= g.P) return;
    int f = 0, sw = 0, changes = 0;
    const bool x0 = T[(size_t)p * g.nu].is > 0.0f;
    bool prev = x0;
    for (int au = 0; au < g.nu; ++au) {
        const bool xd = T[(size_t)p * g.nu + au].is > 0.0f;
        f |= xd ? 1 : 2;
        if (sw == 0 && xd != x0) sw = au;
        changes += xd != prev;
        prev = xd;
    }
    vdom[p] = f | (x0 ? kVdomX0 : 0) | (changes <= 1 ? kVdomOneSwitch | (sw << kVdomSwitchShift) : 0);
    vshift[p] = (kTU - sw % kTU) % kTU;
}

// Exact transpose of the cone-beam line-intersection projector
// (k_project_T_slab), gathered per voxel instead of scattered per sample.
// Voxel (ix, iy, iz) receives, from every ray that crosses the slab of its
// plane (x = ix -+ 1/2 for x-dominant rays, y = iy -+ 1/2 for y-dominant
// ones) through it, the ray's value times the fraction of the slab spent
// inside the voxel and the ray's step length: the A_ij of the forward
// model, summed over i.  With the slab parameter s in [0, 1], the ray is
// inside the voxel's b range on one interval of s and inside its c range on
// another (the coordinates are linear in s), and the weight is the length
// of their intersection.  Such rays have |f_b - i_b| < 1 and |f_c - iz| < 1
// at the plane.  Along a plane a ray's b coordinate depends on its detector
// column only, f_b = (o_b + D t(u)) / vox + C_b with D the plane's distance
// from the source along the dominant axis and t = r_b / r_a a
// linear-fractional function of u; inverting it at f_b = i_b -+ 1 gives the
// few candidate columns (all columns where the inverse interval wraps
// through infinity), each of which is tested exactly with the projector's
// dominant axis from the column table.  Its c coordinate is linear in the
// detector row: each row of a candidate column feeds the voxels of the
// work-item's z chunk its slab crosses, accumulated in per-work-item LDS
// slots.  Views are summed in FP32 over a group and added to FP64, as in
// B_un; no atomics, so the result is deterministic.  (The Joseph transpose,
// k_project_T_sheets below, shares the staging, the column table and the
// candidate columns.)
constexpr int kATS = kZC + 1;   // LDS slots per work-item (odd stride across banks)

// The s in [0, 1] on which lo <= d + (s - 1/2) g < lo + 1: the slab
// parameters where a coordinate with centre offset d and slope g per slab
// lies in one voxel (lo = -1/2 for the voxel at offset 0).
__device__ __forceinline__ void slab_interval(float d, float g, float &s0, float &s1) {
    if (g == 0.0f) {
        const bool in = d >= -0.5f && d < 0.5f;
        s0 = in ? 0.0f : 1.0f;
        s1 = in ? 1.0f : 0.0f;
        return;
    }
    const float ig = 1.0f / g;
    const float a = fmaf(-0.5f - d, ig, 0.5f), b = fmaf(0.5f - d, ig, 0.5f);
    s0 = fmaxf(fminf(a, b), 0.0f);
    s1 = fminf(fmaxf(a, b), 1.0f);
}

// Step weights of the cone-beam transpose applied once per ray: ys = y *
// step, with step = vox |r| / |r_a| = |is| sqrt(v^2 + r_x^2 + r_y^2) from the
// column table, so that the transpose reads one value per ray and row.
template <typename InT>
__global__ __launch_bounds__(256) void k_ray_step_scale(GeomK g, const InT *__restrict__ y, float *__restrict__ ys,
                                                        const int *__restrict__ stop) {
    if (stop && *stop) return;
    // one detector row (view p, row av) per wavefront, lanes along the row
    const int rows = g.P * g.nv;
    const int wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const float Cvf = (float)(0.5 * (g.nv - 1)), dvf = (float)g.dv;
    for (int row = (int)blockIdx.x * 4 + wave; row < rows; row += (int)gridDim.x * 4) {
        const int p = row / g.nv, av = row - p * g.nv;
        const float vv = ((float)av - Cvf) * dvf;
        const ColT *T = g.colT + (size_t)p * g.nu;
        const size_t base = (size_t)row * g.nu;
        for (int au = lane; au < g.nu; au += 64)
            ys[base + au] = fabsf(T[au].is) * sqrtf(fmaf(vv, vv, T[au].sxy)) * to_f(y[base + au]);
    }
}

// Detector columns [a_lo, a_hi] of a view whose rays, on the sampling plane
// at distance D from the source along the dominant axis (axis 0: planes
// x = const, b = y; axis 1: planes y = const, b = x), have in-plane
// coordinate f_b with lo < f_b - ib < hi, where e0 = o_b - (ib - C_b) vox
// so that f_b - ib = (e0 + D t) / vox with t = r_b / r_a.  t is a
// linear-fractional function of the column, inverted at the two ends; all
// columns when the inverse interval wraps through infinity, none
// (a_hi < a_lo) when it misses the detector.
__device__ __forceinline__ void column_range(const GeomK &g, int axis, double c, double s, double D, double e0,
                                             double lo, double hi, int &a_lo, int &a_hi) {
    const double Cu = 0.5 * (g.nu - 1);
    const double al = axis ? -s : c, be = axis ? -g.sdd * c : -g.sdd * s;
    const double ga = axis ? c : -s, de = axis ? -g.sdd * s : -g.sdd * c;
    const double iD = 1.0 / D, tm = (lo * g.vox - e0) * iD, tp = (hi * g.vox - e0) * iD;
    const double dm = ga * tm - al, dp = ga * tp - al;
    a_lo = 0;
    a_hi = g.nu - 1;
    if ((dm > 0.0 && dp > 0.0) || (dm < 0.0 && dp < 0.0)) {
        const double um = (be - de * tm) / dm, up = (be - de * tp) / dp;
        const double alo = fmin(um, up) / g.du + Cu, ahi = fmax(um, up) / g.du + Cu;
        a_lo = alo > -1.0 ? max((int)floor(alo), 0) : 0;
        a_hi = ahi < (double)g.nu ? min((int)ceil(ahi), g.nu - 1) : g.nu - 1;
        if (alo >= (double)g.nu || ahi <= -1.0) a_hi = -1;
    }
}

// The cone-beam transpose with each view's footprint of the step-weighted
// data staged in LDS (as the back-projector stages its footprint): per
// group of kTVG views, the box of detector cells whose rays can sample the
// workgroup's voxel block (the projection of the block widened by one
// voxel on every side, the reach of a weight, with a cell of margin) is
// copied with 16-byte loads, and the candidate rows of every candidate
// column are read from there instead of from global memory.  Candidate
// columns, weights and the z splat are described above.  A group whose box
// does not fit the tile reads the data from global memory.
constexpr int kTVG = 3;               // views per staged group
constexpr int kTSU = 36, kTSV = 32;   // staged detector columns / rows per view

__global__ __launch_bounds__(256) void k_project_T_slab(GeomK g, const float *__restrict__ ys, float *__restrict__ x,
                                                          const float *__restrict__ scale,
                                                          const int *__restrict__ stop) {
    if (stop && *stop) return;
    __shared__ float s_acc[256 * kATS];
    __shared__ float4 tile4[kTVG * kTSV * kTSU / 4];
    __shared__ int s_box[kTVG][2];
    __shared__ int s_fit;
    const float *tile = (const float *)tile4;
    const int tid = threadIdx.y * 16 + threadIdx.x;
    const int ix0 = blockIdx.x * 16, iy0 = blockIdx.y * 16, iz0 = blockIdx.z * kZC;
    const int ix = ix0 + threadIdx.x, iy = iy0 + threadIdx.y;
    const bool active = ix < g.nx && iy < g.ny;   // the others stage and meet the barriers
    float *slot = s_acc + tid * kATS;
#pragma unroll
    for (int z = 0; z < kZC; ++z) slot[z] = 0.0f;
    const int nu = g.nu, nv = g.nv, P = g.P;
    const double vox = g.vox, ivox = 1.0 / vox;
    const double Cx = 0.5 * (g.nx - 1), Cy = 0.5 * (g.ny - 1), Cz = 0.5 * (g.nz - 1), Cu = 0.5 * (nu - 1);
    const float Cvf = (float)(0.5 * (nv - 1));
    const float zoff = (float)(0.5 * (g.nz - 1) - iz0);   // f_c - iz0 = zoff + a1 (av - Cv)
    const double xc = (ix - Cx) * vox, yc = (iy - Cy) * vox;
    // the block widened by one voxel (the reach of a weight) in every axis
    const double bx0 = (ix0 - 1 - Cx) * vox, bx1 = (min(ix0 + 15, g.nx - 1) + 1 - Cx) * vox;
    const double by0 = (iy0 - 1 - Cy) * vox, by1 = (min(iy0 + 15, g.ny - 1) + 1 - Cy) * vox;
    const double bz0 = (iz0 - 1 - Cz) * vox, bz1 = (min(iz0 + kZC - 1, g.nz - 1) + 1 - Cz) * vox;
    constexpr int Q = kTSU / 4;                      // 16-byte cells per staged row
    constexpr int kCells = kTVG * kTSV * Q;
    double acc[kZC];
#pragma unroll
    for (int z = 0; z < kZC; ++z) acc[z] = 0.0;
    for (int p0 = 0; p0 < P; p0 += kTVG) {
        __syncthreads();   // the previous group's readers are done with the tile and boxes
        if (tid == 0) s_fit = 1;
        if (tid < kTVG && p0 + tid < P) {
            const int p = p0 + tid;
            const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
            double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
            for (int k = 0; k < 4; ++k) {
                const double px = (k & 1) ? bx1 : bx0, py = (k & 2) ? by1 : by0;
                const double U = g.sod - (px * c + py * s);
                const double M = g.sdd / U;
                const double fu = M * (py * c - px * s) / g.du + Cu;
                umin = fmin(umin, fu); umax = fmax(umax, fu);
                const double va = M * bz0 / g.dv + 0.5 * (nv - 1), vb = M * bz1 / g.dv + 0.5 * (nv - 1);
                vmin = fmin(vmin, fmin(va, vb)); vmax = fmax(vmax, fmax(va, vb));
            }
            const int u0 = ((int)floor(umin) - 1) & ~3, u1 = (int)floor(umax) + 2;
            const int v0 = (int)floor(vmin) - 1, v1 = (int)floor(vmax) + 2;
            s_box[tid][0] = u0;
            s_box[tid][1] = v0;
            if (u1 - u0 >= kTSU || v1 - v0 >= kTSV || !(umin > -1e6 && umax < 1e6 && vmin > -1e6 && vmax < 1e6))
                atomicAnd(&s_fit, 0);
        }
        __syncthreads();
        const bool fit = s_fit != 0;
        if (fit) {
            for (int q = tid; q < kCells; q += 256) {
                const int vv = q / (kTSV * Q), r = (q / Q) % kTSV, c4 = 4 * (q % Q);
                const int p = p0 + vv;
                float4 e = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (p < P) {
                    const int v = s_box[vv][1] + r, u = s_box[vv][0] + c4;
                    if ((unsigned)v < (unsigned)nv) {
                        const float *row = ys + ((size_t)p * nv + v) * nu;
                        if ((nu & 3) == 0 && (unsigned)u <= (unsigned)(nu - 4)) {
                            e = *reinterpret_cast<const float4 *>(row + u);
                        } else {
                            float t4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                if (u + k >= 0 && u + k < nu) t4[k] = row[u + k];
                            e = make_float4(t4[0], t4[1], t4[2], t4[3]);
                        }
                    }
                }
                tile4[q] = e;
            }
        }
        __syncthreads();
        if (active) {
            for (int vv = 0; vv < kTVG && p0 + vv < P; ++vv) {
                const int p = p0 + vv;
                const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
                const double ox = g.sod * c, oy = g.sod * s;
                const float *yp = ys + (size_t)p * nv * nu;
                const float *tv = tile + vv * kTSV * kTSU;
                const int bu0 = s_box[vv][0], bv0 = s_box[vv][1];
                const ColT *Tp = g.colT + (size_t)p * nu;
                const int vd = g.vdom[p];
#pragma unroll 1
                for (int axis = 0; axis < 2; ++axis) {
                    if (!(vd & (1 << axis))) continue;
                    const double D = axis ? yc - oy : xc - ox;
                    const int ib = axis ? ix : iy;
                    const double e0 = (axis ? ox : oy) - (ib - (axis ? Cx : Cy)) * vox;
                    int a_lo, a_hi;
                    column_range(g, axis, c, s, D, e0, -1.0, 1.0, a_lo, a_hi);
                    const float Df = (float)D;
                    for (int au = a_lo; au <= a_hi; ++au) {
                        const ColT T = Tp[au];
                        if ((T.is > 0.0f) != (axis == 0)) continue;
                        const float db = (float)((e0 + D * T.t) * ivox);
                        float lb, hb;
                        slab_interval(db, (float)T.t, lb, hb);
                        if (!(hb > lb)) continue;
                        const float wb = 1.0f;
                        const float a1 = Df * T.ar, ia1 = 1.0f / a1;
                        const float r1 = fmaf(-1.0f - zoff, ia1, Cvf), r2 = fmaf((float)kZC - zoff, ia1, Cvf);
                        const int v0 = max((int)ceilf(fminf(r1, r2)), 0), v1 = min((int)floorf(fmaxf(r1, r2)), nv - 1);
                        // this column's staged cells (clamped into the tile: the
                        // box covers every row and column that can carry a
                        // weight here, up to rounding)
                        const int lu = min(max(au - bu0, 0), kTSU - 1);
                        for (int av = v0; av <= v1; ++av) {
                            const float dv = (float)av - Cvf;
                            const float yv = fit ? tv[min(max(av - bv0, 0), kTSV - 1) * kTSU + lu] : yp[(size_t)av * nu + au];
                            const float val = wb * yv;
                            // the slab's c range, [zc + q -+ gc/2] with zc = zoff + 1/2
                            // (an exact integer or half-integer) and q = a1 dv: the
                            // crossing is taken relative to zc, so that a small slope
                            // does not divide the rounding of the absolute coordinate
                            const float gc = T.ar * (float)vox * dv, q = a1 * dv, zc = zoff + 0.5f;
                            const float r0 = fmaf(-0.5f, gc, q), r1 = fmaf(0.5f, gc, q);
                            const float k0f = floorf(zc + r0), k1f = floorf(zc + r1);
                            const float sc = k0f == k1f ? 1.0f : ((fmaxf(k0f, k1f) - zc) - r0) / gc;
                            const float f0 = fmaxf(fminf(sc, hb) - lb, 0.0f);
                            const float f1 = k0f == k1f ? 0.0f : fmaxf(hb - fmaxf(sc, lb), 0.0f);
                            const int k0 = (int)k0f, k1 = (int)k1f;
                            if ((unsigned)k0 < (unsigned)kZC) slot[k0] = fmaf(f0, val, slot[k0]);
                            if ((unsigned)k1 < (unsigned)kZC && k1 != k0) slot[k1] = fmaf(f1, val, slot[k1]);
                        }
                    }
                }
            }
            // views summed in FP32 over the group, then in FP64
#pragma unroll
            for (int z = 0; z < kZC; ++z) { acc[z] += (double)slot[z]; slot[z] = 0.0f; }
        }
    }
    if (!active) return;
    const double sc = scale ? (double)*scale : 1.0;
#pragma unroll
    for (int z = 0; z < kZC; ++z) {
        const int iz = iz0 + z;
        if (iz < g.nz) x[((size_t)iz * g.ny + iy) * g.nx + ix] = (float)(acc[z] * sc);
    }
}


// The cone-beam Joseph transpose, factored by detector column.  On a
// sampling plane all rows of one detector column share the in-plane
// coordinate f_b, so a voxel's weight in ray (u, v) is tent(f_b(u) - ib)
// times tent(f_c(u, v) - iz): per view, the column's rows are first
// splatted in z onto the plane, z_sheet(u, plane)[iz] = sum over rows of
// tent(f_c - iz) ys(u, v), once per (plane, column) of the workgroup's
// block, and each voxel column then gathers its two or three candidate
// columns' sheets with weight tent(f_b - ib).  The splat, which the
// per-voxel form repeated for every voxel column that a detector column
// reaches (two or three), is done once.  Sheets live in LDS (17-float
// stride and an odd plane stride, across banks); the footprint of the
// step-weighted data and the column table entries of its columns are
// staged as in k_project_T_slab.  Per (view, axis) the pairs to splat are
// listed (each plane's column range cut to the axis's columns), so that
// views whose fan spans both axes split the work instead of doubling it.  A
// (view, axis) whose plane needs more than kZU columns falls back to the
// per-voxel splat, in the same LDS.
constexpr int kZU = 24;              // detector columns per plane in the z sheets
constexpr int kZS = kZC + 1;         // floats per sheet
constexpr int kTG = 2;               // zero guard rows on either side of a staged view
constexpr int kPS = kZU * kZS + 1;   // floats per plane of sheets (odd: planes on distinct banks)

// LDS-qualified view of staged data: rows are addressed by 32-bit byte offsets
typedef __attribute__((address_space(3))) const float lds_cfloat;

// Eight voxels of one z sheet from the staged rows of a detector column
// (t: LDS byte address of tile row 0 of the column, the first kTG rows
// guards; rows kTSU floats apart): voxel zz takes the
// rows around tile position vr = vrb + zz / a1 (row position relative to
// the first guard row) with weights 1 - |a1| |v - vr| clipped at zero.  For
// |a1| < 1 those are rows floor(vr) - 1 .. floor(vr) + 2, the inner two
// always weighted; for |a1| >= 1 only floor(vr) and floor(vr) + 1.  Inside
// the volume vr >= 1 (the box holds the rows with a row of margin), so
// truncation is the floor; CLAMP keeps the rows of voxels beyond the volume
// (last chunk) in the tile.  Weights lie in [0, 1], so clipping at zero is
// the FMA's clamp.
template <bool CLAMP>
__device__ __forceinline__ void sheet_rows(float *out, uint32_t t, float vrb, float ia1, float aa, float am) {
    constexpr int kRows = kTSV + 2 * kTG;
    constexpr uint32_t kRB = kTSU * sizeof(float);   // bytes per tile row
    if (aa < 1.0f) {
        const float am2 = am - aa;
#pragma unroll
        for (int zz = 0; zz < kZC / 2; ++zz) {
            const float vr = fmaf((float)zz, ia1, vrb);
            const float f = __builtin_amdgcn_fractf(vr);
            const uint32_t iv = CLAMP ? (uint32_t)min(max((int)vr, 1), kRows - 3) : (uint32_t)(int)vr;
            lds_cfloat *tr = (lds_cfloat *)(size_t)(__umul24(iv, kRB) + (t - kRB));
            const float w0 = __builtin_amdgcn_fmed3f(fmaf(-aa, f, am), 0.0f, 1.0f), w1 = fmaf(-aa, f, 1.0f);
            const float w2 = fmaf(aa, f, am), w3 = __builtin_amdgcn_fmed3f(fmaf(aa, f, am2), 0.0f, 1.0f);
            out[zz] = fmaf(w0, tr[0], fmaf(w1, tr[kTSU], fmaf(w2, tr[2 * kTSU], w3 * tr[3 * kTSU])));
        }
    } else {
#pragma unroll
        for (int zz = 0; zz < kZC / 2; ++zz) {
            const float vr = fmaf((float)zz, ia1, vrb);
            const float f = __builtin_amdgcn_fractf(vr);
            const uint32_t iv = CLAMP ? (uint32_t)min(max((int)vr, 0), kRows - 2) : (uint32_t)(int)vr;
            lds_cfloat *tr = (lds_cfloat *)(size_t)(__umul24(iv, kRB) + t);
            const float w1 = __builtin_amdgcn_fmed3f(fmaf(-aa, f, 1.0f), 0.0f, 1.0f);
            const float w2 = __builtin_amdgcn_fmed3f(fmaf(aa, f, am), 0.0f, 1.0f);
            out[zz] = fmaf(w1, tr[0], w2 * tr[kTSU]);
        }
    }
}

__global__ __launch_bounds__(256, 3) void k_project_T_sheets(GeomK g, const float *__restrict__ ys, float *__restrict__ x,
                                                          const float *__restrict__ scale,
                                                          const int *__restrict__ stop) {
    if (stop && *stop) return;
    __shared__ float s_z[16 * kPS];
    __shared__ double s_fb[16 * kZU];       // f_b of each (plane, column) pair
    // staged footprint with kTG zero guard rows above and below each view's rows
    constexpr int kTVS = (kTSV + 2 * kTG) * kTSU;
    __shared__ float4 tile4[kTVG * kTVS / 4];
    __shared__ int s_box[kTVG][2];
    __shared__ int s_rng[kTVG][2][16][2];   // per view, axis, plane: first column, column count
    // per view, axis, plane: the column (relative to the first) whose ray
    // meets the plane at f_b (relative to the block's first voxel column),
    // col(f_b) = (n0 + n1 f_b) / (d0 + d1 f_b) + Cu - first, as (n0, n1, d0, d1)
    __shared__ float4 s_cf[kTVG][2][16];
    // the (plane, column) pairs of each view and axis (see the range phase
    // for the packing), and their count
    __shared__ unsigned short s_list[kTVG][2][16 * kZU];
    __shared__ int s_npairs[kTVG][2];
    // column table entries (t, then a_r and the signed step factor) of the
    // staged columns of each view
    __shared__ double s_Tt[kTVG][kTSU];
    __shared__ float2 s_Tai[kTVG][kTSU];
    __shared__ int s_wide[kTVG][2];
    __shared__ int s_fit;
    static_assert(256 * kATS <= 16 * kPS, "per-voxel fallback slots fit the sheets");
    const float *tile = (const float *)tile4;
    const int tid = threadIdx.y * 16 + threadIdx.x;
    const int ix0 = blockIdx.x * 16, iy0 = blockIdx.y * 16, iz0 = blockIdx.z * kZC;
    const int ix = ix0 + threadIdx.x, iy = iy0 + threadIdx.y;
    const bool active = ix < g.nx && iy < g.ny;   // the others stage and meet the barriers
    const int nu = g.nu, nv = g.nv, P = g.P;
    const double vox = g.vox, ivox = 1.0 / vox;
    const double Cx = 0.5 * (g.nx - 1), Cy = 0.5 * (g.ny - 1), Cz = 0.5 * (g.nz - 1), Cu = 0.5 * (nu - 1);
    const double Cv = 0.5 * (nv - 1), inv_du = 1.0 / g.du, inv_dv = 1.0 / g.dv;
    const float Cvf = (float)(0.5 * (nv - 1));
    const float zoff = (float)(0.5 * (g.nz - 1) - iz0);   // f_c - iz0 = zoff + a1 (av - Cv)
    const double bx0 = (ix0 - 1 - Cx) * vox, bx1 = (min(ix0 + 15, g.nx - 1) + 1 - Cx) * vox;
    const double by0 = (iy0 - 1 - Cy) * vox, by1 = (min(iy0 + 15, g.ny - 1) + 1 - Cy) * vox;
    const double bz0 = (iz0 - 1 - Cz) * vox, bz1 = (min(iz0 + kZC - 1, g.nz - 1) + 1 - Cz) * vox;
    constexpr int Q = kTSU / 4;
    constexpr int kCells = kTVG * kTSV * Q;
    for (int q = tid; q < kTVG * 2 * kTG * kTSU; q += 256) {   // guard rows, once
        const int vv = q / (2 * kTG * kTSU), r = (q / kTSU) % (2 * kTG), c = q % kTSU;
        const_cast<float *>(tile)[vv * kTVS + (r < kTG ? r : kTSV + r) * kTSU + c] = 0.0f;
    }
    const int zmax = min(kZC, g.nz - iz0);   // voxels of the chunk inside the volume
    double acc[kZC];
    float accz[kZC];
#pragma unroll
    for (int z = 0; z < kZC; ++z) { acc[z] = 0.0; accz[z] = 0.0f; }
    // z splat of detector column au (its table entry T) on the plane at
    // distance D from the source into the 16 slots at sl (rows feeding the
    // chunk [iz0 - 1, iz0 + kZC]); w scales every contribution
    auto splat = [&](float *sl, float ar, double D, int p, int au, float w, bool fit, int bu0, int bv0,
                     const float *tv) {
        const float a1 = (float)D * ar, ia1 = 1.0f / a1;
        const float r1 = fmaf(-1.0f - zoff, ia1, Cvf), r2 = fmaf((float)kZC - zoff, ia1, Cvf);
        const int v0 = max((int)ceilf(fminf(r1, r2)), 0), v1 = min((int)floorf(fmaxf(r1, r2)), nv - 1);
        const int lu = min(max(au - bu0, 0), kTSU - 1);
        const float *yp = ys + (size_t)p * nv * nu + au;
        for (int av = v0; av <= v1; ++av) {
            const float zf = fmaf(a1, (float)av - Cvf, zoff);
            const float zl = floorf(zf), w1 = zf - zl;
            const int zi = (int)zl;
            const float yv = fit ? tv[min(max(av - bv0, 0), kTSV - 1) * kTSU + lu] : yp[(size_t)av * nu];
            const float val = w * yv;
            if ((unsigned)zi < (unsigned)kZC) sl[zi] = fmaf(1.0f - w1, val, sl[zi]);
            if ((unsigned)(zi + 1) < (unsigned)kZC) sl[zi + 1] = fmaf(w1, val, sl[zi + 1]);
        }
    };
    for (int p0 = 0; p0 < P; p0 += kTVG) {
        __syncthreads();   // the previous group's readers are done with the tile, sheets and tables
        if (tid == 0) s_fit = 1;
        if (tid < 4 * kTVG) {
            // footprint of each view from the block's four corner columns,
            // one corner per lane, reduced over the view's four lanes
            const int vv = tid >> 2, k = tid & 3;
            const int p = min(p0 + vv, P - 1);
            const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
            const double px = (k & 1) ? bx1 : bx0, py = (k & 2) ? by1 : by0;
            const double U = g.sod - (px * c + py * s);
            const double M = g.sdd / U;
            const double fu = M * (py * c - px * s) * inv_du + Cu;
            const double va = M * bz0 * inv_dv + Cv, vb = M * bz1 * inv_dv + Cv;
            const double vlo = fmin(va, vb), vhi = fmax(va, vb);
            int bad = !(fu > -1e6 && fu < 1e6 && vlo > -1e6 && vhi < 1e6);
            int ulo = bad ? 0 : (int)floor(fu), uhi = ulo;
            int vl = bad ? 0 : (int)floor(vlo), vh = bad ? 0 : (int)floor(vhi);
#pragma unroll
            for (int m = 1; m < 4; m <<= 1) {
                ulo = min(ulo, __shfl_xor(ulo, m));
                uhi = max(uhi, __shfl_xor(uhi, m));
                vl = min(vl, __shfl_xor(vl, m));
                vh = max(vh, __shfl_xor(vh, m));
                bad |= __shfl_xor(bad, m);
            }
            if (k == 0 && p0 + vv < P) {
                const int u0 = (ulo - 1) & ~3, u1 = uhi + 2;
                const int v0 = vl - 1, v1 = vh + 2;
                s_box[vv][0] = u0;
                s_box[vv][1] = v0;
                if (bad || u1 - u0 >= kTSU || v1 - v0 >= kTSV) atomicAnd(&s_fit, 0);
            }
        }
        if (tid < kTVG * 2) s_wide[tid / 2][tid % 2] = 0;
        __syncthreads();
        // column range of every (view, axis, plane) of the block: the columns
        // whose f_b at the plane lies within one voxel of the block's b range
        if (tid >= 64 && tid < 64 + kTVG * 32) {
            const int q = tid - 64, vv = q / 32, a = (q / 16) % 2, jj = q % 16;
            const int p = p0 + vv;
            int first = 0, cnt = 0;
            const int vd = p < P ? g.vdom[p] : 0;
            if (p < P && (vd & (1 << a)) && (a ? iy0 + jj < g.ny : ix0 + jj < g.nx)) {
                const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
                const double ox = g.sod * c, oy = g.sod * s;
                const double D = a ? (iy0 + jj - Cy) * vox - oy : (ix0 + jj - Cx) * vox - ox;
                const int ib0 = a ? ix0 : iy0, nb = min(16, (a ? g.nx : g.ny) - ib0);
                const double e0 = (a ? ox : oy) - (ib0 - (a ? Cx : Cy)) * vox;
                int lo, hi;
                column_range(g, a, c, s, D, e0, -1.0, (double)nb, lo, hi);
                if (vd & kVdomOneSwitch) {
                    // the axis's columns are one interval: keep the range within it
                    const int sw = vd >> kVdomSwitchShift;
                    const bool first_is_a = ((vd & kVdomX0) != 0) == (a == 0);
                    if (first_is_a) {
                        if (sw > 0) hi = min(hi, sw - 1);
                    } else {
                        lo = max(lo, sw);
                    }
                }
                first = lo;
                cnt = hi >= lo ? hi - lo + 1 : 0;
                if (cnt > kZU) atomicOr(&s_wide[vv][a], 1);
                // the inverse map of column_range, written out for the gather
                const double al = a ? -s : c, be = a ? -g.sdd * c : -g.sdd * s;
                const double ga = a ? c : -s, de = a ? -g.sdd * s : -g.sdd * c;
                s_cf[vv][a][jj] = make_float4((float)((be * D + de * e0) * inv_du), (float)(-de * vox * inv_du),
                                              (float)(-ga * e0 - al * D), (float)(ga * vox));
            }
            s_rng[vv][a][jj][0] = first;
            s_rng[vv][a][jj][1] = cnt;
            // list of the pairs: exclusive scan of the planes' counts over
            // the 16 lanes of (view, axis)
            const int cl = min(cnt, kZU);
            int inc = cl;
#pragma unroll
            for (int d = 1; d < 16; d <<= 1) {
                const int o = __shfl_up(inc, d, 16);
                if (jj >= d) inc += o;
            }
            // entry: column within the plane's range | plane << 5 | column
            // within the staged box << 9; a column outside the box sends the
            // (view, axis) to the per-voxel path
            bool outside = false;
            for (int kk = 0; kk < cl; ++kk) {
                const int lc = first + kk - s_box[vv][0];
                outside |= (unsigned)lc >= (unsigned)kTSU;
                s_list[vv][a][inc - cl + kk] = (unsigned short)(kk | jj << 5 | (lc & 127) << 9);
            }
            if (outside) atomicOr(&s_wide[vv][a], 1);
            if (jj == 15) s_npairs[vv][a] = inc;
        }
        const bool fit = s_fit != 0;
        if (fit) {
            for (int q = tid; q < kCells; q += 256) {
                const int vv = q / (kTSV * Q), r = (q / Q) % kTSV, c4 = 4 * (q % Q);
                const int p = p0 + vv;
                float4 e = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (p < P) {
                    const int v = s_box[vv][1] + r, u = s_box[vv][0] + c4;
                    if ((unsigned)v < (unsigned)nv) {
                        const float *row = ys + ((size_t)p * nv + v) * nu;
                        if ((nu & 3) == 0 && (unsigned)u <= (unsigned)(nu - 4)) {
                            e = *reinterpret_cast<const float4 *>(row + u);
                        } else {
                            float t4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                if (u + k >= 0 && u + k < nu) t4[k] = row[u + k];
                            e = make_float4(t4[0], t4[1], t4[2], t4[3]);
                        }
                    }
                }
                tile4[(vv * kTVS + (r + kTG) * kTSU) / 4 + c4 / 4] = e;
            }
            for (int q = tid; q < kTVG * kTSU; q += 256) {
                const int vv = q / kTSU, cc = q % kTSU;
                const int p = p0 + vv, u = s_box[vv][0] + cc;
                double t = 0.0;
                float2 ai = make_float2(0.0f, 0.0f);
                if (p < P && (unsigned)u < (unsigned)nu) {
                    const ColT &T = g.colT[(size_t)p * nu + u];
                    t = T.t;
                    ai = make_float2(T.ar, T.is);
                }
                s_Tt[vv][cc] = t;
                s_Tai[vv][cc] = ai;
            }
        }
        __syncthreads();
        for (int vv = 0; vv < kTVG && p0 + vv < P; ++vv) {
            const int p = p0 + vv;
            const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
            const double ox = g.sod * c, oy = g.sod * s;
            const float *tv = tile + vv * kTVS + kTG * kTSU;   // first staged row
            const int bu0 = s_box[vv][0], bv0 = s_box[vv][1];
            const ColT *Tp = g.colT + (size_t)p * nu;
            const int vd = g.vdom[p];
#pragma unroll 1
            for (int a = 0; a < 2; ++a) {
                if (!(vd & (1 << a))) continue;   // uniform: no column of this view has this axis
                // this work-item's voxel column on the axis's planes
                const int jj = a ? (int)threadIdx.y : (int)threadIdx.x;
                const int ib = a ? ix : iy;
                const double D = a ? (iy - Cy) * vox - oy : (ix - Cx) * vox - ox;
                const double e0 = (a ? ox : oy) - (ib - (a ? Cx : Cy)) * vox;
                const double eb0 = (a ? ox : oy) - ((a ? ix0 : iy0) - (a ? Cx : Cy)) * vox;
                const double Dp0 = a ? (iy0 - Cy) * vox - oy : (ix0 - Cx) * vox - ox;   // the block's first plane
                if (fit && !s_wide[vv][a]) {
                    // splat: (plane, column) pairs of the block, z by z in
                    // registers.  Voxel z takes the rows with |f_c - z| < 1,
                    // f_c - z = a1 (v - vc(z)), vc(z) = Cv + (z - zoff) / a1:
                    // with |a1| in (1/2, 2) (one row per voxel within a factor
                    // of two) those are among floor(vc) - 1 .. floor(vc) + 2,
                    // with tent weights 1 - |a1| |v - vc| clipped at zero.
                    // Half a pair (8 voxels of z) per step, over the listed
                    // pairs, first halves then second halves.  The first half
                    // also records the column's f_b on the plane relative to
                    // the block's first voxel column (NaN for a column of the
                    // other axis, possible where the axis changes twice).
                    const int npairs = s_npairs[vv][a];
                    for (int h = tid; h < 2 * npairs; h += 256) {
                        const int half = h >= npairs;
                        const int e = s_list[vv][a][half ? h - npairs : h];
                        const int k = e & 31, pj = (e >> 5) & 15, lc = e >> 9, zh = half * (kZC / 2);
                        const int q = pj * kZU + k;
                        // the column's table entry, staged with the data
                        const double Tt = s_Tt[vv][lc];
                        const float2 ai = s_Tai[vv][lc];
                        const float Tar = ai.x, Tis = ai.y;
                        const int au = bu0 + lc;
                        const bool other = (Tis > 0.0f) != (a == 0);   // the projector's dominant axis
                        const double Dp = fma((double)pj, vox, Dp0);
                        if (zh == 0) s_fb[q] = other ? __builtin_nan("") : (eb0 + Dp * Tt) * ivox;
                        if (other) continue;
                        float *sl = s_z + pj * kPS + k * kZS;
                        const float a1 = (float)Dp * Tar, aa = fabsf(a1);
                        if (!(aa > 0.5f && aa < 2.0f)) {   // steep or flat rows: row by row
                            if (zh == 0) {
#pragma unroll
                                for (int z = 0; z < kZC; ++z) sl[z] = 0.0f;
                                splat(sl, Tar, Dp, p, au, 1.0f, true, bu0, bv0, tv);
                            }
                            continue;
                        }
                        // 1 / a1: the hardware reciprocal and one Newton step
                        const float r0 = __builtin_amdgcn_rcpf(a1);
                        const float ia1 = fmaf(fmaf(-a1, r0, 1.0f), r0, r0);
                        const float am = 1.0f - aa;
                        // row positions relative to the first guard row
                        const float vrb = fmaf((float)zh, ia1, fmaf(-zoff, ia1, Cvf - (float)(bv0 - kTG)));
                        const uint32_t t = (uint32_t)(size_t)(lds_cfloat *)(tv - kTG * kTSU + lc);
                        float out[kZC / 2];
                        if (zmax == kZC) sheet_rows<false>(out, t, vrb, ia1, aa, am);
                        else sheet_rows<true>(out, t, vrb, ia1, aa, am);
#pragma unroll
                        for (int zz = 0; zz < kZC / 2; ++zz) sl[zh + zz] = out[zz];
                    }
                    __syncthreads();
                    if (active) {
                        // candidate columns: f_b within one voxel of this column's,
                        // i.e. strictly between col(jb - 1) and col(jb + 1) where the
                        // map has no pole in between (FP32, 1e-3 column of margin)
                        const int first = s_rng[vv][a][jj][0], cnt = s_rng[vv][a][jj][1];
                        const int jbi = ib - (a ? ix0 : iy0);
                        const float4 cf = s_cf[vv][a][jj];
                        const float fm = (float)(jbi - 1), fp = (float)(jbi + 1);
                        const float dm = fmaf(cf.w, fm, cf.z), dp = fmaf(cf.w, fp, cf.z);
                        int k0 = 0, k1 = cnt - 1;
                        if ((dm > 0.0f && dp > 0.0f) || (dm < 0.0f && dp < 0.0f)) {
                            const float c0 = (float)(Cu - first);
                            const float um = fmaf(cf.y, fm, cf.x) * __builtin_amdgcn_rcpf(dm) + c0;
                            const float up = fmaf(cf.y, fp, cf.x) * __builtin_amdgcn_rcpf(dp) + c0;
                            k0 = max(k0, (int)ceilf(fminf(um, up) - 1e-3f));
                            k1 = min(k1, (int)floorf(fmaxf(um, up) + 1e-3f));
                        }
                        const double jb = (double)jbi;
                        for (int k = k0; k <= k1; ++k) {
                            const float wb = 1.0f - fabsf((float)(s_fb[jj * kZU + k] - jb));
                            if (!(wb > 0.0f)) continue;   // NaN: a column of the other axis
                            const float *sl = s_z + jj * kPS + k * kZS;
#pragma unroll
                            for (int z = 0; z < kZC; ++z) accz[z] = fmaf(wb, sl[z], accz[z]);
                        }
                    }
                    __syncthreads();   // sheets read before the next splat
                } else {
                    // planes wider than the sheets, a column outside the staged
                    // box, or a group that does not fit: each voxel column
                    // splats its own candidates into private slots (the
                    // sheets' LDS), from the staged data where it has them
                    float *sl = s_z + tid * kATS;
                    if (active) {
#pragma unroll
                        for (int z = 0; z < kZC; ++z) sl[z] = 0.0f;
                        int a_lo, a_hi;
                        column_range(g, a, c, s, D, e0, -1.0, 1.0, a_lo, a_hi);
                        for (int au = a_lo; au <= a_hi; ++au) {
                            const ColT T = Tp[au];
                            if ((T.is > 0.0f) != (a == 0)) continue;
                            const float wb = 1.0f - fabsf((float)((e0 + D * T.t) * ivox));
                            if (!(wb > 0.0f)) continue;
                            splat(sl, T.ar, D, p, au, wb, fit && (unsigned)(au - bu0) < (unsigned)kTSU, bu0, bv0, tv);
                        }
#pragma unroll
                        for (int z = 0; z < kZC; ++z) accz[z] += sl[z];
                    }
                    __syncthreads();   // private slots overlap the next sheets
                }
            }
        }
        // views summed in FP32 over the group, then in FP64
#pragma unroll
        for (int z = 0; z < kZC; ++z) { acc[z] += (double)accz[z]; accz[z] = 0.0f; }
    }
    if (!active) return;
    const double sc = scale ? (double)*scale : 1.0;
#pragma unroll
    for (int z = 0; z < kZC; ++z) {
        const int iz = iz0 + z;
        if (iz < g.nz) x[((size_t)iz * g.ny + iy) * g.nx + ix] = (float)(acc[z] * sc);
    }
}

// --------------------------------------------------------------- B_un

// ------------------------------------------- line-intersection projector
// A_ij = length of ray i inside voxel j (the forward model the paper uses,
// Sec. III).  One work-item per ray walks the voxels the ray crosses: the
// ray enters and leaves the grid at the parameters of the slab test, and per
// axis the parameter of the next boundary plane advances by d/|r_a| at each
// crossing of that axis.  Every step adds (t_next - t) x[voxel]; parameters
// and sums are FP64 (the walk over hundreds of planes would lose 1e-4 of a
// voxel in FP32, and FP64 runs at the FP32 rate here).  The loop stops at the
// exit parameter or when an index leaves the grid, whichever comes first, and
// is bounded by nx + ny + nz + 2 steps, so no read is out of range.  Rays
// lying exactly on a boundary plane give their length to one neighbour.
struct SiddonWalk {
    double t, t_out;            // current and exit parameter (length units)
    double tn0, tn1, tn2;       // parameter of the next boundary per axis
    double dt0, dt1, dt2;       // parameter step between boundaries per axis
    int i0, i1, i2;             // current voxel
    int st0, st1, st2;          // step direction per axis (0: parallel)
    bool hit;
};

__device__ __forceinline__ void siddon_axis(double o, double r, double lo, double vox, int N, double t_in,
                                            bool hit, int &i, int &st, double &dt, double &tn) {
    const double f = hit ? (o + t_in * r - lo) / vox : 0.0;
    int k = (int)floor(f);
    k = k < 0 ? 0 : (k >= N ? N - 1 : k);   // the entry face rounds either way
    i = k;
    if (r > 0.0) {
        st = 1; dt = vox / r; tn = (lo + (k + 1) * vox - o) / r;
    } else if (r < 0.0) {
        st = -1; dt = -vox / r; tn = (lo + k * vox - o) / r;
    } else {
        st = 0; dt = 0.0; tn = 1e300;
    }
}

template <bool CONE>
__device__ __forceinline__ SiddonWalk siddon_setup(const GeomK &g, int p, int av, int au) {
    const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
    double ox, oy, rx, ry, rz;
    if (CONE) {
        const double u = (au - 0.5 * (g.nu - 1)) * g.du, v = (av - 0.5 * (g.nv - 1)) * g.dv;
        ox = g.sod * c; oy = g.sod * s;
        rx = -g.sdd * c - u * s; ry = -g.sdd * s + u * c; rz = v;
    } else {
        const double sa = (au - 0.5 * (g.nu - 1)) * g.du;
        ox = sa * c; oy = sa * s;
        rx = -s; ry = c; rz = 0.0;
    }
    const double inv = 1.0 / sqrt(rx * rx + ry * ry + rz * rz);   // unit speed: parameters are lengths
    rx *= inv; ry *= inv; rz *= inv;
    const double lox = -0.5 * g.nx * g.vox, loy = -0.5 * g.ny * g.vox, loz = -0.5 * g.nz * g.vox;
    SiddonWalk w;
    w.hit = true;
    double t_in = -1e300, t_out = 1e300;
    auto slab = [&](double o, double r, double lo) {
        if (r == 0.0) {
            if (!(o > lo && o < -lo)) w.hit = false;
            return;
        }
        const double t1 = (lo - o) / r, t2 = (-lo - o) / r;
        t_in = fmax(t_in, fmin(t1, t2));
        t_out = fmin(t_out, fmax(t1, t2));
    };
    slab(ox, rx, lox);
    slab(oy, ry, loy);
    slab(0.0, rz, loz);
    if (!(t_in < t_out)) w.hit = false;
    w.t = t_in;
    w.t_out = t_out;
    siddon_axis(ox, rx, lox, g.vox, g.nx, t_in, w.hit, w.i0, w.st0, w.dt0, w.tn0);
    siddon_axis(oy, ry, loy, g.vox, g.ny, t_in, w.hit, w.i1, w.st1, w.dt1, w.tn1);
    siddon_axis(0.0, rz, loz, g.vox, g.nz, t_in, w.hit, w.i2, w.st2, w.dt2, w.tn2);
    return w;
}

// One step of the walk: the segment [t, min(next boundary, exit)] lies in the
// current voxel; returns its length and advances to the next voxel.  `more`
// turns false at the exit or when the index leaves the grid.
__device__ __forceinline__ double siddon_step(const GeomK &g, SiddonWalk &w, long &idx, bool &more) {
    const bool a0 = w.tn0 <= w.tn1 && w.tn0 <= w.tn2;
    const bool a1 = !a0 && w.tn1 <= w.tn2;
    const double tb = a0 ? w.tn0 : (a1 ? w.tn1 : w.tn2);
    const double tn = fmin(tb, w.t_out);
    const double len = tn - w.t;
    w.t = tn;
    more = tb < w.t_out;
    if (a0) {
        w.tn0 += w.dt0; w.i0 += w.st0; idx += w.st0;
        more = more && w.i0 >= 0 && w.i0 < g.nx;
    } else if (a1) {
        w.tn1 += w.dt1; w.i1 += w.st1; idx += (long)w.st1 * g.nx;
        more = more && w.i1 >= 0 && w.i1 < g.ny;
    } else {
        w.tn2 += w.dt2; w.i2 += w.st2; idx += (long)w.st2 * g.nx * g.ny;
        more = more && w.i2 >= 0 && w.i2 < g.nz;
    }
    return len;
}

// Sum over the voxels one ray crosses of length x value, walking the plain
// volume.  The walk does not depend on the data: it advances eight steps,
// then issues their eight gathers together (a finished walk repeats its last
// voxel with length 0); 8 beat 4 and 2 at 256^3 (12.8, 13.3, 17.2 ms).
template <bool CONE>
__device__ __forceinline__ double siddon_walk_sum(const GeomK &g, const float *__restrict__ x, int p, int av,
                                                  int au) {
    SiddonWalk w = siddon_setup<CONE>(g, p, av, au);
    double acc = 0.0;
    if (w.hit) {
        constexpr int U = 8;
        long idx = w.i0 + (long)w.i1 * g.nx + (long)w.i2 * g.nx * g.ny;
        const int steps = g.nx + g.ny + g.nz + 2;
        bool more = true;
        for (int k = 0; k < steps && more; k += U) {
            long at[U];
            double len[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                at[u] = idx;
                len[u] = 0.0;
                if (more) {
                    const long cur = idx;
                    len[u] = siddon_step(g, w, idx, more);
                    at[u] = cur;
                    if (!more) idx = cur;   // keep the index of a voxel inside the grid
                }
            }
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = x[at[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) acc = fma(len[u], (double)v[u], acc);
        }
    }
    return acc;
}

// One work-item per ray (2D geometries; cone geometries take the staged
// kernel).
template <bool CONE, typename OutT>
__global__ __launch_bounds__(256) void k_siddon(GeomK g, const float *__restrict__ x, OutT *__restrict__ y,
                                                const float *__restrict__ out_scale,
                                                const int *__restrict__ stop) {
    if (stop && *stop) return;
    const int au = blockIdx.x * blockDim.x + threadIdx.x;
    const int av = blockIdx.y * blockDim.y + threadIdx.y;
    const int p = blockIdx.z;
    if (au >= g.nu || av >= g.nv) return;
    float val = (float)siddon_walk_sum<CONE>(g, x, p, av, au);
    if (out_scale) val *= *out_scale;
    y[((size_t)p * g.nv + av) * g.nu + au] = from_f<OutT>(val);
}

// transpose: the same walk, scattering y_i * length into x with FP32 atomics
template <bool CONE, typename InT>
__global__ __launch_bounds__(256) void k_siddon_T(GeomK g, const InT *__restrict__ y, float *__restrict__ x,
                                                  const float *__restrict__ in_scale,
                                                  const int *__restrict__ stop) {
    if (stop && *stop) return;
    const int au = blockIdx.x * blockDim.x + threadIdx.x;
    const int av = blockIdx.y * blockDim.y + threadIdx.y;
    const int p = blockIdx.z;
    if (au >= g.nu || av >= g.nv) return;
    double yv = (double)to_f(y[((size_t)p * g.nv + av) * g.nu + au]);
    if (in_scale) yv *= (double)*in_scale;
    if (yv == 0.0) return;
    SiddonWalk w = siddon_setup<CONE>(g, p, av, au);
    if (!w.hit) return;
    long idx = w.i0 + (long)w.i1 * g.nx + (long)w.i2 * g.nx * g.ny;
    const int steps = g.nx + g.ny + g.nz + 2;
    bool more = true;
    for (int k = 0; k < steps && more; ++k) {
        const long at = idx;
        const double len = siddon_step(g, w, idx, more);
        if (len > 0.0) unsafeAtomicAdd(x + at, (float)(yv * len));
    }
}

// ---------------------------------------------- staged 3D back-projector
// A workgroup is 16 x 16 columns (x, y) times kZC voxels in z.  For groups of
// kVG views it copies each view's footprint (kSV rows x kSU columns of the
// detector, zero outside it) into LDS with 16-byte loads, then every column
// reads its bilinear taps for all kZC voxels from LDS.  The footprint of a
// view comes from the workgroup's four corner columns: u is monotone along
// x and y at fixed view, v is monotone in z and along the view direction.
// Workgroups with any footprint larger than the tile take the direct path.
constexpr int kVG = 5;               // views per staged group (4: 2.17 ms at 256^3, 5: 2.14; LDS holds 5 workgroups per CU either way)
constexpr int kSU = 36, kSV = 32;    // staged detector columns / rows per view
constexpr int kMaxViewsStaged = 2048;

__device__ __forceinline__ void project_point(const GeomK &g, double px, double py, double c, double s,
                                              double &fu, double &M) {
    const double U = g.sod - (px * c + py * s);
    M = g.sdd / U;
    fu = M * (py * c - px * s) / g.du + 0.5 * (g.nu - 1);
}

template <typename InT>
__global__ __launch_bounds__(256, 5) void k_bp_cone_staged(GeomK g, const InT *__restrict__ y, float *__restrict__ x,
                                                        const float *__restrict__ in_scale,
                                                        const int *__restrict__ stop) {
    if (stop && *stop) return;
    __shared__ float4 tile4[kVG * kSV * kSU / 4];
    __shared__ short s_box[kMaxViewsStaged][2];
    __shared__ int s_bad;
    const float *tile = (const float *)tile4;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 16 + tx;
    const int ix0 = blockIdx.x * 16, iy0 = blockIdx.y * 16, iz0 = blockIdx.z * kZC;
    const int ix = ix0 + tx, iy = iy0 + ty;
    const bool active = ix < g.nx && iy < g.ny;
    const int nu = g.nu, nv = g.nv, P = g.P;
    if (tid == 0) s_bad = P > kMaxViewsStaged;
    __syncthreads();
    const double inv_dv = 1.0 / g.dv;
    const double cv = 0.5 * (nv - 1);
    // footprint of each view from the corner columns and the chunk's z range
    if (!s_bad) {
        const int ix1 = min(ix0 + 15, g.nx - 1), iy1 = min(iy0 + 15, g.ny - 1), iz1 = min(iz0 + kZC - 1, g.nz - 1);
        const double pza = (iz0 - 0.5 * (g.nz - 1)) * g.vox, pzb = (iz1 - 0.5 * (g.nz - 1)) * g.vox;
        for (int p = tid; p < P; p += 256) {
            const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
            double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
            for (int k = 0; k < 4; ++k) {
                const double px = ((k & 1 ? ix1 : ix0) - 0.5 * (g.nx - 1)) * g.vox;
                const double py = ((k & 2 ? iy1 : iy0) - 0.5 * (g.ny - 1)) * g.vox;
                double fu, M;
                project_point(g, px, py, c, s, fu, M);
                umin = fmin(umin, fu); umax = fmax(umax, fu);
                const double va = M * pza * inv_dv + cv, vb = M * pzb * inv_dv + cv;
                vmin = fmin(vmin, fmin(va, vb)); vmax = fmax(vmax, fmax(va, vb));
            }
            // one cell of margin each side; u start aligned to 4 for 16-byte loads
            const int u0 = ((int)floor(umin) - 1) & ~3, u1 = (int)floor(umax) + 2;
            const int v0 = (int)floor(vmin) - 1, v1 = (int)floor(vmax) + 2;
            if (u1 - u0 >= kSU || v1 - v0 >= kSV || u0 < -32000 || v0 < -32000 || u0 > 32000 || v0 > 32000)
                s_bad = 1;
            s_box[p][0] = (short)u0;
            s_box[p][1] = (short)v0;
        }
    }
    __syncthreads();
    const double px = (ix - 0.5 * (g.nx - 1)) * g.vox;
    const double py = (iy - 0.5 * (g.ny - 1)) * g.vox;
    const double pz0 = (iz0 - 0.5 * (g.nz - 1)) * g.vox;
    const double wconst = g.vox * g.vox * g.vox / (g.du * g.dv);
    double acc[kZC];
    float grp[kZC];
#pragma unroll
    for (int z = 0; z < kZC; ++z) { acc[z] = 0.0; grp[z] = 0.0f; }
    if (s_bad) {
        // direct path: masked gathers from global memory
        if (active) {
            for (int p = 0; p < P; ++p) {
                const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
                double fu, M;
                project_point(g, px, py, c, s, fu, M);
                const float dfv = (float)(M * g.vox * inv_dv);
                const float w = (float)(M * M * wconst);
                const float fuf = (float)fu;
                const float iuf = floorf(fuf);
                const float wu = fuf - iuf;
                const int iu = (int)iuf;
                const bool u0 = iu >= 0 && iu < nu, u1 = iu + 1 >= 0 && iu + 1 < nu;
                const float wu0 = u0 ? (1.0f - wu) * w : 0.0f, wu1 = u1 ? wu * w : 0.0f;
                const int c0 = u0 ? iu : 0, c1 = u1 ? iu + 1 : 0;
                const InT *yp = y + (size_t)p * nv * nu;
                const float fv0f = (float)(M * pz0 * inv_dv + cv);
#pragma unroll
                for (int z = 0; z < kZC; ++z) {
                    const float fv = fmaf((float)z, dfv, fv0f);
                    const float ivf = floorf(fv);
                    const float wv = fv - ivf;
                    const int iv = (int)ivf;
                    const bool v0 = iv >= 0 && iv < nv, v1 = iv + 1 >= 0 && iv + 1 < nv;
                    const size_t r0 = (size_t)(v0 ? iv : 0) * nu, r1 = (size_t)(v1 ? iv + 1 : 0) * nu;
                    const float a = wu0 * to_f(yp[r0 + c0]) + wu1 * to_f(yp[r0 + c1]);
                    const float b = wu0 * to_f(yp[r1 + c0]) + wu1 * to_f(yp[r1 + c1]);
                    grp[z] += (v0 ? 1.0f - wv : 0.0f) * a + (v1 ? wv : 0.0f) * b;
                }
                if ((p & 3) == 3 || p == P - 1) {
#pragma unroll
                    for (int z = 0; z < kZC; ++z) { acc[z] += (double)grp[z]; grp[z] = 0.0f; }
                }
            }
        }
    } else {
        constexpr int Q = kSU / 4;   // 16-byte chunks per staged row
        // per-column set-up in FP32 (positions within ~2e-5 detector cells)
        const float pxf = (float)px, pyf = (float)py;
        const float sodf = (float)g.sod, sddf = (float)g.sdd, inv_duf = (float)(1.0 / g.du);
        const float cuf = (float)(0.5 * (nu - 1)), cvf = (float)cv;
        const float dzf = (float)(g.vox * inv_dv), pz0f = (float)(pz0 * inv_dv), wcf = (float)wconst;
        // rows a multiple of four: 16-byte staging loads of FP32 data,
        // 8-byte loads of four FP16 values
        const bool vec4 = sizeof(InT) == 4 && (nu & 3) == 0 && ((uintptr_t)y & 15) == 0;
        const bool vec4h = sizeof(InT) == 2 && (nu & 3) == 0 && ((uintptr_t)y & 7) == 0;
        // Each work-item stages the same cells (view within the group, row,
        // 16-byte column) of every view group, so their coordinates are
        // computed once; a view's box is one LDS word (u0 low, v0 high).
        constexpr int kCells = kVG * kSV * Q, kCPT = (kCells + 255) / 256;
        uint32_t cell[kCPT];   // view in group | row << 8 | first column << 16
#pragma unroll
        for (int i = 0; i < kCPT; ++i) {
            const int q = tid + 256 * i;
            cell[i] = (uint32_t)(q / (kSV * Q)) | (uint32_t)((q / Q) % kSV) << 8 | (uint32_t)(4 * (q % Q)) << 16;
        }
        const uint32_t *boxw = reinterpret_cast<const uint32_t *>(&s_box[0][0]);
        for (int p0 = 0; p0 < P; p0 += kVG) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < kCPT; ++i) {
                const int q = tid + 256 * i;
                if (kCells % 256 != 0 && q >= kCells) break;
                const int p = p0 + (int)(cell[i] & 0xffu);
                float4 e = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (p < P) {
                    const uint32_t bx = boxw[p];
                    const int v = (int)(short)(bx >> 16) + (int)((cell[i] >> 8) & 0xffu);
                    const int u = (int)(short)(bx & 0xffffu) + (int)(cell[i] >> 16);
                    if ((unsigned)v < (unsigned)nv) {
                        const InT *row = y + (size_t)(uint32_t)(p * nv + v) * (uint32_t)nu;
                        if (vec4 && (unsigned)u <= (unsigned)(nu - 4)) {
                            e = *reinterpret_cast<const float4 *>(reinterpret_cast<const float *>(row) + u);
                        } else if (vec4h && (unsigned)u <= (unsigned)(nu - 4)) {
                            const uint2 h = *reinterpret_cast<const uint2 *>(row + u);
                            const float2 lo = __half22float2(__builtin_bit_cast(__half2, h.x));
                            const float2 hi = __half22float2(__builtin_bit_cast(__half2, h.y));
                            e = make_float4(lo.x, lo.y, hi.x, hi.y);
                        } else {
                            float t4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                if (u + k >= 0 && u + k < nu) t4[k] = to_f(row[u + k]);
                            e = make_float4(t4[0], t4[1], t4[2], t4[3]);
                        }
                    }
                }
                tile4[q] = e;
            }
            __syncthreads();
            // Rows: within a chunk whose kZC planes all lie in the volume the
            // box bounds every voxel's row with a cell of margin (v is
            // linear in z and linear-fractional across the columns, so its
            // extremes are at the corner columns and the end planes), and
            // the row index needs no clamp; the last, partial chunk keeps it.
            auto views = [&](auto clamp_rows) {
                constexpr bool kClampRows = decltype(clamp_rows)::value;
                for (int vv = 0; vv < kVG && p0 + vv < P; ++vv) {
                    const int p = p0 + vv;
                    const float c = g.cs32[2 * p], s = g.cs32[2 * p + 1];
                    const float M = sddf * __builtin_amdgcn_rcpf(fmaf(-pxf, c, fmaf(-pyf, s, sodf)));
                    const float dfv = M * dzf;
                    const float w = M * M * wcf;
                    // coordinates relative to the staged box are >= 1 (one
                    // cell of margin), so truncation is floor; the clamps only
                    // guard the tile against rounding
                    const float fur = fmaf(M * inv_duf, fmaf(pyf, c, -pxf * s), cuf - (float)s_box[p][0]);
                    const float wu = __builtin_amdgcn_fractf(fur);
                    const int lu = min(max((int)fur, 0), kSU - 2);
                    const float fv0r = fmaf(M, pz0f, cvf - (float)s_box[p][1]);
                    // the column's byte offset in the tile, kept whole in a
                    // register so that each row address is one 24-bit
                    // multiply-add (lv lies in [0, kSV - 2])
                    uint32_t tvb = (uint32_t)(vv * kSV * kSU + lu) * 4u;
                    asm("" : "+v"(tvb));
                    // the rows of voxel z + 1 are read while voxel z is
                    // interpolated (the scheduling barriers keep that order)
                    auto rows = [&](int z, float &r0, float &r1, float &r2, float &r3) {
                        const float fv = fmaf((float)z, dfv, fv0r);
                        const int lv = kClampRows ? min(max((int)fv, 0), kSV - 2) : (int)fv;
                        const float *t = reinterpret_cast<const float *>(
                            reinterpret_cast<const char *>(tile) + (__umul24((uint32_t)lv, (uint32_t)(kSU * 4)) + tvb));
                        r0 = t[0];
                        r1 = t[1];
                        r2 = t[kSU];
                        r3 = t[kSU + 1];
                    };
                    float q0, q1, q2, q3;
                    rows(0, q0, q1, q2, q3);
#pragma unroll
                    for (int z = 0; z < kZC; ++z) {
                        const float c0 = q0, c1 = q1, c2 = q2, c3 = q3;
                        if (z + 1 < kZC) rows(z + 1, q0, q1, q2, q3);
                        __builtin_amdgcn_sched_barrier(0);
                        const float wv = __builtin_amdgcn_fractf(fmaf((float)z, dfv, fv0r));
                        const float a = fmaf(wu, c1 - c0, c0);
                        const float b = fmaf(wu, c3 - c2, c2);
                        grp[z] = fmaf(w, fmaf(wv, b - a, a), grp[z]);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            };
            if (active) {
                if (iz0 + kZC <= g.nz) views(std::false_type{});
                else views(std::true_type{});
#pragma unroll
                for (int z = 0; z < kZC; ++z) { acc[z] += (double)grp[z]; grp[z] = 0.0f; }
            }
        }
    }
    if (!active) return;
    const double sc = in_scale ? (double)*in_scale : 1.0;
#pragma unroll
    for (int z = 0; z < kZC; ++z) {
        const int iz = iz0 + z;
        if (iz < g.nz) x[((size_t)iz * g.ny + iy) * g.nx + ix] = (float)(acc[z] * sc);
    }
}

template <typename InT>
__global__ __launch_bounds__(256) void k_bp_par(GeomK g, const InT *__restrict__ y, float *__restrict__ x,
                                                const float *__restrict__ in_scale,
                                                const int *__restrict__ stop) {
    if (stop && *stop) return;
    const int ix = blockIdx.x * 16 + threadIdx.x, iy = blockIdx.y * 16 + threadIdx.y;
    if (ix >= g.nx || iy >= g.ny) return;
    const double inv_du = 1.0 / g.du;
    const double px = (ix - 0.5 * (g.nx - 1)) * g.vox * inv_du;
    const double py = (iy - 0.5 * (g.ny - 1)) * g.vox * inv_du;
    const double cu = 0.5 * (g.nu - 1);
    const int nu = g.nu;
    // views summed in FP32 in groups of four, groups in FP64
    double acc = 0.0;
    float grp = 0.0f;
    for (int p = 0; p < g.P; ++p) {
        const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
        const float fu = (float)(px * c + py * s + cu);
        const float iuf = floorf(fu);
        const float wu = fu - iuf;
        const int iu = (int)iuf;
        const bool u0 = iu >= 0 && iu < nu, u1 = iu + 1 >= 0 && iu + 1 < nu;
        const InT *yp = y + (size_t)p * nu;
        const float a = u0 ? to_f(yp[u0 ? iu : 0]) : 0.0f;
        const float b = u1 ? to_f(yp[u1 ? iu + 1 : 0]) : 0.0f;
        grp += fmaf(wu, b - a, a);
        if ((p & 3) == 3 || p == g.P - 1) { acc += (double)grp; grp = 0.0f; }
    }
    const double sc = in_scale ? (double)*in_scale : 1.0;
    x[(size_t)iy * g.nx + ix] = (float)(acc * (g.vox * g.vox * inv_du) * sc);
}

// 2D Joseph A^T gathered per pixel, deterministic.  For a parallel-beam
// view with direction d = (-sin t, cos t) and dominant component r_a
// (sin t for x-major views, whose samples lie on the columns x = const;
// cos t for y-major views), the sample of ray a on the pixel's plane lies
// (s_a - p.n) / r_a from the pixel centre along the other axis, s_a the
// bin's offset and p.n the pixel centre projected on n = (cos t, sin t).
// The pixel's weight in that ray is therefore tent((s_a - p.n) / (r_a vox))
// times the step vox / |r_a|: a tent on the detector of half-width
// |r_a| vox, which covers at most three bins.  The dominant axis is the
// forward projector's (the per-view table with the integer tie rule).
// Views are summed in FP32 in groups of four, groups in FP64.
template <typename InT>
__global__ __launch_bounds__(256) void k_project_T_par(GeomK g, const InT *__restrict__ y, float *__restrict__ x,
                                                       const float *__restrict__ in_scale,
                                                       const int *__restrict__ stop) {
    if (stop && *stop) return;
    const int ix = blockIdx.x * 16 + threadIdx.x, iy = blockIdx.y * 16 + threadIdx.y;
    if (ix >= g.nx || iy >= g.ny) return;
    const double px = (ix - 0.5 * (g.nx - 1)) * g.vox, py = (iy - 0.5 * (g.ny - 1)) * g.vox;
    const double cu = 0.5 * (g.nu - 1), inv_du = 1.0 / g.du;
    const int nu = g.nu;
    double acc = 0.0;
    float grp = 0.0f;
    for (int p = 0; p < g.P; ++p) {
        const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
        const double ra = fabs(g.axis[p] == 0 ? s : c);
        const double pn = px * c + py * s, hw = ra * g.vox;
        const double lo = (pn - hw) * inv_du + cu, hi = (pn + hw) * inv_du + cu;
        const int a0 = max((int)ceil(lo), 0), a1 = min((int)floor(hi), nu - 1);
        const InT *yp = y + (size_t)p * nu;
        float v = 0.0f;
        for (int a = a0; a <= a1; ++a) {
            const double w = 1.0 - fabs(((a - cu) * g.du - pn) / hw);
            if (w > 0.0) v = fmaf((float)w, to_f(yp[a]), v);
        }
        grp = fmaf((float)(g.vox / ra), v, grp);
        if ((p & 3) == 3 || p == g.P - 1) { acc += (double)grp; grp = 0.0f; }
    }
    const double sc = in_scale ? (double)*in_scale : 1.0;
    x[(size_t)iy * g.nx + ix] = (float)(acc * sc);
}

// ----------------------------------------------------------------- F
// Generic row filter: one workgroup per row, one output per lane (rows of
// any length up to 4096).
template <typename InT, typename OutT>
__global__ __launch_bounds__(256) void k_ramp(const InT *__restrict__ q, OutT *__restrict__ out,
                                              const float *__restrict__ taps, int nu,
                                              const int *__restrict__ stop) {
    if (stop && *stop) return;
    extern __shared__ float sm[];
    float *qs = sm;            // [nu zeros][row][nu zeros]
    float *hs = sm + 3 * nu;   // du * h[j]
    const size_t row = blockIdx.x;
    const InT *qr = q + row * nu;
    for (int i = threadIdx.x; i < nu; i += blockDim.x) {
        qs[i] = 0.0f;
        qs[nu + i] = to_f(qr[i]);
        qs[2 * nu + i] = 0.0f;
        hs[i] = taps[i];
    }
    __syncthreads();
    for (int a = threadIdx.x; a < nu; a += blockDim.x) {
        const float *qa = qs + nu + a;
        float acc = hs[0] * qa[0];
        for (int j = 1; j < nu; j += 2) acc = fmaf(hs[j], qa[-j] + qa[j], acc);
        out[row * nu + a] = from_f<OutT>(acc);
    }
}

// Register-blocked row filter: one wavefront per row, RB consecutive outputs
// per lane (nu <= 64 RB).  For odd tap j the lane needs q[a-j] and q[a+j] for
// its RB outputs; stepping j by two shifts both windows by two, so each step
// reads four new values from LDS and does RB adds and RB FMAs.  The
// symmetric, odd-only Ram-Lak taps (h[even] = 0) halve the work of a dense
// convolution.  Four rows per workgroup.
template <int RB, typename InT, typename OutT>
__global__ __launch_bounds__(256) void k_ramp_rb(const InT *__restrict__ q, OutT *__restrict__ out,
                                                 const float *__restrict__ taps, int nu, size_t rows,
                                                 const int *__restrict__ stop) {
    if (stop && *stop) return;
    constexpr int W = 64 * RB;                 // padded row length handled
    constexpr int E = 4;                       // guard cells: the last window shift reads past +-W
    __shared__ float qs[4][3 * W + 2 * E];     // [E + W zeros][row][W + E zeros]
    __shared__ float hs[W];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const size_t row = (size_t)blockIdx.x * 4 + wv;
    for (int i = threadIdx.x; i < W; i += 256) hs[i] = i < nu ? taps[i] : 0.0f;
    float *qw = qs[wv];
    for (int i = lane; i < 3 * W + 2 * E; i += 64) {
        const int a = i - W - E;
        qw[i] = (row < rows && a >= 0 && a < nu) ? to_f(q[row * nu + a]) : 0.0f;
    }
    __syncthreads();
    if (row >= rows) return;
    const int a0 = lane * RB;
    const float *qc = qw + E + W + a0;         // q[a0 + r] = qc[r]
    float acc[RB], L[RB], U[RB];
    const float h0 = hs[0];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = h0 * qc[r];
    // window for j = 1: L[r] = q[a0 + r - 1], U[r] = q[a0 + r + 1]
#pragma unroll
    for (int r = 0; r < RB; ++r) { L[r] = qc[r - 1]; U[r] = qc[r + 1]; }
    for (int j = 1; j < nu; j += 2) {
        const float h = hs[j];
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[r] = fmaf(h, L[r] + U[r], acc[r]);
        // shift to j + 2
#pragma unroll
        for (int r = RB - 1; r >= 2; --r) L[r] = L[r - 2];
        L[1] = qc[-j - 1];
        L[0] = qc[-j - 2];
#pragma unroll
        for (int r = 0; r < RB - 2; ++r) U[r] = U[r + 2];
        U[RB - 2] = qc[RB - 2 + j + 2];
        U[RB - 1] = qc[RB - 1 + j + 2];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
        if (a0 + r < nu) out[row * nu + a0 + r] = from_f<OutT>(acc[r]);
}


// ------------------------------------------------ batched 2D problems
// Workgroup b belongs to problem s with pfx[s] <= b < pfx[s+1].  The search
// is uniform across the workgroup, so its loads are scalar.
__device__ __forceinline__ int find_slice(const int *__restrict__ pfx, int count, int b) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pfx[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// XCD-aware order: the hardware deals workgroups round-robin to the eight
// XCDs; remap so that each XCD receives a contiguous range of logical
// workgroups (neighbouring rays / pixels of the same problems, whose image
// and data then stay in that XCD's L2).  False for the padding workgroups.
__device__ __forceinline__ bool xcd_block(int nblk, int &b) {
    const int per = (nblk + 7) >> 3;
    const int hw = blockIdx.x;
    if ((hw >> 3) >= per) return false;
    b = (hw & 7) * per + (hw >> 3);
    return b < nblk;
}

__global__ __launch_bounds__(256) void k_bpad2d(const BSlice *__restrict__ sl, int count,
                                                const int *__restrict__ pfx, const float *__restrict__ vec,
                                                float *__restrict__ pad) {
    const int s = find_slice(pfx, count, blockIdx.x);
    const BSlice &S = sl[s];
    if (*S.stop) return;
    const int t = blockIdx.x - pfx[s];
    const int ntx = (S.g.nx + 31) / 32;
    pad_tile(vec + S.voff, pad + S.pvx, pad + S.pvy, S.g.nx, S.g.ny, S.L, (t % ntx) * 32, (t / ntx) * 32, 0);
}

// Samples of one 2D ray, in groups of four summed in FP32 and added to FP64
// (the same order as the single-problem projector, so results agree bit for
// bit), U samples' loads in flight per step.
template <int U>
__device__ __forceinline__ double samples2d(const RaySetup &R, __amdgpu_buffer_rsrc_t rs, uint32_t base,
                                            uint32_t S, int ja, int jb) {
    static_assert(U % 4 == 0, "groups of four");
    double acc = 0.0;
    int j = ja;
    for (; j + U - 1 <= jb; j += U) {
        float2 v[U];
        float w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const float fb = fmaf((float)(j + u), R.gb, R.fb0);
            const float ibf = floorf(fb);
            w[u] = fb - ibf;
            v[u] = ld2(rs, base + __umul24((uint32_t)(j + u), S) + (uint32_t)(int)ibf);
        }
#pragma unroll
        for (int g4 = 0; g4 < U / 4; ++g4) {
            float grp = 0.0f;
#pragma unroll
            for (int u = 4 * g4; u < 4 * g4 + 4; ++u) grp += fmaf(w[u], v[u].y - v[u].x, v[u].x);
            acc += (double)grp;
        }
    }
    for (; j + 3 <= jb; j += 4) {
        float2 v[4];
        float w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float fb = fmaf((float)(j + u), R.gb, R.fb0);
            const float ibf = floorf(fb);
            w[u] = fb - ibf;
            v[u] = ld2(rs, base + __umul24((uint32_t)(j + u), S) + (uint32_t)(int)ibf);
        }
        float grp = 0.0f;
#pragma unroll
        for (int u = 0; u < 4; ++u) grp += fmaf(w[u], v[u].y - v[u].x, v[u].x);
        acc += (double)grp;
    }
    for (; j <= jb; ++j) {
        const float fb = fmaf((float)j, R.gb, R.fb0);
        const float ibf = floorf(fb);
        const float wb = fb - ibf;
        const float2 a = ld2(rs, base + __umul24((uint32_t)j, S) + (uint32_t)(int)ibf);
        acc += (double)fmaf(wb, a.y - a.x, a.x);
    }
    return acc;
}

// One work-item per ray; 256 consecutive rays of one problem (view-major)
// per workgroup.
template <int U>
__global__ __launch_bounds__(256) void k_bproject2d(const BSlice *__restrict__ sl, int count,
                                                    const int *__restrict__ pfx, int nblk,
                                                    const float *__restrict__ pad, uint32_t pad_elems,
                                                    float *__restrict__ q) {
    int b;
    if (!xcd_block(nblk, b)) return;
    const int s = find_slice(pfx, count, b);
    const BSlice &S = sl[s];
    if (*S.stop) return;
    const int r = (b - pfx[s]) * 256 + (int)threadIdx.x;
    const int nu = S.g.nu;
    if (r >= S.g.P * nu) return;
    const int p = r / nu, a = r - p * nu;
    const RaySetup R = ray_setup<false>(S.g, S.L, p, 0, a);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(pad, pad_elems);
    const bool isx = R.ax == 0;
    const double acc = samples2d<U>(R, rs, isx ? S.pvx : S.pvy, isx ? S.L.sx : S.L.sy, R.j0, R.j1);
    q[S.roff + r] = (float)(acc * (double)R.step);
}

// Voxel-driven B_un for 2D problems: a workgroup covers 16 columns x 16 PPT
// rows, each work-item PPT pixels 16 rows apart.  Per pixel the views are
// summed in FP32 in groups of four and the groups in FP64, as in the
// single-problem kernel.
template <int PPT>
__global__ __launch_bounds__(256) void k_bbp2d(const BSlice *__restrict__ sl, int count,
                                               const int *__restrict__ pfx, int nblk,
                                               const float *__restrict__ q, float *__restrict__ z) {
    int b;
    if (!xcd_block(nblk, b)) return;
    const int s = find_slice(pfx, count, b);
    const BSlice &S = sl[s];
    if (*S.stop) return;
    const GeomK &g = S.g;
    const int t = b - pfx[s];
    const int ntx = (g.nx + 15) / 16;
    const int ix = (t % ntx) * 16 + (int)(threadIdx.x & 15);
    const int iy0 = (t / ntx) * 16 * PPT + (int)(threadIdx.x >> 4);
    if (ix >= g.nx || iy0 >= g.ny) return;
    const float *y = q ? q + S.roff : S.b;
    const double inv_du = 1.0 / g.du;
    const double px = (ix - 0.5 * (g.nx - 1)) * g.vox * inv_du;
    double py[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) py[i] = (iy0 + 16 * i - 0.5 * (g.ny - 1)) * g.vox * inv_du;
    const double cu = 0.5 * (g.nu - 1);
    const int nu = g.nu;
    double acc[PPT];
    float grp[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) { acc[i] = 0.0; grp[i] = 0.0f; }
    for (int p = 0; p < g.P; ++p) {
        const double c = g.cs[2 * p], sn = g.cs[2 * p + 1];
        const float *yp = y + (size_t)p * nu;
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const float fu = (float)(px * c + py[i] * sn + cu);
            const float iuf = floorf(fu);
            const float wu = fu - iuf;
            const int iu = (int)iuf;
            const bool u0 = iu >= 0 && iu < nu, u1 = iu + 1 >= 0 && iu + 1 < nu;
            const float va = u0 ? yp[u0 ? iu : 0] : 0.0f;
            const float vb = u1 ? yp[u1 ? iu + 1 : 0] : 0.0f;
            grp[i] += fmaf(wu, vb - va, va);
        }
        if ((p & 3) == 3 || p == g.P - 1) {
#pragma unroll
            for (int i = 0; i < PPT; ++i) { acc[i] += (double)grp[i]; grp[i] = 0.0f; }
        }
    }
    const double wgt = g.vox * g.vox * inv_du;
    float *zs = z + S.voff;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int iy = iy0 + 16 * i;
        if (iy < g.ny) zs[(size_t)iy * g.nx + ix] = (float)(acc[i] * wgt);
    }
}

// Ram-Lak filter of one detector row of one problem per workgroup (rows of
// up to max_nu bins staged in LDS with zeros on both sides); the same
// multiply-add order as the single-problem filters.
__global__ __launch_bounds__(256) void k_bramp(const BSlice *__restrict__ sl, int count,
                                               const int *__restrict__ pfx, const float *__restrict__ q,
                                               float *__restrict__ out) {
    extern __shared__ float sm[];
    const int s = find_slice(pfx, count, blockIdx.x);
    const BSlice &S = sl[s];
    if (*S.stop) return;
    const int nu = S.g.nu;
    const int row = blockIdx.x - pfx[s];
    float *qs = sm;            // [nu zeros][row][nu zeros]
    float *hs = sm + 3 * nu;
    const float *qr = (q ? q + S.roff : S.b) + (size_t)row * nu;
    for (int i = threadIdx.x; i < nu; i += blockDim.x) {
        qs[i] = 0.0f;
        qs[nu + i] = qr[i];
        qs[2 * nu + i] = 0.0f;
        hs[i] = S.ramp[i];
    }
    __syncthreads();
    float *orow = out + S.roff + (size_t)row * nu;
    for (int a = threadIdx.x; a < nu; a += blockDim.x) {
        const float *qa = qs + nu + a;
        float acc = hs[0] * qa[0];
        for (int j = 1; j < nu; j += 2) acc = fmaf(hs[j], qa[-j] + qa[j], acc);
        orow[a] = acc;
    }
}


// Ram-Lak filter on the matrix cores.  Split by the parity of the output
// index, the filter is two dense Toeplitz products per detector row, because
// only odd lags carry non-zero taps:
//   out[2i]   = h0 q[2i]   + sum_m hh[2(i-m) - 1] q[2m+1]
//   out[2i+1] = h0 q[2i+1] + sum_m hh[2(i-m) + 1] q[2m]
// (hh[j] = du h[|j|]), half the multiply-adds of the dense convolution.  A
// workgroup takes 16 NRG rows and the two parities in turn: it stages the
// inputs of the other parity (half of each row) in LDS, next to the taps as
// a table over signed lags, and its wavefronts take tasks of 16 outputs for
// all the rows: v_mfma_f32_16x16x4f32 with M = output index, N = row,
// K = input index, the A operand (16 x 4 Toeplitz block) read from the tap
// table and the B operand from the staged half-rows, one accumulator per
// 16-row group; the h0 term is read from global memory and added last.
template <typename InT, typename OutT, int NRG>
__global__ __launch_bounds__(256) void k_ramp_mfma(const InT *__restrict__ q, OutT *__restrict__ out,
                                                   const float *__restrict__ taps, int nu, size_t rows,
                                                   int vec_in, const int *__restrict__ stop) {
    if (stop && *stop) return;
    extern __shared__ float sm[];
    constexpr int R = 16 * NRG;
    constexpr int TPR = 256 / R;   // staging work-items per row
    const int ne = (nu + 1) / 2, no = nu / 2;
    const int nep = (ne + 15) & ~15, nop = (no + 15) & ~15;
    const int ss = ((nep > nop ? nep : nop) + 31 & ~31) + 2;   // half-row stride = 2 (mod 32 banks)
    const int lmax = 2 * (nep > nop ? nep : nop) + 1;
    float *Qs = sm, *hsym = sm + R * ss;
    const size_t r0 = (size_t)blockIdx.x * R;
    const int tid = threadIdx.x;
    for (int t = tid; t <= 2 * lmax; t += 256) {
        const int L = t - lmax, aL = L < 0 ? -L : L;
        hsym[t] = aL < nu ? taps[aL] : 0.0f;
    }
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll 1
    for (int par = 0; par < 2; ++par) {
        // inputs of the other parity: q[2m + 1 - par], m < K
        const int K = par ? nep : nop, kcnt = par ? ne : no;
        __syncthreads();   // previous phase's readers are done; taps written
        {
            const int r = tid / TPR, c = tid % TPR;
            float *dst = Qs + r * ss;
            if (r0 + r < rows) {
                const InT *src = q + (r0 + r) * nu;
                int m = 0;
                if (vec_in) {
                    // this parity's two elements of each 4-element load
                    // (nu divisible by 4, so kcnt = nu / 2)
                    for (int j = c; 4 * j < nu; j += TPR) {
                        const float4 v = ld4f(src + 4 * j);
                        dst[2 * j] = par ? v.x : v.y;
                        dst[2 * j + 1] = par ? v.z : v.w;
                    }
                    m = nu / 2;
                }
                for (m += c; m < ss; m += TPR) dst[m] = m < kcnt ? to_f(src[2 * m + 1 - par]) : 0.0f;
            } else {
                for (int m = c; m < ss; m += TPR) dst[m] = 0.0f;
            }
        }
        __syncthreads();
        const float h0 = hsym[lmax];
        const int cnt = par ? no : ne;           // outputs of this parity
        const int ntask = (par ? nop : nep) / 16;
        for (int task = wave; task < ntask; task += 4) {
            const int i0 = 16 * task;
            // the h0 term's inputs are loaded first and added after the
            // products, so that their latency hides behind the matrix cores
            float self[NRG][4];
            f4 acc[NRG];
#pragma unroll
            for (int g = 0; g < NRG; ++g) {
                const size_t row = r0 + 16 * g + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + 4 * lk + r;
                    self[g][r] = (row < rows && i < cnt) ? to_f(q[row * nu + 2 * i + par]) : 0.0f;
                    acc[g][r] = 0.0f;
                }
            }
            // A[i][k] = hh[2((i0 + i) - (m0 + k)) + 2 par - 1] at lane (i = li, k = lk)
            const float *ap = hsym + lmax + 2 * (i0 + li - lk) + 2 * par - 1;
            const float *bp = Qs + li * ss + lk;
            for (int m0 = 0; m0 < K; m0 += 4) {
                const float av = ap[-2 * m0];
#pragma unroll
                for (int g = 0; g < NRG; ++g)
                    acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bp[16 * g * ss + m0], acc[g], 0, 0, 0);
            }
#pragma unroll
            for (int g = 0; g < NRG; ++g) {
                const size_t row = r0 + 16 * g + li;
                if (row < rows)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = i0 + 4 * lk + r;
                        if (i < cnt) out[row * nu + 2 * i + par] = from_f<OutT>(acc[g][r] + h0 * self[g][r]);
                    }
            }
        }
    }
}

// The same filter with whole rows staged: for rows short enough that 16 of
// them (both parities) fit in LDS, 16 work-items stage each row with 16-byte
// loads where the row allows (no index division), and a wavefront computes
// two adjacent 16-output blocks of both parities, adds the h0 terms from LDS
// and stores the interleaved outputs of each row as contiguous 16-byte
// vectors.  Input and output move once, in full lines.  The two blocks share
// the input operand, and the Toeplitz block of the upper outputs at input m
// is the lower block's at input m - 16, so its operand comes from a four-step
// register ring rather than from LDS.  Outputs per parity are padded to 32;
// the padded outputs are computed from zeros and not stored.
template <typename InT, typename OutT>
__global__ __launch_bounds__(256) void k_ramp_rows(const InT *__restrict__ q, OutT *__restrict__ out,
                                                   const float *__restrict__ taps, int nu, size_t rows,
                                                   int vec_in, int vec_out, const int *__restrict__ stop) {
    if (stop && *stop) return;
    extern __shared__ float sm[];
    const int ne = (nu + 1) / 2, no = nu / 2;
    const int nep = (ne + 15) & ~15, nop = (no + 15) & ~15;
    const int P2 = ((nep > nop ? nep : nop) + 31) & ~31;   // outputs per parity, padded to 32
    const int ss = 2 * P2 + 1;                             // odd row stride: rows start on different banks
    const int lmax = 2 * P2 + 33;                          // the ring reaches 16 inputs before m = 0
    float *Qs = sm, *hsym = sm + 16 * ss;
    const size_t r0 = (size_t)blockIdx.x * 16;
    const int tid = threadIdx.x;
    for (int t = tid; t <= 2 * lmax; t += 256) {
        const int L = t - lmax, aL = L < 0 ? -L : L;
        hsym[t] = aL < nu ? taps[aL] : 0.0f;
    }
    {
        const int r = tid >> 4, c = tid & 15;   // 16 work-items per row
        float *dst = Qs + r * ss;
        if (r0 + r < rows) {
            const InT *src = q + (r0 + r) * nu;
            int m = 0;
            if (vec_in) {
                for (int m4 = 4 * c; m4 < nu; m4 += 64) {
                    const float4 v = ld4f(src + m4);
                    dst[m4] = v.x;
                    dst[m4 + 1] = v.y;
                    dst[m4 + 2] = v.z;
                    dst[m4 + 3] = v.w;
                }
                m = nu;
            }
            for (m += c; m < ss; m += 16) dst[m] = m < nu ? to_f(src[m]) : 0.0f;
        } else {
            for (int m = c; m < ss; m += 16) dst[m] = 0.0f;
        }
    }
    __syncthreads();
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const float h0 = hsym[lmax];
    const size_t row = r0 + li;
    typedef float f4 __attribute__((ext_vector_type(4)));
    for (int task = wave; task < P2 / 32; task += 4) {
        const int i0 = 32 * task;
        // outputs 2i + par from the inputs of the other parity, q[2m + 1 - par]
        // (nop <= nep <= nop + 16); four independent accumulation chains
        const float *ap0 = hsym + lmax + 2 * (i0 + li - lk) - 1, *ap1 = ap0 + 2;
        const float *bp0 = Qs + li * ss + 2 * lk + 1, *bp1 = bp0 - 1;
        f4 e0 = {0.0f, 0.0f, 0.0f, 0.0f}, o0 = e0, e1 = e0, o1 = e0;
        float ra0 = ap0[32], rb0 = ap0[24], rc0 = ap0[16], rd0 = ap0[8];
        float ra1 = ap1[32], rb1 = ap1[24], rc1 = ap1[16], rd1 = ap1[8];
#define CT_RAMP_STEP(M, R0, R1)                                             \
    {                                                                       \
        const float x0 = ap0[-2 * (M)], x1 = ap1[-2 * (M)];                 \
        const float b0 = bp0[2 * (M)], b1 = bp1[2 * (M)];                   \
        e0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0, b0, e0, 0, 0, 0);     \
        o0 = __builtin_amdgcn_mfma_f32_16x16x4f32(x1, b1, o0, 0, 0, 0);     \
        e1 = __builtin_amdgcn_mfma_f32_16x16x4f32(R0, b0, e1, 0, 0, 0);     \
        o1 = __builtin_amdgcn_mfma_f32_16x16x4f32(R1, b1, o1, 0, 0, 0);     \
        R0 = x0;                                                            \
        R1 = x1;                                                            \
    }
        int m0 = 0;
        for (; m0 + 16 <= nop; m0 += 16) {
            CT_RAMP_STEP(m0, ra0, ra1)
            CT_RAMP_STEP(m0 + 4, rb0, rb1)
            CT_RAMP_STEP(m0 + 8, rc0, rc1)
            CT_RAMP_STEP(m0 + 12, rd0, rd1)
        }
#undef CT_RAMP_STEP
        for (int m = m0; m < nep; m += 4) {
            if (m < nop) {
                e0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ap0[-2 * m], bp0[2 * m], e0, 0, 0, 0);
                e1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ap0[32 - 2 * m], bp0[2 * m], e1, 0, 0, 0);
            }
            o0 = __builtin_amdgcn_mfma_f32_16x16x4f32(ap1[-2 * m], bp1[2 * m], o0, 0, 0, 0);
            o1 = __builtin_amdgcn_mfma_f32_16x16x4f32(ap1[32 - 2 * m], bp1[2 * m], o1, 0, 0, 0);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const f4 ev = h ? e1 : e0, od = h ? o1 : o0;
            const int ib = i0 + 16 * h;
            float o[8];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = li * ss + 2 * (ib + 4 * lk + r);
                o[2 * r] = ev[r] + h0 * Qs[c];
                o[2 * r + 1] = od[r] + h0 * Qs[c + 1];
            }
            if (row < rows) {
                const int col0 = 2 * (ib + 4 * lk);   // this lane's 8 consecutive outputs of the row
                OutT *dst = out + row * nu + col0;
                if (vec_out && col0 + 8 <= nu) {
                    if (sizeof(OutT) == 4) {
                        reinterpret_cast<float4 *>(dst)[0] = make_float4(o[0], o[1], o[2], o[3]);
                        reinterpret_cast<float4 *>(dst)[1] = make_float4(o[4], o[5], o[6], o[7]);
                    } else {
#pragma unroll
                        for (int k = 0; k < 8; ++k) dst[k] = from_f<OutT>(o[k]);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        if (col0 + k < nu) dst[k] = from_f<OutT>(o[k]);
                }
            }
        }
    }
}

static size_t ramp_rows_lds(int nu) {
    const int ne = (nu + 1) / 2, no = nu / 2;
    const int nep = (ne + 15) & ~15, nop = (no + 15) & ~15;
    const int P2 = ((nep > nop ? nep : nop) + 31) & ~31;
    return sizeof(float) * ((size_t)16 * (2 * P2 + 1) + 2 * (size_t)(2 * P2 + 33) + 1);
}

// LDS bytes of k_ramp_mfma for a row length and row-group count
static size_t ramp_mfma_lds(int nu, int nrg) {
    const int ne = (nu + 1) / 2, no = nu / 2;
    const int nep = (ne + 15) & ~15, nop = (no + 15) & ~15;
    const int ss = ((nep > nop ? nep : nop) + 31 & ~31) + 2;
    const int lmax = 2 * (nep > nop ? nep : nop) + 1;
    return sizeof(float) * ((size_t)16 * nrg * ss + 2 * (size_t)lmax + 1);
}

// FBP / FDK pre-weighting: out = scale * w(u, v) * y with the cone-beam
// cosine weight w = SDD / sqrt(SDD^2 + u^2 + v^2) (1 in 2D).
template <typename InT>
__global__ __launch_bounds__(256) void k_fbp_weight(GeomK g, const InT *__restrict__ y, float *__restrict__ out,
                                                    size_t n, double scale) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double w = scale;
        if (g.kind == 1) {
            const int au = (int)(i % g.nu), av = (int)((i / g.nu) % g.nv);
            const double u = (au - 0.5 * (g.nu - 1)) * g.du, v = (av - 0.5 * (g.nv - 1)) * g.dv;
            w *= g.sdd / sqrt(g.sdd * g.sdd + u * u + v * v);
        }
        out[i] = (float)(w * (double)to_f(y[i]));
    }
}
}  // namespace

// ------------------------------------------------------------ launchers
int launch_pad_zero(const ct_geometry *g, float *vx, float *vy, hipStream_t s) {
    const PadLayout &L = g->pad;
    const size_t per_x = (size_t)2 * L.pz * L.rx + (size_t)g->k.nz * (L.rx - g->k.ny);
    const size_t per_y = (size_t)2 * L.pz * L.ry + (size_t)g->k.nz * (L.ry - g->k.nx);
    const size_t tot = per_x * g->k.nx + per_y * g->k.ny;
    size_t blocks = (tot + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_pad_zero, dim3((unsigned)blocks), dim3(256), 0, s, vx, vy, g->k.nx, g->k.ny,
                       g->k.nz, L);
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int launch_pad_copy(const ct_geometry *g, const void *x, int x_dtype, float *vx, float *vy, const int *stop,
                    hipStream_t s) {
    dim3 grid((g->k.nx + 31) / 32, (g->k.ny + 31) / 32, g->k.nz);
    if (x_dtype == CT_F16)
        hipLaunchKernelGGL(k_pad_copy<__half>, grid, dim3(256), 0, s, (const __half *)x, vx, vy, g->k.nx, g->k.ny,
                           g->pad, stop);
    else
        hipLaunchKernelGGL(k_pad_copy<float>, grid, dim3(256), 0, s, (const float *)x, vx, vy, g->k.nx, g->k.ny,
                           g->pad, stop);
    CT_LAUNCH_CHECK();
    return CT_OK;
}

static void ray_grid(const ct_geometry *g, dim3 &grid, dim3 &block) {
    if (g->k.kind == CT_CONE_CIRCULAR_3D) block = dim3(64, 4);
    else block = dim3(256, 1);
    grid = dim3((g->k.nu + block.x - 1) / block.x, (g->k.nv + block.y - 1) / block.y, g->k.P);
}

// Dynamic LDS that holds a 256-work-item kernel to at most `target`
// resident workgroups per CU (0 if it already is), found with the runtime's
// occupancy calculator and cached per device, kernel and target.
static unsigned lds_for_occupancy(const void *kernel, int target) {
    static std::mutex mu;
    static std::map<std::pair<std::pair<int, int>, const void *>, unsigned> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_pair(std::make_pair(dev, target), kernel);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    unsigned extra = 0;
    for (unsigned e = 0; e <= 64u * 1024u; e += 256u) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, e) != hipSuccess) break;
        if (nb <= target) { extra = e; break; }
    }
    cache[key] = extra;
    return extra;
}

// The staged projector re-reads each tile's planes from L2 for the
// neighbouring views of its group.  While the padded copies fit the 256 MB
// last-level cache the misses are cheap and the kernel is bound by VALU
// issue, so it runs at full occupancy (eight workgroups per CU) with groups
// of ten views (ms per launch at 256^3, 360 views: groups of 6: 4.50,
// 10: 4.44, 16: 4.56, 24: 4.58; four workgroups per CU: 5.43).  Beyond
// that the misses go to HBM, and fewer resident tiles per XCD and smaller
// view groups keep more of each tile's planes in L2.  At 1024 x 1024 x 300
// with 180 views: groups of ten at 7, 5, 4, 3 and 2 workgroups per CU took
// 77.2, 68.0, 63.2, 64.1 and 80.3 ms; at four per CU, groups of 2, 3, 4, 6,
// 8, 16 and 24 took 56.4, 54.2, 55.4, 55.3, 58.1, 70.7 and 77.3 ms (groups
// of 3 at 3, 5 and 7 per CU: 62.2 (groups of 4), 58.7, 85.9).  The band
// order (xcd_tile, negative vgrp) then keeps the slab of the volume that a
// band of detector rows sees in the last-level cache: at four per CU,
// groups of 1, 2, 3, 4, 6, 8, 10 and 12 took 80.2, 53.6, 49.4, 47.9, 49.1,
// 52.2, 54.8 and 60.5 ms, against 54.7 ms for the XCD-contiguous order with
// groups of six (groups of 6 at 3, 5 and 8 per CU: 53.5, 58.5, 81.7; the
// band order without view groups, views innermost across XCDs: 86.4).
constexpr double kLlcBytes = 256.0 * 1024 * 1024;
constexpr int kVGrpCached = 10;
constexpr int kVGrpBig = -4;   // band order, groups of four views
constexpr int kBigVolumeWgPerCu = 4;

// Launch setting of the staged projector: vgrp > 0 deals the workgroups in
// the XCD-contiguous order with groups of vgrp views, vgrp < 0 in the band
// order with groups of -vgrp views (xcd_tile); wgcu > 0 holds the resident
// workgroups per CU to wgcu with dynamic LDS, 0 leaves as many as fit.
// Only the order and residency of the workgroups change, not what any of
// them computes.
struct StagedCfg {
    int vgrp, wgcu;
};
constexpr int kMaxVGrp = 64, kMaxBandGrp = 16, kMaxWgPerCu = 8;

static bool staged_cfg_valid(int vgrp, int wgcu) {
    return ((vgrp >= 1 && vgrp <= kMaxVGrp) || (vgrp <= -1 && vgrp >= -kMaxBandGrp)) && wgcu >= 0 &&
           wgcu <= kMaxWgPerCu;
}

static uint64_t pack_cfg(StagedCfg c) { return (uint64_t)(uint32_t)c.vgrp | (uint64_t)(uint32_t)c.wgcu << 32; }

// The geometry's setting, or the size heuristic: while the padded copies
// fit the last-level cache, groups of ten views in the XCD order at full
// occupancy; beyond it, the band order with groups of four at four
// workgroups per CU.
static StagedCfg staged_cfg(const ct_geometry *g) {
    const uint64_t v = g->a_cfg.load(std::memory_order_relaxed);
    if (v != 0) return StagedCfg{(int)(uint32_t)v, (int)(uint32_t)(v >> 32)};
    return 4.0 * (double)(g->pad.nvx + g->pad.nvy) > kLlcBytes ? StagedCfg{kVGrpBig, kBigVolumeWgPerCu}
                                                               : StagedCfg{kVGrpCached, 0};
}

template <typename OutT, bool SID>
static int launch_staged(const ct_geometry *g, StagedCfg cfg, dim3 grid, const float *vx, uint32_t offy, void *y,
                         const float *out_scale, const int *stop, hipStream_t s) {
    const void *kern = (const void *)&k_project_staged<OutT, SID>;
    const unsigned lds = cfg.wgcu > 0 ? lds_for_occupancy(kern, cfg.wgcu) : 0u;
    hipLaunchKernelGGL((k_project_staged<OutT, SID>), grid, dim3(kTU, kTV), lds, s, g->k, g->pad, vx, offy,
                       (OutT *)y, out_scale, stop, cfg.vgrp);
    return CT_OK;
}

int launch_project(const ct_geometry *g, const float *vx, const float *vy, void *y, int y_dtype,
                   const float *out_scale, const int *stop, hipStream_t s) {
    dim3 grid, block;
    ray_grid(g, grid, block);
    const bool cone = g->k.kind == CT_CONE_CIRCULAR_3D;
    // the two copies must be carved back to back (one buffer resource)
    const ptrdiff_t dy = vy - vx;
    if (dy < (ptrdiff_t)g->pad.nvx || (double)(dy + g->pad.nvy) * 4.0 >= 4294967296.0) {
        set_error("launch_project: padded volume copies are not contiguous or exceed 4 GiB");
        return CT_ERR_UNSUPPORTED;
    }
    const uint32_t offy = (uint32_t)dy;
    ProfScope prof(PROF_A, s);
    if (cone) {
        // 16 x 16 ray tiles, flat grid remapped per XCD inside the kernel
        const long ntiles = (long)staged_tile_cols(g->k.nu) * ((g->k.nv + kTV - 1) / kTV);
        const StagedCfg cfg = staged_cfg(g);   // read once: the grid and the kernel agree
        const int vgrp = cfg.vgrp;
        long per;   // workgroups per XCD
        if (vgrp < 0) {
            // band order: whole runs of one group's tile row per XCD
            const long G = -vgrp, run = (long)staged_tile_cols(g->k.nu) * G;
            const long nlog = (long)((g->k.nv + kTV - 1) / kTV) * ((g->k.P + G - 1) / G) * run;
            per = (nlog + 8 * run - 1) / (8 * run) * run;
        } else {
            const long nlog = (long)((g->k.P + vgrp - 1) / vgrp) * ntiles * vgrp;
            per = (nlog + 7) / 8;
        }
        if (8 * per > 2147483647L) {
            set_error("launch_project: too many ray tiles");
            return CT_ERR_UNSUPPORTED;
        }
        const dim3 sgrid((unsigned)(8 * per));
        if (g->k.proj == CT_SIDDON) {
            if (y_dtype == CT_F32) launch_staged<float, true>(g, cfg, sgrid, vx, offy, y, out_scale, stop, s);
            else launch_staged<__half, true>(g, cfg, sgrid, vx, offy, y, out_scale, stop, s);
        } else {
            if (y_dtype == CT_F32) launch_staged<float, false>(g, cfg, sgrid, vx, offy, y, out_scale, stop, s);
            else launch_staged<__half, false>(g, cfg, sgrid, vx, offy, y, out_scale, stop, s);
        }
    } else {
        if (y_dtype == CT_F32) hipLaunchKernelGGL((k_project<false, float>), grid, block, 0, s, g->k, g->pad, vx, offy, (float *)y, out_scale, stop);
        else hipLaunchKernelGGL((k_project<false, __half>), grid, block, 0, s, g->k, g->pad, vx, offy, (__half *)y, out_scale, stop);
    }
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int launch_col_table(ct_geometry *g) {
    dim3 grid((g->k.nu + 255) / 256, g->k.P), block(256);
    hipLaunchKernelGGL(k_ray_columns, grid, block, 0, 0, g->k, g->d_rcol);
    CT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_col_table, grid, block, 0, 0, g->k, g->d_colT);
    CT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_view_dom, dim3((g->k.P + 255) / 256), dim3(256), 0, 0, g->k, g->d_colT, g->d_vdom,
                       g->d_vshift);
    CT_LAUNCH_CHECK();
    if (hipStreamSynchronize(0) != hipSuccess) {
        set_error("ct_geometry_create: column table kernel failed");
        return CT_ERR_HIP;
    }
    return CT_OK;
}

int launch_project_T_gather(const ct_geometry *g, const void *y, int y_dtype, float *x, const float *scale,
                            const int *stop, hipStream_t s, float *ys) {
    if (!ys) {
        set_error("A^T: no scratch for the step-weighted data");
        return CT_ERR_ARG;
    }
    ProfScope prof(PROF_AT, s);
    size_t blocks = ((size_t)g->k.P * g->k.nv + 3) / 4;   // four rows per workgroup
    if (blocks > 16384) blocks = 16384;
    if (y_dtype == CT_F32)
        hipLaunchKernelGGL(k_ray_step_scale<float>, dim3((unsigned)blocks), dim3(256), 0, s, g->k, (const float *)y, ys, stop);
    else
        hipLaunchKernelGGL(k_ray_step_scale<__half>, dim3((unsigned)blocks), dim3(256), 0, s, g->k, (const __half *)y, ys, stop);
    CT_LAUNCH_CHECK();
    dim3 grid((g->k.nx + 15) / 16, (g->k.ny + 15) / 16, (g->k.nz + kZC - 1) / kZC), block(16, 16);
    if (g->k.proj == CT_SIDDON)
        hipLaunchKernelGGL(k_project_T_slab, grid, block, 0, s, g->k, (const float *)ys, x, scale, stop);
    else
        hipLaunchKernelGGL(k_project_T_sheets, grid, block, 0, s, g->k, (const float *)ys, x, scale, stop);
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int launch_project_T_par(const ct_geometry *g, const void *y, int y_dtype, float *x, const float *scale,
                         const int *stop, hipStream_t s) {
    ProfScope prof(PROF_AT, s);
    dim3 grid((g->k.nx + 15) / 16, (g->k.ny + 15) / 16), block(16, 16);
    if (y_dtype == CT_F32)
        hipLaunchKernelGGL(k_project_T_par<float>, grid, block, 0, s, g->k, (const float *)y, x, scale, stop);
    else
        hipLaunchKernelGGL(k_project_T_par<__half>, grid, block, 0, s, g->k, (const __half *)y, x, scale, stop);
    CT_LAUNCH_CHECK();
    return CT_OK;
}



int launch_siddon(const ct_geometry *g, const float *x, void *y, int y_dtype, const float *out_scale,
                  const int *stop, hipStream_t s) {
    dim3 grid, block;
    ray_grid(g, grid, block);
    ProfScope prof(PROF_A, s);
    const bool cone = g->k.kind == CT_CONE_CIRCULAR_3D;
    if (y_dtype == CT_F32) {
        if (cone) hipLaunchKernelGGL((k_siddon<true, float>), grid, block, 0, s, g->k, x, (float *)y, out_scale, stop);
        else hipLaunchKernelGGL((k_siddon<false, float>), grid, block, 0, s, g->k, x, (float *)y, out_scale, stop);
    } else {
        if (cone) hipLaunchKernelGGL((k_siddon<true, __half>), grid, block, 0, s, g->k, x, (__half *)y, out_scale, stop);
        else hipLaunchKernelGGL((k_siddon<false, __half>), grid, block, 0, s, g->k, x, (__half *)y, out_scale, stop);
    }
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int launch_siddon_T(const ct_geometry *g, const void *y, int y_dtype, float *x, const float *in_scale,
                    const int *stop, hipStream_t s) {
    dim3 grid, block;
    ray_grid(g, grid, block);
    ProfScope prof(PROF_AT, s);
    const bool cone = g->k.kind == CT_CONE_CIRCULAR_3D;
    if (y_dtype == CT_F32) {
        if (cone) hipLaunchKernelGGL((k_siddon_T<true, float>), grid, block, 0, s, g->k, (const float *)y, x, in_scale, stop);
        else hipLaunchKernelGGL((k_siddon_T<false, float>), grid, block, 0, s, g->k, (const float *)y, x, in_scale, stop);
    } else {
        if (cone) hipLaunchKernelGGL((k_siddon_T<true, __half>), grid, block, 0, s, g->k, (const __half *)y, x, in_scale, stop);
        else hipLaunchKernelGGL((k_siddon_T<false, __half>), grid, block, 0, s, g->k, (const __half *)y, x, in_scale, stop);
    }
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int launch_backproject(const ct_geometry *g, const void *y, int y_dtype, float *x, const float *in_scale,
                       const int *stop, hipStream_t s) {
    const bool cone = g->k.kind == CT_CONE_CIRCULAR_3D;
    ProfScope prof(PROF_B, s);
    dim3 block(16, 16);
    if (cone) {
        dim3 grid((g->k.nx + 15) / 16, (g->k.ny + 15) / 16, (g->k.nz + kZC - 1) / kZC);
        if (y_dtype == CT_F32) hipLaunchKernelGGL((k_bp_cone_staged<float>), grid, block, 0, s, g->k, (const float *)y, x, in_scale, stop);
        else hipLaunchKernelGGL((k_bp_cone_staged<__half>), grid, block, 0, s, g->k, (const __half *)y, x, in_scale, stop);
    } else {
        dim3 grid((g->k.nx + 15) / 16, (g->k.ny + 15) / 16, 1);
        if (y_dtype == CT_F32) hipLaunchKernelGGL((k_bp_par<float>), grid, block, 0, s, g->k, (const float *)y, x, in_scale, stop);
        else hipLaunchKernelGGL((k_bp_par<__half>), grid, block, 0, s, g->k, (const __half *)y, x, in_scale, stop);
    }
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int launch_ramp(const ct_geometry *g, const void *q, int q_dtype, void *out, int out_dtype, size_t rows,
                const int *stop, hipStream_t s) {
    const int nu = g->k.nu;
    ProfScope prof(PROF_F, s);
    const size_t shm = sizeof(float) * 4 * (size_t)nu;
    if (shm > 64 * 1024) {
        set_error("ramp filter: detector rows longer than 4096 are not supported");
        return CT_ERR_UNSUPPORTED;
    }
    if (ramp_rows_lds(nu) <= 64 * 1024) {
        // whole rows staged (rows up to about 900 bins)
        const size_t lds = ramp_rows_lds(nu);
        dim3 rgrid((unsigned)((rows + 15) / 16)), rblock(256);
        const size_t es = out_dtype == CT_F16 ? 2 : 4;
        const int vec_out = (nu % 4 == 0) && ((uintptr_t)out % 16 == 0) && (es == 4 || nu % 8 == 0);
        const size_t is = q_dtype == CT_F16 ? 2 : 4;
        const int vec_in = (nu % 4 == 0) && ((uintptr_t)q % (4 * is) == 0);
#define CT_RAMP_ROWS(IT, OT) \
    hipLaunchKernelGGL((k_ramp_rows<IT, OT>), rgrid, rblock, lds, s, (const IT *)q, (OT *)out, g->d_ramp, nu, rows, \
                       vec_in, vec_out, stop)
        if (q_dtype == CT_F32 && out_dtype == CT_F32) CT_RAMP_ROWS(float, float);
        else if (q_dtype == CT_F16 && out_dtype == CT_F16) CT_RAMP_ROWS(__half, __half);
        else if (q_dtype == CT_F16 && out_dtype == CT_F32) CT_RAMP_ROWS(__half, float);
        else CT_RAMP_ROWS(float, __half);
#undef CT_RAMP_ROWS
        CT_LAUNCH_CHECK();
        return CT_OK;
    }
    {
        // matrix-core path, one 16-row group per workgroup: larger groups
        // share the tap reads but hold more LDS, and the extra workgroups in
        // flight measured faster (rows of 384 bins: 0.36 ms at 16 rows, 0.39
        // at 32, 0.48 at 64 for 138240 rows); rows longer than 1600 bins
        // exceed 64 KB of LDS and take the per-row FIR below
        constexpr int nrg = 1;
        const size_t lds = ramp_mfma_lds(nu, nrg);
        if (lds <= 64 * 1024) {
            const size_t rpb = 16 * (size_t)nrg;
            const int vec_in = (nu % 4 == 0) && ((uintptr_t)q % (q_dtype == CT_F16 ? 8 : 16) == 0);
            dim3 mgrid((unsigned)((rows + rpb - 1) / rpb)), mblock(256);
#define CT_RAMP_MFMA(NRGV)                                                                                        \
    do {                                                                                                          \
        if (q_dtype == CT_F32 && out_dtype == CT_F32)                                                             \
            hipLaunchKernelGGL((k_ramp_mfma<float, float, NRGV>), mgrid, mblock, lds, s, (const float *)q,        \
                               (float *)out, g->d_ramp, nu, rows, vec_in, stop);                                  \
        else if (q_dtype == CT_F16 && out_dtype == CT_F16)                                                        \
            hipLaunchKernelGGL((k_ramp_mfma<__half, __half, NRGV>), mgrid, mblock, lds, s, (const __half *)q,     \
                               (__half *)out, g->d_ramp, nu, rows, vec_in, stop);                                 \
        else if (q_dtype == CT_F16 && out_dtype == CT_F32)                                                        \
            hipLaunchKernelGGL((k_ramp_mfma<__half, float, NRGV>), mgrid, mblock, lds, s, (const __half *)q,      \
                               (float *)out, g->d_ramp, nu, rows, vec_in, stop);                                  \
        else                                                                                                      \
            hipLaunchKernelGGL((k_ramp_mfma<float, __half, NRGV>), mgrid, mblock, lds, s, (const float *)q,       \
                               (__half *)out, g->d_ramp, nu, rows, vec_in, stop);                                 \
    } while (0)
            CT_RAMP_MFMA(nrg);
#undef CT_RAMP_MFMA
            CT_LAUNCH_CHECK();
            return CT_OK;
        }
    }
    if (nu <= 64 * 8) {
        // register-blocked path: RB outputs per lane, four rows per workgroup
        const int rb = nu <= 128 ? 2 : nu <= 256 ? 4 : nu <= 384 ? 6 : 8;
        dim3 rgrid((unsigned)((rows + 3) / 4)), rblock(256);
#define CT_RAMP_RB(RBV)                                                                                   \
    do {                                                                                                  \
        if (q_dtype == CT_F32 && out_dtype == CT_F32)                                                     \
            hipLaunchKernelGGL((k_ramp_rb<RBV, float, float>), rgrid, rblock, 0, s, (const float *)q,     \
                               (float *)out, g->d_ramp, nu, rows, stop);                                  \
        else if (q_dtype == CT_F16 && out_dtype == CT_F16)                                                \
            hipLaunchKernelGGL((k_ramp_rb<RBV, __half, __half>), rgrid, rblock, 0, s, (const __half *)q,  \
                               (__half *)out, g->d_ramp, nu, rows, stop);                                 \
        else if (q_dtype == CT_F16 && out_dtype == CT_F32)                                                \
            hipLaunchKernelGGL((k_ramp_rb<RBV, __half, float>), rgrid, rblock, 0, s, (const __half *)q,   \
                               (float *)out, g->d_ramp, nu, rows, stop);                                  \
        else                                                                                              \
            hipLaunchKernelGGL((k_ramp_rb<RBV, float, __half>), rgrid, rblock, 0, s, (const float *)q,    \
                               (__half *)out, g->d_ramp, nu, rows, stop);                                 \
    } while (0)
        switch (rb) {
        case 2: CT_RAMP_RB(2); break;
        case 4: CT_RAMP_RB(4); break;
        case 6: CT_RAMP_RB(6); break;
        default: CT_RAMP_RB(8); break;
        }
#undef CT_RAMP_RB
        CT_LAUNCH_CHECK();
        return CT_OK;
    }
    dim3 grid((unsigned)rows), block(256);
    if (q_dtype == CT_F32 && out_dtype == CT_F32)
        hipLaunchKernelGGL((k_ramp<float, float>), grid, block, shm, s, (const float *)q, (float *)out, g->d_ramp, nu, stop);
    else if (q_dtype == CT_F16 && out_dtype == CT_F16)
        hipLaunchKernelGGL((k_ramp<__half, __half>), grid, block, shm, s, (const __half *)q, (__half *)out, g->d_ramp, nu, stop);
    else if (q_dtype == CT_F16 && out_dtype == CT_F32)
        hipLaunchKernelGGL((k_ramp<__half, float>), grid, block, shm, s, (const __half *)q, (float *)out, g->d_ramp, nu, stop);
    else
        hipLaunchKernelGGL((k_ramp<float, __half>), grid, block, shm, s, (const float *)q, (__half *)out, g->d_ramp, nu, stop);
    CT_LAUNCH_CHECK();
    return CT_OK;
}


// ------------------------------------------------ batched launchers
int launch_bpad_copy(const BSlice *sl, int count, const int *pfx, int nblk, const float *vec, float *pad,
                     hipStream_t s) {
    if (nblk <= 0) return CT_OK;
    hipLaunchKernelGGL(k_bpad2d, dim3(nblk), dim3(256), 0, s, sl, count, pfx, vec, pad);
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int launch_bproject2d(const BSlice *sl, int count, const int *pfx, int nblk, int variant, const float *pad,
                      size_t pad_elems, float *q, hipStream_t s) {
    if (nblk <= 0) return CT_OK;
    if ((double)pad_elems * 4.0 >= 4294967296.0) {
        set_error("batched projector: padded buffer exceeds 4 GiB");
        return CT_ERR_UNSUPPORTED;
    }
    ProfScope prof(PROF_A, s);
    const dim3 grid((unsigned)(8 * ((nblk + 7) / 8)));
    if (variant == 1)
        hipLaunchKernelGGL(k_bproject2d<8>, grid, dim3(256), 0, s, sl, count, pfx, nblk, pad, (uint32_t)pad_elems, q);
    else
        hipLaunchKernelGGL(k_bproject2d<4>, grid, dim3(256), 0, s, sl, count, pfx, nblk, pad, (uint32_t)pad_elems, q);
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int launch_bbackproject2d(const BSlice *sl, int count, const int *pfx, int nblk, int variant, const float *q,
                          float *z, hipStream_t s) {
    if (nblk <= 0) return CT_OK;
    ProfScope prof(PROF_B, s);
    const dim3 grid((unsigned)(8 * ((nblk + 7) / 8)));
    switch (variant) {
    case 0: hipLaunchKernelGGL(k_bbp2d<1>, grid, dim3(256), 0, s, sl, count, pfx, nblk, q, z); break;
    case 1: hipLaunchKernelGGL(k_bbp2d<2>, grid, dim3(256), 0, s, sl, count, pfx, nblk, q, z); break;
    default: hipLaunchKernelGGL(k_bbp2d<4>, grid, dim3(256), 0, s, sl, count, pfx, nblk, q, z); break;
    }
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int launch_bramp(const BSlice *sl, int count, const int *pfx, int nblk, int max_nu, const float *q, float *out,
                 hipStream_t s) {
    if (nblk <= 0) return CT_OK;
    const size_t shm = sizeof(float) * 4 * (size_t)max_nu;
    if (shm > 64 * 1024) {
        set_error("batched ramp filter: detector rows longer than 4096 are not supported");
        return CT_ERR_UNSUPPORTED;
    }
    ProfScope prof(PROF_F, s);
    hipLaunchKernelGGL(k_bramp, dim3(nblk), dim3(256), shm, s, sl, count, pfx, q, out);
    CT_LAUNCH_CHECK();
    return CT_OK;
}

// ------------------------------------------------------- composite ops
static size_t dtype_size(int dt) { return dt == CT_F16 ? 2 : 4; }

size_t op_scratch_bytes(const ct_geometry *g, int op, int data_dtype) {
    switch (op) {
    case CT_OP_A:
        return align_up(g->pad.nvx * 4) + align_up(g->pad.nvy * 4);
    case CT_OP_AT:   // step-weighted data of the cone-beam transpose (2D: none)
        return g->k.kind == CT_CONE_CIRCULAR_3D ? align_up(g->n_rays * 4) : 0;
    case CT_OP_B_RAMP:
        return align_up(g->n_rays * dtype_size(data_dtype));
    case CT_OP_FBP:
        return 2 * align_up(g->n_rays * 4);
    default:
        return 0;
    }
}

OpScratch carve_op_scratch(const ct_geometry *g, int op, int data_dtype, void *ws) {
    OpScratch sc;
    char *p = (char *)ws;
    if (op == CT_OP_A) {
        sc.vx = (float *)p;
        p += align_up(g->pad.nvx * 4);
        sc.vy = (float *)p;
    } else if (op == CT_OP_AT) {
        if (g->k.kind == CT_CONE_CIRCULAR_3D) sc.filt = p;
    } else if (op == CT_OP_B_RAMP) {
        sc.filt = p;
    }
    (void)data_dtype;
    return sc;
}

int apply_A(const ct_geometry *g, const void *x, void *y, int y_dtype, OpScratch &sc, bool pad_ready,
            const float *out_scale, const int *stop, hipStream_t s, int x_dtype) {
    if (g->k.proj == CT_SIDDON && g->k.kind != CT_CONE_CIRCULAR_3D) {
        if (x_dtype != CT_F32) {
            set_error("A: the 2D line-intersection projector reads FP32 input only");
            return CT_ERR_UNSUPPORTED;
        }
        return launch_siddon(g, (const float *)x, y, y_dtype, out_scale, stop, s);
    }
    if (!pad_ready) CT_TRY(launch_pad_zero(g, sc.vx, sc.vy, s));
    CT_TRY(launch_pad_copy(g, x, x_dtype, sc.vx, sc.vy, stop, s));
    return launch_project(g, sc.vx, sc.vy, y, y_dtype, out_scale, stop, s);
}

int apply_B(const ct_geometry *g, int which, const void *y, int y_dtype, float *x, OpScratch &sc,
            const float *in_scale, const int *stop, hipStream_t s) {
    if (which == CT_B_UNMATCHED) return launch_backproject(g, y, y_dtype, x, in_scale, stop, s);
    if (which == CT_B_RAMP) {
        CT_TRY(launch_ramp(g, y, y_dtype, sc.filt, y_dtype, (size_t)g->k.P * g->k.nv, stop, s));
        return launch_backproject(g, sc.filt, y_dtype, x, in_scale, stop, s);
    }
    if (g->k.kind == CT_CONE_CIRCULAR_3D)
        return launch_project_T_gather(g, y, y_dtype, x, in_scale, stop, s, (float *)sc.filt);
    if (g->k.proj == CT_SIDDON) {
        // the 2D line-intersection transpose scatters straight into x
        CT_TRY(launch_fill(x, g->n_vox, 0.0f, s));
        return launch_siddon_T(g, y, y_dtype, x, in_scale, stop, s);
    }
    // 2D Joseph A^T: gathered per pixel
    return launch_project_T_par(g, y, y_dtype, x, in_scale, stop, s);
}

}  // namespace ct

using namespace ct;

// ------------------------------------------------------------------ ABI
static int check_dtype(int dt) { return dt == CT_F32 || dt == CT_F16; }

extern "C" int ct_op_workspace_bytes(const ct_geometry *g, int op, int batch, size_t *bytes) {
    clear_error();
    CT_ARG_CHECK(g && bytes, "ct_op_workspace_bytes: NULL argument");
    CT_ARG_CHECK(op >= CT_OP_A && op <= CT_OP_FBP, "ct_op_workspace_bytes: unknown op");
    CT_ARG_CHECK(batch >= 0, "ct_op_workspace_bytes: negative batch");
    // items are processed one after another; the scratch is reused
    *bytes = op_scratch_bytes(g, op, CT_F32);
    return CT_OK;
}

extern "C" int ct_project_A(const ct_geometry *g, const float *x, void *y, int y_dtype, int batch, void *ws,
                            size_t ws_bytes, void *stream) {
    clear_error();
    CT_ARG_CHECK(g, "ct_project_A: geometry is NULL");
    CT_ARG_CHECK(batch >= 0, "ct_project_A: negative batch");
    CT_ARG_CHECK(check_dtype(y_dtype), "ct_project_A: bad y_dtype");
    if (batch == 0) return CT_OK;
    CT_ARG_CHECK(x && y, "ct_project_A: NULL array");
    const size_t need = op_scratch_bytes(g, CT_OP_A, CT_F32);
    CT_ARG_CHECK(ws && ws_bytes >= need, "ct_project_A: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    OpScratch sc = carve_op_scratch(g, CT_OP_A, CT_F32, ws);
    const size_t es = y_dtype == CT_F16 ? 2 : 4;
    for (int b = 0; b < batch; ++b)
        CT_TRY(apply_A(g, x + (size_t)b * g->n_vox, (char *)y + (size_t)b * g->n_rays * es, y_dtype, sc,
                       b > 0, nullptr, nullptr, s));
    return CT_OK;
}

// ------------------------------------------- allocation-free projection
// The padded volume copies of ct_project_A_noalloc live in this array, one
// per GPU that the library runs on (each GPU holds its own copy until the
// process ends).  Host code never passes the array's name to a kernel: its
// device address, per device, comes from hipGetSymbolAddress on the first
// call made with that device current.
static __device__ __align__(256) unsigned char scratch[CT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

int noalloc_scratch(void **out) {
    int dev = 0;
    CT_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) {
        set_error("ct_project_A_noalloc: device index beyond the scratch table");
        return CT_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        CT_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("ct_project_A_noalloc: no device address for the scratch array");
            return CT_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CT_OK;
}

// kernel timing records hipEvents; none are created inside this entry point
struct NoProfile {
    const bool was = ProfScope::suppressed();
    NoProfile() { ProfScope::suppress(true); }
    ~NoProfile() { ProfScope::suppress(was); }
};
}  // namespace

extern "C" int ct_project_A_noalloc(const ct_geometry *g, const float *x, void *y, int y_dtype, int batch,
                                    void *stream) {
    clear_error();
    CT_ARG_CHECK(g, "ct_project_A_noalloc: geometry is NULL");
    CT_ARG_CHECK(batch >= 0, "ct_project_A_noalloc: negative batch");
    CT_ARG_CHECK(check_dtype(y_dtype), "ct_project_A_noalloc: bad y_dtype");
    if (batch == 0) return CT_OK;
    CT_ARG_CHECK(x && y, "ct_project_A_noalloc: NULL array");
    const size_t need = op_scratch_bytes(g, CT_OP_A, CT_F32);
    if (need > (size_t)CT_NOALLOC_SCRATCH_BYTES) {
        set_error("ct_project_A_noalloc: this geometry's padded volume copies need " + std::to_string(need) +
                  " bytes; the allocation-free scratch holds " +
                  std::to_string((size_t)CT_NOALLOC_SCRATCH_BYTES) + " (use ct_project_A with a workspace)");
        return CT_ERR_UNSUPPORTED;
    }
    void *ws = nullptr;
    CT_TRY(noalloc_scratch(&ws));
    NoProfile np;
    hipStream_t s = (hipStream_t)stream;
    // the copies' zero border is rewritten by the first item of every call,
    // so the previous call's contents (any geometry) do not matter
    OpScratch sc = carve_op_scratch(g, CT_OP_A, CT_F32, ws);
    const size_t es = y_dtype == CT_F16 ? 2 : 4;
    for (int b = 0; b < batch; ++b)
        CT_TRY(apply_A(g, x + (size_t)b * g->n_vox, (char *)y + (size_t)b * g->n_rays * es, y_dtype, sc,
                       b > 0, nullptr, nullptr, s));
    return CT_OK;
}

extern "C" int ct_backproject_B(const ct_geometry *g, const void *y, int y_dtype, float *x, int ramp_filter,
                                int batch, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    CT_ARG_CHECK(g, "ct_backproject_B: geometry is NULL");
    CT_ARG_CHECK(batch >= 0, "ct_backproject_B: negative batch");
    CT_ARG_CHECK(check_dtype(y_dtype), "ct_backproject_B: bad y_dtype");
    if (batch == 0) return CT_OK;
    CT_ARG_CHECK(x && y, "ct_backproject_B: NULL array");
    const int op = ramp_filter ? CT_OP_B_RAMP : CT_OP_B;
    const size_t need = op_scratch_bytes(g, op, CT_F32);
    CT_ARG_CHECK(need == 0 || (ws && ws_bytes >= need), "ct_backproject_B: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const size_t es = y_dtype == CT_F16 ? 2 : 4;
    for (int b = 0; b < batch; ++b) {
        const char *yb = (const char *)y + (size_t)b * g->n_rays * es;
        float *xb = x + (size_t)b * g->n_vox;
        if (ramp_filter) {
            // filtered data kept in FP32 whatever the input type
            CT_TRY(launch_ramp(g, yb, y_dtype, ws, CT_F32, (size_t)g->k.P * g->k.nv, nullptr, s));
            CT_TRY(launch_backproject(g, ws, CT_F32, xb, nullptr, nullptr, s));
        } else {
            CT_TRY(launch_backproject(g, yb, y_dtype, xb, nullptr, nullptr, s));
        }
    }
    return CT_OK;
}

extern "C" int ct_backproject_AT(const ct_geometry *g, const void *y, int y_dtype, float *x, int batch,
                                 void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    CT_ARG_CHECK(g, "ct_backproject_AT: geometry is NULL");
    CT_ARG_CHECK(batch >= 0, "ct_backproject_AT: negative batch");
    CT_ARG_CHECK(check_dtype(y_dtype), "ct_backproject_AT: bad y_dtype");
    if (batch == 0) return CT_OK;
    CT_ARG_CHECK(x && y, "ct_backproject_AT: NULL array");
    const size_t need = op_scratch_bytes(g, CT_OP_AT, CT_F32);
    CT_ARG_CHECK(need == 0 || (ws && ws_bytes >= need), "ct_backproject_AT: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    OpScratch sc = carve_op_scratch(g, CT_OP_AT, CT_F32, ws);
    const size_t es = y_dtype == CT_F16 ? 2 : 4;
    for (int b = 0; b < batch; ++b)
        CT_TRY(apply_B(g, CT_B_AT, (const char *)y + (size_t)b * g->n_rays * es, y_dtype,
                       x + (size_t)b * g->n_vox, sc, nullptr, nullptr, s));
    return CT_OK;
}

extern "C" int ct_ramp_filter(const ct_geometry *g, const float *q, float *y, int batch, void *stream) {
    clear_error();
    CT_ARG_CHECK(g, "ct_ramp_filter: geometry is NULL");
    CT_ARG_CHECK(batch >= 0, "ct_ramp_filter: negative batch");
    if (batch == 0) return CT_OK;
    CT_ARG_CHECK(q && y && q != y, "ct_ramp_filter: bad arrays");
    return launch_ramp(g, q, CT_F32, y, CT_F32, (size_t)batch * g->k.P * g->k.nv, nullptr,
                       (hipStream_t)stream);
}

extern "C" int ct_fbp(const ct_geometry *g, const void *y, int y_dtype, float *x, int batch, void *ws,
                      size_t ws_bytes, void *stream) {
    clear_error();
    CT_ARG_CHECK(g, "ct_fbp: geometry is NULL");
    CT_ARG_CHECK(batch >= 0, "ct_fbp: negative batch");
    CT_ARG_CHECK(check_dtype(y_dtype), "ct_fbp: bad y_dtype");
    if (batch == 0) return CT_OK;
    CT_ARG_CHECK(x && y, "ct_fbp: NULL array");
    const size_t need = op_scratch_bytes(g, CT_OP_FBP, CT_F32);
    CT_ARG_CHECK(ws && ws_bytes >= need, "ct_fbp: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const GeomK &k = g->k;
    const double scale = k.kind == CT_PARALLEL_2D
                             ? (M_PI / k.P) * k.du / (k.vox * k.vox)
                             : (M_PI / k.P) * (k.sod / k.sdd) * k.du * k.dv / (k.vox * k.vox * k.vox);
    float *wy = (float *)ws;
    float *fy = (float *)((char *)ws + align_up(g->n_rays * 4));
    const size_t es = y_dtype == CT_F16 ? 2 : 4;
    size_t blocks = (g->n_rays + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    for (int b = 0; b < batch; ++b) {
        const char *yb = (const char *)y + (size_t)b * g->n_rays * es;
        if (y_dtype == CT_F32)
            hipLaunchKernelGGL(k_fbp_weight<float>, dim3((unsigned)blocks), dim3(256), 0, s, k, (const float *)yb, wy,
                               g->n_rays, scale);
        else
            hipLaunchKernelGGL(k_fbp_weight<__half>, dim3((unsigned)blocks), dim3(256), 0, s, k, (const __half *)yb,
                               wy, g->n_rays, scale);
        CT_LAUNCH_CHECK();
        CT_TRY(launch_ramp(g, wy, CT_F32, fy, CT_F32, (size_t)k.P * k.nv, nullptr, s));
        CT_TRY(launch_backproject(g, fy, CT_F32, x + (size_t)b * g->n_vox, nullptr, nullptr, s));
    }
    return CT_OK;
}

// ------------------------------------------- projector launch setting
namespace {
// pseudo-random values in [0, 1) for the tuner's scratch volume (a hash of
// the index; the projector's time depends a little on the data)
__global__ void k_fill_hash(float *__restrict__ p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t h = (uint32_t)i * 2654435761u;
        h ^= h >> 15;
        h *= 2246822519u;
        h ^= h >> 13;
        p[i] = (float)(h >> 8) * (1.0f / 16777216.0f);
    }
}

// the tuner's device scratch and events, released on every return path
// (after the stream has drained)
struct TuneScratch {
    hipStream_t s = nullptr;
    float *vol = nullptr, *y = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneScratch() {
        (void)hipStreamSynchronize(s);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (vol) (void)hipFree(vol);
        if (y) (void)hipFree(y);
    }
};

// puts the setting back unless the tuner finished
struct RestoreCfg {
    ct_geometry *g;
    uint64_t v;
    bool done = false;
    ~RestoreCfg() {
        if (!done) g->a_cfg.store(v);
    }
};
}  // namespace

extern "C" int ct_projector_config(ct_geometry *g, int vgrp, int wg_per_cu) {
    clear_error();
    CT_ARG_CHECK(g, "ct_projector_config: geometry is NULL");
    if (vgrp == 0 && wg_per_cu == 0) {
        g->a_cfg.store(0);
        return CT_OK;
    }
    if (g->k.kind != CT_CONE_CIRCULAR_3D) {
        set_error("ct_projector_config: only cone-beam geometries have a staged projector setting");
        return CT_ERR_UNSUPPORTED;
    }
    CT_ARG_CHECK(staged_cfg_valid(vgrp, wg_per_cu),
                 "ct_projector_config: vgrp must be 1..64 or -16..-1 and wg_per_cu 0..8");
    g->a_cfg.store(pack_cfg(StagedCfg{vgrp, wg_per_cu}));
    return CT_OK;
}

extern "C" int ct_projector_get_config(const ct_geometry *g, int *vgrp, int *wg_per_cu) {
    clear_error();
    CT_ARG_CHECK(g && vgrp && wg_per_cu, "ct_projector_get_config: NULL argument");
    if (g->k.kind != CT_CONE_CIRCULAR_3D) {
        *vgrp = 0;
        *wg_per_cu = 0;
        return CT_OK;
    }
    const StagedCfg c = staged_cfg(g);
    *vgrp = c.vgrp;
    *wg_per_cu = c.wgcu;
    return CT_OK;
}

extern "C" int ct_tune_projector(ct_geometry *g, int reps, int cap, int *vgrp, int *wg_per_cu, double *ms, int *count,
                                 void *stream) {
    clear_error();
    CT_ARG_CHECK(g, "ct_tune_projector: geometry is NULL");
    CT_ARG_CHECK(reps >= 1 && reps <= 100, "ct_tune_projector: reps must be 1..100");
    CT_ARG_CHECK(cap >= 0, "ct_tune_projector: negative cap");
    CT_ARG_CHECK(cap == 0 || (vgrp && wg_per_cu && ms), "ct_tune_projector: NULL output array");
    if (count) *count = 0;
    if (g->k.kind != CT_CONE_CIRCULAR_3D) return CT_OK;
    std::vector<StagedCfg> cands = {{4, 0}, {6, 0}, {8, 0}, {10, 0}, {12, 0}, {16, 0}};
    if (4.0 * (double)(g->pad.nvx + g->pad.nvy) > kLlcBytes)
        for (int grp : {2, 4, 6})
            for (int w : {3, 4, 5}) cands.push_back(StagedCfg{-grp, w});
    TuneScratch sc;
    sc.s = (hipStream_t)stream;
    const size_t nvol = g->pad.nvx + g->pad.nvy;
    if (hipMalloc((void **)&sc.vol, nvol * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&sc.y, g->n_rays * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("ct_tune_projector: device allocation of the scratch volume and sinogram failed");
        return CT_ERR_ALLOC;
    }
    CT_HIP_CHECK(hipEventCreate(&sc.e0));
    CT_HIP_CHECK(hipEventCreate(&sc.e1));
    hipLaunchKernelGGL(k_fill_hash, dim3(4096), dim3(256), 0, sc.s, sc.vol, nvol);
    CT_LAUNCH_CHECK();
    NoProfile np;   // the tuner's launches stay out of the kernel timing
    RestoreCfg restore{g, g->a_cfg.load()};
    double best = 0.0;
    StagedCfg win = cands[0];
    for (size_t i = 0; i < cands.size(); ++i) {
        g->a_cfg.store(pack_cfg(cands[i]));
        CT_TRY(launch_project(g, sc.vol, sc.vol + g->pad.nvx, sc.y, CT_F32, nullptr, nullptr, sc.s));   // warm-up
        CT_HIP_CHECK(hipEventRecord(sc.e0, sc.s));
        for (int r = 0; r < reps; ++r)
            CT_TRY(launch_project(g, sc.vol, sc.vol + g->pad.nvx, sc.y, CT_F32, nullptr, nullptr, sc.s));
        CT_HIP_CHECK(hipEventRecord(sc.e1, sc.s));
        CT_HIP_CHECK(hipEventSynchronize(sc.e1));
        float t = 0.0f;
        CT_HIP_CHECK(hipEventElapsedTime(&t, sc.e0, sc.e1));
        const double m = (double)t / reps;
        if ((int)i < cap) {
            vgrp[i] = cands[i].vgrp;
            wg_per_cu[i] = cands[i].wgcu;
            ms[i] = m;
        }
        if (i == 0 || m < best) {
            best = m;
            win = cands[i];
        }
    }
    g->a_cfg.store(pack_cfg(win));
    restore.done = true;
    if (count) *count = (int)cands.size();
    return CT_OK;
}
