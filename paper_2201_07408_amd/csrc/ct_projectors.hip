// CT operators of the ABBA method on gfx950: Joseph forward projector A,
// its exact scatter transpose A^T, the voxel-driven back-projector B_un and
// the Ram-Lak ramp filter F (Sec. III of the paper names A, B_un, F and
// B_FBP = B_un F; the discretisations are the ones stated in ct.h).
//
// None of these is a dense contraction, so none uses MFMA.  The design:
//  * A is ray-driven, one work-item per ray.  A workgroup is a tile of one
//    view's detector (64 u x 4 v in 3D), so stores are coalesced along u.
//    Per-ray set-up (direction, dominant axis, plane range) is FP64; the
//    plane loop is FP32, with each sample position computed from the plane
//    index by one FMA.  Samples are read from a zero-padded copy of the
//    volume permuted so that the in-plane axis that varies across a
//    wavefront (y for x-major views, x for y-major views) is contiguous;
//    the padding removes every bounds test from the loop and the reads go
//    through a buffer resource whose range check returns 0 outside.
//  * A^T walks the same samples and scatters with FP32 atomics into padded
//    copies, which are then summed back into the volume.
//  * B_un is voxel-driven: one work-item per (x, y) column and a chunk of z.
//    The view's perspective set-up (U, M, u-taps, weight) is FP64 and shared
//    by the whole chunk; the z loop is FP32 with FMA-from-index.
//  * F convolves each detector row in LDS.
#include <cmath>

#include "ct_common.h"

namespace ct {

namespace {

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, size_t elems) {
    // gfx9 raw buffer: stride 0, num_records in bytes, range-checked.
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0,
                                             (int)(uint32_t)(elems * 4u), 0x00020000);
}

__device__ __forceinline__ float ldf(__amdgpu_buffer_rsrc_t r, uint32_t elem) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)(elem * 4u), 0, 0));
}

// two adjacent floats (4-byte alignment is enough for buffer loads on gfx9)
__device__ __forceinline__ float2 ld2(__amdgpu_buffer_rsrc_t r, uint32_t elem) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)(elem * 4u), 0, 0);
    return make_float2(__builtin_bit_cast(float, (uint32_t)v[0]), __builtin_bit_cast(float, (uint32_t)v[1]));
}

__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(__half v) { return __half2float(v); }
template <typename T> __device__ __forceinline__ T from_f(float v);
template <> __device__ __forceinline__ float from_f<float>(float v) { return v; }
template <> __device__ __forceinline__ __half from_f<__half>(float v) { return __float2half_rn(v); }

// ------------------------------------------------------------- padding
// Zero only the border cells of both padded copies.
__global__ void k_pad_zero(float *__restrict__ vx, float *__restrict__ vy, int nx, int ny,
                           int nz, PadLayout L) {
    // cells per plane: full border rows + two side strips of kPad per interior row
    const size_t per_x = (size_t)2 * L.pz * L.rx + (size_t)nz * 2 * kPad;
    const size_t per_y = (size_t)2 * L.pz * L.ry + (size_t)nz * 2 * kPad;
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
            const size_t q2 = q - full;
            row = (uint32_t)(L.pz + q2 / (2 * kPad));
            const uint32_t c = (uint32_t)(q2 % (2 * kPad));
            col = c < (uint32_t)kPad ? c : (uint32_t)nb + c;
        }
        float *dst = isx ? vx : vy;
        dst[plane * S + (size_t)row * R + col] = 0.0f;
    }
}

// x[z][y][x] -> Vx[x][z+pz][y+kPad] and Vy[y][z+pz][x+kPad] (interior only).
__global__ __launch_bounds__(256) void k_pad_copy(const float *__restrict__ x, float *__restrict__ vx,
                                                  float *__restrict__ vy, int nx, int ny, PadLayout L,
                                                  const int *__restrict__ stop) {
    if (stop && *stop) return;
    __shared__ float tile[32][33];
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, z = blockIdx.z;
    const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
    const size_t zoff = (size_t)z * ny * nx;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int yy = y0 + ty + 8 * r, xx = x0 + tx;
        if (yy < ny && xx < nx) {
            const float v = x[zoff + (size_t)yy * nx + xx];
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

// x[z][y][x] = Vx[x][z+pz][y+kPad] + Vy[y][z+pz][x+kPad]
__global__ __launch_bounds__(256) void k_unpad_sum(const float *__restrict__ vx, const float *__restrict__ vy,
                                                   float *__restrict__ x, int nx, int ny, PadLayout L,
                                                   const float *__restrict__ scale,
                                                   const int *__restrict__ stop) {
    if (stop && *stop) return;
    __shared__ float tile[32][33];
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, z = blockIdx.z;
    const int tx = threadIdx.x, ty = threadIdx.y;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int xx = x0 + ty + 8 * r, yy = y0 + tx;
        if (yy < ny && xx < nx)
            tile[ty + 8 * r][tx] = vx[(size_t)xx * L.sx + (size_t)(z + L.pz) * L.rx + yy + kPad];
    }
    __syncthreads();
    const size_t zoff = (size_t)z * ny * nx;
    const float sc = scale ? *scale : 1.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int yy = y0 + ty + 8 * r, xx = x0 + tx;
        if (yy < ny && xx < nx)
            x[zoff + (size_t)yy * nx + xx] =
                sc * (tile[tx][ty + 8 * r] + vy[(size_t)yy * L.sy + (size_t)(z + L.pz) * L.ry + xx + kPad]);
    }
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

template <bool CONE>
__device__ __forceinline__ RaySetup ray_setup(const GeomK &g, const PadLayout &L, int p, int av, int au) {
    const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
    double ox, oy, rx, ry, rz;
    if (CONE) {
        const double u = (au - 0.5 * (g.nu - 1)) * g.du;
        const double v = (av - 0.5 * (g.nv - 1)) * g.dv;
        ox = g.sod * c;
        oy = g.sod * s;
        rx = -g.sdd * c - u * s;
        ry = -g.sdd * s + u * c;
        rz = v;
    } else {
        const double sa = (au - 0.5 * (g.nu - 1)) * g.du;
        ox = sa * c;
        oy = sa * s;
        rx = -s;
        ry = c;
        rz = 0.0;
    }
    RaySetup R;
    R.ax = CONE ? (fabs(rx) >= fabs(ry) ? 0 : 1) : g.axis[p];
    const double ra = R.ax == 0 ? rx : ry, rb = R.ax == 0 ? ry : rx;
    const double oa = R.ax == 0 ? ox : oy, ob = R.ax == 0 ? oy : ox;
    const int Na = R.ax == 0 ? g.nx : g.ny, Nb = R.ax == 0 ? g.ny : g.nx;
    const double inv_vox = 1.0 / g.vox;
    const double inv_ra = 1.0 / ra;
    const double base = -0.5 * (Na - 1) - oa * inv_vox;   // plane j at j + base (voxel units from o)
    const double gb = rb * inv_ra;
    const double fb0 = ob * inv_vox + 0.5 * (Nb - 1) + gb * base;
    double jlo = 0.0, jhi = (double)(Na - 1);
    auto clip = [&](double f0, double gg, int N) {
        if (gg == 0.0) {
            if (!(f0 > -1.0 && f0 < (double)N)) { jlo = 1.0; jhi = 0.0; }
            return;
        }
        const double t1 = (-1.0 - f0) / gg, t2 = ((double)N - f0) / gg;
        jlo = fmax(jlo, floor(fmin(t1, t2)) + 1.0);
        jhi = fmin(jhi, ceil(fmax(t1, t2)) - 1.0);
    };
    clip(fb0, gb, Nb);
    double gc = 0.0, fc0 = 0.0;
    if (CONE) {
        gc = rz * inv_ra;
        fc0 = 0.5 * (g.nz - 1) + gc * base;   // source at z = 0
        clip(fc0, gc, g.nz);
    }
    if (!(jlo <= jhi)) { jlo = 1.0; jhi = 0.0; }
    R.j0 = (int)jlo;
    R.j1 = (int)jhi;
    R.fb0 = (float)(fb0 + kPad);
    R.gb = (float)gb;
    R.fc0 = (float)(fc0 + L.pz);
    R.gc = (float)gc;
    R.step = (float)(g.vox * sqrt(rx * rx + ry * ry + rz * rz) * fabs(inv_ra));
    return R;
}

// `vol` holds Vx at element 0 and Vy at element `offy`; one buffer
// resource covers both so that the descriptor stays wave-uniform while the
// copy (and strides) are chosen per ray.
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
    const uint32_t S = isx ? L.sx : L.sy, Rw = isx ? L.rx : L.ry;
    const uint32_t base = isx ? 0u : offy;
    // the plane loop is unrolled by four so that eight (3D) or four (2D)
    // loads are in flight before the first interpolation; each group of four
    // samples is summed in FP32 and added to an FP64 accumulator (FP32
    // accumulation over hundreds of samples costs more accuracy than the
    // sample positions do)
    double acc = 0.0;
    int j = R.j0;
    for (; j + 3 <= R.j1; j += 4) {
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
    for (; j <= R.j1; ++j) {
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
    float val = (float)(acc * (double)R.step);
    if (out_scale) val *= *out_scale;
    y[((size_t)p * g.nv + av) * g.nu + au] = from_f<OutT>(val);
}

__device__ __forceinline__ uint32_t clampu(int v, int hi) { return (uint32_t)min(max(v, 0), hi); }

template <bool CONE, typename InT>
__global__ __launch_bounds__(256) void k_project_T(GeomK g, PadLayout L, const InT *__restrict__ y,
                                                   float *__restrict__ vx, float *__restrict__ vy,
                                                   const int *__restrict__ stop) {
    if (stop && *stop) return;
    const int au = blockIdx.x * blockDim.x + threadIdx.x;
    const int av = blockIdx.y * blockDim.y + threadIdx.y;
    const int p = blockIdx.z;
    if (au >= g.nu || av >= g.nv) return;
    const float yv = to_f(y[((size_t)p * g.nv + av) * g.nu + au]);
    if (yv == 0.0f) return;
    const RaySetup R = ray_setup<CONE>(g, L, p, av, au);
    const bool isx = R.ax == 0;
    float *V = isx ? vx : vy;
    const uint32_t S = isx ? L.sx : L.sy, Rw = isx ? L.rx : L.ry;
    // clamping keeps every address inside the padded copy; a clamped tap can
    // only be a border tap, whose accumulated value is discarded
    const int bmax = (int)Rw - 2;
    const int cmax = g.nz + 2 * L.pz - 2;
    const float val = yv * R.step;
    for (int j = R.j0; j <= R.j1; ++j) {
        const float fj = (float)j;
        const float fb = fmaf(fj, R.gb, R.fb0);
        const float ibf = floorf(fb);
        const float wb = fb - ibf;
        uint32_t off = (uint32_t)j * S + clampu((int)ibf, bmax);
        if (CONE) {
            const float fc = fmaf(fj, R.gc, R.fc0);
            const float icf = floorf(fc);
            const float wc = fc - icf;
            off += clampu((int)icf, cmax) * Rw;
            const float a0 = val * (1.0f - wc), a1 = val * wc;
            unsafeAtomicAdd(V + off, a0 * (1.0f - wb));
            unsafeAtomicAdd(V + off + 1, a0 * wb);
            unsafeAtomicAdd(V + off + Rw, a1 * (1.0f - wb));
            unsafeAtomicAdd(V + off + Rw + 1, a1 * wb);
        } else {
            unsafeAtomicAdd(V + off, val * (1.0f - wb));
            unsafeAtomicAdd(V + off + 1, val * wb);
        }
    }
}

// --------------------------------------------------------------- B_un
constexpr int kZC = 16;   // z voxels per work-item in the cone back-projector

template <typename InT>
__global__ __launch_bounds__(256) void k_bp_cone(GeomK g, const InT *__restrict__ y, float *__restrict__ x,
                                                 const float *__restrict__ in_scale,
                                                 const int *__restrict__ stop) {
    if (stop && *stop) return;
    const int ix = blockIdx.x * 16 + threadIdx.x, iy = blockIdx.y * 16 + threadIdx.y;
    const int iz0 = blockIdx.z * kZC;
    if (ix >= g.nx || iy >= g.ny) return;
    const double px = (ix - 0.5 * (g.nx - 1)) * g.vox;
    const double py = (iy - 0.5 * (g.ny - 1)) * g.vox;
    const double pz0 = (iz0 - 0.5 * (g.nz - 1)) * g.vox;
    const double inv_du = 1.0 / g.du, inv_dv = 1.0 / g.dv;
    const double wconst = g.vox * g.vox * g.vox * inv_du * inv_dv;
    const double cu = 0.5 * (g.nu - 1), cv = 0.5 * (g.nv - 1);
    const int nu = g.nu, nv = g.nv;
    // views are summed in FP32 in groups of four, groups in FP64
    double acc[kZC];
    float grp[kZC];
#pragma unroll
    for (int z = 0; z < kZC; ++z) { acc[z] = 0.0; grp[z] = 0.0f; }
    const size_t view = (size_t)nv * nu;
    for (int p = 0; p < g.P; ++p) {
        const double c = g.cs[2 * p], s = g.cs[2 * p + 1];
        const double U = g.sod - (px * c + py * s);
        const double M = g.sdd / U;
        const double fu = M * (py * c - px * s) * inv_du + cu;
        const double fv0 = M * pz0 * inv_dv + cv;
        const float dfv = (float)(M * g.vox * inv_dv);
        const float w = (float)(M * M * wconst);
        const float fuf = (float)fu;
        const float iuf = floorf(fuf);
        const float wu = fuf - iuf;
        const int iu = (int)iuf;
        const bool u0 = iu >= 0 && iu < nu, u1 = iu + 1 >= 0 && iu + 1 < nu;
        const float wu0 = u0 ? (1.0f - wu) * w : 0.0f, wu1 = u1 ? wu * w : 0.0f;
        const int c0 = u0 ? iu : 0, c1 = u1 ? iu + 1 : 0;
        const InT *yp = y + (size_t)p * view;
        const float fv0f = (float)fv0;
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
        if ((p & 3) == 3 || p == g.P - 1) {
#pragma unroll
            for (int z = 0; z < kZC; ++z) { acc[z] += (double)grp[z]; grp[z] = 0.0f; }
        }
    }
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

// ----------------------------------------------------------------- F
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

}  // namespace

// ------------------------------------------------------------ launchers
int launch_pad_zero(const ct_geometry *g, float *vx, float *vy, hipStream_t s) {
    const PadLayout &L = g->pad;
    const size_t per_x = (size_t)2 * L.pz * L.rx + (size_t)g->k.nz * 2 * kPad;
    const size_t per_y = (size_t)2 * L.pz * L.ry + (size_t)g->k.nz * 2 * kPad;
    const size_t tot = per_x * g->k.nx + per_y * g->k.ny;
    size_t blocks = (tot + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_pad_zero, dim3((unsigned)blocks), dim3(256), 0, s, vx, vy, g->k.nx, g->k.ny,
                       g->k.nz, L);
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int launch_pad_copy(const ct_geometry *g, const float *x, float *vx, float *vy, const int *stop,
                    hipStream_t s) {
    dim3 grid((g->k.nx + 31) / 32, (g->k.ny + 31) / 32, g->k.nz);
    hipLaunchKernelGGL(k_pad_copy, grid, dim3(32, 8), 0, s, x, vx, vy, g->k.nx, g->k.ny, g->pad, stop);
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int launch_unpad_sum(const ct_geometry *g, const float *vx, const float *vy, float *x, const float *scale,
                     const int *stop, hipStream_t s) {
    dim3 grid((g->k.nx + 31) / 32, (g->k.ny + 31) / 32, g->k.nz);
    hipLaunchKernelGGL(k_unpad_sum, grid, dim3(32, 8), 0, s, vx, vy, x, g->k.nx, g->k.ny, g->pad, scale, stop);
    CT_LAUNCH_CHECK();
    return CT_OK;
}

static void ray_grid(const ct_geometry *g, dim3 &grid, dim3 &block) {
    if (g->k.kind == CT_CONE_CIRCULAR_3D) block = dim3(64, 4);
    else block = dim3(256, 1);
    grid = dim3((g->k.nu + block.x - 1) / block.x, (g->k.nv + block.y - 1) / block.y, g->k.P);
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
    if (y_dtype == CT_F32) {
        if (cone) hipLaunchKernelGGL((k_project<true, float>), grid, block, 0, s, g->k, g->pad, vx, offy, (float *)y, out_scale, stop);
        else hipLaunchKernelGGL((k_project<false, float>), grid, block, 0, s, g->k, g->pad, vx, offy, (float *)y, out_scale, stop);
    } else {
        if (cone) hipLaunchKernelGGL((k_project<true, __half>), grid, block, 0, s, g->k, g->pad, vx, offy, (__half *)y, out_scale, stop);
        else hipLaunchKernelGGL((k_project<false, __half>), grid, block, 0, s, g->k, g->pad, vx, offy, (__half *)y, out_scale, stop);
    }
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int launch_project_T(const ct_geometry *g, const void *y, int y_dtype, float *vx, float *vy,
                     const int *stop, hipStream_t s) {
    dim3 grid, block;
    ray_grid(g, grid, block);
    const bool cone = g->k.kind == CT_CONE_CIRCULAR_3D;
    if (y_dtype == CT_F32) {
        if (cone) hipLaunchKernelGGL((k_project_T<true, float>), grid, block, 0, s, g->k, g->pad, (const float *)y, vx, vy, stop);
        else hipLaunchKernelGGL((k_project_T<false, float>), grid, block, 0, s, g->k, g->pad, (const float *)y, vx, vy, stop);
    } else {
        if (cone) hipLaunchKernelGGL((k_project_T<true, __half>), grid, block, 0, s, g->k, g->pad, (const __half *)y, vx, vy, stop);
        else hipLaunchKernelGGL((k_project_T<false, __half>), grid, block, 0, s, g->k, g->pad, (const __half *)y, vx, vy, stop);
    }
    CT_LAUNCH_CHECK();
    return CT_OK;
}

int launch_backproject(const ct_geometry *g, const void *y, int y_dtype, float *x, const float *in_scale,
                       const int *stop, hipStream_t s) {
    const bool cone = g->k.kind == CT_CONE_CIRCULAR_3D;
    dim3 block(16, 16);
    if (cone) {
        dim3 grid((g->k.nx + 15) / 16, (g->k.ny + 15) / 16, (g->k.nz + kZC - 1) / kZC);
        if (y_dtype == CT_F32) hipLaunchKernelGGL((k_bp_cone<float>), grid, block, 0, s, g->k, (const float *)y, x, in_scale, stop);
        else hipLaunchKernelGGL((k_bp_cone<__half>), grid, block, 0, s, g->k, (const __half *)y, x, in_scale, stop);
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
    const size_t shm = sizeof(float) * 4 * (size_t)nu;
    if (shm > 64 * 1024) {
        set_error("ramp filter: detector rows longer than 4096 are not supported");
        return CT_ERR_UNSUPPORTED;
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

// ------------------------------------------------------- composite ops
static size_t dtype_size(int dt) { return dt == CT_F16 ? 2 : 4; }

size_t op_scratch_bytes(const ct_geometry *g, int op, int data_dtype) {
    switch (op) {
    case CT_OP_A:
    case CT_OP_AT:
        return align_up(g->pad.nvx * 4) + align_up(g->pad.nvy * 4);
    case CT_OP_B_RAMP:
        return align_up(g->n_rays * dtype_size(data_dtype));
    default:
        return 0;
    }
}

OpScratch carve_op_scratch(const ct_geometry *g, int op, int data_dtype, void *ws) {
    OpScratch sc;
    char *p = (char *)ws;
    if (op == CT_OP_A || op == CT_OP_AT) {
        sc.vx = (float *)p;
        p += align_up(g->pad.nvx * 4);
        sc.vy = (float *)p;
    } else if (op == CT_OP_B_RAMP) {
        sc.filt = p;
    }
    (void)data_dtype;
    return sc;
}

int apply_A(const ct_geometry *g, const float *x, void *y, int y_dtype, OpScratch &sc, bool pad_ready,
            const float *out_scale, const int *stop, hipStream_t s) {
    if (!pad_ready) CT_TRY(launch_pad_zero(g, sc.vx, sc.vy, s));
    CT_TRY(launch_pad_copy(g, x, sc.vx, sc.vy, stop, s));
    return launch_project(g, sc.vx, sc.vy, y, y_dtype, out_scale, stop, s);
}

int apply_B(const ct_geometry *g, int which, const void *y, int y_dtype, float *x, OpScratch &sc,
            const float *in_scale, const int *stop, hipStream_t s) {
    if (which == CT_B_UNMATCHED) return launch_backproject(g, y, y_dtype, x, in_scale, stop, s);
    if (which == CT_B_RAMP) {
        CT_TRY(launch_ramp(g, y, y_dtype, sc.filt, y_dtype, (size_t)g->k.P * g->k.nv, stop, s));
        return launch_backproject(g, sc.filt, y_dtype, x, in_scale, stop, s);
    }
    // A^T: scatter into zeroed padded copies, then fold back.  The scatter
    // also writes border cells, so a following A must re-zero the border.
    CT_TRY(launch_fill(sc.vx, g->pad.nvx, 0.0f, s));
    CT_TRY(launch_fill(sc.vy, g->pad.nvy, 0.0f, s));
    CT_TRY(launch_project_T(g, y, y_dtype, sc.vx, sc.vy, stop, s));
    return launch_unpad_sum(g, sc.vx, sc.vy, x, in_scale, stop, s);
}

}  // namespace ct

using namespace ct;

// ------------------------------------------------------------------ ABI
static int check_dtype(int dt) { return dt == CT_F32 || dt == CT_F16; }

extern "C" int ct_op_workspace_bytes(const ct_geometry *g, int op, int batch, size_t *bytes) {
    clear_error();
    CT_ARG_CHECK(g && bytes, "ct_op_workspace_bytes: NULL argument");
    CT_ARG_CHECK(op >= CT_OP_A && op <= CT_OP_AT, "ct_op_workspace_bytes: unknown op");
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
    CT_ARG_CHECK(ws && ws_bytes >= need, "ct_backproject_AT: workspace too small");
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
