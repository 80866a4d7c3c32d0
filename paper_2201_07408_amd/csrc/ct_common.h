// Internal declarations shared by the HIP translation units of libctabba.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "ct.h"

namespace ct {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
void clear_error();

#define CT_HIP_CHECK(expr)                                                     \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) {                                                \
            ::ct::set_error(std::string(#expr) + ": " + hipGetErrorString(e_)); \
            return CT_ERR_HIP;                                                 \
        }                                                                      \
    } while (0)

#define CT_LAUNCH_CHECK()                                                      \
    do {                                                                       \
        hipError_t e_ = hipGetLastError();                                     \
        if (e_ != hipSuccess) {                                                \
            ::ct::set_error(std::string("kernel launch: ") + hipGetErrorString(e_)); \
            return CT_ERR_HIP;                                                 \
        }                                                                      \
    } while (0)

#define CT_ARG_CHECK(cond, msg)                                                \
    do {                                                                       \
        if (!(cond)) {                                                         \
            ::ct::set_error(msg);                                              \
            return CT_ERR_ARG;                                                 \
        }                                                                      \
    } while (0)

#define CT_TRY(expr)                                                           \
    do {                                                                       \
        int s_ = (expr);                                                       \
        if (s_ != CT_OK) return s_;                                            \
    } while (0)

constexpr int kPad = 2;        // zero border of the padded volume copies
constexpr size_t kAlign = 256; // workspace carve alignment

inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------- kernel geometry
// Plain-old-data copy of the geometry passed by value to kernels.
// Per (view, detector column) quantities of a cone-beam ray that do not
// depend on the detector row, for the voxel-driven transpose: the in-plane
// slope t = r_b / r_a along the dominant axis a, dv / (r_a vox), the step
// factor vox / |r_a| (negative for y-dominant columns) and r_x^2 + r_y^2.
struct ColT {
    double t;
    float ar, is, sxy, pad;
};

// Per (view, detector column) part of a cone-beam ray's set-up for the
// projector (see ray_column): 1 / r_a, the plane offset, r_x^2 + r_y^2, the
// plane range allowed by the in-plane coordinate, that coordinate's offset
// (padding included) and slope, and the dominant axis.
struct RayCol {
    double inv_ra, base, sxy, jlo, jhi;
    float fb0, gb;
    int ax, pad;
};

struct GeomK {
    int kind;          // 0 = 2D parallel, 1 = 3D cone
    int proj;          // CT_JOSEPH or CT_SIDDON
    int nx, ny, nz;
    int P, nu, nv;
    double vox, du, dv, sod, sdd;
    const double *cs;  // device: cos, sin per view (2*P)
    const float *cs32; // device: the same table rounded to FP32
    const int *axis;   // device: per-view dominant axis for 2D (0 = x, 1 = y)
    const ColT *colT;  // device: per (view, column) table of cone-beam rays, P x nu
    const RayCol *rcol;  // device, cone: per (view, column) part of the projector's ray set-up, P x nu
    const int *vdom;   // device: per view, bit 0 / bit 1 set if any column is x- / y-dominant
    const int4 *vrect; // device, cone: per view, detector columns [x, y] and rows [z, w] outside
                       // of which no ray meets the volume (bounding box of its shadow)
    const int *vshift; // device, cone: per view, column offset of the projector's ray tiles
};

// Padded, axis-permuted volume copies read by the forward projector and
// accumulated into by the scatter transpose.
//   Vx[ix][iz+pz][iy+kPad], rows of ny+2*kPad rounded up to a multiple of 4,
//   (nz+2*pz) rows per plane
//   Vy[iy][iz+pz][ix+kPad], rows of nx+2*kPad rounded likewise
// with pz = kPad in 3D and 0 in 2D.
struct PadLayout {
    int pz;
    uint32_t rx, sx;   // row / plane stride of Vx (elements)
    uint32_t ry, sy;   // row / plane stride of Vy
    size_t nvx, nvy;   // element counts
};

inline PadLayout pad_layout(const GeomK &g) {
    PadLayout L;
    L.pz = (g.kind == 1) ? kPad : 0;
    // rows are a multiple of four floats so that staged 16-byte loads align
    L.rx = (uint32_t)((g.ny + 2 * kPad + 3) & ~3);
    L.sx = L.rx * (uint32_t)(g.nz + 2 * L.pz);
    L.ry = (uint32_t)((g.nx + 2 * kPad + 3) & ~3);
    L.sy = L.ry * (uint32_t)(g.nz + 2 * L.pz);
    L.nvx = (size_t)L.sx * g.nx;
    L.nvy = (size_t)L.sy * g.ny;
    return L;
}

}  // namespace ct

struct ct_geometry {
    ct_geometry_desc d;            // angles pointer cleared
    int device;
    int uniform;
    std::vector<double> h_cs;      // cos, sin per view (host copy)
    std::vector<int> h_axis;       // 2D dominant axis per view
    double *d_cs = nullptr;
    float *d_cs32 = nullptr;
    ct::ColT *d_colT = nullptr;
    ct::RayCol *d_rcol = nullptr;
    int *d_vdom = nullptr;
    int4 *d_vrect = nullptr;
    int *d_vshift = nullptr;
    int *d_axis = nullptr;
    float *d_ramp = nullptr;       // du * h[j], j = 0..nu-1 (FP32)
    size_t n_vox = 0, n_rays = 0;
    ct::GeomK k;                   // kernel view
    ct::PadLayout pad;
    // Launch setting of the cone-beam projector: its view grouping and
    // workgroup order in the low 32 bits, resident workgroups per CU in the
    // high 32 (0: the size heuristic).  Written by ct_projector_config and
    // ct_tune_projector, read once per launch; every setting gives the same
    // results.
    std::atomic<uint64_t> a_cfg{0};
};

namespace ct {

// -------------------------------------------------------------- profiling
// Brackets one kernel launch with two events on its stream when kernel
// timing is enabled (ct_profile_enable); a no-op otherwise.
enum { PROF_A = 0, PROF_AT, PROF_B, PROF_F, PROF_CGS, PROF_ARNOLDI, kProfClasses };
class ProfScope {
  public:
    // no event pairs while a stream is being captured into a graph
    static void suppress(bool on);
    static bool suppressed();

    ProfScope(int cls, hipStream_t s);
    ~ProfScope();
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;

  private:
    int cls_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

// --------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return CT_OK or CT_ERR_HIP.  `stop`, when
// non-null, points to a device flag; kernels exit at once when it is set.

int launch_fill(float *p, size_t n, float v, hipStream_t s);
int launch_pad_zero(const ct_geometry *g, float *vx, float *vy, hipStream_t s);
int launch_pad_copy(const ct_geometry *g, const void *x, int x_dtype, float *vx, float *vy,
                    const int *stop, hipStream_t s);
int launch_project(const ct_geometry *g, const float *vx, const float *vy, void *y,
                   int y_dtype, const float *out_scale, const int *stop, hipStream_t s);
// fills g->d_rcol and g->d_colT (cone geometries) from the kernel view
int launch_col_table(ct_geometry *g);
// cone-beam A^T gathered per voxel straight into x (times *scale if given);
// ys: n_rays floats of scratch for the step-weighted data
int launch_project_T_gather(const ct_geometry *g, const void *y, int y_dtype, float *x,
                            const float *scale, const int *stop, hipStream_t s, float *ys);
// 2D Joseph A^T gathered per pixel straight into x (times *scale if given)
int launch_project_T_par(const ct_geometry *g, const void *y, int y_dtype, float *x,
                         const float *scale, const int *stop, hipStream_t s);
int launch_backproject(const ct_geometry *g, const void *y, int y_dtype, float *x,
                       const float *in_scale, const int *stop, hipStream_t s);
int launch_ramp(const ct_geometry *g, const void *q, int q_dtype, void *out,
                int out_dtype, size_t rows, const int *stop, hipStream_t s);
// line-intersection projector and its transpose (x read / scattered in its
// own layout, no padded copies; the transpose adds into x); cone geometries
// project through launch_project's staged kernel instead
int launch_siddon(const ct_geometry *g, const float *x, void *y, int y_dtype,
                  const float *out_scale, const int *stop, hipStream_t s);
int launch_siddon_T(const ct_geometry *g, const void *y, int y_dtype, float *x,
                    const float *in_scale, const int *stop, hipStream_t s);

// Composite operators used by the solvers and the ABI: x/y of one item.
struct OpScratch {
    float *vx = nullptr, *vy = nullptr;   // padded copies (A, A^T)
    void *filt = nullptr;                  // filtered data (ramp), dtype as data; step-weighted
                                           // data of the cone-beam A^T (FP32)
};
size_t op_scratch_bytes(const ct_geometry *g, int op, int data_dtype);
OpScratch carve_op_scratch(const ct_geometry *g, int op, int data_dtype, void *ws);

// ------------------------------------------------ batched 2D problems
// A batched solve concatenates the vectors of its problems: image segment
// i starts at voff (a multiple of kBVec floats, zero-padded to the next
// multiple), data segment i at roff (a multiple of 64 floats).  Every
// batched kernel maps its workgroup to a problem through a prefix sum of
// per-problem workgroup counts.
constexpr int kBVec = 4096;

struct BSlice {
    GeomK g;               // 2D parallel geometry (device tables of its handle)
    PadLayout L;
    const float *ramp;     // du * h[j] of its handle
    const float *b;        // caller data [P][nu]
    float *x;              // caller image [ny][nx]
    size_t voff, roff;     // segment offsets in the batched image / data vectors
    uint32_t pvx, pvy;     // Vx / Vy offsets in the batched padded buffer (elements)
    const int *stop;       // the problem's stop flag
};

// workgroups per problem for each batched kernel and variant
inline int bpad_blocks(const GeomK &g) { return ((g.nx + 31) / 32) * ((g.ny + 31) / 32); }
inline int bray_blocks(const GeomK &g) { return (g.P * g.nu + 255) / 256; }
inline int bpix_blocks(const GeomK &g, int ppt) { return ((g.nx + 15) / 16) * ((g.ny + 16 * ppt - 1) / (16 * ppt)); }
constexpr int kBProjVariants = 2;   // plane loop unrolled by 4 or 8
constexpr int kBBackVariants = 3;   // 1, 2 or 4 pixels per work-item
inline int bback_ppt(int variant) { return variant == 0 ? 1 : variant == 1 ? 2 : 4; }

// vec: batched image vector; pad: batched padded buffer (pad_elems floats,
// borders zero).  q == nullptr reads each problem's caller data b.
int launch_bpad_copy(const BSlice *sl, int count, const int *pfx, int nblk, const float *vec, float *pad,
                     hipStream_t s);
int launch_bproject2d(const BSlice *sl, int count, const int *pfx, int nblk, int variant, const float *pad,
                      size_t pad_elems, float *q, hipStream_t s);
int launch_bbackproject2d(const BSlice *sl, int count, const int *pfx, int nblk, int variant, const float *q,
                          float *z, hipStream_t s);
int launch_bramp(const BSlice *sl, int count, const int *pfx, int nblk, int max_nu, const float *q, float *out,
                 hipStream_t s);

// y = A x.  Padding of vx/vy must already be zero (pad_ready) or is zeroed here.
// x is FP32, or FP16 (x_dtype) where A reads the padded copies (not the 2D
// line-intersection projector).
int apply_A(const ct_geometry *g, const void *x, void *y, int y_dtype, OpScratch &sc,
            bool pad_ready, const float *out_scale, const int *stop, hipStream_t s, int x_dtype = CT_F32);
// x = B y with B in {B_un, B_un F, A^T}.
int apply_B(const ct_geometry *g, int which, const void *y, int y_dtype, float *x,
            OpScratch &sc, const float *in_scale, const int *stop, hipStream_t s);

}  // namespace ct
