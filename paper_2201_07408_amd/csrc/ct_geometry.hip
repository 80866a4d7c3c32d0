// Geometry handle, error state and small shared launchers.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "ct_common.h"

namespace ct {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

__global__ void k_fill(float *__restrict__ p, size_t n, float v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

int launch_fill(float *p, size_t n, float v, hipStream_t s) {
    if (n == 0) return CT_OK;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    CT_LAUNCH_CHECK();
    return CT_OK;
}

// ------------------------------------------------------------- profiling
namespace {
struct ProfRec {
    int cls;
    hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_recs;
std::vector<hipEvent_t> g_prof_pool;
long g_prof_launches[kProfClasses] = {};
double g_prof_ms[kProfClasses] = {};
const char *g_prof_names[kProfClasses] = {"A", "AT", "B", "F", "CGS", "ARNOLDI"};
constexpr size_t kProfMax = 65536;

hipEvent_t pool_take() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// fold finished records into the totals; caller holds the lock
int prof_drain() {
    for (ProfRec &r : g_prof_recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            set_error("ct_profile: event timing failed");
            return CT_ERR_HIP;
        }
        g_prof_launches[r.cls] += 1;
        g_prof_ms[r.cls] += ms;
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
    }
    g_prof_recs.clear();
    return CT_OK;
}
}  // namespace

static thread_local bool t_prof_suppressed = false;

void ProfScope::suppress(bool on) { t_prof_suppressed = on; }
bool ProfScope::suppressed() { return t_prof_suppressed; }

ProfScope::ProfScope(int cls, hipStream_t s) : cls_(cls), s_(s) {
    if (t_prof_suppressed) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on || g_prof_recs.size() >= kProfMax) return;
    a_ = pool_take();
    b_ = pool_take();
    if (!a_ || !b_ || hipEventRecord(a_, s_) != hipSuccess) { a_ = b_ = nullptr; return; }
}

ProfScope::~ProfScope() {
    if (!a_) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (hipEventRecord(b_, s_) == hipSuccess) g_prof_recs.push_back(ProfRec{cls_, a_, b_});
}

// Per view of a circular cone-beam geometry: the detector columns
// [x, y] and rows [z, w] that hold the shadow of the volume's box widened by
// one voxel on every side (the reach of an interpolation or intersection
// weight).  The shadow of a box seen from a point in front of it is the
// convex hull of its corners' projections, so a ray through a pixel outside
// the rectangle misses the widened box and its projection is exactly zero.
// A view whose widened box reaches the source plane keeps the whole
// detector.
std::vector<int4> shadow_rects(const ct_geometry_desc &d, const std::vector<double> &cs) {
    std::vector<int4> r((size_t)d.n_views);
    const double hx = (0.5 * d.nx + 1.0) * d.voxel, hy = (0.5 * d.ny + 1.0) * d.voxel,
                 hz = (0.5 * d.nz + 1.0) * d.voxel;
    const double lim = 1.0e9;
    for (int p = 0; p < d.n_views; ++p) {
        const double c = cs[2 * (size_t)p], s = cs[2 * (size_t)p + 1];
        double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
        bool ok = true;
        for (int k = 0; k < 8; ++k) {
            const double X = (k & 1) ? hx : -hx, Y = (k & 2) ? hy : -hy, Z = (k & 4) ? hz : -hz;
            const double dx = X - d.sod * c, dy = Y - d.sod * s;
            const double depth = -(dx * c + dy * s);            // along the central ray
            if (!(depth > 1e-9 * d.sod)) { ok = false; break; }
            const double u = d.sdd * (-dx * s + dy * c) / depth;  // along e_u = (-sin, cos, 0)
            const double v = d.sdd * Z / depth;
            const double au = u / d.du + 0.5 * (d.nu - 1), av = v / d.dv + 0.5 * (d.nv - 1);
            umin = std::fmin(umin, au); umax = std::fmax(umax, au);
            vmin = std::fmin(vmin, av); vmax = std::fmax(vmax, av);
        }
        if (!ok) {
            r[p] = make_int4(0, d.nu - 1, 0, d.nv - 1);
            continue;
        }
        const auto lo = [&](double a) { return (int)std::fmax(std::floor(a) - 1.0, -lim); };
        const auto hi = [&](double a) { return (int)std::fmin(std::ceil(a) + 1.0, lim); };
        r[p] = make_int4(lo(umin), hi(umax), lo(vmin), hi(vmax));
    }
    return r;
}

}  // namespace ct

using namespace ct;

extern "C" int ct_profile_enable(int on) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return CT_OK;
}

extern "C" int ct_profile_reset(void) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_prof_mu);
    CT_TRY(prof_drain());
    for (int i = 0; i < kProfClasses; ++i) { g_prof_launches[i] = 0; g_prof_ms[i] = 0.0; }
    return CT_OK;
}

extern "C" int ct_profile_read(const char *name, long *launches, double *total_ms) {
    clear_error();
    CT_ARG_CHECK(name && launches && total_ms, "ct_profile_read: NULL argument");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    CT_TRY(prof_drain());
    for (int i = 0; i < kProfClasses; ++i)
        if (std::strcmp(name, g_prof_names[i]) == 0) {
            *launches = g_prof_launches[i];
            *total_ms = g_prof_ms[i];
            return CT_OK;
        }
    set_error("ct_profile_read: unknown kernel class");
    return CT_ERR_ARG;
}

extern "C" const char *ct_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *ct_version(void) { return "ctabba 0.1 (gfx950)"; }

extern "C" int ct_geometry_create(const ct_geometry_desc *desc, ct_geometry **out) {
    clear_error();
    CT_ARG_CHECK(out != nullptr, "ct_geometry_create: out is NULL");
    *out = nullptr;
    CT_ARG_CHECK(desc != nullptr, "ct_geometry_create: desc is NULL");
    const ct_geometry_desc &d = *desc;
    CT_ARG_CHECK(d.kind == CT_PARALLEL_2D || d.kind == CT_CONE_CIRCULAR_3D,
                 "ct_geometry_create: unknown kind");
    CT_ARG_CHECK(d.nx >= 1 && d.ny >= 1 && d.nz >= 1, "ct_geometry_create: volume sizes must be >= 1");
    CT_ARG_CHECK(d.projector == CT_JOSEPH || d.projector == CT_SIDDON, "ct_geometry_create: unknown projector");
    CT_ARG_CHECK(d.n_views >= 1 && d.nu >= 1 && d.nv >= 1, "ct_geometry_create: detector sizes must be >= 1");
    CT_ARG_CHECK(std::isfinite(d.voxel) && d.voxel > 0, "ct_geometry_create: voxel must be > 0");
    CT_ARG_CHECK(std::isfinite(d.du) && d.du > 0, "ct_geometry_create: du must be > 0");
    if (d.kind == CT_PARALLEL_2D) {
        CT_ARG_CHECK(d.nz == 1 && d.nv == 1, "ct_geometry_create: 2D geometry needs nz = nv = 1");
    } else {
        CT_ARG_CHECK(std::isfinite(d.dv) && d.dv > 0, "ct_geometry_create: dv must be > 0");
        CT_ARG_CHECK(std::isfinite(d.sod) && d.sod > 0, "ct_geometry_create: sod must be > 0");
        CT_ARG_CHECK(std::isfinite(d.sdd) && d.sdd > d.sod, "ct_geometry_create: sdd must exceed sod");
        double hx = 0.5 * d.nx * d.voxel, hy = 0.5 * d.ny * d.voxel;
        CT_ARG_CHECK(std::sqrt(hx * hx + hy * hy) < d.sod,
                     "ct_geometry_create: the volume reaches the source circle");
        double vmax = 0.5 * (d.nv - 1) * d.dv;
        if (!(vmax * std::sqrt(2.0) < d.sdd)) {
            set_error("ct_geometry_create: cone angle allows z-dominant rays");
            return CT_ERR_UNSUPPORTED;
        }
    }
    // 32-bit element offsets in the kernels
    const double lim = 4294967296.0 / 4.0;
    if ((double)d.nx * (d.ny + 2 * kPad) * (d.nz + 4 * kPad) >= lim ||
        (double)d.ny * (d.nx + 2 * kPad) * (d.nz + 4 * kPad) >= lim ||
        (double)d.n_views * d.nv * d.nu >= 2147483647.0) {
        set_error("ct_geometry_create: volume or data too large for 32-bit offsets");
        return CT_ERR_UNSUPPORTED;
    }

    ct_geometry *g = new (std::nothrow) ct_geometry();
    if (!g) {
        set_error("ct_geometry_create: host allocation failed");
        return CT_ERR_ALLOC;
    }
    g->d = d;
    g->d.angles = nullptr;
    g->uniform = (d.angles == nullptr);
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        set_error("ct_geometry_create: hipGetDevice failed");
        return CT_ERR_HIP;
    }
    const int P = d.n_views;
    g->h_cs.resize(2 * (size_t)P);
    g->h_axis.resize(P);
    const double span = (d.kind == CT_PARALLEL_2D) ? M_PI : 2.0 * M_PI;
    for (int p = 0; p < P; ++p) {
        double th = g->uniform ? (span * p) / P : d.angles[p];
        if (!std::isfinite(th)) {
            delete g;
            set_error("ct_geometry_create: non-finite angle");
            return CT_ERR_ARG;
        }
        double c = std::cos(th), s = std::sin(th);
        g->h_cs[2 * p] = c;
        g->h_cs[2 * p + 1] = s;
        int ax;
        if (g->uniform) ax = (P <= 4 * p && 4 * p <= 3 * P) ? 0 : 1;
        else ax = (std::fabs(s) >= std::fabs(c)) ? 0 : 1;
        g->h_axis[p] = ax;
    }
    std::vector<float> taps(d.nu);
    for (int j = 0; j < d.nu; ++j) {
        double h;
        if (j == 0) h = 1.0 / (4.0 * d.du);
        else if (j % 2 == 0) h = 0.0;
        else h = -1.0 / (M_PI * M_PI * (double)j * (double)j * d.du);
        taps[j] = (float)h;   // du * h[j]
    }
    std::vector<float> cs32(2 * (size_t)P);
    for (size_t i = 0; i < cs32.size(); ++i) cs32[i] = (float)g->h_cs[i];
    bool ok = hipMalloc(&g->d_cs, sizeof(double) * 2 * P) == hipSuccess &&
              hipMalloc(&g->d_cs32, sizeof(float) * 2 * P) == hipSuccess &&
              hipMalloc(&g->d_axis, sizeof(int) * P) == hipSuccess &&
              hipMalloc(&g->d_ramp, sizeof(float) * d.nu) == hipSuccess;
    if (!ok) {
        ct_geometry_destroy(g);
        set_error("ct_geometry_create: hipMalloc failed");
        return CT_ERR_ALLOC;
    }
    ok = hipMemcpy(g->d_cs, g->h_cs.data(), sizeof(double) * 2 * P, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(g->d_cs32, cs32.data(), sizeof(float) * 2 * P, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(g->d_axis, g->h_axis.data(), sizeof(int) * P, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(g->d_ramp, taps.data(), sizeof(float) * d.nu, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        ct_geometry_destroy(g);
        set_error("ct_geometry_create: hipMemcpy failed");
        return CT_ERR_HIP;
    }
    g->n_vox = (size_t)d.nx * d.ny * d.nz;
    g->n_rays = (size_t)P * d.nv * d.nu;
    GeomK &k = g->k;
    k.kind = d.kind;
    k.proj = d.projector;
    k.nx = d.nx; k.ny = d.ny; k.nz = d.nz;
    k.P = P; k.nu = d.nu; k.nv = d.nv;
    k.vox = d.voxel; k.du = d.du; k.dv = (d.kind == CT_PARALLEL_2D) ? 1.0 : d.dv;
    k.sod = d.sod; k.sdd = d.sdd;
    k.cs = g->d_cs;
    k.cs32 = g->d_cs32;
    k.axis = g->d_axis;
    k.colT = nullptr;
    k.rcol = nullptr;
    k.vdom = nullptr;
    k.vrect = nullptr;
    k.vshift = nullptr;
    g->pad = pad_layout(k);
    if (d.kind == CT_CONE_CIRCULAR_3D) {
        if (hipMalloc(&g->d_colT, sizeof(ColT) * (size_t)P * d.nu) != hipSuccess ||
            hipMalloc(&g->d_rcol, sizeof(RayCol) * (size_t)P * d.nu) != hipSuccess ||
            hipMalloc(&g->d_vdom, sizeof(int) * (size_t)P) != hipSuccess ||
            hipMalloc(&g->d_vrect, sizeof(int4) * (size_t)P) != hipSuccess ||
            hipMalloc(&g->d_vshift, sizeof(int) * (size_t)P) != hipSuccess) {
            ct_geometry_destroy(g);
            set_error("ct_geometry_create: hipMalloc failed");
            return CT_ERR_ALLOC;
        }
        const std::vector<int4> rect = shadow_rects(d, g->h_cs);
        if (hipMemcpy(g->d_vrect, rect.data(), sizeof(int4) * (size_t)P, hipMemcpyHostToDevice) != hipSuccess) {
            ct_geometry_destroy(g);
            set_error("ct_geometry_create: hipMemcpy failed");
            return CT_ERR_HIP;
        }
        k.colT = g->d_colT;
        k.rcol = g->d_rcol;
        k.vdom = g->d_vdom;
        k.vrect = g->d_vrect;
        k.vshift = g->d_vshift;
        const int st = launch_col_table(g);
        if (st != CT_OK) {
            ct_geometry_destroy(g);
            return st;
        }
    }
    *out = g;
    return CT_OK;
}

extern "C" void ct_geometry_destroy(ct_geometry *g) {
    if (!g) return;
    if (g->d_cs) (void)hipFree(g->d_cs);
    if (g->d_cs32) (void)hipFree(g->d_cs32);
    if (g->d_colT) (void)hipFree(g->d_colT);
    if (g->d_rcol) (void)hipFree(g->d_rcol);
    if (g->d_vdom) (void)hipFree(g->d_vdom);
    if (g->d_vrect) (void)hipFree(g->d_vrect);
    if (g->d_vshift) (void)hipFree(g->d_vshift);
    if (g->d_axis) (void)hipFree(g->d_axis);
    if (g->d_ramp) (void)hipFree(g->d_ramp);
    delete g;
}

extern "C" int ct_geometry_sizes(const ct_geometry *g, size_t *n_vox, size_t *n_rays) {
    clear_error();
    CT_ARG_CHECK(g != nullptr, "ct_geometry_sizes: geometry is NULL");
    if (n_vox) *n_vox = g->n_vox;
    if (n_rays) *n_rays = g->n_rays;
    return CT_OK;
}
