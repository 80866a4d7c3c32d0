/*
 * FP64 CPU oracle for the CT operators of the ABBA method (Sidky, Hansen,
 * Jorgensen and Pan, "Iterative image reconstruction for CT with unmatched
 * projection matrices using the generalized minimal residual algorithm").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is plain, slow and meant to be read
 * against the definitions.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header or table
 * with the HIP library.
 *
 * Operators (Sec. III of the paper names them; the formulas are the readings
 * written out below because the paper defers the discretisation to a
 * textbook):
 *   A     ray-driven forward projector, one of
 *         Joseph's method (projector 0): for the dominant axis a of the ray
 *         direction r, sample the ray in every voxel-centre plane along a,
 *         interpolate bilinearly (linearly in 2D) in the plane with zero
 *         outside the grid, sum, and multiply by vox*|r|/|r_a|;
 *         the line-intersection method the paper uses (projector 1,
 *         Siddon's): A_ij is the length of the part of ray i inside voxel j.
 *   A^T   exact transpose of the same weights (scatter form).
 *   B_un  voxel-driven back-projector: project each voxel centre onto the
 *         detector, interpolate the data linearly (bilinearly in 3D) with zero
 *         outside the detector, weight, and sum over views.  2D weight
 *         vox^2/du; 3D weight vox^3 M^2/(du dv), M the magnification.
 *   F     Ram-Lak ramp filter along u (Sec. III, B_FBP = B_un F):
 *         (Fq)[a] = du * sum_a' h[a-a'] q[a'], h[0] = 1/(4 du^2),
 *         h[even != 0] = 0, h[odd j] = -1/(pi^2 j^2 du^2); zero-padded
 *         linear convolution per view and detector row.
 *
 * Conventions (shared with the library by definition, not by code):
 *   volume  x[(iz*ny + iy)*nx + ix], voxel centre (i - (N-1)/2)*vox per axis;
 *   2D      nz = nv = 1; view p: n = (cos t, sin t), d = (-sin t, cos t),
 *           bin a at s = (a - (nu-1)/2)*du, ray {s n + t d};
 *   3D      source (SOD cos t, SOD sin t, 0), detector centre
 *           source - SDD (cos t, sin t, 0), e_u = (-sin t, cos t, 0),
 *           e_v = (0,0,1), pixel (a_u, a_v) at centre + u e_u + v e_v with
 *           u = (a_u - (nu-1)/2) du, v = (a_v - (nv-1)/2) dv;
 *   data    y[(p*nv + av)*nu + au];
 *   ties    the dominant axis goes to the lowest axis index on ties; for the
 *           uniform 2D view set t_p = pi p / P the choice is made in
 *           integers: x-major iff P <= 4p <= 3P.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int kind;              /* 0: 2D parallel beam, 1: 3D circular cone beam */
    int nx, ny, nz;
    double vox;
    int nviews;
    const double *angles;  /* nviews angles (radians), always given */
    int uniform;           /* 1 if angles are the uniform set (tie rule) */
    int nu, nv;
    double du, dv;
    double sod, sdd;
    int projector;         /* 0: Joseph, 1: line intersection (Siddon) */
} orc_geom;

static const double PI = 3.14159265358979323846;

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Origin o and direction r of ray (p, av, au). */
static void ray_of(const orc_geom *g, int p, int av, int au, double o[3], double r[3])
{
    double th = g->angles[p];
    double c = cos(th), s = sin(th);
    if (g->kind == 0) {
        double sa = (au - 0.5 * (g->nu - 1)) * g->du;
        o[0] = sa * c; o[1] = sa * s; o[2] = 0.0;
        r[0] = -s;     r[1] = c;      r[2] = 0.0;
    } else {
        double src[3] = { g->sod * c, g->sod * s, 0.0 };
        double cen[3] = { src[0] - g->sdd * c, src[1] - g->sdd * s, 0.0 };
        double u = (au - 0.5 * (g->nu - 1)) * g->du;
        double v = (av - 0.5 * (g->nv - 1)) * g->dv;
        double pix[3] = { cen[0] - u * s, cen[1] + u * c, cen[2] + v };
        o[0] = src[0]; o[1] = src[1]; o[2] = src[2];
        r[0] = pix[0] - src[0]; r[1] = pix[1] - src[1]; r[2] = pix[2] - src[2];
    }
}

static int dominant_axis(const orc_geom *g, int p, const double r[3])
{
    if (g->kind == 0 && g->uniform) {
        int P = g->nviews;
        return (P <= 4 * p && 4 * p <= 3 * P) ? 0 : 1;
    }
    double ax = fabs(r[0]), ay = fabs(r[1]), az = fabs(r[2]);
    if (ax >= ay && ax >= az) return 0;
    if (ay >= az) return 1;
    return 2;
}

static inline long vidx(const orc_geom *g, const int i[3])
{
    return ((long)i[2] * g->ny + i[1]) * (long)g->nx + i[0];
}

/*
 * Walk the Joseph samples of one ray.  mode 0: return sum of interpolated
 * values of x; mode 1: scatter val * weight into xo (A^T); mode 2: count
 * samples whose point lies inside (-1, N_b) x (-1, N_c).
 */
static double joseph_walk(const orc_geom *g, int p, int av, int au,
                          const double *x, double *xo, double val, int mode,
                          long *count)
{
    double o[3], r[3];
    int N[3] = { g->nx, g->ny, g->nz };
    ray_of(g, p, av, au, o, r);
    int a = dominant_axis(g, p, r);
    int b = (a + 1) % 3, c = (a + 2) % 3;
    double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double step = g->vox * rn / fabs(r[a]);
    double acc = 0.0;
    for (int j = 0; j < N[a]; ++j) {
        double ca = (j - 0.5 * (N[a] - 1)) * g->vox;
        double t = (ca - o[a]) / r[a];
        double fb = (o[b] + t * r[b]) / g->vox + 0.5 * (N[b] - 1);
        double fc = (o[c] + t * r[c]) / g->vox + 0.5 * (N[c] - 1);
        if (!(fb > -1.0 && fb < N[b] && fc > -1.0 && fc < N[c])) continue;
        if (mode == 2) { (*count)++; continue; }
        int ib = (int)floor(fb), ic = (int)floor(fc);
        double wb = fb - ib, wc = fc - ic;
        for (int db = 0; db < 2; ++db) {
            int kb = ib + db;
            if (kb < 0 || kb >= N[b]) continue;
            double w_b = db ? wb : 1.0 - wb;
            for (int dc = 0; dc < 2; ++dc) {
                int kc = ic + dc;
                if (kc < 0 || kc >= N[c]) continue;
                double w = w_b * (dc ? wc : 1.0 - wc);
                int ii[3];
                ii[a] = j; ii[b] = kb; ii[c] = kc;
                if (mode == 0) acc += w * x[vidx(g, ii)];
                else xo[vidx(g, ii)] += w * val * step;
            }
        }
    }
    return acc * step;
}


static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/*
 * Line-intersection walk of one ray {o + t r}: every parameter where the ray
 * crosses a voxel boundary plane inside the volume box is collected and
 * sorted; each segment between consecutive parameters lies in one voxel,
 * found from the segment's midpoint, and has length (t2 - t1) |r|.  mode 0:
 * return sum of length * x; mode 1: scatter val * length into xo; mode 2:
 * count segments of positive length.  2D rays have r_z = 0 and o_z = 0 and
 * never leave the single slice.
 */
static double siddon_walk(const orc_geom *g, int p, int av, int au,
                          const double *x, double *xo, double val, int mode,
                          long *count)
{
    double o[3], r[3];
    int N[3] = { g->nx, g->ny, g->nz };
    ray_of(g, p, av, au, o, r);
    double lo[3], t_in = -INFINITY, t_out = INFINITY;
    for (int a = 0; a < 3; ++a) {
        lo[a] = -0.5 * N[a] * g->vox;
        double hi = -lo[a];
        if (r[a] == 0.0) {
            if (!(o[a] > lo[a] && o[a] < hi)) return 0.0;
            continue;
        }
        double t1 = (lo[a] - o[a]) / r[a], t2 = (hi - o[a]) / r[a];
        t_in = fmax(t_in, fmin(t1, t2));
        t_out = fmin(t_out, fmax(t1, t2));
    }
    if (!(t_in < t_out)) return 0.0;
    int cap = N[0] + N[1] + N[2] + 2, n = 0;
    double *ts = (double *)malloc(sizeof(double) * (size_t)cap);
    if (!ts) return NAN;
    ts[n++] = t_in;
    for (int a = 0; a < 3; ++a) {
        if (r[a] == 0.0) continue;
        for (int k = 1; k < N[a]; ++k) {
            double t = (lo[a] + k * g->vox - o[a]) / r[a];
            if (t > t_in && t < t_out) ts[n++] = t;
        }
    }
    ts[n++] = t_out;
    qsort(ts, (size_t)n, sizeof(double), cmp_double);
    double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    double acc = 0.0;
    for (int k = 0; k + 1 < n; ++k) {
        double len = (ts[k + 1] - ts[k]) * rn;
        if (!(len > 0.0)) continue;
        double tm = 0.5 * (ts[k] + ts[k + 1]);
        int ii[3];
        for (int a = 0; a < 3; ++a) {
            int i = (int)floor((o[a] + tm * r[a] - lo[a]) / g->vox);
            ii[a] = i < 0 ? 0 : (i >= N[a] ? N[a] - 1 : i);
        }
        if (mode == 0) acc += len * x[vidx(g, ii)];
        else if (mode == 1) xo[vidx(g, ii)] += val * len;
        else (*count)++;
    }
    free(ts);
    return acc;
}

static double ray_walk(const orc_geom *g, int p, int av, int au, const double *x, double *xo, double val,
                       int mode, long *count)
{
    if (g->projector == 1) return siddon_walk(g, p, av, au, x, xo, val, mode, count);
    return joseph_walk(g, p, av, au, x, xo, val, mode, count);
}

/* y = A x */
void orc_project_A(const orc_geom *g, const double *x, double *y)
{
    long nrays = (long)g->nviews * g->nv * g->nu;
#pragma omp parallel for schedule(dynamic, 64)
    for (long rid = 0; rid < nrays; ++rid) {
        int au = (int)(rid % g->nu);
        int av = (int)((rid / g->nu) % g->nv);
        int p = (int)(rid / ((long)g->nu * g->nv));
        y[rid] = ray_walk(g, p, av, au, x, NULL, 0.0, 0, NULL);
    }
}

/* A applied to selected rays only: out[i] = (A x)[ray_ids[i]] */
void orc_project_A_rays(const orc_geom *g, const double *x, long nsel,
                        const int64_t *ray_ids, double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (long i = 0; i < nsel; ++i) {
        long rid = ray_ids[i];
        int au = (int)(rid % g->nu);
        int av = (int)((rid / g->nu) % g->nv);
        int p = (int)(rid / ((long)g->nu * g->nv));
        out[i] = ray_walk(g, p, av, au, x, NULL, 0.0, 0, NULL);
    }
}

/* x = A^T y, scatter form; per-thread buffers summed in thread order. */
void orc_backproject_AT(const orc_geom *g, const double *y, double *x)
{
    long n = (long)g->nx * g->ny * g->nz;
    long nrays = (long)g->nviews * g->nv * g->nu;
    int nt = orc_num_threads();
    double *buf = (double *)calloc((size_t)nt * (size_t)n, sizeof(double));
    if (!buf) { for (long i = 0; i < n; ++i) x[i] = NAN; return; }
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = buf + (size_t)tid * (size_t)n;
#pragma omp for schedule(static)
        for (long rid = 0; rid < nrays; ++rid) {
            double val = y[rid];
            if (val == 0.0) continue;
            int au = (int)(rid % g->nu);
            int av = (int)((rid / g->nu) % g->nv);
            int p = (int)(rid / ((long)g->nu * g->nv));
            ray_walk(g, p, av, au, NULL, mine, val, 1, NULL);
        }
    }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t) s += buf[(size_t)t * (size_t)n + i];
        x[i] = s;
    }
    free(buf);
}

/* Exact number of A-updates: Joseph samples whose point lies inside the open
 * support box of the grid (bilinear taps touch the volume), or, for the
 * line-intersection projector, ray-voxel segments (siddon_count). */
/* Line-intersection updates of one ray: 1 + the number of voxel boundary
 * planes crossed strictly inside the grid (coinciding crossings counted
 * separately), 0 for a ray that misses the grid. */
static long siddon_count(const orc_geom *g, int p, int av, int au)
{
    double o[3], r[3];
    int N[3] = { g->nx, g->ny, g->nz };
    ray_of(g, p, av, au, o, r);
    double lo[3], t_in = -INFINITY, t_out = INFINITY;
    for (int a = 0; a < 3; ++a) {
        lo[a] = -0.5 * N[a] * g->vox;
        if (r[a] == 0.0) {
            if (!(o[a] > lo[a] && o[a] < -lo[a])) return 0;
            continue;
        }
        double t1 = (lo[a] - o[a]) / r[a], t2 = (-lo[a] - o[a]) / r[a];
        t_in = fmax(t_in, fmin(t1, t2));
        t_out = fmin(t_out, fmax(t1, t2));
    }
    if (!(t_in < t_out)) return 0;
    long n = 1;
    for (int a = 0; a < 3; ++a) {
        if (r[a] == 0.0) continue;
        double f1 = (o[a] + t_in * r[a] - lo[a]) / g->vox, f2 = (o[a] + t_out * r[a] - lo[a]) / g->vox;
        double fmn = fmin(f1, f2), fmx = fmax(f1, f2);
        long k0 = (long)floor(fmn) + 1, k1 = (long)ceil(fmx) - 1;
        if (k0 < 1) k0 = 1;
        if (k1 > N[a] - 1) k1 = N[a] - 1;
        if (k1 >= k0) n += k1 - k0 + 1;
    }
    return n;
}

int64_t orc_count_A_updates(const orc_geom *g)
{
    long nrays = (long)g->nviews * g->nv * g->nu;
    long total = 0;
    if (g->projector == 1) {
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : total)
        for (long rid = 0; rid < nrays; ++rid) {
            int au = (int)(rid % g->nu);
            int av = (int)((rid / g->nu) % g->nv);
            int p = (int)(rid / ((long)g->nu * g->nv));
            total += siddon_count(g, p, av, au);
        }
        return (int64_t)total;
    }
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : total)
    for (long rid = 0; rid < nrays; ++rid) {
        int au = (int)(rid % g->nu);
        int av = (int)((rid / g->nu) % g->nv);
        int p = (int)(rid / ((long)g->nu * g->nv));
        long c = 0;
        ray_walk(g, p, av, au, NULL, NULL, 0.0, 2, &c);
        total += c;
    }
    return (int64_t)total;
}

/* B_un at one voxel (ix, iy, iz): sum over views of weight * interp(y_p). */
static double bp_voxel(const orc_geom *g, const double *y, int ix, int iy, int iz)
{
    double px = (ix - 0.5 * (g->nx - 1)) * g->vox;
    double py = (iy - 0.5 * (g->ny - 1)) * g->vox;
    double pz = (iz - 0.5 * (g->nz - 1)) * g->vox;
    double acc = 0.0;
    for (int p = 0; p < g->nviews; ++p) {
        double th = g->angles[p];
        double c = cos(th), s = sin(th);
        double fu, fv, w;
        if (g->kind == 0) {
            double sp = px * c + py * s;
            fu = sp / g->du + 0.5 * (g->nu - 1);
            fv = 0.0;
            w = g->vox * g->vox / g->du;
        } else {
            double U = g->sod - (px * c + py * s);
            double M = g->sdd / U;
            double u = M * (-px * s + py * c);
            double v = M * pz;
            fu = u / g->du + 0.5 * (g->nu - 1);
            fv = v / g->dv + 0.5 * (g->nv - 1);
            w = g->vox * g->vox * g->vox * M * M / (g->du * g->dv);
        }
        int iu = (int)floor(fu), iv = (int)floor(fv);
        double wu = fu - iu, wv = fv - iv;
        const double *yp = y + (long)p * g->nv * g->nu;
        double val = 0.0;
        for (int dv_ = 0; dv_ < 2; ++dv_) {
            int kv = iv + dv_;
            if (kv < 0 || kv >= g->nv) continue;
            double w_v = dv_ ? wv : 1.0 - wv;
            for (int du_ = 0; du_ < 2; ++du_) {
                int ku = iu + du_;
                if (ku < 0 || ku >= g->nu) continue;
                val += w_v * (du_ ? wu : 1.0 - wu) * yp[(long)kv * g->nu + ku];
            }
        }
        acc += w * val;
    }
    return acc;
}

/* x = B_un y */
void orc_backproject_B(const orc_geom *g, const double *y, double *x)
{
    long n = (long)g->nx * g->ny * g->nz;
#pragma omp parallel for schedule(dynamic, 256)
    for (long i = 0; i < n; ++i) {
        int ix = (int)(i % g->nx);
        int iy = (int)((i / g->nx) % g->ny);
        int iz = (int)(i / ((long)g->nx * g->ny));
        x[i] = bp_voxel(g, y, ix, iy, iz);
    }
}

/* B_un at selected voxels only */
void orc_backproject_B_voxels(const orc_geom *g, const double *y, long nsel,
                              const int64_t *vox_ids, double *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (long k = 0; k < nsel; ++k) {
        long i = vox_ids[k];
        int ix = (int)(i % g->nx);
        int iy = (int)((i / g->nx) % g->ny);
        int iz = (int)(i / ((long)g->nx * g->ny));
        out[k] = bp_voxel(g, y, ix, iy, iz);
    }
}

static double ramlak_tap(int j, double du)
{
    if (j == 0) return 1.0 / (4.0 * du * du);
    if (j % 2 == 0) return 0.0;
    return -1.0 / (PI * PI * (double)j * (double)j * du * du);
}

/* out = F y, row by row (rows of length nu, nviews*nv rows) */
void orc_ramp(const orc_geom *g, const double *y, double *out)
{
    long rows = (long)g->nviews * g->nv;
    int nu = g->nu;
#pragma omp parallel for schedule(dynamic, 16)
    for (long rw = 0; rw < rows; ++rw) {
        const double *q = y + rw * nu;
        double *o = out + rw * nu;
        for (int a = 0; a < nu; ++a) {
            double acc = 0.0;
            for (int a2 = 0; a2 < nu; ++a2) acc += ramlak_tap(a - a2, g->du) * q[a2];
            o[a] = g->du * acc;
        }
    }
}
