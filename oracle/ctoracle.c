/*
 * FP64 CPU oracle for the cone-beam projector hot path -- TEST INFRASTRUCTURE.
 *
 * Plain, slow, obviously correct definitions that the HIP library is checked
 * against.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it; the product path never calls it.  It shares no code,
 * header or table with the HIP library.
 *
 * Geometry (default circular cone beam, the paper's section on geometric
 * flexibility and its geometry-parameter appendix):
 *   world frame Oxyz in mm, object static, source rotating about +z;
 *   view angle theta: source S = DSO (cos t, sin t, 0), unit vector
 *   e = (cos t, sin t, 0) from the origin towards the source, detector centre
 *   S - DSD e, detector axes u = (-sin t, cos t, 0), v = (0, 0, 1);
 *   pixel (iv, iu) centre at u = (iu + 1/2 - nu/2) du + off_u,
 *                            v = (iv + 1/2 - nv/2) dv + off_v
 *   (index 0 is the bottom-left corner of the detector);
 *   voxel (iz, iy, ix) is the half-open cell [lo_x + ix dx, lo_x + (ix+1) dx)
 *   x ..., lo_x = off_x - nx dx / 2; volume is C-order [nz][ny][nx].
 * The paper states that D lies at distance DSO from the origin; read as S at
 * DSO from O and the detector at DSD from S (the names' meaning in the
 * geometry table).
 *
 * Operators (the paper's linear model Ax + e = b, section 2.1):
 *   orc_forward_siddon  -- exact radiological path (Siddon 1985): per ray
 *                          the sorted plane crossings, midpoint rule for the
 *                          cell, length in mm.
 *   orc_forward_interp  -- trilinear ray marching: samples at t_k = k ds
 *                          from the source, ds = accuracy * min voxel size,
 *                          trilinear tent weights, zero outside the grid.
 *   orc_backward_*      -- exact transposes, by ray-driven scatter.
 *   orc_*_adjoint_voxels-- the same transposes evaluated per chosen voxel by
 *                          brute force (independent of the scatter code).
 *   orc_bfdk            -- FDK backprojector (Feldkamp 1984): bilinear
 *                          detector sample times (DSO/U)^2.
 *   orc_fdk_filter      -- cosine weight, optional Wang weight, Ram-Lak ramp
 *                          by direct linear convolution, angular scale.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double DSD, DSO;
    int64_t nz, ny, nx;
    double dz, dy, dx;
    double oz, oy, ox;
    int64_t nv, nu;
    double dv, du;
    double ov, ou;
    double accuracy;
} orc_geo;

/* ------------------------------------------------------------ geometry -- */

/* Per-view geometry (the paper's section on geometric flexibility: Euler ZYZ
 * gantry angles, centre-of-rotation shift, in-place detector rotation, and
 * every parameter settable per projection).  Readings:
 *   machine frame before the gantry rotation: source (DSO, COR, 0), detector
 *   centre (DSO - DSD, COR, 0), detector axes u = (0, 1, 0), v = (0, 0, 1),
 *   normal (1, 0, 0) towards the source;
 *   detector rotation about its centre (roll about the normal x, pitch about
 *   u = y, yaw about v = z): R_d = Rx(roll) Ry(pitch) Rz(yaw);
 *   detector offsets are taken along the rotated detector axes;
 *   gantry rotation about the origin: R_g = Rz(z1) Ry(y1) Rz(z2);
 *   offOrigin moves the volume: rays are expressed relative to it.
 * With (z1, 0, 0) and everything else zero this is the circular default. */
typedef struct {
    double z1, y1, z2;
    double DSO, DSD;
    double oz, oy, ox;   /* volume centre (mm) */
    double ov, ou;       /* detector offset (mm) */
    double cor;          /* mm */
    double roll, pitch, yaw;
} orc_view;

/* when set, ray_endpoints and the footprints use these frames instead of the
 * circular default (the Python wrapper sets it around one call) */
static const orc_view* g_views = NULL;
static int64_t g_nviews = 0;

void orc_set_views(const orc_view* v, int64_t n)
{
    g_views = n > 0 ? v : NULL;
    g_nviews = n;
}

static void rot_x(double a, const double in[3], double out[3])
{
    const double c = cos(a), s = sin(a);
    out[0] = in[0];
    out[1] = c * in[1] - s * in[2];
    out[2] = s * in[1] + c * in[2];
}

static void rot_y(double a, const double in[3], double out[3])
{
    const double c = cos(a), s = sin(a);
    out[0] = c * in[0] + s * in[2];
    out[1] = in[1];
    out[2] = -s * in[0] + c * in[2];
}

static void rot_z(double a, const double in[3], double out[3])
{
    const double c = cos(a), s = sin(a);
    out[0] = c * in[0] - s * in[1];
    out[1] = s * in[0] + c * in[1];
    out[2] = in[2];
}

/* world (volume-relative) source, detector centre and unit detector axes of
 * view k */
static void view_frame(const orc_view* w, double S[3], double D[3], double eu[3], double ev[3])
{
    double t[3], t2[3];
    const double s0[3] = {w->DSO, w->cor, 0.0}, d0[3] = {w->DSO - w->DSD, w->cor, 0.0};
    const double u0[3] = {0.0, 1.0, 0.0}, v0[3] = {0.0, 0.0, 1.0};
    double ud[3], vd[3];
    /* detector rotation: yaw, then pitch, then roll */
    rot_z(w->yaw, u0, t); rot_y(w->pitch, t, t2); rot_x(w->roll, t2, ud);
    rot_z(w->yaw, v0, t); rot_y(w->pitch, t, t2); rot_x(w->roll, t2, vd);
    const double* in[4] = {s0, d0, ud, vd};
    double* out[4] = {S, D, eu, ev};
    for (int i = 0; i < 4; ++i) {
        rot_z(w->z2, in[i], t); rot_y(w->y1, t, t2); rot_z(w->z1, t2, out[i]);
    }
    const double o[3] = {w->ox, w->oy, w->oz};
    for (int a = 0; a < 3; ++a) {
        S[a] -= o[a];
        D[a] -= o[a];
    }
}

/* Source position and the centre of pixel (iv, iu) of view k. */
static void ray_endpoints(const orc_geo* g, const double* angles, int64_t k, double iv, double iu, double S[3],
                          double P[3])
{
    if (g_views) {
        const orc_view* w = &g_views[k];
        double D[3], eu[3], ev[3];
        view_frame(w, S, D, eu, ev);
        const double u = (iu + 0.5 - 0.5 * (double)g->nu) * g->du + w->ou;
        const double v = (iv + 0.5 - 0.5 * (double)g->nv) * g->dv + w->ov;
        for (int a = 0; a < 3; ++a) P[a] = D[a] + u * eu[a] + v * ev[a];
        return;
    }
    const double theta = angles[k];
    const double c = cos(theta), s = sin(theta);
    const double u = (iu + 0.5 - 0.5 * (double)g->nu) * g->du + g->ou;
    const double v = (iv + 0.5 - 0.5 * (double)g->nv) * g->dv + g->ov;
    S[0] = g->DSO * c;
    S[1] = g->DSO * s;
    S[2] = 0.0;
    /* detector centre S - DSD e, plus u * (-s, c, 0) + v * (0, 0, 1) */
    P[0] = S[0] - g->DSD * c - u * s;
    P[1] = S[1] - g->DSD * s + u * c;
    P[2] = v;
}

void orc_ray_endpoints(const orc_geo* g, double theta, double iv, double iu, double* S, double* P)
{
    ray_endpoints(g, &theta, 0, iv, iu, S, P);
}

/* volume box: lo[a], cell size h[a], count n[a] for a = x, y, z */
static void vol_box(const orc_geo* g, double lo[3], double h[3], int64_t n[3])
{
    n[0] = g->nx; n[1] = g->ny; n[2] = g->nz;
    h[0] = g->dx; h[1] = g->dy; h[2] = g->dz;
    lo[0] = g->ox - 0.5 * (double)g->nx * g->dx;
    lo[1] = g->oy - 0.5 * (double)g->ny * g->dy;
    lo[2] = g->oz - 0.5 * (double)g->nz * g->dz;
}

static int64_t lin_index(const orc_geo* g, int64_t ix, int64_t iy, int64_t iz)
{
    return (iz * g->ny + iy) * g->nx + ix;
}

/* --------------------------------------------------------------- Siddon -- */

/* Crossings of the planes of one axis with alpha strictly inside (amin, amax),
 * written in increasing alpha order.  Returns how many. */
static int64_t axis_crossings(double S, double d, double lo, double h, int64_t n, double amin, double amax,
                              double* out)
{
    int64_t m = 0;
    if (d == 0.0) return 0;
    for (int64_t q = 0; q <= n; ++q) {
        const int64_t k = d > 0 ? q : n - q;      /* increasing alpha */
        const double a = (lo + (double)k * h - S) / d;
        if (a > amin && a < amax) out[m++] = a;
    }
    return m;
}

/* Siddon segments of the ray S -> P: cell[m] (linear index) and len[m] (mm).
 * Work buffer `wa` must hold nx + ny + nz + 3 doubles.  Returns the count. */
static int64_t siddon_segments(const orc_geo* g, const double S[3], const double P[3], int64_t* cell,
                               double* len, double* wa)
{
    double lo[3], h[3];
    int64_t n[3];
    vol_box(g, lo, h, n);
    double d[3] = {P[0] - S[0], P[1] - S[1], P[2] - S[2]};
    const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double amin = 0.0, amax = 1.0;
    for (int a = 0; a < 3; ++a) {
        const double hi = lo[a] + (double)n[a] * h[a];
        if (d[a] != 0.0) {
            const double a0 = (lo[a] - S[a]) / d[a], a1 = (hi - S[a]) / d[a];
            amin = fmax(amin, fmin(a0, a1));
            amax = fmin(amax, fmax(a0, a1));
        } else if (!(S[a] >= lo[a] && S[a] < hi)) {
            return 0;
        }
    }
    if (!(amin < amax)) return 0;
    double* ax = wa;
    const int64_t mx = axis_crossings(S[0], d[0], lo[0], h[0], n[0], amin, amax, ax);
    double* ay = ax + mx;
    const int64_t my = axis_crossings(S[1], d[1], lo[1], h[1], n[1], amin, amax, ay);
    double* az = ay + my;
    const int64_t mz = axis_crossings(S[2], d[2], lo[2], h[2], n[2], amin, amax, az);
    /* merge the three increasing lists, closing with amax */
    int64_t px = 0, py = 0, pz = 0, m = 0;
    double cur = amin;
    for (;;) {
        double nxt = amax;
        if (px < mx && ax[px] < nxt) nxt = ax[px];
        if (py < my && ay[py] < nxt) nxt = ay[py];
        if (pz < mz && az[pz] < nxt) nxt = az[pz];
        if (nxt > cur) {
            const double mid = 0.5 * (cur + nxt);
            int64_t idx[3];
            for (int a = 0; a < 3; ++a) {
                int64_t i = (int64_t)floor((S[a] + mid * d[a] - lo[a]) / h[a]);
                if (i < 0) i = 0;
                if (i > n[a] - 1) i = n[a] - 1;
                idx[a] = i;
            }
            cell[m] = lin_index(g, idx[0], idx[1], idx[2]);
            len[m] = (nxt - cur) * L;
            ++m;
        }
        if (nxt >= amax) break;
        while (px < mx && ax[px] <= nxt) ++px;
        while (py < my && ay[py] <= nxt) ++py;
        while (pz < mz && az[pz] <= nxt) ++pz;
        cur = nxt;
    }
    return m;
}

/* ---------------------------------------------------------- interpolated -- */

typedef struct {
    double S[3], dhat[3], ds;
    int64_t k0, k1;            /* sample indices t_k = k ds, k0..k1 inclusive */
} interp_ray_t;

/* Clip the ray to the open box where trilinear interpolation can be nonzero
 * (voxel-centre coordinates in (-1, n)), within [0, |P - S|]. */
static int interp_setup(const orc_geo* g, const double S[3], const double P[3], interp_ray_t* r)
{
    double lo[3], h[3];
    int64_t n[3];
    vol_box(g, lo, h, n);
    double d[3] = {P[0] - S[0], P[1] - S[1], P[2] - S[2]};
    const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double hmin = fmin(h[0], fmin(h[1], h[2]));
    r->ds = g->accuracy * hmin;
    double t0 = 0.0, t1 = L;
    for (int a = 0; a < 3; ++a) {
        r->S[a] = S[a];
        r->dhat[a] = d[a] / L;
        const double glo = lo[a] - 0.5 * h[a];                 /* centre coord -1 */
        const double ghi = lo[a] + ((double)n[a] + 0.5) * h[a]; /* centre coord n  */
        if (r->dhat[a] != 0.0) {
            const double ta = (glo - S[a]) / r->dhat[a], tb = (ghi - S[a]) / r->dhat[a];
            t0 = fmax(t0, fmin(ta, tb));
            t1 = fmin(t1, fmax(ta, tb));
        } else if (!(S[a] > glo && S[a] < ghi)) {
            return 0;
        }
    }
    if (!(t0 < t1)) return 0;
    r->k0 = (int64_t)ceil(t0 / r->ds);
    r->k1 = (int64_t)floor(t1 / r->ds);
    return r->k1 >= r->k0;
}

/* Trilinear corners of sample k: up to 8 (cell, weight) pairs inside the grid. */
static int interp_corners(const orc_geo* g, const interp_ray_t* r, int64_t k, int64_t cell[8], double w[8])
{
    double lo[3], h[3];
    int64_t n[3];
    vol_box(g, lo, h, n);
    const double t = (double)k * r->ds;
    int64_t j0[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        const double c = (r->S[a] + t * r->dhat[a] - lo[a]) / h[a] - 0.5;   /* voxel-centre coordinate */
        j0[a] = (int64_t)floor(c);
        f[a] = c - (double)j0[a];
    }
    int m = 0;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                const int64_t ix = j0[0] + cx, iy = j0[1] + cy, iz = j0[2] + cz;
                if (ix < 0 || iy < 0 || iz < 0 || ix >= n[0] || iy >= n[1] || iz >= n[2]) continue;
                const double wx = cx ? f[0] : 1.0 - f[0];
                const double wy = cy ? f[1] : 1.0 - f[1];
                const double wz = cz ? f[2] : 1.0 - f[2];
                cell[m] = lin_index(g, ix, iy, iz);
                w[m] = wx * wy * wz;
                ++m;
            }
    return m;
}

/* ---------------------------------------------------------- operators -- */

enum { ORC_SIDDON = 0, ORC_INTERP = 1 };

static double ray_sum(const orc_geo* g, int kind, const double S[3], const double P[3], const double* vol,
                      int64_t* cell, double* len, double* wa)
{
    double acc = 0.0;
    if (kind == ORC_SIDDON) {
        const int64_t m = siddon_segments(g, S, P, cell, len, wa);
        for (int64_t i = 0; i < m; ++i) acc += len[i] * vol[cell[i]];
    } else {
        interp_ray_t r;
        if (!interp_setup(g, S, P, &r)) return 0.0;
        int64_t c8[8];
        double w8[8];
        for (int64_t k = r.k0; k <= r.k1; ++k) {
            const int m = interp_corners(g, &r, k, c8, w8);
            for (int i = 0; i < m; ++i) acc += w8[i] * vol[c8[i]];
        }
        acc *= r.ds;
    }
    return acc;
}

static void ray_scatter(const orc_geo* g, int kind, const double S[3], const double P[3], double y, double* acc,
                        int64_t* cell, double* len, double* wa)
{
    if (kind == ORC_SIDDON) {
        const int64_t m = siddon_segments(g, S, P, cell, len, wa);
        for (int64_t i = 0; i < m; ++i) acc[cell[i]] += len[i] * y;
    } else {
        interp_ray_t r;
        if (!interp_setup(g, S, P, &r)) return;
        int64_t c8[8];
        double w8[8];
        for (int64_t k = r.k0; k <= r.k1; ++k) {
            const int m = interp_corners(g, &r, k, c8, w8);
            for (int i = 0; i < m; ++i) acc[c8[i]] += r.ds * w8[i] * y;
        }
    }
}

static int64_t seg_cap(const orc_geo* g) { return g->nx + g->ny + g->nz + 8; }

/* proj[view][iv][iu] = (A vol) for every ray. */
void orc_forward(const orc_geo* g, int kind, const double* angles, int64_t nviews, const double* vol,
                 double* proj)
{
    const int64_t nrow = nviews * g->nv;
    #pragma omp parallel
    {
        const int64_t cap = seg_cap(g);
        int64_t* cell = (int64_t*)malloc(sizeof(int64_t) * cap);
        double* len = (double*)malloc(sizeof(double) * cap);
        double* wa = (double*)malloc(sizeof(double) * cap);
        #pragma omp for schedule(dynamic, 4)
        for (int64_t row = 0; row < nrow; ++row) {
            const int64_t k = row / g->nv, iv = row % g->nv;
            for (int64_t iu = 0; iu < g->nu; ++iu) {
                double S[3], P[3];
                ray_endpoints(g, angles, k, (double)iv, (double)iu, S, P);
                proj[row * g->nu + iu] = ray_sum(g, kind, S, P, vol, cell, len, wa);
            }
        }
        free(cell); free(len); free(wa);
    }
}

/* Arbitrary rays: out[i] = (A vol) for ray (view[i], iv[i], iu[i]). */
void orc_forward_rays(const orc_geo* g, int kind, const double* angles, const double* vol, int64_t nrays,
                      const int64_t* view, const int64_t* iv, const int64_t* iu, double* out)
{
    #pragma omp parallel
    {
        const int64_t cap = seg_cap(g);
        int64_t* cell = (int64_t*)malloc(sizeof(int64_t) * cap);
        double* len = (double*)malloc(sizeof(double) * cap);
        double* wa = (double*)malloc(sizeof(double) * cap);
        #pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < nrays; ++i) {
            double S[3], P[3];
            ray_endpoints(g, angles, view[i], (double)iv[i], (double)iu[i], S, P);
            out[i] = ray_sum(g, kind, S, P, vol, cell, len, wa);
        }
        free(cell); free(len); free(wa);
    }
}

/* vol = A^T proj, by ray-driven scatter into per-thread FP64 volumes that
 * are summed in thread order (deterministic for a fixed thread count). */
void orc_backward(const orc_geo* g, int kind, const double* angles, int64_t nviews, const double* proj,
                  double* vol)
{
    const int64_t nvox = g->nx * g->ny * g->nz;
    const int64_t nrow = nviews * g->nv;
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double* part = (double*)calloc((size_t)nt * (size_t)nvox, sizeof(double));
    #pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* acc = part + (size_t)tid * (size_t)nvox;
        const int64_t cap = seg_cap(g);
        int64_t* cell = (int64_t*)malloc(sizeof(int64_t) * cap);
        double* len = (double*)malloc(sizeof(double) * cap);
        double* wa = (double*)malloc(sizeof(double) * cap);
        #pragma omp for schedule(static)
        for (int64_t row = 0; row < nrow; ++row) {
            const int64_t k = row / g->nv, iv = row % g->nv;
            for (int64_t iu = 0; iu < g->nu; ++iu) {
                const double y = proj[row * g->nu + iu];
                if (y == 0.0) continue;
                double S[3], P[3];
                ray_endpoints(g, angles, k, (double)iv, (double)iu, S, P);
                ray_scatter(g, kind, S, P, y, acc, cell, len, wa);
            }
        }
        free(cell); free(len); free(wa);
    }
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nvox; ++j) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t) s += part[(size_t)t * (size_t)nvox + j];
        vol[j] = s;
    }
    free(part);
}

/* ------------------------------------------- brute-force adjoint per voxel -- */

/* Length (mm) of the segment S -> P inside the axis-aligned box [bl, bh]. */
static double box_chord(const double S[3], const double P[3], const double bl[3], const double bh[3])
{
    double d[3] = {P[0] - S[0], P[1] - S[1], P[2] - S[2]};
    const double L = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double a0 = 0.0, a1 = 1.0;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0) {
            const double p = (bl[a] - S[a]) / d[a], q = (bh[a] - S[a]) / d[a];
            a0 = fmax(a0, fmin(p, q));
            a1 = fmin(a1, fmax(p, q));
        } else if (!(S[a] >= bl[a] && S[a] < bh[a])) {
            return 0.0;
        }
    }
    return a1 > a0 ? (a1 - a0) * L : 0.0;
}

/* Detector pixel index range [iu0, iu1] x [iv0, iv1] that can see the box
 * [bl, bh] in view theta: project its 8 corners, pad by one pixel. */
static int box_footprint(const orc_geo* g, const double* angles, int64_t k, const double bl[3], const double bh[3],
                         int64_t* iu0, int64_t* iu1, int64_t* iv0, int64_t* iv1)
{
    double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
    /* pixel index coordinates of the central projection of each box corner:
     * from the pixel grid of view k (pixel (0,0) centre, axis steps) */
    double S[3], P00[3], P10[3], P01[3];
    ray_endpoints(g, angles, k, 0.0, 0.0, S, P00);
    ray_endpoints(g, angles, k, 0.0, 1.0, S, P10);
    ray_endpoints(g, angles, k, 1.0, 0.0, S, P01);
    double eu[3], ev[3], n[3];
    for (int a = 0; a < 3; ++a) {
        eu[a] = P10[a] - P00[a];
        ev[a] = P01[a] - P00[a];
    }
    n[0] = eu[1] * ev[2] - eu[2] * ev[1];
    n[1] = eu[2] * ev[0] - eu[0] * ev[2];
    n[2] = eu[0] * ev[1] - eu[1] * ev[0];
    const double eu2 = eu[0] * eu[0] + eu[1] * eu[1] + eu[2] * eu[2];
    const double ev2 = ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2];
    double dn = 0.0;   /* (P00 - S) . n */
    for (int a = 0; a < 3; ++a) dn += (P00[a] - S[a]) * n[a];
    for (int q = 0; q < 8; ++q) {
        const double X[3] = {(q & 1) ? bh[0] : bl[0], (q & 2) ? bh[1] : bl[1], (q & 4) ? bh[2] : bl[2]};
        double xn = 0.0;
        for (int a = 0; a < 3; ++a) xn += (X[a] - S[a]) * n[a];
        /* the corner must lie beyond the source, on the detector's side */
        if (!(xn / dn > 0.0)) return 0;
        const double t = dn / xn;   /* S + t (X - S) lies on the detector plane */
        double pu = 0.0, pv = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double d = S[a] + t * (X[a] - S[a]) - P00[a];
            pu += d * eu[a];
            pv += d * ev[a];
        }
        const double fu = pu / eu2, fv = pv / ev2;
        umin = fmin(umin, fu); umax = fmax(umax, fu);
        vmin = fmin(vmin, fv); vmax = fmax(vmax, fv);
    }
    *iu0 = (int64_t)floor(umin) - 1; *iu1 = (int64_t)ceil(umax) + 1;
    *iv0 = (int64_t)floor(vmin) - 1; *iv1 = (int64_t)ceil(vmax) + 1;
    if (*iu0 < 0) *iu0 = 0;
    if (*iv0 < 0) *iv0 = 0;
    if (*iu1 > g->nu - 1) *iu1 = g->nu - 1;
    if (*iv1 > g->nv - 1) *iv1 = g->nv - 1;
    return *iu0 <= *iu1 && *iv0 <= *iv1;
}

/* out[i] = (A^T proj)_j for voxel j = (iz[i], iy[i], ix[i]), Siddon weights:
 * a_ij = length of ray i inside the cell of voxel j. */
void orc_siddon_adjoint_voxels(const orc_geo* g, const double* angles, int64_t nviews, const double* proj,
                               int64_t nsel, const int64_t* iz, const int64_t* iy, const int64_t* ix,
                               double* out)
{
    double lo[3], h[3];
    int64_t n[3];
    vol_box(g, lo, h, n);
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nsel; ++i) {
        const double bl[3] = {lo[0] + ix[i] * h[0], lo[1] + iy[i] * h[1], lo[2] + iz[i] * h[2]};
        const double bh[3] = {bl[0] + h[0], bl[1] + h[1], bl[2] + h[2]};
        double acc = 0.0;
        for (int64_t k = 0; k < nviews; ++k) {
            int64_t u0, u1, v0, v1;
            if (!box_footprint(g, angles, k, bl, bh, &u0, &u1, &v0, &v1)) continue;
            for (int64_t iv = v0; iv <= v1; ++iv)
                for (int64_t iu = u0; iu <= u1; ++iu) {
                    double S[3], P[3];
                    ray_endpoints(g, angles, k, (double)iv, (double)iu, S, P);
                    const double w = box_chord(S, P, bl, bh);
                    if (w > 0.0) acc += w * proj[(k * g->nv + iv) * g->nu + iu];
                }
        }
        out[i] = acc;
    }
}

/* Same for the interpolated projector: a_ij = ds * sum_k phi(c_k - j), phi the
 * trilinear tent evaluated directly on every sample in the tent's support. */
void orc_interp_adjoint_voxels(const orc_geo* g, const double* angles, int64_t nviews, const double* proj,
                               int64_t nsel, const int64_t* iz, const int64_t* iy, const int64_t* ix,
                               double* out)
{
    double lo[3], h[3];
    int64_t n[3];
    vol_box(g, lo, h, n);
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nsel; ++i) {
        const int64_t j[3] = {ix[i], iy[i], iz[i]};
        double bl[3], bh[3];          /* tent support of voxel j: centre +- one cell */
        for (int a = 0; a < 3; ++a) {
            bl[a] = lo[a] + ((double)j[a] - 0.5) * h[a];
            bh[a] = lo[a] + ((double)j[a] + 1.5) * h[a];
        }
        double acc = 0.0;
        for (int64_t k = 0; k < nviews; ++k) {
            int64_t u0, u1, v0, v1;
            if (!box_footprint(g, angles, k, bl, bh, &u0, &u1, &v0, &v1)) continue;
            for (int64_t iv = v0; iv <= v1; ++iv)
                for (int64_t iu = u0; iu <= u1; ++iu) {
                    double S[3], P[3];
                    ray_endpoints(g, angles, k, (double)iv, (double)iu, S, P);
                    interp_ray_t r;
                    if (!interp_setup(g, S, P, &r)) continue;
                    /* phi(. - j) vanishes outside the support box: only the
                     * samples with t_k inside the segment's clip to [bl, bh]
                     * can contribute (the others are skipped, not approximated) */
                    double t0 = 0.0, t1 = 1e300;
                    for (int a = 0; a < 3; ++a) {
                        if (r.dhat[a] != 0.0) {
                            const double ta = (bl[a] - r.S[a]) / r.dhat[a], tb = (bh[a] - r.S[a]) / r.dhat[a];
                            t0 = fmax(t0, fmin(ta, tb));
                            t1 = fmin(t1, fmax(ta, tb));
                        }
                    }
                    if (!(t0 < t1)) continue;
                    const int64_t qa = (int64_t)floor(t0 / r.ds) - 1, qb = (int64_t)ceil(t1 / r.ds) + 1;
                    double w = 0.0;
                    for (int64_t q = qa > r.k0 ? qa : r.k0; q <= (qb < r.k1 ? qb : r.k1); ++q) {
                        const double t = (double)q * r.ds;
                        double phi = 1.0;
                        for (int a = 0; a < 3 && phi > 0.0; ++a) {
                            const double c = (r.S[a] + t * r.dhat[a] - lo[a]) / h[a] - 0.5;
                            phi *= fmax(0.0, 1.0 - fabs(c - (double)j[a]));
                        }
                        w += phi;
                    }
                    if (w > 0.0) acc += r.ds * w * proj[(k * g->nv + iv) * g->nu + iu];
                }
        }
        out[i] = acc;
    }
}

/* out[i] = 2 (A^T (A x - y))_j for the listed voxels j: for every ray i of
 * the voxel's footprint with a_ij != 0, the full ray sum (A x)_i minus y_i,
 * times a_ij (cell chord or tent sum), doubled.  The gradient of
 * |A x - y|^2 evaluated entry by entry. */
void orc_gradient_voxels(const orc_geo* g, int kind, const double* angles, int64_t nviews, const double* x,
                         const double* y, int64_t nsel, const int64_t* iz, const int64_t* iy, const int64_t* ix,
                         double* out)
{
    double lo[3], h[3];
    int64_t n[3];
    vol_box(g, lo, h, n);
    #pragma omp parallel
    {
        const int64_t cap = seg_cap(g);
        int64_t* cell = (int64_t*)malloc(sizeof(int64_t) * cap);
        double* len = (double*)malloc(sizeof(double) * cap);
        double* wa = (double*)malloc(sizeof(double) * cap);
        #pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < nsel; ++i) {
            const int64_t j[3] = {ix[i], iy[i], iz[i]};
            double bl[3], bh[3];
            for (int a = 0; a < 3; ++a) {
                const double pad = kind == ORC_SIDDON ? 0.0 : 0.5;   /* cell, or tent support */
                bl[a] = lo[a] + ((double)j[a] - pad) * h[a];
                bh[a] = lo[a] + ((double)j[a] + 1.0 + pad) * h[a];
            }
            double acc = 0.0;
            for (int64_t k = 0; k < nviews; ++k) {
                int64_t u0, u1, v0, v1;
                if (!box_footprint(g, angles, k, bl, bh, &u0, &u1, &v0, &v1)) continue;
                for (int64_t iv = v0; iv <= v1; ++iv)
                    for (int64_t iu = u0; iu <= u1; ++iu) {
                        double S[3], P[3];
                        ray_endpoints(g, angles, k, (double)iv, (double)iu, S, P);
                        double a_ij = 0.0;
                        if (kind == ORC_SIDDON) {
                            a_ij = box_chord(S, P, bl, bh);
                        } else {
                            interp_ray_t r;
                            if (!interp_setup(g, S, P, &r)) continue;
                            for (int64_t q = r.k0; q <= r.k1; ++q) {
                                const double t = (double)q * r.ds;
                                double phi = 1.0;
                                for (int a = 0; a < 3 && phi > 0.0; ++a) {
                                    const double c = (r.S[a] + t * r.dhat[a] - lo[a]) / h[a] - 0.5;
                                    phi *= fmax(0.0, 1.0 - fabs(c - (double)j[a]));
                                }
                                a_ij += phi;
                            }
                            a_ij *= r.ds;
                        }
                        if (a_ij == 0.0) continue;
                        const double res = ray_sum(g, kind, S, P, x, cell, len, wa) - y[(k * g->nv + iv) * g->nu + iu];
                        acc += a_ij * res;
                    }
            }
            out[i] = 2.0 * acc;
        }
        free(cell); free(len); free(wa);
    }
}

/* Explicit system matrix (rows = rays in [view][iv][iu] order, cols = voxels),
 * every entry evaluated from its definition: cell chord (Siddon) or the
 * tent sum over all samples (interpolated).  For tiny problems only. */
void orc_dense_matrix(const orc_geo* g, int kind, const double* angles, int64_t nviews, double* M)
{
    double lo[3], h[3];
    int64_t n[3];
    vol_box(g, lo, h, n);
    const int64_t nvox = g->nx * g->ny * g->nz;
    const int64_t nray = nviews * g->nv * g->nu;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nray; ++r) {
        const int64_t k = r / (g->nv * g->nu), iv = (r / g->nu) % g->nv, iu = r % g->nu;
        double S[3], P[3];
        ray_endpoints(g, angles, k, (double)iv, (double)iu, S, P);
        interp_ray_t ir;
        const int has = kind == ORC_INTERP ? interp_setup(g, S, P, &ir) : 0;
        for (int64_t jz = 0; jz < n[2]; ++jz)
            for (int64_t jy = 0; jy < n[1]; ++jy)
                for (int64_t jx = 0; jx < n[0]; ++jx) {
                    const int64_t col = lin_index(g, jx, jy, jz);
                    double w = 0.0;
                    if (kind == ORC_SIDDON) {
                        const double bl[3] = {lo[0] + jx * h[0], lo[1] + jy * h[1], lo[2] + jz * h[2]};
                        const double bh[3] = {bl[0] + h[0], bl[1] + h[1], bl[2] + h[2]};
                        w = box_chord(S, P, bl, bh);
                    } else if (has) {
                        const int64_t j[3] = {jx, jy, jz};
                        for (int64_t q = ir.k0; q <= ir.k1; ++q) {
                            const double t = (double)q * ir.ds;
                            double phi = 1.0;
                            for (int a = 0; a < 3; ++a) {
                                const double c = (ir.S[a] + t * ir.dhat[a] - lo[a]) / h[a] - 0.5;
                                phi *= fmax(0.0, 1.0 - fabs(c - (double)j[a]));
                            }
                            w += phi;
                        }
                        w *= ir.ds;
                    }
                    M[r * nvox + col] = w;
                }
    }
}

/* ------------------------------------------------------------------ FDK -- */

/* Bilinear sample of one detector image at pixel-index coordinates (fu, fv),
 * pixel centres at integers, zero outside the detector. */
static double bilinear(const orc_geo* g, const double* img, double fu, double fv)
{
    const double u0 = floor(fu), v0 = floor(fv);
    const double au = fu - u0, av = fv - v0;
    double s = 0.0;
    for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
            const int64_t iu = (int64_t)u0 + a, iv = (int64_t)v0 + b;
            if (iu < 0 || iv < 0 || iu >= g->nu || iv >= g->nv) continue;
            s += (a ? au : 1.0 - au) * (b ? av : 1.0 - av) * img[iv * g->nu + iu];
        }
    return s;
}

/* vol[j] = sum_views (DSO/U)^2 * bilinear(q_view; u_j, v_j), U = DSO - X.e */
void orc_bfdk(const orc_geo* g, const double* angles, int64_t nviews, const double* proj, double* vol)
{
    double lo[3], h[3];
    int64_t n[3];
    vol_box(g, lo, h, n);
    #pragma omp parallel for collapse(2) schedule(static)
    for (int64_t iz = 0; iz < n[2]; ++iz)
        for (int64_t iy = 0; iy < n[1]; ++iy)
            for (int64_t ix = 0; ix < n[0]; ++ix) {
                const double X = lo[0] + (ix + 0.5) * h[0];
                const double Y = lo[1] + (iy + 0.5) * h[1];
                const double Z = lo[2] + (iz + 0.5) * h[2];
                double acc = 0.0;
                for (int64_t k = 0; k < nviews; ++k) {
                    const double c = cos(angles[k]), s = sin(angles[k]);
                    const double U = g->DSO - (X * c + Y * s);
                    const double ud = g->DSD / U * (-X * s + Y * c);
                    const double vd = g->DSD / U * Z;
                    const double fu = (ud - g->ou) / g->du + 0.5 * (double)g->nu - 0.5;
                    const double fv = (vd - g->ov) / g->dv + 0.5 * (double)g->nv - 0.5;
                    const double w = (g->DSO / U) * (g->DSO / U);
                    acc += w * bilinear(g, proj + k * g->nv * g->nu, fu, fv);
                }
                vol[lin_index(g, ix, iy, iz)] = acc;
            }
}

/* The FDK backprojector at the listed voxels only (same definition). */
void orc_bfdk_voxels(const orc_geo* g, const double* angles, int64_t nviews, const double* proj, int64_t nsel,
                     const int64_t* iz, const int64_t* iy, const int64_t* ix, double* out)
{
    double lo[3], h[3];
    int64_t n[3];
    vol_box(g, lo, h, n);
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nsel; ++i) {
        const double X = lo[0] + (ix[i] + 0.5) * h[0];
        const double Y = lo[1] + (iy[i] + 0.5) * h[1];
        const double Z = lo[2] + (iz[i] + 0.5) * h[2];
        double acc = 0.0;
        for (int64_t k = 0; k < nviews; ++k) {
            const double c = cos(angles[k]), s = sin(angles[k]);
            const double U = g->DSO - (X * c + Y * s);
            const double fu = (g->DSD / U * (-X * s + Y * c) - g->ou) / g->du + 0.5 * (double)g->nu - 0.5;
            const double fv = (g->DSD / U * Z - g->ov) / g->dv + 0.5 * (double)g->nv - 0.5;
            acc += (g->DSO / U) * (g->DSO / U) * bilinear(g, proj + k * g->nv * g->nu, fu, fv);
        }
        out[i] = acc;
    }
}

/* Wang redundancy weight for a laterally offset detector (Wang 2002):
 * overlap half-width D = nu du / 2 - |off_u|, u' = u sign(off_u);
 * w = sin^2(pi/4 (u' + D) / D) on [-D, D], 1 beyond D, 0 below -D. */
double orc_wang_weight(const orc_geo* g, double u)
{
    if (g->ou == 0.0) return 1.0;
    const double D = 0.5 * (double)g->nu * g->du - fabs(g->ou);
    const double up = g->ou > 0 ? u : -u;
    if (up >= D) return 1.0;
    if (up <= -D) return 0.0;
    const double s = sin(M_PI / 4.0 * (up + D) / D);
    return s * s;
}

/* FDK filtering of projections q[nviews][nv][nu] (Kak & Slaney ch. 3):
 * 1. cosine weight DSD / sqrt(DSD^2 + u^2 + v^2);  2. optional Wang weight;
 * 3. Ram-Lak ramp on the iso-scaled grid tau = du DSO / DSD as a linear
 *    convolution q2[m] = tau sum_n h[m - n] q1[n], h[0] = 1/(4 tau^2),
 *    h[odd n] = -1/(n^2 pi^2 tau^2), h[even n != 0] = 0;
 * 4. angular scale dtheta / 2 with dtheta = 2 pi / ntotal (dtheta alone when
 *    the Wang weight already removes the redundancy). */
void orc_fdk_filter(const orc_geo* g, int64_t nviews, int64_t ntotal, int wang, const double* proj, double* out)
{
    const int64_t nu = g->nu, nv = g->nv;
    const double tau = g->du * g->DSO / g->DSD;
    const double dtheta = 2.0 * M_PI / (double)ntotal;
    const double scale = wang ? dtheta : 0.5 * dtheta;
    double* h = (double*)malloc(sizeof(double) * (size_t)(2 * nu));
    for (int64_t m = 0; m < 2 * nu; ++m) {
        const int64_t k = m - nu;  /* h index in [-nu, nu) */
        if (k == 0) h[m] = 1.0 / (4.0 * tau * tau);
        else if (k % 2 != 0) h[m] = -1.0 / ((double)(k * k) * M_PI * M_PI * tau * tau);
        else h[m] = 0.0;
    }
    #pragma omp parallel
    {
        double* q1 = (double*)malloc(sizeof(double) * (size_t)nu);
        #pragma omp for schedule(static)
        for (int64_t row = 0; row < nviews * nv; ++row) {
            const int64_t iv = row % nv;
            const double v = (iv + 0.5 - 0.5 * (double)nv) * g->dv + g->ov;
            for (int64_t iu = 0; iu < nu; ++iu) {
                const double u = (iu + 0.5 - 0.5 * (double)nu) * g->du + g->ou;
                double w = g->DSD / sqrt(g->DSD * g->DSD + u * u + v * v);
                if (wang) w *= orc_wang_weight(g, u);
                q1[iu] = proj[row * nu + iu] * w;
            }
            for (int64_t m = 0; m < nu; ++m) {
                double s = 0.0;
                for (int64_t k = 0; k < nu; ++k) s += h[m - k + nu] * q1[k];
                out[row * nu + m] = tau * s * scale;
            }
        }
        free(q1);
    }
    free(h);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the following calls (timing runs); n < 1 is ignored. */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
