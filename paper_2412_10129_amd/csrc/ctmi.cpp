// Host side of libctmi: argument validation, the FP64 per-view geometry
// plan, the FFT filter tables and the exported C entry points.  Every check
// runs before anything is enqueued, so a failing call has no side effect.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "ctmi_internal.h"

namespace ctmi {
size_t reduce_ws_bytes();
}

using ctmi::Plan;
using ctmi::ViewGeo;

namespace {

thread_local char g_err[512] = "no error";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(CTMI_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Sizes shared by every plan: counts, spacings, the interpolation step and
// the index ranges the kernels rely on.
int check_sizes(const ctmi_geometry* g, int64_t nviews)
{
    if (!g) return fail(CTMI_EINVAL, "geometry is NULL");
    if (nviews < 1) return fail(CTMI_EINVAL, "nviews must be >= 1 (got %lld)", (long long)nviews);
    for (int a = 0; a < 3; ++a) {
        if (g->nVoxel[a] < 1) return fail(CTMI_EINVAL, "nVoxel[%d] must be >= 1", a);
        if (!finite_pos(g->dVoxel[a])) return fail(CTMI_EINVAL, "dVoxel[%d] must be finite and > 0", a);
    }
    for (int a = 0; a < 2; ++a) {
        if (g->nDetector[a] < 1) return fail(CTMI_EINVAL, "nDetector[%d] must be >= 1", a);
        if (!finite_pos(g->dDetector[a])) return fail(CTMI_EINVAL, "dDetector[%d] must be finite and > 0", a);
    }
    if (!finite_pos(g->accuracy)) return fail(CTMI_EINVAL, "accuracy must be finite and > 0");
    const int64_t nz = g->nVoxel[0], ny = g->nVoxel[1], nx = g->nVoxel[2];
    if (nx > (1 << 20) || ny > (1 << 20) || nz > (1 << 20)) return fail(CTMI_EOVERFLOW, "volume dimension too large");
    if ((double)nx * ny * nz >= 2147483648.0) return fail(CTMI_EOVERFLOW, "volume must hold < 2^31 voxels");
    const int64_t nv = g->nDetector[0], nu = g->nDetector[1];
    if (nu > 4096 || nv > (1 << 20)) return fail(CTMI_EOVERFLOW, "detector must have nu <= 4096");
    // the adjoints count a group of 8 views' footprint pixels in int32
    if (nu * nv >= (int64_t)1 << 28) return fail(CTMI_EOVERFLOW, "detector must hold < 2^28 pixels");
    if (nviews > (1 << 24)) return fail(CTMI_EOVERFLOW, "too many views");
    // the interpolated projector's samples of one ray inside the volume (its
    // diagonal over the step) must stay below 2^15
    const double hmin = std::fmin(g->dVoxel[0], std::fmin(g->dVoxel[1], g->dVoxel[2]));
    const double diag = std::sqrt((double)nx * nx * g->dVoxel[2] * g->dVoxel[2] +
                                  (double)ny * ny * g->dVoxel[1] * g->dVoxel[1] +
                                  (double)nz * nz * g->dVoxel[0] * g->dVoxel[0]);
    if (diag / (g->accuracy * hmin) + 8.0 >= 32768.0)
        return fail(CTMI_EOVERFLOW, "more than 2^15 interpolation samples per ray: raise accuracy");
    return CTMI_OK;
}

int check_geometry(const ctmi_geometry* g, const double* angles, int64_t nviews)
{
    int rc;
    if ((rc = check_sizes(g, nviews))) return rc;
    if (!angles) return fail(CTMI_EINVAL, "angles is NULL");
    if (!finite_pos(g->DSO) || !finite_pos(g->DSD)) return fail(CTMI_EINVAL, "DSO and DSD must be finite and > 0");
    if (!(g->DSD > g->DSO)) return fail(CTMI_EINVAL, "DSD must exceed DSO");
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(g->offOrigin[a])) return fail(CTMI_EINVAL, "offOrigin[%d] is not finite", a);
        if (!std::isfinite(g->rotDetector[a])) return fail(CTMI_EINVAL, "rotDetector[%d] is not finite", a);
    }
    for (int a = 0; a < 2; ++a)
        if (!std::isfinite(g->offDetector[a])) return fail(CTMI_EINVAL, "offDetector[%d] is not finite", a);
    if (!std::isfinite(g->COR)) return fail(CTMI_EINVAL, "COR is not finite");
    for (int64_t k = 0; k < nviews; ++k)
        if (!std::isfinite(angles[k])) return fail(CTMI_EINVAL, "angle %lld is not finite", (long long)k);
    if (g->COR != 0.0)
        return fail(CTMI_EUNSUPPORTED, "COR != 0 needs per-view geometry (ctmi_plan_create_views)");
    if (g->rotDetector[0] != 0.0 || g->rotDetector[1] != 0.0 || g->rotDetector[2] != 0.0)
        return fail(CTMI_EUNSUPPORTED, "rotDetector != 0 needs per-view geometry (ctmi_plan_create_views)");
    // the volume's circumscribed sphere, grown by one voxel, must lie strictly
    // between the source and the detector plane for every view
    double half2 = 0.0, off2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double h = 0.5 * (double)g->nVoxel[a] * g->dVoxel[a] + g->dVoxel[a];
        half2 += h * h;
        off2 += g->offOrigin[a] * g->offOrigin[a];
    }
    const double R = std::sqrt(half2) + std::sqrt(off2);
    if (!(g->DSO > R)) return fail(CTMI_EINVAL, "the source passes within the volume (DSO %.6g <= radius %.6g)", g->DSO, R);
    if (!(g->DSD - g->DSO > R))
        return fail(CTMI_EINVAL, "the detector cuts the volume (DSD - DSO %.6g <= radius %.6g)", g->DSD - g->DSO, R);
    return CTMI_OK;
}

// Per-view table in FP64, rounded once to FP32 (out), and its FP64 ray part (out64, optional).
void view_table(const ctmi_geometry* g, const double* angles, int64_t nviews, ViewGeo* out,
                ctmi::ViewGeo64* out64 = nullptr)
{
    const double nz = (double)g->nVoxel[0], ny = (double)g->nVoxel[1], nx = (double)g->nVoxel[2];
    const double hz = g->dVoxel[0], hy = g->dVoxel[1], hx = g->dVoxel[2];
    const double lo[3] = {g->offOrigin[2] - 0.5 * nx * hx, g->offOrigin[1] - 0.5 * ny * hy,
                          g->offOrigin[0] - 0.5 * nz * hz};
    const double h[3] = {hx, hy, hz};
    const double nu = (double)g->nDetector[1], nv = (double)g->nDetector[0];
    const double du = g->dDetector[1], dv = g->dDetector[0];
    const double ou = g->offDetector[1], ov = g->offDetector[0];
    const double u0 = (0.5 - 0.5 * nu) * du + ou, v0 = (0.5 - 0.5 * nv) * dv + ov;
    const double DSO = g->DSO, DSD = g->DSD;
    for (int64_t k = 0; k < nviews; ++k) {
        const double c = std::cos(angles[k]), s = std::sin(angles[k]);
        const double S[3] = {DSO * c, DSO * s, 0.0};
        const double P00[3] = {S[0] - DSD * c - u0 * s, S[1] - DSD * s + u0 * c, v0};
        const double DU[3] = {-du * s, du * c, 0.0};
        const double DV[3] = {0.0, 0.0, dv};
        ViewGeo& o = out[k];
        std::memset(&o, 0, sizeof o);
        for (int a = 0; a < 3; ++a) {
            o.S[a] = (float)((S[a] - lo[a]) / h[a]);
            o.P00[a] = (float)((P00[a] - lo[a]) / h[a]);
            o.DU[a] = (float)(DU[a] / h[a]);
            o.DV[a] = (float)(DV[a] / h[a]);
        }
        if (out64) {
            ctmi::ViewGeo64& o64 = out64[k];
            std::memset(&o64, 0, sizeof o64);
            for (int a = 0; a < 3; ++a) {
                o64.S[a] = (S[a] - lo[a]) / h[a];
                o64.P00[a] = (P00[a] - lo[a]) / h[a];
                o64.DU[a] = DU[a] / h[a];
                o64.DV[a] = DV[a] / h[a];
            }
        }
        // world position of voxel centre index c: X = lo + (c + 1/2) h
        const double X0 = lo[0] + 0.5 * hx, Y0 = lo[1] + 0.5 * hy, Z0 = lo[2] + 0.5 * hz;
        // W = U / DSO = 1 - (X c + Y s) / DSO
        const double MW[4] = {-hx * c / DSO, -hy * s / DSO, 0.0, 1.0 - (X0 * c + Y0 * s) / DSO};
        // fu W = (DSD/DSO (-X s + Y c) - ou W) / du + (nu/2 - 1/2) W
        const double ku = 0.5 * nu - 0.5 - ou / du, kv = 0.5 * nv - 0.5 - ov / dv;
        const double mag = DSD / DSO;
        const double MU[4] = {mag * (-s * hx) / du + ku * MW[0], mag * (c * hy) / du + ku * MW[1], 0.0,
                              mag * (-s * X0 + c * Y0) / du + ku * MW[3]};
        // fv W = (DSD/DSO Z - ov W) / dv + (nv/2 - 1/2) W
        const double MV[4] = {kv * MW[0], kv * MW[1], mag * hz / dv, mag * Z0 / dv + kv * MW[3]};
        for (int a = 0; a < 4; ++a) {
            o.MU[a] = (float)MU[a];
            o.MV[a] = (float)MV[a];
            o.MW[a] = (float)MW[a];
        }
    }
}

// 3x3 rotations (row-major) and products for the per-view frames.
struct Rot {
    double m[3][3];
};

Rot rot_axis(int axis, double a)
{
    const double c = std::cos(a), s = std::sin(a);
    Rot r{};
    const int i = (axis + 1) % 3, j = (axis + 2) % 3;   // the plane the rotation acts in
    r.m[axis][axis] = 1.0;
    r.m[i][i] = c;
    r.m[i][j] = -s;
    r.m[j][i] = s;
    r.m[j][j] = c;
    return r;
}

Rot mul(const Rot& A, const Rot& B)
{
    Rot C{};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k) C.m[i][j] += A.m[i][k] * B.m[k][j];
    return C;
}

void apply(const Rot& R, const double v[3], double out[3])
{
    for (int i = 0; i < 3; ++i) out[i] = R.m[i][0] * v[0] + R.m[i][1] * v[1] + R.m[i][2] * v[2];
}

// World frame of one view, relative to its volume centre: source S, centre
// of pixel (0, 0) P00, unit detector axes eu, ev (mm).
void view_frame(const ctmi_geometry* g, const ctmi_view& w, double S[3], double P00[3], double eu[3], double ev[3])
{
    // gantry Rz(z1) Ry(y1) Rz(z2); detector Rx(roll) Ry(pitch) Rz(yaw) about
    // its centre, in the machine frame (x towards the source, u = y, v = z)
    const Rot G = mul(rot_axis(2, w.angles[0]), mul(rot_axis(1, w.angles[1]), rot_axis(2, w.angles[2])));
    const Rot Dt = mul(rot_axis(0, w.rotDetector[0]), mul(rot_axis(1, w.rotDetector[1]), rot_axis(2, w.rotDetector[2])));
    const Rot GD = mul(G, Dt);
    const double s0[3] = {w.DSO, w.COR, 0.0}, d0[3] = {w.DSO - w.DSD, w.COR, 0.0};
    const double ux[3] = {0.0, 1.0, 0.0}, vx[3] = {0.0, 0.0, 1.0};
    double D[3];
    apply(G, s0, S);
    apply(G, d0, D);
    apply(GD, ux, eu);
    apply(GD, vx, ev);
    const double o[3] = {w.offOrigin[2], w.offOrigin[1], w.offOrigin[0]};   // x, y, z
    const double nu = (double)g->nDetector[1], nv = (double)g->nDetector[0];
    const double u0 = (0.5 - 0.5 * nu) * g->dDetector[1] + w.offDetector[1];
    const double v0 = (0.5 - 0.5 * nv) * g->dDetector[0] + w.offDetector[0];
    for (int a = 0; a < 3; ++a) {
        S[a] -= o[a];
        P00[a] = D[a] - o[a] + u0 * eu[a] + v0 * ev[a];
    }
}

// Per-view table for general frames.  Rays as in view_table (voxel-cell
// coordinates); the 3x4 rows give (fu W, fv W, W) from voxel-centre indices
// with W = 1 on the detector plane and 0 on the source's parallel plane
// (only fu, fv = ratios are used: detector footprints).
void view_table_general(const ctmi_geometry* g, const ctmi_view* views, int64_t nviews, ViewGeo* out,
                        ctmi::ViewGeo64* out64)
{
    const double h[3] = {g->dVoxel[2], g->dVoxel[1], g->dVoxel[0]};
    const double lo[3] = {-0.5 * (double)g->nVoxel[2] * h[0], -0.5 * (double)g->nVoxel[1] * h[1],
                          -0.5 * (double)g->nVoxel[0] * h[2]};
    const double du = g->dDetector[1], dv = g->dDetector[0];
    for (int64_t k = 0; k < nviews; ++k) {
        double S[3], P00[3], eu[3], ev[3];
        view_frame(g, views[k], S, P00, eu, ev);
        ViewGeo& o = out[k];
        std::memset(&o, 0, sizeof o);
        ctmi::ViewGeo64& o64 = out64[k];
        std::memset(&o64, 0, sizeof o64);
        for (int a = 0; a < 3; ++a) {
            o64.S[a] = (S[a] - lo[a]) / h[a];
            o64.P00[a] = (P00[a] - lo[a]) / h[a];
            o64.DU[a] = du * eu[a] / h[a];
            o64.DV[a] = dv * ev[a] / h[a];
            o.S[a] = (float)o64.S[a];
            o.P00[a] = (float)o64.P00[a];
            o.DU[a] = (float)o64.DU[a];
            o.DV[a] = (float)o64.DV[a];
        }
        // central projection of world point X onto the detector plane:
        // W = (X - S).n / (P00 - S).n, then (fu W, fv W) = ((S - P00) W + X - S).(eu / du, ev / dv)
        const double n[3] = {eu[1] * ev[2] - eu[2] * ev[1], eu[2] * ev[0] - eu[0] * ev[2], eu[0] * ev[1] - eu[1] * ev[0]};
        double den = 0.0, spu = 0.0, spv = 0.0;
        for (int a = 0; a < 3; ++a) {
            den += (P00[a] - S[a]) * n[a];
            spu += (S[a] - P00[a]) * eu[a];
            spv += (S[a] - P00[a]) * ev[a];
        }
        // X = lo + (c + 1/2) h; X - S = (lo + h/2 - S) + c h
        double MW[4] = {0.0, 0.0, 0.0, 0.0}, MU[4] = {0.0, 0.0, 0.0, 0.0}, MV[4] = {0.0, 0.0, 0.0, 0.0};
        for (int a = 0; a < 3; ++a) {
            MW[a] = h[a] * n[a] / den;
            MU[a] = (spu * MW[a] + h[a] * eu[a]) / du;
            MV[a] = (spv * MW[a] + h[a] * ev[a]) / dv;
            const double x0 = lo[a] + 0.5 * h[a] - S[a];
            MW[3] += x0 * n[a] / den;
        }
        for (int a = 0; a < 3; ++a) {
            const double x0 = lo[a] + 0.5 * h[a] - S[a];
            MU[3] += x0 * eu[a] / du;
            MV[3] += x0 * ev[a] / dv;
        }
        MU[3] += spu * MW[3] / du;
        MV[3] += spv * MW[3] / dv;
        for (int a = 0; a < 4; ++a) {
            o.MU[a] = (float)MU[a];
            o.MV[a] = (float)MV[a];
            o.MW[a] = (float)MW[a];
        }
    }
}

// Per-view checks: finite values, the volume's circumscribed sphere (grown by
// one voxel) in front of the source and on the source's side of the
// detector plane, by more than its radius.
int check_views(const ctmi_geometry* g, const ctmi_view* views, int64_t nviews)
{
    double half2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        const double hh = 0.5 * (double)g->nVoxel[a] * g->dVoxel[a] + g->dVoxel[a];
        half2 += hh * hh;
    }
    const double R = std::sqrt(half2);
    for (int64_t k = 0; k < nviews; ++k) {
        const ctmi_view& w = views[k];
        bool ok = std::isfinite(w.DSO) && std::isfinite(w.DSD) && std::isfinite(w.COR);
        for (int a = 0; a < 3; ++a)
            ok = ok && std::isfinite(w.angles[a]) && std::isfinite(w.offOrigin[a]) && std::isfinite(w.rotDetector[a]);
        ok = ok && std::isfinite(w.offDetector[0]) && std::isfinite(w.offDetector[1]);
        if (!ok) return fail(CTMI_EINVAL, "view %lld has a non-finite parameter", (long long)k);
        if (!(w.DSO > 0.0) || !(w.DSD > w.DSO)) return fail(CTMI_EINVAL, "view %lld: need 0 < DSO < DSD", (long long)k);
        double S[3], P00[3], eu[3], ev[3];
        view_frame(g, w, S, P00, eu, ev);
        const double n[3] = {eu[1] * ev[2] - eu[2] * ev[1], eu[2] * ev[0] - eu[0] * ev[2], eu[0] * ev[1] - eu[1] * ev[0]};
        // orient n from the detector towards the source
        double sd = 0.0;
        for (int a = 0; a < 3; ++a) sd += (S[a] - P00[a]) * n[a];
        const double sg = sd > 0.0 ? 1.0 : -1.0;
        double cs = 0.0, cd = 0.0;   // volume centre (origin) to the source's and the detector's planes
        for (int a = 0; a < 3; ++a) {
            cs += (S[a] - 0.0) * n[a] * sg;
            cd += (0.0 - P00[a]) * n[a] * sg;
        }
        if (!(cs > R)) return fail(CTMI_EINVAL, "view %lld: the source passes within the volume", (long long)k);
        if (!(cd > R)) return fail(CTMI_EINVAL, "view %lld: the detector cuts the volume", (long long)k);
    }
    return CTMI_OK;
}

int bitrev(int x, int bits)
{
    int r = 0;
    for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i);
    return r;
}

// Frequency response of the zero-padded Ram-Lak kernel on the iso grid
// tau = du DSO / DSD: H[k] = tau (h[0] + 2 sum_{n odd < nu} h[n] cos(2 pi k n / L)),
// times 1/L for the inverse transform, stored in bit-reversed order.
void ramp_tables(const ctmi_geometry* g, int L, int logL, std::vector<float>& Hbr, std::vector<float>& tw)
{
    const int64_t nu = g->nDetector[1];
    const double tau = g->dDetector[1] * g->DSO / g->DSD;
    const double pi = 3.14159265358979323846;
    std::vector<double> H(L);
    for (int k = 0; k < L; ++k) {
        double acc = 1.0 / (4.0 * tau * tau);
        for (int64_t n = 1; n < nu; n += 2)
            acc += 2.0 * (-1.0 / ((double)n * n * pi * pi * tau * tau)) * std::cos(2.0 * pi * (double)k * n / L);
        H[k] = tau * acc / (double)L;
    }
    Hbr.resize(L);
    for (int k = 0; k < L; ++k) Hbr[k] = (float)H[bitrev(k, logL)];
    tw.resize(L);  // L/2 complex values
    for (int k = 0; k < L / 2; ++k) {
        tw[2 * k] = (float)std::cos(-2.0 * pi * k / L);
        tw[2 * k + 1] = (float)std::sin(-2.0 * pi * k / L);
    }
}

int check_plan(const ctmi_plan* p)
{
    if (!p) return fail(CTMI_EINVAL, "plan is NULL");
    return CTMI_OK;
}

int check_views(const Plan* p, int64_t view0, int64_t nviews)
{
    if (view0 < 0 || nviews < 0 || view0 > p->nviews || nviews > p->nviews - view0)
        return fail(CTMI_EINVAL, "view range [%lld, %lld) outside the plan's %lld views", (long long)view0,
                    (long long)(view0 + nviews), (long long)p->nviews);
    return CTMI_OK;
}

int check_ptr(const void* ptr, const char* name)
{
    if (!ptr) return fail(CTMI_EINVAL, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(ptr) % 4 != 0) return fail(CTMI_EINVAL, "%s is not 4-byte aligned", name);
    return CTMI_OK;
}

int check_device(const Plan* p)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != p->device) return fail(CTMI_EINVAL, "plan was created on device %d but device %d is current", p->device, dev);
    return CTMI_OK;
}

int launched(hipError_t e, const char* what) { return e == hipSuccess ? CTMI_OK : hip_fail(e, what); }

}  // namespace

int ctmi::api_fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int ctmi::api_hip(hipError_t e, const char* what) { return hip_fail(e, what); }

extern "C" {

const char* ctmi_last_error(void) { return g_err; }

const char* ctmi_version(void) { return "ctmi 0.1 (gfx950)"; }

int ctmi_geometry_check(const ctmi_geometry* geo, const double* angles, int64_t nviews)
{
    return check_geometry(geo, angles, nviews);
}

int ctmi_view_table(const ctmi_geometry* geo, const double* angles, int64_t nviews, float* out)
{
    int rc = check_geometry(geo, angles, nviews);
    if (rc) return rc;
    if (!out) return fail(CTMI_EINVAL, "out is NULL");
    std::vector<ViewGeo> t(nviews);
    view_table(geo, angles, nviews, t.data());
    std::memcpy(out, t.data(), sizeof(ViewGeo) * (size_t)nviews);
    return CTMI_OK;
}

static int create_plan(const ctmi_geometry* geo, const double* angles, const ctmi_view* views, int64_t nviews,
                       ctmi_plan** out)
{
    ctmi_plan* p = new (std::nothrow) ctmi_plan();
    if (!p) return fail(CTMI_EINVAL, "out of host memory");
    p->geo = *geo;
    p->nviews = nviews;
    p->vol.nz = (int)geo->nVoxel[0];
    p->vol.ny = (int)geo->nVoxel[1];
    p->vol.nx = (int)geo->nVoxel[2];
    p->vol.hz = (float)geo->dVoxel[0];
    p->vol.hy = (float)geo->dVoxel[1];
    p->vol.hx = (float)geo->dVoxel[2];
    p->det.nv = (int)geo->nDetector[0];
    p->det.nu = (int)geo->nDetector[1];
    p->ds = (float)(geo->accuracy * std::fmin(geo->dVoxel[0], std::fmin(geo->dVoxel[1], geo->dVoxel[2])));
    // bounds that size the adjoints' fixed-point scales: one Siddon term is
    // a chord of one cell (at most its diagonal); one interpolation term is
    // a sample's tent weight (<= 1) times ds
    {
        double hdiag2 = 0.0;
        for (int a = 0; a < 3; ++a) hdiag2 += geo->dVoxel[a] * geo->dVoxel[a];
        const double hdiag = std::sqrt(hdiag2);
        p->entry_siddon = (float)(hdiag * 1.0001);
        // one ray crosses a cell once, and items end on cell boundaries, so a
        // ray adds at most one chord to one cell
        p->round_siddon = (float)(hdiag * 1.0001);
        // samples of one ray inside a 2x2x2-voxel support: the chord is at most
        // 2 sqrt(3) voxel units and samples are at least ds / h_max apart
        // (one more for FP32 rounding of the positions)
        const double hmax = std::fmax(geo->dVoxel[0], std::fmax(geo->dVoxel[1], geo->dVoxel[2]));
        const double K = std::floor(2.0 * std::sqrt(3.0) * hmax / (double)p->ds) + 2.0;
        p->round_interp = (float)(K * (double)p->ds * 1.0001);
    }
    int L = 1, logL = 0;
    while (L < 2 * p->det.nu - 1 || L < 2) {
        L <<= 1;
        ++logL;
    }
    p->fft_len = L;
    p->fft_log2 = logL;

    std::vector<ViewGeo> t(nviews);
    std::vector<ctmi::ViewGeo64> t64(nviews);
    p->circular = views == nullptr;
    if (views)
        view_table_general(geo, views, nviews, t.data(), t64.data());
    else
        view_table(geo, angles, nviews, t.data(), t64.data());
    std::vector<float> Hbr, tw;
    ramp_tables(geo, L, logL, Hbr, tw);

    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipGetDevice");
    }
    const size_t tb = sizeof(ViewGeo) * (size_t)nviews;
    const size_t t64b = sizeof(ctmi::ViewGeo64) * (size_t)nviews;
    const size_t hb = sizeof(float) * (size_t)L;
    const size_t wb = sizeof(float) * (size_t)L;  // L/2 float2
    char* mem = nullptr;
    e = hipMalloc(reinterpret_cast<void**>(&mem), tb + t64b + hb + wb);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipMalloc(plan tables)");
    }
    p->d_views = reinterpret_cast<ViewGeo*>(mem);
    p->d_views64 = reinterpret_cast<ctmi::ViewGeo64*>(mem + tb);
    p->d_filter = reinterpret_cast<float*>(mem + tb + t64b);
    p->d_twiddle = reinterpret_cast<float2*>(mem + tb + t64b + hb);
    if ((e = hipMemcpy(p->d_views, t.data(), tb, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->d_views64, t64.data(), t64b, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->d_filter, Hbr.data(), hb, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->d_twiddle, tw.data(), wb, hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(mem);
        delete p;
        return hip_fail(e, "hipMemcpy(plan tables)");
    }
    *out = p;
    return CTMI_OK;
}

int ctmi_plan_create(const ctmi_geometry* geo, const double* angles, int64_t nviews, ctmi_plan** out)
{
    if (!out) return fail(CTMI_EINVAL, "out is NULL");
    int rc = check_geometry(geo, angles, nviews);
    if (rc) return rc;
    return create_plan(geo, angles, nullptr, nviews, out);
}

int ctmi_plan_create_views(const ctmi_geometry* geo, const ctmi_view* views, int64_t nviews, ctmi_plan** out)
{
    if (!out) return fail(CTMI_EINVAL, "out is NULL");
    if (!views) return fail(CTMI_EINVAL, "views is NULL");
    if (!geo) return fail(CTMI_EINVAL, "geometry is NULL");
    if (nviews < 1) return fail(CTMI_EINVAL, "nviews must be >= 1 (got %lld)", (long long)nviews);
    int rc;
    if ((rc = check_sizes(geo, nviews))) return rc;
    if ((rc = check_views(geo, views, nviews))) return rc;
    return create_plan(geo, nullptr, views, nviews, out);
}

int ctmi_plan_destroy(ctmi_plan* plan)
{
    if (!plan) return CTMI_OK;
    int rc = CTMI_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) rc = hip_fail(e, "hipDeviceSynchronize");
    e = hipFree(plan->d_views);
    if (e != hipSuccess && rc == CTMI_OK) rc = hip_fail(e, "hipFree");
    delete plan;
    return rc;
}

int ctmi_forward(const ctmi_plan* plan, int projector, const float* vol, float* proj, int64_t view0, int64_t nviews,
                 void* stream)
{
    int rc;
    if ((rc = check_plan(plan)) || (rc = check_views(plan, view0, nviews))) return rc;
    if (projector != CTMI_SIDDON && projector != CTMI_INTERP)
        return fail(CTMI_EINVAL, "unknown projector %d", projector);
    if (nviews == 0) return CTMI_OK;
    if ((rc = check_ptr(vol, "vol")) || (rc = check_ptr(proj, "proj")) || (rc = check_device(plan))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return projector == CTMI_SIDDON
               ? launched(ctmi::launch_forward_siddon(*plan, vol, proj, view0, nviews, s), "forward (Siddon)")
               : launched(ctmi::launch_forward_interp(*plan, vol, proj, view0, nviews, s), "forward (interpolated)");
}

static size_t op_workspace(const Plan& p, int op)
{
    switch (op) {
    case CTMI_OP_BACKPROJECT_INTERP: return ctmi::interp_adjoint_ws_bytes(p);
    case CTMI_OP_FOV_SQ_ERR: return ctmi::reduce_ws_bytes();
    default: return 0;
    }
}

int ctmi_workspace_size(const ctmi_plan* plan, int op, size_t* bytes)
{
    int rc;
    if ((rc = check_plan(plan))) return rc;
    if (!bytes) return fail(CTMI_EINVAL, "bytes is NULL");
    if (op < CTMI_OP_FORWARD_SIDDON || op > CTMI_OP_FOV_SQ_ERR) return fail(CTMI_EINVAL, "unknown operation %d", op);
    *bytes = op_workspace(*plan, op);
    return CTMI_OK;
}

int ctmi_stream_check(void* stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamQuery(s);
    if (e != hipSuccess && e != hipErrorNotReady) return hip_fail(e, "stream");
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "device");
    return CTMI_OK;
}

}  // extern "C"

// Checks shared by the backprojection entry points (everything except the
// workspace).
int ctmi::check_backproject(const ctmi_plan* plan, int bp, const float* proj, float* vol, int64_t view0, int64_t nviews,
                            float beta)
{
    int rc;
    if ((rc = check_plan(plan)) || (rc = check_views(plan, view0, nviews))) return rc;
    if (bp != CTMI_BP_SIDDON && bp != CTMI_BP_INTERP && bp != CTMI_BP_FDK)
        return fail(CTMI_EINVAL, "unknown backprojector %d", bp);
    if (bp == CTMI_BP_FDK && !plan->circular)
        return fail(CTMI_EUNSUPPORTED, "the FDK backprojector needs a circular-orbit plan");
    if (!std::isfinite(beta)) return fail(CTMI_EINVAL, "beta is not finite");
    if ((rc = check_ptr(vol, "vol")) || (nviews > 0 && (rc = check_ptr(proj, "proj"))) ||
        (rc = check_device(plan)))
        return rc;
    return CTMI_OK;
}

int ctmi::run_backproject(const ctmi_plan* plan, int bp, const float* proj, float* vol, int64_t view0, int64_t nviews,
                          float beta, float* ws, void* stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    // nviews == 0 still applies vol = beta * vol (proj is not read)
    switch (bp) {
    case CTMI_BP_SIDDON:
        return launched(ctmi::launch_backward_siddon(*plan, proj, vol, view0, nviews, beta, s), "backproject (Siddon)");
    case CTMI_BP_INTERP:
        return launched(ctmi::launch_backward_interp(*plan, proj, vol, view0, nviews, beta, ws, s),
                        "backproject (interpolated)");
    default:
        return launched(ctmi::launch_backward_fdk(*plan, proj, vol, view0, nviews, beta, s), "backproject (FDK)");
    }
}

extern "C" {

int ctmi_backproject(const ctmi_plan* plan, int bp, const float* proj, float* vol, int64_t view0, int64_t nviews,
                     float beta, void* ws, size_t ws_bytes, void* stream)
{
    int rc;
    if ((rc = ctmi::check_backproject(plan, bp, proj, vol, view0, nviews, beta))) return rc;
    if (bp == CTMI_BP_INTERP) {
        const size_t need = ctmi::interp_adjoint_ws_bytes(*plan);
        if (!ws) return fail(CTMI_EWORKSPACE, "the interpolated backprojector needs a workspace of %zu bytes", need);
        if (reinterpret_cast<uintptr_t>(ws) % 16 != 0) return fail(CTMI_EINVAL, "workspace is not 16-byte aligned");
        if (ws_bytes < need)
            return fail(CTMI_EWORKSPACE, "workspace of %zu bytes is below the %zu required", ws_bytes, need);
    }
    return ctmi::run_backproject(plan, bp, proj, vol, view0, nviews, beta, static_cast<float*>(ws), stream);
}

int ctmi_fdk_filter(const ctmi_plan* plan, int wang, const float* proj, float* out, int64_t view0, int64_t nviews,
                    void* stream)
{
    int rc;
    if ((rc = check_plan(plan)) || (rc = check_views(plan, view0, nviews))) return rc;
    if (!plan->circular) return fail(CTMI_EUNSUPPORTED, "the FDK filter needs a circular-orbit plan");
    if (nviews == 0) return CTMI_OK;
    if ((rc = check_ptr(proj, "proj")) || (rc = check_ptr(out, "out")) || (rc = check_device(plan))) return rc;
    if (wang && plan->geo.offDetector[1] != 0.0 &&
        !(0.5 * (double)plan->det.nu * plan->geo.dDetector[1] > std::fabs(plan->geo.offDetector[1])))
        return fail(CTMI_EINVAL, "Wang weighting needs an overlap: |offDetector_u| must be < nu du / 2");
    return launched(ctmi::launch_fdk_filter(*plan, wang, proj, out, view0, nviews, static_cast<hipStream_t>(stream)),
                    "FDK filter");
}

size_t ctmi_reduce_workspace_bytes(int64_t n)
{
    (void)n;
    return ctmi::reduce_ws_bytes();
}

static int check_ws(const void* ws, size_t ws_bytes)
{
    if (!ws) return fail(CTMI_EWORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 8 != 0) return fail(CTMI_EINVAL, "workspace is not 8-byte aligned");
    if (ws_bytes < ctmi::reduce_ws_bytes())
        return fail(CTMI_EWORKSPACE, "workspace of %zu bytes is below the %zu required", ws_bytes,
                    ctmi::reduce_ws_bytes());
    return CTMI_OK;
}

static int check_n(int64_t n)
{
    if (n < 0) return fail(CTMI_EINVAL, "negative length");
    return CTMI_OK;
}

int ctmi_dot(const float* a, const float* b, int64_t n, double* out, void* ws, size_t ws_bytes, void* stream)
{
    int rc;
    if ((rc = check_n(n)) || (rc = check_ptr(a, "a")) || (rc = check_ptr(b, "b")) || (rc = check_ws(ws, ws_bytes)))
        return rc;
    if (!out || reinterpret_cast<uintptr_t>(out) % 8) return fail(CTMI_EINVAL, "out must be an aligned double");
    return launched(ctmi::launch_dot(a, b, n, out, static_cast<double*>(ws), static_cast<hipStream_t>(stream)), "dot");
}

int ctmi_axpby(int64_t n, float a, const float* x, float b, float* y, void* stream)
{
    int rc;
    if ((rc = check_n(n))) return rc;
    if (n == 0) return CTMI_OK;
    if ((rc = check_ptr(x, "x")) || (rc = check_ptr(y, "y"))) return rc;
    return launched(ctmi::launch_axpby(n, a, x, b, y, static_cast<hipStream_t>(stream)), "axpby");
}

int ctmi_cgls_xr(float* x, const float* p, int64_t nvol, float* r, const float* q, int64_t nproj, const double* gamma,
                 const double* delta, double* rnorm2, void* ws, size_t ws_bytes, void* stream)
{
    int rc;
    if ((rc = check_n(nvol)) || (rc = check_n(nproj)) || (rc = check_ptr(x, "x")) || (rc = check_ptr(p, "p")) ||
        (rc = check_ptr(r, "r")) || (rc = check_ptr(q, "q")) || (rc = check_ws(ws, ws_bytes)))
        return rc;
    if (!gamma || !delta || !rnorm2) return fail(CTMI_EINVAL, "gamma, delta and rnorm2 must be device doubles");
    return launched(ctmi::launch_cgls_xr(x, p, nvol, r, q, nproj, gamma, delta, rnorm2, static_cast<double*>(ws),
                                         static_cast<hipStream_t>(stream)),
                    "cgls_xr");
}

int ctmi_cgls_p(float* p, const float* s, int64_t n, const double* gamma_old, const double* gamma_new, void* stream)
{
    int rc;
    if ((rc = check_n(n)) || (rc = check_ptr(p, "p")) || (rc = check_ptr(s, "s"))) return rc;
    if (!gamma_old || !gamma_new) return fail(CTMI_EINVAL, "gamma_old and gamma_new must be device doubles");
    if (n == 0) return CTMI_OK;
    return launched(ctmi::launch_cgls_p(p, s, n, gamma_old, gamma_new, static_cast<hipStream_t>(stream)), "cgls_p");
}

int ctmi_recip_or_zero(const float* in, float* out, int64_t n, void* stream)
{
    int rc;
    if ((rc = check_n(n)) || (rc = check_ptr(in, "in")) || (rc = check_ptr(out, "out"))) return rc;
    if (n == 0) return CTMI_OK;
    return launched(ctmi::launch_recip(in, out, n, static_cast<hipStream_t>(stream)), "recip_or_zero");
}

int ctmi_sart_residual(const float* b, const float* ax, const float* w, float* out, int64_t n, void* stream)
{
    int rc;
    if ((rc = check_n(n)) || (rc = check_ptr(b, "b")) || (rc = check_ptr(ax, "ax")) || (rc = check_ptr(w, "w")) ||
        (rc = check_ptr(out, "out")))
        return rc;
    if (n == 0) return CTMI_OK;
    return launched(ctmi::launch_sart_residual(b, ax, w, out, n, static_cast<hipStream_t>(stream)), "sart_residual");
}

int ctmi_sart_update(float* x, const float* v, const float* bp, int64_t n, float lam, int nonneg, void* stream)
{
    int rc;
    if ((rc = check_n(n)) || (rc = check_ptr(x, "x")) || (rc = check_ptr(v, "v")) || (rc = check_ptr(bp, "bp")))
        return rc;
    if (!std::isfinite(lam)) return fail(CTMI_EINVAL, "lam is not finite");
    if (n == 0) return CTMI_OK;
    return launched(ctmi::launch_sart_update(x, v, bp, n, lam, nonneg, static_cast<hipStream_t>(stream)),
                    "sart_update");
}

int ctmi_awtv_grad(const float* x, float* g, int64_t nz, int64_t ny, int64_t nx, float delta, float eps, void* stream)
{
    int rc;
    if ((rc = check_ptr(x, "x")) || (rc = check_ptr(g, "g"))) return rc;
    if (nz < 1 || ny < 1 || nx < 1) return fail(CTMI_EINVAL, "volume dimensions must be >= 1");
    if (nx > (1 << 20) || ny > (1 << 20) || nz > (1 << 20) || (double)nx * ny * nz >= 2147483648.0)
        return fail(CTMI_EOVERFLOW, "volume must hold < 2^31 voxels");
    if (x == g) return fail(CTMI_EINVAL, "g must not alias x");
    if (std::isnan(delta)) return fail(CTMI_EINVAL, "delta is NaN");
    if (!(eps >= 0.0f) || !std::isfinite(eps)) return fail(CTMI_EINVAL, "eps must be finite and >= 0");
    return launched(ctmi::launch_awtv_grad(x, g, (int)nz, (int)ny, (int)nx, delta, eps, static_cast<hipStream_t>(stream)),
                    "awtv_grad");
}

int ctmi_tv_step(float* x, const float* g, int64_t n, const double* gnorm2, float step, void* stream)
{
    int rc;
    if ((rc = check_n(n)) || (rc = check_ptr(x, "x")) || (rc = check_ptr(g, "g"))) return rc;
    if (!gnorm2) return fail(CTMI_EINVAL, "gnorm2 is NULL");
    if (!std::isfinite(step)) return fail(CTMI_EINVAL, "step is not finite");
    if (n == 0) return CTMI_OK;
    return launched(ctmi::launch_tv_step(x, g, n, gnorm2, step, static_cast<hipStream_t>(stream)), "tv_step");
}

int ctmi_em_ratio(const float* b, const float* ax, float* out, int64_t n, void* stream)
{
    int rc;
    if ((rc = check_n(n)) || (rc = check_ptr(b, "b")) || (rc = check_ptr(ax, "ax")) || (rc = check_ptr(out, "out")))
        return rc;
    if (n == 0) return CTMI_OK;
    return launched(ctmi::launch_em_ratio(b, ax, out, n, static_cast<hipStream_t>(stream)), "em_ratio");
}

int ctmi_em_update(float* x, const float* v, const float* bp, int64_t n, void* stream)
{
    int rc;
    if ((rc = check_n(n)) || (rc = check_ptr(x, "x")) || (rc = check_ptr(v, "v")) || (rc = check_ptr(bp, "bp")))
        return rc;
    if (n == 0) return CTMI_OK;
    return launched(ctmi::launch_em_update(x, v, bp, n, static_cast<hipStream_t>(stream)), "em_update");
}

int ctmi_fov_sq_err(const ctmi_plan* plan, const float* x, const float* gt, double* out, void* ws, size_t ws_bytes,
                    void* stream)
{
    int rc;
    if ((rc = check_plan(plan)) || (rc = check_ptr(x, "x")) || (rc = check_ptr(gt, "gt")) ||
        (rc = check_ws(ws, ws_bytes)) || (rc = check_device(plan)))
        return rc;
    if (!out) return fail(CTMI_EINVAL, "out is NULL");
    return launched(ctmi::launch_fov_sq_err(*plan, x, gt, out, static_cast<double*>(ws), static_cast<hipStream_t>(stream)),
                    "fov_sq_err");
}

/* -------------------------------------------------- curved detectors -- */
int ctmi_flatten_curved(const ctmi_plan* plan, const ctmi_curved_detector* cd, const float* curved, float* flat,
                        int64_t view0, int64_t nviews, void* stream)
{
    int rc;
    if ((rc = check_plan(plan)) || (rc = check_views(plan, view0, nviews))) return rc;
    if (!cd) return fail(CTMI_EINVAL, "curved detector is NULL");
    if (!plan->circular) return fail(CTMI_EUNSUPPORTED, "flattening needs a circular-orbit plan");
    for (int a = 0; a < 2; ++a) {
        if (cd->nDetector[a] < 1) return fail(CTMI_EINVAL, "curved detector sizes must be >= 1");
        if (!(cd->dDetector[a] > 0.0) || !std::isfinite(cd->dDetector[a]))
            return fail(CTMI_EINVAL, "curved detector pitch must be finite and > 0");
        if (!std::isfinite(cd->offDetector[a])) return fail(CTMI_EINVAL, "curved detector offset is not finite");
    }
    if (cd->nDetector[1] > 65536 || (double)cd->nDetector[0] * (double)cd->nDetector[1] >= 268435456.0)
        return fail(CTMI_EOVERFLOW, "curved detector must hold nu <= 65536 and fewer than 2^28 pixels");
    if (!std::isfinite(cd->radius) || !(cd->radius > 0.5 * plan->geo.DSD))
        return fail(CTMI_EINVAL, "arc radius must be finite and > DSD / 2 (the source inside the cylinder)");
    if (nviews == 0) return CTMI_OK;
    if ((rc = check_ptr(curved, "curved")) || (rc = check_ptr(flat, "flat")) || (rc = check_device(plan))) return rc;
    if (static_cast<const void*>(curved) == static_cast<const void*>(flat))
        return fail(CTMI_EINVAL, "flat must not alias curved");
    ctmi::CurvedDet c;
    c.nv = (int)cd->nDetector[0];
    c.nu = (int)cd->nDetector[1];
    c.dv = cd->dDetector[0];
    c.du = cd->dDetector[1];
    c.ov = cd->offDetector[0];
    c.ou = cd->offDetector[1];
    c.R = cd->radius;
    return launched(ctmi::launch_flatten_curved(*plan, c, curved, flat, nviews, static_cast<hipStream_t>(stream)),
                    "flatten_curved");
}

/* ------------------------------------------------------- ceilings -- */
int ctmi_ceiling_copy(const float* src, float* dst, int64_t n, void* stream)
{
    int rc;
    if ((rc = check_n(n))) return rc;
    if (n % 4) return fail(CTMI_EINVAL, "n must be a multiple of 4");
    if (n == 0) return CTMI_OK;
    if (!src || !dst || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
        return fail(CTMI_EINVAL, "src and dst must be 16-byte aligned device pointers");
    return launched(ctmi::launch_stream_copy(src, dst, n, static_cast<hipStream_t>(stream)), "ceiling copy");
}

int64_t ctmi_ceiling_fma_per_lane(int iters) { return (int64_t)ctmi::fma_loop_chains() * (int64_t)iters; }

int ctmi_ceiling_fma(float* out, int blocks, int iters, void* stream)
{
    int rc;
    if ((rc = check_ptr(out, "out"))) return rc;
    if (blocks < 1 || iters < 1) return fail(CTMI_EINVAL, "blocks and iters must be >= 1");
    return launched(ctmi::launch_fma_loop(out, blocks, iters, static_cast<hipStream_t>(stream)), "ceiling fma");
}

}  // extern "C"
