// Curved detectors (section 2.4: curved detectors are taken in through a
// flattening transformation): projections measured on a cylindrically
// curved detector are resampled onto the plan's flat detector, after which
// every operator of the flat geometry applies to them.
//
// The arc's axis is parallel to v, at distance R from the flat detector's
// centre towards the source (R = DSD: every pixel of a row equidistant
// from the source); u pixel positions are arc lengths.  A flat pixel's ray
// meets the cylinder at parameter t along source -> flat pixel, the
// positive root of (DSD^2 + u^2) t^2 - 2 DSD (DSD - R) t + (DSD - R)^2 - R^2
// = 0, at arc length R atan2(t u, t DSD - DSD + R) and height t v; the flat
// value is the curved projection there, bilinear between pixel centres and
// 0 outside the curved detector.  The map is the same for every view of a
// circular orbit and for every row of a column except the height, so each
// thread owns one (view, column), forms its column's arc position once in
// FP64 (the arc coordinates of a large radius cancel heavily), and walks the
// rows; neighbouring lanes hold neighbouring columns, so the writes and most
// reads coalesce.  HBM-bound: one read and one write per pixel.
#include "ctmi_internal.h"

namespace ctmi {

namespace {

__global__ void __launch_bounds__(256) k_flatten_curved(const float* __restrict__ curved, float* __restrict__ flat,
                                                        int nviews, FlatDet f, CurvedDet c, double DSD)
{
    const int iu = blockIdx.x * blockDim.x + threadIdx.x;
    if (iu >= f.nu) return;
    const double R = c.R;
    const double uf = ((double)iu + 0.5 - 0.5 * f.nu) * f.du + f.ou;
    const double a = DSD * DSD + uf * uf;
    const double b = -2.0 * DSD * (DSD - R);
    const double cc = (DSD - R) * (DSD - R) - R * R;
    const double t = (-b + sqrt(b * b - 4.0 * a * cc)) / (2.0 * a);
    const double s = R * atan2(t * uf, t * DSD - DSD + R);
    const double cu = (s - c.ou) / c.du + 0.5 * c.nu - 0.5;
    const double fl_u = floor(cu);
    const int u0 = (int)fl_u;
    const float wu1 = (float)(cu - fl_u), wu0 = 1.0f - wu1;
    const bool ok0 = u0 >= 0 && u0 < c.nu, ok1 = u0 + 1 >= 0 && u0 + 1 < c.nu;
    // height coordinate: cv = (t v - ov) / dv + nv/2 - 1/2 = kv * iv + cv0
    const double kv = t * f.dv / c.dv;
    const double cv0 = (t * ((0.5 - 0.5 * f.nv) * f.dv + f.ov) - c.ov) / c.dv + 0.5 * c.nv - 0.5;
    for (int view = blockIdx.y; view < nviews; view += gridDim.y) {
        const float* __restrict__ q = curved + (int64_t)view * c.nv * c.nu;
        float* __restrict__ o = flat + (int64_t)view * f.nv * f.nu + iu;
        for (int iv = 0; iv < f.nv; ++iv) {
            const double cv = __builtin_fma((double)iv, kv, cv0);
            const double fl_v = floor(cv);
            const int v0 = (int)fl_v;
            const float wv1 = (float)(cv - fl_v), wv0 = 1.0f - wv1;
            float acc = 0.0f;
            if (v0 >= 0 && v0 < c.nv) {
                const float* r = q + (int64_t)v0 * c.nu;
                if (ok0) acc = __builtin_fmaf(wv0 * wu0, r[u0], acc);
                if (ok1) acc = __builtin_fmaf(wv0 * wu1, r[u0 + 1], acc);
            }
            if (v0 + 1 >= 0 && v0 + 1 < c.nv) {
                const float* r = q + (int64_t)(v0 + 1) * c.nu;
                if (ok0) acc = __builtin_fmaf(wv1 * wu0, r[u0], acc);
                if (ok1) acc = __builtin_fmaf(wv1 * wu1, r[u0 + 1], acc);
            }
            o[(int64_t)iv * f.nu] = acc;
        }
    }
}

}  // namespace

hipError_t launch_flatten_curved(const Plan& p, const CurvedDet& c, const float* curved, float* flat, int64_t nviews,
                                 hipStream_t s)
{
    FlatDet f;
    f.nu = p.det.nu;
    f.nv = p.det.nv;
    f.du = p.geo.dDetector[1];
    f.dv = p.geo.dDetector[0];
    f.ou = p.geo.offDetector[1];
    f.ov = p.geo.offDetector[0];
    const dim3 grid((unsigned)((f.nu + 255) / 256), (unsigned)std::min<int64_t>(nviews, 65535));
    hipLaunchKernelGGL(k_flatten_curved, grid, dim3(256), 0, s, curved, flat, (int)nviews, f, c, p.geo.DSD);
    return hipGetLastError();
}

}  // namespace ctmi
