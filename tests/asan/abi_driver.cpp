// Host-side checks of libctmi's C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer: every entry point is called with arguments it
// must reject (NULL pointers, misaligned pointers, bad sizes, non-finite
// values, unknown enums) and with valid ones that need no GPU, and each
// return code is checked.  Built and run by tests/test_abi_asan.py on a
// machine without a GPU: calls that reach the device return an error there.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

#include "../../include/ctmi.h"

static int failures = 0;

static void expect(bool ok, const char* what)
{
    if (!ok) {
        std::fprintf(stderr, "FAIL: %s (last error: %s)\n", what, ctmi_last_error());
        ++failures;
    }
}

static ctmi_geometry good_geometry()
{
    ctmi_geometry g;
    std::memset(&g, 0, sizeof g);
    g.DSD = 1536.0;
    g.DSO = 1000.0;
    g.nVoxel[0] = g.nVoxel[1] = g.nVoxel[2] = 64;
    g.dVoxel[0] = g.dVoxel[1] = g.dVoxel[2] = 1.0;
    g.nDetector[0] = g.nDetector[1] = 64;
    g.dDetector[0] = g.dDetector[1] = 1.6;
    g.accuracy = 0.5;
    return g;
}

int main()
{
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    std::vector<double> ang(64);
    for (int k = 0; k < 64; ++k) ang[k] = 2.0 * M_PI * k / 64;

    expect(std::strstr(ctmi_version(), "gfx950") != nullptr, "version string");
    expect(ctmi_last_error() != nullptr, "last error is never NULL");

    // geometry validation
    ctmi_geometry g = good_geometry();
    expect(ctmi_geometry_check(&g, ang.data(), 64) == CTMI_OK, "good geometry");
    expect(ctmi_geometry_check(nullptr, ang.data(), 64) == CTMI_EINVAL, "NULL geometry");
    expect(ctmi_geometry_check(&g, nullptr, 64) == CTMI_EINVAL, "NULL angles");
    expect(ctmi_geometry_check(&g, ang.data(), 0) == CTMI_EINVAL, "no views");
    expect(ctmi_geometry_check(&g, ang.data(), -5) == CTMI_EINVAL, "negative views");
    {
        std::vector<double> bad(ang);
        bad[7] = nan;
        expect(ctmi_geometry_check(&g, bad.data(), 64) == CTMI_EINVAL, "NaN angle");
        bad[7] = inf;
        expect(ctmi_geometry_check(&g, bad.data(), 64) == CTMI_EINVAL, "infinite angle");
    }
    struct Mut {
        const char* what;
        void (*apply)(ctmi_geometry&);
        int want;
    } muts[] = {
        {"DSO inside the volume", [](ctmi_geometry& x) { x.DSO = 10.0; }, CTMI_EINVAL},
        {"DSD < DSO", [](ctmi_geometry& x) { x.DSD = 900.0; }, CTMI_EINVAL},
        {"NaN DSD", [](ctmi_geometry& x) { x.DSD = std::nan(""); }, CTMI_EINVAL},
        {"zero voxels", [](ctmi_geometry& x) { x.nVoxel[1] = 0; }, CTMI_EINVAL},
        {"negative voxel size", [](ctmi_geometry& x) { x.dVoxel[2] = -1.0; }, CTMI_EINVAL},
        {"zero detector pitch", [](ctmi_geometry& x) { x.dDetector[0] = 0.0; }, CTMI_EINVAL},
        {"infinite offset", [](ctmi_geometry& x) { x.offOrigin[1] = std::numeric_limits<double>::infinity(); },
         CTMI_EINVAL},
        {"zero accuracy", [](ctmi_geometry& x) { x.accuracy = 0.0; }, CTMI_EINVAL},
        {"COR", [](ctmi_geometry& x) { x.COR = 1.0; }, CTMI_EUNSUPPORTED},
        {"detector rotation", [](ctmi_geometry& x) { x.rotDetector[2] = 0.1; }, CTMI_EUNSUPPORTED},
        {"2^31 voxels", [](ctmi_geometry& x) { x.nVoxel[0] = x.nVoxel[1] = x.nVoxel[2] = 1300; x.dVoxel[0] = x.dVoxel[1] = x.dVoxel[2] = 0.1; },
         CTMI_EOVERFLOW},
        {"too wide detector", [](ctmi_geometry& x) { x.nDetector[1] = 5000; x.dDetector[1] = 0.1; }, CTMI_EOVERFLOW},
        {"huge sizes", [](ctmi_geometry& x) { x.nVoxel[0] = (int64_t)1 << 62; }, CTMI_EOVERFLOW},
    };
    for (const Mut& m : muts) {
        ctmi_geometry b = good_geometry();
        m.apply(b);
        const int rc = ctmi_geometry_check(&b, ang.data(), 64);
        if (rc != m.want) std::fprintf(stderr, "  %s: got %d want %d\n", m.what, rc, m.want);
        expect(rc == m.want, m.what);
        expect(std::strlen(ctmi_last_error()) > 0, "message set");
    }

    // view table (host only)
    std::vector<float> tab(32 * 64);
    expect(ctmi_view_table(&g, ang.data(), 64, tab.data()) == CTMI_OK, "view table");
    expect(ctmi_view_table(&g, ang.data(), 64, nullptr) == CTMI_EINVAL, "view table NULL out");
    for (float v : tab) expect(std::isfinite(v), "view table finite");

    // plan-free entry points reject NULL plans and bad arguments before any device work
    float buf[64] = {0};
    double dbuf[16] = {0};
    expect(ctmi_forward(nullptr, CTMI_SIDDON, buf, buf, 0, 1, nullptr) == CTMI_EINVAL, "forward NULL plan");
    expect(ctmi_backproject(nullptr, CTMI_BP_INTERP, buf, buf, 0, 1, 0.0f, nullptr, 0, nullptr) == CTMI_EINVAL,
           "backproject NULL plan");
    expect(ctmi_fdk_filter(nullptr, 0, buf, buf, 0, 1, nullptr) == CTMI_EINVAL, "filter NULL plan");
    size_t nb = 0;
    expect(ctmi_workspace_size(nullptr, CTMI_OP_BACKPROJECT_INTERP, &nb) == CTMI_EINVAL, "workspace NULL plan");
    expect(ctmi_flatten_curved(nullptr, nullptr, buf, buf, 0, 1, nullptr) == CTMI_EINVAL, "flatten NULL plan");
    expect(ctmi_plan_destroy(nullptr) == CTMI_OK, "destroy NULL");
    ctmi_plan* plan = nullptr;
    expect(ctmi_plan_create(&g, ang.data(), 64, nullptr) == CTMI_EINVAL, "plan NULL out");
    {
        ctmi_geometry b = good_geometry();
        b.DSO = 10.0;
        expect(ctmi_plan_create(&b, ang.data(), 64, &plan) == CTMI_EINVAL && plan == nullptr, "plan bad geometry");
    }
    expect(ctmi_plan_create_views(&g, nullptr, 4, &plan) == CTMI_EINVAL, "plan views NULL");

    // vector entry points
    const size_t ws = ctmi_reduce_workspace_bytes(1000);
    expect(ws >= 8, "reduce workspace size");
    expect(ctmi_dot(buf, buf, -1, dbuf, dbuf, ws, nullptr) == CTMI_EINVAL, "dot negative n");
    expect(ctmi_dot(nullptr, buf, 4, dbuf, dbuf, ws, nullptr) == CTMI_EINVAL, "dot NULL a");
    expect(ctmi_dot(buf, buf, 4, dbuf, nullptr, ws, nullptr) == CTMI_EWORKSPACE, "dot NULL workspace");
    expect(ctmi_dot(buf, buf, 4, dbuf, dbuf, 8, nullptr) == CTMI_EWORKSPACE, "dot small workspace");
    expect(ctmi_dot(reinterpret_cast<float*>(reinterpret_cast<char*>(buf) + 2), buf, 4, dbuf, dbuf, ws, nullptr) ==
               CTMI_EINVAL,
           "dot misaligned");
    expect(ctmi_axpby(-1, 1.0f, buf, 1.0f, buf, nullptr) == CTMI_EINVAL, "axpby negative n");
    expect(ctmi_axpby(0, 1.0f, nullptr, 1.0f, nullptr, nullptr) == CTMI_OK, "axpby empty");
    expect(ctmi_sart_update(buf, buf, buf, 4, std::nanf(""), 1, nullptr) == CTMI_EINVAL, "sart NaN lambda");
    expect(ctmi_tv_step(buf, buf, 4, nullptr, 0.1f, nullptr) == CTMI_EINVAL, "tv step NULL norm");
    expect(ctmi_awtv_grad(buf, buf, 2, 2, 2, 1.0f, 1e-8f, nullptr) == CTMI_EINVAL, "awtv aliasing");
    expect(ctmi_awtv_grad(buf, buf + 16, 0, 2, 2, 1.0f, 1e-8f, nullptr) == CTMI_EINVAL, "awtv zero dim");
    expect(ctmi_awtv_grad(buf, buf + 16, 2, 2, 2, std::nanf(""), 1e-8f, nullptr) == CTMI_EINVAL, "awtv NaN delta");
    expect(ctmi_em_ratio(buf, nullptr, buf, 4, nullptr) == CTMI_EINVAL, "em ratio NULL");
    expect(ctmi_ceiling_copy(buf, buf + 32, 6, nullptr) == CTMI_EINVAL, "ceiling copy n % 4");
    expect(ctmi_ceiling_fma(buf, 0, 10, nullptr) == CTMI_EINVAL, "ceiling fma blocks");
    expect(ctmi_ceiling_fma_per_lane(10) > 0, "fma per lane");

    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("abi driver: all checks passed\n");
    return 0;
}
