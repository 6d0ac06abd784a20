/*
 * ctmi -- cone-beam CT projectors and reconstruction updates for MI355X (gfx950).
 *
 * C ABI of libctmi.so.  The operations are those of the iterative cone-beam
 * reconstruction hot path described in TIGRE v3 (arXiv 2412.10129): the
 * forward projector A and its adjoint of the linear model A x + e = b
 * (section 2.1, Eq. 1), the FDK direct method with its filter and weights
 * (section 2.1, direct methods), the CGLS Krylov updates (section 2.1 list of
 * Krylov methods; section 2.2.1) and the ordered-subset SART step (section
 * 2.2.2, Eq. 6), in the circular cone-beam geometry of section 2.4 and the
 * geometry table of the appendix on geometric parameters.
 *
 * Conventions, shared by every call:
 *   - world frame Oxyz in mm; the object is static; the source rotates about
 *     +z: S = DSO (cos t, sin t, 0); detector centre S - DSD (cos t, sin t, 0);
 *     detector axes u = (-sin t, cos t, 0), v = (0, 0, 1); pixel (iv, iu)
 *     centre at u = (iu + 1/2 - nu/2) du + offDetector[1],
 *                  v = (iv + 1/2 - nv/2) dv + offDetector[0];
 *   - voxel (iz, iy, ix) is the cell [lo + i d, lo + (i+1) d) per axis with
 *     lo = offOrigin - n d / 2;
 *   - volumes are float32 C-order [nz][ny][nx] (x fastest); projections are
 *     float32 C-order [nviews][nv][nu] (u fastest);
 *   - every per-axis array of the volume is ordered (z, y, x), every
 *     per-axis array of the detector (v, u).
 *
 * Memory and streams: all array arguments are DEVICE pointers, 4-byte
 * aligned, owned by the caller, and so are the workspaces that some calls
 * take (ctmi_workspace_size gives their size).  The library never allocates
 * or frees per call and keeps no pointer after a call returns.  Every call
 * is asynchronous on `stream` (a hipStream_t; NULL = the null stream) and
 * returns after enqueueing its kernels.  A plan owns one small device
 * allocation made on the device that is current when the plan is created:
 * the per-view geometry tables (256 bytes per view) and the ramp filter's
 * tables.  Plans are immutable after creation, so calls on one plan may run
 * concurrently on different streams, each with its own workspace; calls
 * must run with the plan's device current.
 *
 * Errors: every call returns CTMI_OK (0) or a negative code; argument checks
 * happen before anything is enqueued, so a failing call has no effect.
 * ctmi_last_error() returns a thread-local message for the last failure.
 * Faults inside kernels surface asynchronously through the HIP runtime, on a
 * later call or through ctmi_stream_check.
 */
#ifndef CTMI_H
#define CTMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CTMI_OK = 0,
    CTMI_EINVAL = -1,       /* bad geometry, pointer, range or size */
    CTMI_EUNSUPPORTED = -2, /* a geometry feature the library does not model */
    CTMI_EOVERFLOW = -3,    /* sizes beyond the library's index range */
    CTMI_EWORKSPACE = -4,   /* workspace missing or too small */
    CTMI_EHIP = -5          /* the HIP runtime reported an error */
};

/* Projector models of A (the paper's linear model, section 2.1). */
enum ctmi_projector {
    CTMI_SIDDON = 0, /* exact radiological path: length of ray i in voxel j (Siddon 1985) */
    CTMI_INTERP = 1  /* trilinear ray marching, samples t_k = k ds from the source */
};

/* Backprojectors. */
enum ctmi_backprojector {
    CTMI_BP_SIDDON = 0, /* exact transpose of CTMI_SIDDON */
    CTMI_BP_INTERP = 1, /* exact transpose of CTMI_INTERP */
    CTMI_BP_FDK = 2     /* FDK backprojector: sum_views (DSO/U)^2 bilinear(q; u, v) */
};

/* Geometry parameters (the paper's geometry-parameter table).  The table's
 * total sizes sVoxel / sDetector are n * d and are not passed.  COR and
 * rotDetector must be 0 and accuracy > 0 (default 0.5 voxel). */
typedef struct {
    double DSD;            /* source -> detector distance, mm */
    double DSO;            /* source -> origin distance, mm */
    int64_t nVoxel[3];     /* (nz, ny, nx) */
    double dVoxel[3];      /* (dz, dy, dx) mm */
    double offOrigin[3];   /* (z, y, x) mm: volume centre */
    int64_t nDetector[2];  /* (nv, nu) */
    double dDetector[2];   /* (dv, du) mm */
    double offDetector[2]; /* (v, u) mm */
    double COR;            /* centre-of-rotation shift, must be 0 */
    double rotDetector[3]; /* detector in-place rotation, must be 0 */
    double accuracy;       /* interpolated-projector step in voxels (min voxel size) */
} ctmi_geometry;

typedef struct ctmi_plan ctmi_plan;

/* Operations, for ctmi_workspace_size. */
enum ctmi_op {
    CTMI_OP_FORWARD_SIDDON = 0,
    CTMI_OP_FORWARD_INTERP = 1,
    CTMI_OP_BACKPROJECT_SIDDON = 2,
    CTMI_OP_BACKPROJECT_INTERP = 3,
    CTMI_OP_BACKPROJECT_FDK = 4,
    CTMI_OP_FDK_FILTER = 5,
    CTMI_OP_FOV_SQ_ERR = 6
};

/* Thread-local description of the last error (never NULL). */
const char* ctmi_last_error(void);

/* Library version string. */
const char* ctmi_version(void);

/* Validate a geometry without touching the GPU.  Checks: positive sizes and
 * spacings, DSD > DSO, the volume's circumscribed sphere (grown by one voxel)
 * strictly between the source and the detector plane, finite angles,
 * nvox < 2^31, nu <= 4096 and nu * nv < 2^28 detector pixels.  Returns
 * CTMI_OK, CTMI_EINVAL, CTMI_EUNSUPPORTED or
 * CTMI_EOVERFLOW.  `angles` is a HOST array of nviews z1 angles (rad). */
int ctmi_geometry_check(const ctmi_geometry* geo, const double* angles, int64_t nviews);

/* Per-view geometry as used on the device (host copy, for inspection):
 * writes 32 floats per view into `out` (host memory, 32 * nviews floats).
 * Layout: [0:3] source, [3:6] centre of pixel (0,0), [6:9] step per iu,
 * [9:12] step per iv, all in voxel-cell coordinates (volume corner at 0,
 * one unit per voxel); [12:16], [16:20], [20:24] the rows of the 3x4 matrix
 * taking voxel-centre indices (ix, iy, iz, 1) to (fu W, fv W, W), W = U/DSO,
 * (fu, fv) pixel-index coordinates.  No GPU needed. */
int ctmi_view_table(const ctmi_geometry* geo, const double* angles, int64_t nviews, float* out);

/* Create a plan for `nviews` views (angles: HOST array, z1 angles in rad).
 * Validates as ctmi_geometry_check, computes the per-view table in FP64 and
 * uploads it in FP32 to the current device (synchronous).  *out is set on
 * success only. */
int ctmi_plan_create(const ctmi_geometry* geo, const double* angles, int64_t nviews, ctmi_plan** out);

/* Geometry of one projection for plans with per-view geometry (the paper's
 * section on geometric flexibility and its geometry-parameter table: Euler
 * ZYZ gantry angles, centre-of-rotation shift, in-place detector rotation,
 * and every parameter except the image and detector sizes per projection).
 * Machine frame before the gantry rotation: source (DSO, COR, 0), detector
 * centre (DSO - DSD, COR, 0), detector axes u = (0, 1, 0), v = (0, 0, 1)
 * (x points at the source).  The detector turns about its centre by
 * Rx(roll) Ry(pitch) Rz(yaw); offDetector moves the pixel grid along the
 * turned axes; the gantry turns everything about the origin by
 * Rz(z1) Ry(y1) Rz(z2); offOrigin places the volume centre.  Angles in rad,
 * lengths in mm; (z1, 0, 0) with zero COR and rotation is the circular orbit
 * of ctmi_plan_create. */
typedef struct {
    double angles[3];      /* z1, y1, z2 */
    double DSD, DSO;
    double offOrigin[3];   /* z, y, x */
    double offDetector[2]; /* v, u */
    double COR;
    double rotDetector[3]; /* roll (about the detector normal), pitch (about u), yaw (about v) */
} ctmi_view;

/* Create a plan from per-view geometry: `views` is a HOST array of nviews
 * records; from `geo` only the sizes are used (nVoxel, dVoxel, nDetector,
 * dDetector, accuracy).  Checks the sizes as ctmi_geometry_check, and per
 * view finite values, 0 < DSO < DSD, and the volume's circumscribed sphere
 * (grown by one voxel) in front of the source and on the source's side of
 * the detector plane.  The projectors and their adjoints accept such plans;
 * the FDK filter and backprojector (defined for the circular orbit) return
 * CTMI_EUNSUPPORTED on them. */
int ctmi_plan_create_views(const ctmi_geometry* geo, const ctmi_view* views, int64_t nviews, ctmi_plan** out);

/* Destroy a plan; waits for the device, then frees the plan's table.  No
 * call using the plan may be in flight.  NULL is accepted. */
int ctmi_plan_destroy(ctmi_plan* plan);

/* Device workspace (bytes) that operation `op` (enum ctmi_op) needs on this
 * plan, for any view range; 0 when it needs none.  The interpolated
 * backprojector needs 553 floats per 16x16x8 voxel brick (about 27 % of
 * the volume's size: the bricks' upper shells, handed to their neighbours);
 * the FOV error needs ctmi_reduce_workspace_bytes.  Errors: CTMI_EINVAL for
 * a NULL plan or bytes, or an unknown op.  No GPU work. */
int ctmi_workspace_size(const ctmi_plan* plan, int op, size_t* bytes);

/* Reports errors that the device raised asynchronously: CTMI_EHIP (with the
 * runtime's message) when the stream (a hipStream_t; NULL = the null
 * stream) is in an error state or the runtime holds an error from an
 * earlier launch (which this call clears), else CTMI_OK.  Does not wait for
 * the stream. */
int ctmi_stream_check(void* stream);

/* proj = A vol for views [view0, view0 + nviews) of the plan.
 * vol: [nz][ny][nx]; proj: [nviews][nv][nu] holding only those views.
 * projector: CTMI_SIDDON or CTMI_INTERP.  Overwrites proj.
 * (Section 2.1, Eq. 1: the line integrals of the discretised image.) */
int ctmi_forward(const ctmi_plan* plan, int projector, const float* vol, float* proj, int64_t view0,
                 int64_t nviews, void* stream);

/* vol = beta * vol + B proj for views [view0, view0 + nviews).
 * bp = CTMI_BP_SIDDON / CTMI_BP_INTERP: B is the exact transpose A^T of the
 * matching projector (the adjoint the Krylov methods of section 2.2.1
 * require), computed brick-by-brick with one writer per voxel.  A voxel
 * that a ray with a NaN or infinite value reaches (a Siddon piece of
 * positive length, or a corner of an interpolation sample) is set to NaN;
 * the other voxels get the sum over the finite values.
 * bp = CTMI_BP_FDK: B is the FDK backprojector (DSO/U)^2-weighted bilinear
 * detector sampling (section 2.1, FDK).  beta = 0 ignores the old contents
 * of vol (NaNs included).
 * ws: device workspace of ws_bytes >= ctmi_workspace_size(plan,
 * CTMI_OP_BACKPROJECT_INTERP) bytes, 16-byte aligned, for bp =
 * CTMI_BP_INTERP (contents need not be initialised; the call overwrites
 * them, so concurrent calls need distinct workspaces); ignored (may be NULL)
 * otherwise.  Errors: CTMI_EINVAL (plan, range, pointers, beta not finite,
 * FDK on a non-circular plan gives CTMI_EUNSUPPORTED), CTMI_EWORKSPACE
 * (workspace missing or too small). */
int ctmi_backproject(const ctmi_plan* plan, int bp, const float* proj, float* vol, int64_t view0,
                     int64_t nviews, float beta, void* ws, size_t ws_bytes, void* stream);

/* FDK filtering of views [view0, view0 + nviews): out = scale * tau *
 * (h * (w_cos * w_wang * proj)) row by row, h the Ram-Lak kernel on the iso
 * grid tau = du DSO / DSD (h[0] = 1/(4 tau^2), h[odd n] = -1/(n^2 pi^2 tau^2)),
 * applied as a linear convolution (zero-padded FFT), w_cos = DSD /
 * sqrt(DSD^2 + u^2 + v^2), w_wang the Wang offset-detector weight when
 * `wang` is nonzero, scale = pi / N (wang = 0) or 2 pi / N (wang != 0), N the
 * plan's view count.  proj and out may alias.  (Section 2.1, direct
 * methods: FDK with filters and Wang weights.) */
int ctmi_fdk_filter(const ctmi_plan* plan, int wang, const float* proj, float* out, int64_t view0,
                    int64_t nviews, void* stream);

/* ------------------------------------------------------------ vectors -- */
/* Workspace (device, bytes) needed by the reductions for n elements. */
size_t ctmi_reduce_workspace_bytes(int64_t n);

/* *out = sum_i a[i] * b[i], accumulated in FP64, deterministic (fixed
 * blocking and order).  out: one device double.  ws: device workspace of at
 * least ctmi_reduce_workspace_bytes(n) bytes.  a and b may alias. */
int ctmi_dot(const float* a, const float* b, int64_t n, double* out, void* ws, size_t ws_bytes, void* stream);

/* y = a * x + b * y (float scalars). */
int ctmi_axpby(int64_t n, float a, const float* x, float b, float* y, void* stream);

/* CGLS step (Hestenes-Stiefel, section 2.2.1): alpha = gamma / delta read
 * from device doubles (alpha = 0 when delta == 0); x += alpha p (nvol
 * elements); r -= alpha q (nproj elements); then *rnorm2 = |r|^2 in FP64.
 * ws: ctmi_reduce_workspace_bytes(nproj) bytes. */
int ctmi_cgls_xr(float* x, const float* p, int64_t nvol, float* r, const float* q, int64_t nproj,
                 const double* gamma, const double* delta, double* rnorm2, void* ws, size_t ws_bytes,
                 void* stream);

/* CGLS direction: beta = gamma_new / gamma_old (device doubles; 0 when
 * gamma_old == 0); p = s + beta p. */
int ctmi_cgls_p(float* p, const float* s, int64_t n, const double* gamma_old, const double* gamma_new,
                void* stream);

/* SART weights: out[i] = 1 / in[i], or 0 where in[i] == 0 (the row / column
 * sums W = 1/(A 1), V = 1/(A^T 1)).  in and out may alias. */
int ctmi_recip_or_zero(const float* in, float* out, int64_t n, void* stream);

/* SART residual: out = w * (b - ax).  out may alias ax. */
int ctmi_sart_residual(const float* b, const float* ax, const float* w, float* out, int64_t n, void* stream);

/* SART update (section 2.2.2, Eq. 6 with the descent sign): x = x + lam * v *
 * bp, then x = max(x, 0) when nonneg != 0. */
int ctmi_sart_update(float* x, const float* v, const float* bp, int64_t n, float lam, int nonneg,
                     void* stream);

/* Gradient of the adaptive-weighted total variation (section 2.2.3, the
 * AwTV norm, written there in 2-D; here with the z axis added the same way)
 * of a volume x[nz][ny][nx] (x fastest), into g (same layout; must not alias
 * x).  With backward differences d_a(u) = x_u - x_{u - e_a} at every voxel u
 * whose three backward neighbours exist, weights w_a = exp(-(d_a/delta)^2)
 * (plain isotropic TV when delta <= 0 or infinite) and
 * s_u = sqrt(sum_a w_a d_a^2 + eps):
 *     g_v = sum_a w_a(v) d_a(v) / s_v - sum_a w_a(v+e_a) d_a(v+e_a) / s_{v+e_a}
 * (terms with s = 0 contribute 0; the weights are held at their current
 * values, not differentiated).  Used by the TV steps of ASD-POCS.  Errors:
 * CTMI_EINVAL (NULL/misaligned pointers, aliasing, dims < 1, NaN delta,
 * eps < 0), CTMI_EOVERFLOW (2^31 voxels or more). */
int ctmi_awtv_grad(const float* x, float* g, int64_t nz, int64_t ny, int64_t nx, float delta, float eps,
                   void* stream);

/* TV steepest-descent step of ASD-POCS: x -= step * g / sqrt(*gnorm2), with
 * gnorm2 a device double (e.g. ctmi_dot(g, g)); no change when *gnorm2 is
 * 0.  x, g: n device floats. */
int ctmi_tv_step(float* x, const float* g, int64_t n, const double* gnorm2, float step, void* stream);

/* MLEM / OSEM ratio (section 2.2, the update for the Kullback-Leibler data
 * term, and its ordered-subsets form, section 2.2.2): out = b / ax where
 * ax > 0, else 0.  b, ax, out: n device floats (projections of one block);
 * out may alias ax.  Errors: CTMI_EINVAL for NULL or misaligned pointers or
 * n < 0. */
int ctmi_em_ratio(const float* b, const float* ax, float* out, int64_t n, void* stream);

/* MLEM / OSEM multiplicative update: x = x * v * bp, with v = 1 / (A_s^T 1)
 * (ctmi_recip_or_zero of the block's sensitivity; 0 where no ray reaches)
 * and bp = A_s^T (ratio).  x, v, bp: n device floats (volumes); x is
 * updated in place.  Errors as ctmi_em_ratio. */
int ctmi_em_update(float* x, const float* v, const float* bp, int64_t n, void* stream);

/* Squared error inside the field of view (section 2.2.3 ground-truth error
 * history): out[0] = sum (x - gt)^2 and out[1] = voxel count, over voxels
 * whose centre lies inside the volume's inscribed cylinder, FP64.
 * ws: ctmi_reduce_workspace_bytes(nvox) bytes. */
int ctmi_fov_sq_err(const ctmi_plan* plan, const float* x, const float* gt, double* out, void* ws,
                    size_t ws_bytes, void* stream);

/* ------------------------------------------- allocation-free calls -- */
/* ctmi_backproject without the workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The interpolated adjoint's brick
 * shells go to a scratch array inside the library instead: 160 MiB on every
 * GPU that loads the library, held until the process ends, enough for
 * volumes of up to 75 846 bricks of 16x16x8 voxels (a 512^3 volume has
 * 65 536); larger volumes return CTMI_EWORKSPACE.  All calls on one GPU
 * share that GPU's scratch, so calls that overlap on one GPU (on different
 * streams) race and must not be issued; each call writes all the scratch it
 * reads, so nothing needs clearing.  The Siddon and FDK backprojectors need
 * no scratch.  Otherwise exactly as ctmi_backproject (same kernels). */
int ctmi_backproject_noalloc(const ctmi_plan* plan, int bp, const float* proj, float* vol, int64_t view0,
                             int64_t nviews, float beta, void* stream);

/* ------------------------------------------------ curved detectors -- */
/* A cylindrically curved detector (section 2.4 on geometric flexibility:
 * curved detectors, taken in through a flattening transformation).  The
 * pixel rows follow an arc whose axis is parallel to v and passes at
 * distance `radius` from the flat detector's centre towards the source
 * (radius = DSD: every pixel of a row at the same distance from the
 * source).  u positions and du are arc lengths. */
typedef struct {
    int64_t nDetector[2];  /* (nv, nu) */
    double dDetector[2];   /* (dv, du) mm, du along the arc */
    double offDetector[2]; /* (v, u) mm, u along the arc */
    double radius;         /* mm, finite and > DSD / 2 */
} ctmi_curved_detector;

/* Flattening transformation: flat = the curved projections `curved`
 * ([nviews][cd.nv][cd.nu], views [view0, view0 + nviews) of the plan)
 * resampled onto the plan's flat detector ([nviews][nv][nu]).  Flat pixel
 * (u, v) takes the curved projection where its ray meets the cylinder: at
 * parameter t along source -> flat pixel, the positive root of
 * (DSD^2 + u^2) t^2 - 2 DSD (DSD - R) t + (DSD - R)^2 - R^2 = 0, i.e. arc
 * length R atan2(t u, t DSD - DSD + R) and height t v; bilinear between
 * curved pixel centres, 0 outside the curved detector.  The line integral
 * along a ray does not depend on where the ray meets a detector, so the
 * flattened projections feed every flat-geometry operator (FDK, the
 * iterative solvers).  Circular-orbit plans only (CTMI_EUNSUPPORTED
 * otherwise); flat must not alias curved.  Errors: CTMI_EINVAL (sizes,
 * pitches, offsets, radius <= DSD / 2, pointers), CTMI_EOVERFLOW (nu > 65536
 * or 2^28 pixels or more). */
int ctmi_flatten_curved(const ctmi_plan* plan, const ctmi_curved_detector* cd, const float* curved, float* flat,
                        int64_t view0, int64_t nviews, void* stream);

/* --------------------------------------------------------- ceilings -- */
/* Measurement kernels that compute nothing of the reconstruction: the two
 * machine ceilings that the projector, filter and vector kernels are rated
 * against.  ctmi_ceiling_copy copies n floats (n a multiple of 4; src and dst
 * 16-byte aligned device arrays, not overlapping) with 16-byte accesses: 8 n
 * bytes of HBM traffic.  ctmi_ceiling_fma runs blocks x 256 lanes, each
 * executing ctmi_ceiling_fma_per_lane(iters) independent non-packed FP32
 * fused multiply-adds, and writes one float per lane to out (blocks x 256
 * device floats).  Errors: CTMI_EINVAL for bad sizes or pointers. */
int ctmi_ceiling_copy(const float* src, float* dst, int64_t n, void* stream);
int64_t ctmi_ceiling_fma_per_lane(int iters);
int ctmi_ceiling_fma(float* out, int blocks, int iters, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CTMI_H */
