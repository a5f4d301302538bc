/*
 * hsd.h -- C ABI of the MI355X H^-s surface-distance library (libhsd.so).
 *
 * The library compares a closed triangulated surface with the unit sphere
 * S^2, or with a second triangulated surface, through the inhomogeneous
 * Sobolev norm of negative order of the difference of their surface measures
 * (Sections 2.1-2.2 of the paper; eq. sobolev_2 via the Plancherel theorem).
 *
 * Convention.  Transforms are taken with exp(-i xi.x) (no 2*pi in the
 * exponent), so the sphere's transform is 4*pi*sin|xi|/|xi| (eq.
 * ft_nsphere_sinc rescaled) and the squared distance carries the Plancherel
 * factor (2*pi)^-3:
 *
 *     d^2 = (2*pi)^-3 * sum_k w_k (1+|xi_k|^2)^-s |mu_h^(xi_k) - nu^(xi_k)|^2
 *
 * over the nodes xi_k / weights w_k of a frequency quadrature (Section 3.2).
 * mu_h^ is the sum over triangles of the exact triangle transform (eq.
 * simplex32_ft, Section 2.2) or, with HSD_METHOD_NUFFT3, of the transform of
 * its quadrature point cloud (eqs. change_variable_approx, def_nufft_type1).
 *
 * Conventions common to every entry point:
 *  - Every function returns an hsd_status: 0 (HSD_OK) on success, 1
 *    (HSD_PENDING) for a request still running, a negative code on error.
 *    On error a message is available from hsd_last_error() (thread-local).
 *    No C++ exception crosses this boundary.
 *  - Input arrays are copied; the caller may free them when the call
 *    returns.  Handles are owned by the library and freed with the matching
 *    *_destroy call.  Output arrays are owned by the caller.
 *  - mem_kind arguments say where a pointer lives: HSD_MEM_HOST (pageable or
 *    pinned host memory) or HSD_MEM_DEVICE (device memory of the context's
 *    device, e.g. a torch tensor's data_ptr()).  Device outputs are written
 *    on the context's stream; host outputs are complete when the call
 *    returns.
 *  - Layouts: vertices are row-major [nv][3] float64; triangles are
 *    row-major [nt][3] int32 vertex indices (0-based); frequency nodes are
 *    [n][3] float64; complex outputs are interleaved (re, im) float64.
 *  - A context is used by one host thread at a time (the serving loop
 *    uses its own internal streams and threads).
 */
#ifndef HSD_H
#define HSD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hsd_status;

#define HSD_OK           0
#define HSD_PENDING      1
#define HSD_EINVAL      (-1)  /* bad argument: index out of range, NaN/Inf, bad s or rule */
#define HSD_ENOMEM      (-2)  /* device memory budget or allocation failure          */
#define HSD_EDEVICE     (-3)  /* HIP runtime error                                    */
#define HSD_EAGAIN      (-4)  /* request queue full                                   */
#define HSD_ECANCELED   (-5)  /* request cancelled                                    */
#define HSD_ENOTFOUND   (-6)  /* unknown ticket                                       */

#define HSD_MEM_HOST     0
#define HSD_MEM_DEVICE   1

#define HSD_FORM_FP64    0   /* all arithmetic in FP64                                */
#define HSD_FORM_MIXED   1   /* FP64 phases/reduction/series branch, FP32 sin/cos and
                                per-pair arithmetic, FP64 accumulation of partials   */

#define HSD_METHOD_DIRECT 0  /* exact triangle transform summed over all pairs        */
#define HSD_METHOD_NUFFT3 1  /* triangle quadrature points + type-3 NUFFT             */

#define HSD_RULE_SPHERICAL_PRODUCT 0  /* ball rule centred at 0 (end of Section 3.2) */
#define HSD_RULE_EXPLICIT          1  /* caller-given nodes and weights               */
#define HSD_RULE_CUBE_TRAPEZOID    2  /* eqs. def_trap_grid, trap_rule_R3             */

#define HSD_TRI_DUNAVANT7 0  /* 7-point degree-5 symmetric triangle rule              */
#define HSD_TRI_GL8X8     1  /* 8x8 Gauss-Legendre as an iterated integral (Sec. 3.1) */

typedef struct hsd_ctx hsd_ctx;
typedef struct hsd_mesh hsd_mesh;
typedef struct hsd_rule hsd_rule;
typedef struct hsd_server hsd_server;

/* Frequency quadrature description (Section 3.2).
 *  SPHERICAL_PRODUCT: |xi| <= r_max; radial Gauss-Legendre on n_panels equal
 *    panels with n_per_panel nodes each; Gauss-Legendre in cos(theta) with
 *    n_cos nodes; trapezoid in phi with n_phi nodes, phi_j = 2*pi*j/n_phi.
 *    Node weight w = w_r r^2 w_mu 2*pi/n_phi.  Node order: direction-major
 *    (cos(theta) index, then phi index), radial index fastest.
 *  EXPLICIT: n_nodes nodes [n_nodes][3] and weights [n_nodes] (host arrays,
 *    copied).
 *  CUBE_TRAPEZOID: lattice h*Z^3 on [-xi_max, xi_max]^3, h = 2*xi_max/M
 *    (M even), weights h^3 times 1, 1/2, 1/4, 1/8 (interior, faces, edges,
 *    corners); node order i (x) slowest, k (z) fastest. */
typedef struct {
    int32_t kind;
    double r_max;
    int32_t n_panels, n_per_panel, n_cos, n_phi;
    const double *nodes;
    const double *weights;
    int64_t n_nodes;
    double xi_max;
    int32_t M;
} hsd_rule_desc;

/* Per-call parameters.  Fill with hsd_params_default() first. */
typedef struct {
    double s;            /* Sobolev order: weight (1+|xi|^2)^-s; finite, s >= 0   */
    int32_t form;        /* HSD_FORM_*                                             */
    int32_t method;      /* HSD_METHOD_*                                           */
    double taylor_tau;   /* series branch when the phase spread G < tau (1e-2);
                            FP64: (0, 0.05]; mixed: (0, 0.75], and the mixed
                            form uses max(tau, 0.75) with a longer series      */
    int32_t tri_rule;    /* HSD_TRI_* (NUFFT3 only)                                */
    double nufft_tol;    /* requested NUFFT accuracy (sets the width if width==0)  */
    int32_t nufft_width; /* ES kernel width in grid points (0: from tol)           */
    double nufft_sigma;  /* oversampling factor (2.0)                              */
    int32_t k_splits;    /* triangle splits of the direct sum (0: automatic)       */
    int32_t reserved0;
    double freq_unit;    /* kappa in the weight (1+(|xi|/kappa)^2)^-s; 1 (or 0):
                            the library's exp(-i xi.x) convention; 2 pi: the
                            paper's exp(-2 pi i eta.x) convention (section 2.1)
                            with nodes xi = 2 pi eta, which makes d2 the paper's
                            H_{-s} norm of eq. sobolev_2 (s >= 0 here is the
                            paper's -s)                                          */
    int32_t reserved[4];
} hsd_params;

typedef struct {
    double d2;              /* squared distance                                    */
    double rel_err_stated;  /* stated relative error bound of d2 for this form     */
    double pairs;           /* triangle x node pairs evaluated (direct) or points  */
    double device_ms;       /* device time of the call's kernels (HIP events)      */
    double transform_ms;    /* device time of the transform stage alone (direct-sum
                               or NUFFT kernels), HIP events on the same stream     */
    int32_t status;         /* status of a served request                          */
    int32_t reserved;
} hsd_result;

/* Library version string. */
const char *hsd_version(void);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *hsd_last_error(void);

/* Fill *p with the defaults: s=1, FP64, DIRECT, tau=1e-2, DUNAVANT7,
 * tol 1e-9, width 0, sigma 2, k_splits 0. */
void hsd_params_default(hsd_params *p);

/* Create a context on HIP device `device` with a device-memory budget in
 * bytes for everything the library allocates (0: 90% of free memory).
 * Errors: EINVAL (bad device), EDEVICE. */
hsd_status hsd_init(int device, size_t hbm_budget_bytes, hsd_ctx **out);

/* Bind the stream (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream)
 * on which subsequent calls on this context enqueue their work; NULL selects
 * the default stream. */
hsd_status hsd_ctx_set_stream(hsd_ctx *ctx, void *hip_stream);

/* Bytes of device memory currently allocated by the context. */
size_t hsd_ctx_bytes_in_use(const hsd_ctx *ctx);

/* Stage timing of the NUFFT path (diagnostics).  With enable != 0 the
 * context's later NUFFT3 transforms (hsd_distance, hsd_transform_rule)
 * record HIP events at their stage boundaries on the context's stream.
 * hsd_nufft_stage_stats then gives, for the last such transform, ms[5] the
 * device time and bytes[5] the algorithmic HBM bytes (what each stage must
 * read and write at least) of the stages 0 points, sort and bins, 1 spread,
 * 2 pre-deconvolution, 3 the three FFT passes, 4 read-out (interpolation at
 * the nodes, or the lattice gather of type 1); it waits for the last event.
 * Errors: EINVAL (NULL, or no timed transform yet), EDEVICE. */
hsd_status hsd_ctx_set_stage_timing(hsd_ctx *ctx, int32_t enable);
hsd_status hsd_nufft_stage_stats(hsd_ctx *ctx, double *ms, double *bytes);

/* Destroy the context and everything it still owns. */
void hsd_finalize(hsd_ctx *ctx);

/* Mesh ingest (Section 2.2: each triangle is the affine image L(u) = p0 + A u
 * of the standard simplex, eq. def_affine_simplex).  Copies vertices and
 * triangles (host or device arrays per mem_kind) into device-resident
 * per-triangle records (p0, e1 = p1-p0, e2 = p2-p0, J = |e1 x e2|) and a
 * vertex-to-triangle CSR used by the adjoint.  nt may be 0 (the empty
 * surface).  Degenerate triangles (J = 0) are valid and contribute 0.
 * Vertex order within a triangle is irrelevant.
 * Errors: EINVAL (index outside [0, nv), non-finite vertex, negative sizes),
 * ENOMEM, EDEVICE. */
hsd_status hsd_create_mesh(hsd_ctx *ctx, const double *verts, int64_t nv,
                           const int32_t *tris, int64_t nt, int32_t mem_kind,
                           hsd_mesh **out);
/* A weighted point measure sum_q c_q delta(x - y_q) in place of a mesh: the
 * target of section 5's extension to smooth parametrised surfaces, sampled
 * by a quadrature on the parameter domain (points y_q, weights c_q = quadrature
 * weight times the area element).  Usable wherever a mesh is accepted by
 * hsd_distance, hsd_transform and hsd_transform_rule (as mu or nu), and as
 * nu of hsd_distance_grad.  Stored as n degenerate triangles (y_q, y_q, y_q)
 * with J = 2 c_q, whose exact transform J e[z, z, z] = c_q exp(-i xi.y_q):
 * the direct-sum and NUFFT kernels take it unchanged.
 * points: [n][3] FP64, weights: [n] FP64 (finite, any sign), both host or
 * both device memory per mem_kind, copied; n = 0 gives the zero measure.
 * hsd_mesh_num_vertices/_triangles return n.
 * Errors: EINVAL (negative n, NULL arrays, non-finite values, bad mem_kind),
 * ENOMEM, EDEVICE. */
hsd_status hsd_create_point_measure(hsd_ctx *ctx, const double *points, const double *weights,
                                    int64_t n, int32_t mem_kind, hsd_mesh **out);
/* Smooth surfaces with a built-in parametrisation, as point measures sampled
 * by a quadrature on the parameter domain that converges spectrally
 * (section 5: a smooth target known exactly, compared with its
 * triangulations):
 *  HSD_SURFACE_ELLIPSOID  x = c0 + (a s cos phi, b s sin phi, c u), u = cos theta,
 *      s = sqrt(1 - u^2); n_u Gauss-Legendre nodes in u, n_v trapezoid nodes in
 *      phi; area element sqrt(b^2 c^2 s^2 cos^2 phi + a^2 c^2 s^2 sin^2 phi
 *      + a^2 b^2 u^2) du dphi (a = b = c = 1: the unit sphere);
 *  HSD_SURFACE_TORUS  x = c0 + ((a + b cos v) cos u, (a + b cos v) sin u, b sin v)
 *      (centre-line radius a > b > 0, tube radius b); n_u x n_v trapezoid
 *      nodes; area element b (a + b cos v) du dv.
 * Points are ordered u-major.  The result behaves as hsd_create_point_measure's.
 * Errors: EINVAL (unknown kind, n_u or n_v < 1, non-positive or non-finite
 * radii, a <= b for the torus), ENOMEM, EDEVICE. */
enum { HSD_SURFACE_ELLIPSOID = 0, HSD_SURFACE_TORUS = 1 };
typedef struct {
    int32_t kind;        /* HSD_SURFACE_*                                        */
    int32_t n_u, n_v;    /* quadrature sizes                                     */
    double a, b, c;      /* ellipsoid semi-axes; torus: a, b as above (c unused) */
    double center[3];    /* translation c0                                       */
    int32_t reserved[4];
} hsd_surface_desc;
hsd_status hsd_create_surface_measure(hsd_ctx *ctx, const hsd_surface_desc *desc, hsd_mesh **out);
int64_t hsd_mesh_num_triangles(const hsd_mesh *m);
int64_t hsd_mesh_num_vertices(const hsd_mesh *m);
void hsd_mesh_destroy(hsd_mesh *m);

/* Build a frequency quadrature on the host (Gauss-Legendre nodes by Newton's
 * iteration on the Legendre recurrence) and make it device resident.
 * Errors: EINVAL (non-positive sizes, r_max <= 0, odd M, non-finite nodes,
 * negative weights), ENOMEM, EDEVICE. */
hsd_status hsd_freq_rule(hsd_ctx *ctx, const hsd_rule_desc *desc, hsd_rule **out);
int64_t hsd_rule_num_nodes(const hsd_rule *r);
/* Copy the flattened nodes [n][3] and weights [n] to host arrays (either may
 * be NULL). */
hsd_status hsd_rule_nodes(const hsd_rule *r, double *nodes, double *weights);
void hsd_rule_destroy(hsd_rule *r);

/* Squared H^-s distance between mesh mu and mesh nu (nu == NULL: the unit
 * sphere S^2 with transform 4 pi sin|xi|/|xi|).  Enqueues the direct-sum or
 * NUFFT kernels, the per-node finalize and the two-level deterministic
 * reduction on the context's stream, then waits for the 8-byte result.
 * The result is bitwise reproducible for a given (mesh, rule, params).
 * Errors: EINVAL (s < 0 or non-finite, unknown form/method), ENOMEM,
 * EDEVICE. */
hsd_status hsd_distance(hsd_ctx *ctx, const hsd_mesh *mu, const hsd_mesh *nu,
                        const hsd_rule *rule, const hsd_params *p, hsd_result *out);

/* hsd_distance that allocates no device memory, for callers that cannot
 * allocate: code recorded under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  Same arguments, result and errors as
 * hsd_distance, direct method only (EINVAL for NUFFT3).  The mesh(es) and
 * the rule must exist already (creating them allocates).
 * Every per-call buffer -- the weight and sphere-transform tables for
 * (s, freq_unit), built on the device from the rule's resident nodes and
 * weights; the [K][N] complex partial transforms; the reduction partials --
 * lives in one fixed device array of HSD_NOALLOC_SCRATCH_BYTES bytes per
 * GPU, reserved when the library's code is loaded on that GPU and held
 * until the process ends; hsd_init takes its address once per device.
 * A call needs 16 N + 16 T + 8 (N/256 + 2) bytes plus alignment (N rule
 * nodes; T = radial nodes of a spherical-product rule, else N) and fails
 * with EINVAL, before launching anything, when that exceeds the array; the
 * triangle splits K are reduced until the partials fit, so d2 may differ
 * from hsd_distance's in the last bits (split order, device-built tables).
 * Every call on one GPU uses the same array, which keeps the last call's
 * contents: calls that overlap on one GPU (other threads, other contexts,
 * other streams) race, and the caller must serialise them. */
#define HSD_NOALLOC_SCRATCH_BYTES ((size_t)160 << 20)
hsd_status hsd_distance_noalloc(hsd_ctx *ctx, const hsd_mesh *mu, const hsd_mesh *nu,
                                const hsd_rule *rule, const hsd_params *p, hsd_result *out);

/* Squared distance and its gradient with respect to the vertices of mu,
 * grad[nv][3] (mem_kind says where grad lives).  With nu a mesh, nu is held
 * fixed.  Direct method only (EINVAL for NUFFT3). */
hsd_status hsd_distance_grad(hsd_ctx *ctx, const hsd_mesh *mu, const hsd_mesh *nu,
                             const hsd_rule *rule, const hsd_params *p,
                             double *grad, int32_t mem_kind, hsd_result *out);

/* mu_h^(xi) of one mesh at n arbitrary nodes [n][3] (nodes_mem_kind), written
 * to out_re_im[n][2] (out_mem_kind).  Uses the exact direct sum (form per
 * p->form; method ignored) -- intended for tests and sampled checks. */
hsd_status hsd_transform(hsd_ctx *ctx, const hsd_mesh *m, const double *nodes, int64_t n,
                         int32_t nodes_mem_kind, const hsd_params *p,
                         double *out_re_im, int32_t out_mem_kind);

/* mu_h^ of one mesh at every node of a rule (out_re_im[n_nodes][2], device
 * or host), by the method/form of p (NUFFT3: the point-cloud transform). */
hsd_status hsd_transform_rule(hsd_ctx *ctx, const hsd_mesh *m, const hsd_rule *rule,
                              const hsd_params *p, double *out_re_im, int32_t out_mem_kind);

/* ---------------------------------------------------------------------- */
/* Serving loop: continuous batching of distance requests.                  */
/* ---------------------------------------------------------------------- */

typedef struct {
    int32_t slots;            /* concurrent requests on the device (streams)  */
    int32_t queue_capacity;   /* pending requests before EAGAIN               */
    size_t  hbm_budget_bytes; /* admission budget for request footprints      */
    int64_t chunk_pairs;      /* pairs enqueued per request per quantum       */
    int32_t reserved[8];
} hsd_server_cfg;

typedef struct {
    const double *verts;   int64_t nv;   /* mesh mu (host arrays, copied)         */
    const int32_t *tris;   int64_t nt;
    const double *verts2;  int64_t nv2;  /* mesh nu or NULL (unit sphere)         */
    const int32_t *tris2;  int64_t nt2;
    const hsd_rule *rule;                /* resident rule shared by requests      */
    hsd_params params;
    int64_t tag;                         /* caller's tag, echoed in statistics    */
} hsd_request;

typedef struct {
    double arrival_s;     /* submit time (server clock, seconds)                */
    double admitted_s;    /* admission time                                      */
    double finished_s;    /* result ready                                        */
    int64_t footprint;    /* admitted device bytes                               */
} hsd_request_times;

/* Start the serving thread on ctx's device (own streams, one per slot). */
hsd_status hsd_server_create(hsd_ctx *ctx, const hsd_server_cfg *cfg, hsd_server **out);
/* Submit a request (inputs copied).  EAGAIN when the queue is full; EINVAL
 * for invalid meshes or a footprint larger than the whole budget. */
hsd_status hsd_submit(hsd_server *s, const hsd_request *req, uint64_t *ticket);
/* OK with the result, PENDING, or the request's error.  A completed ticket
 * can be polled again until hsd_release() is called for it. */
hsd_status hsd_poll(hsd_server *s, uint64_t ticket, hsd_result *out, hsd_request_times *times);
/* Block until the ticket completes (timeout_s < 0: no timeout; PENDING on
 * timeout). */
hsd_status hsd_wait(hsd_server *s, uint64_t ticket, double timeout_s, hsd_result *out,
                    hsd_request_times *times);
/* Cancel a queued or running request (ECANCELED result). */
hsd_status hsd_cancel(hsd_server *s, uint64_t ticket);
/* Forget a completed ticket. */
hsd_status hsd_release(hsd_server *s, uint64_t ticket);
/* Drain running work and stop the thread. */
void hsd_server_destroy(hsd_server *s);

#ifdef __cplusplus
}
#endif

#endif /* HSD_H */
