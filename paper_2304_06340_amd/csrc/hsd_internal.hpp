// hsd_internal.hpp -- internal types shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hsd.h"

namespace hsd {

// The mixed form evaluates the closed branch of the triangle transform in
// FP32, where the difference sinc b - sinc a cancels: its rounding error
// grows like eps32 / G relative to the triangle's term at phase spread G.
// These errors are random across triangles, but d^2 is quadratic in mu^, so
// their variance enters d^2 as a positive bias that does not average out.
// Below G = kMixedTau the mixed form therefore sums the power series instead
// (coefficients formed in FP64, no cancellation), through the power
// kMixedSeriesN, whose truncation stays below 5e-12 relative at G = 0.75.
constexpr double kMixedTau = 0.75;
constexpr int kMixedSeriesN = 11;

// The adjoint's closed-branch derivatives (F_a, F_b) lose about eps / G^3 to
// cancellation, 1e-10 at G = 1e-2; its series (twelve terms, truncation
// below 1e-26 at G = 0.05) is therefore used up to G = kAdjointTau.
constexpr double kAdjointTau = 0.05;

// One triangle as the affine image p0 + [e1 e2] u of the standard simplex
// (eq. def_affine_simplex) with its area ratio J = |e1 x e2| (gamma in eq.
// simplex32_ft).  80 bytes, read by whole wavefronts at once (scalar loads).
struct TriRec {
    double p0[3];
    double e1[3];
    double e2[3];
    double J;
};
static_assert(sizeof(TriRec) == 80, "TriRec layout");

void set_error(const char *fmt, ...);
void ctx_retain(hsd_ctx *c);
void ctx_release(hsd_ctx *c);
std::string hip_msg(hipError_t e, const char *what);

#define HSD_HIP_TRY(expr)                                                     \
    do {                                                                      \
        hipError_t _e = (expr);                                               \
        if (_e != hipSuccess) {                                               \
            ::hsd::set_error("%s", ::hsd::hip_msg(_e, #expr).c_str());       \
            return HSD_EDEVICE;                                               \
        }                                                                     \
    } while (0)

// Device allocation accounted against the context budget.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    hsd_ctx *ctx = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf();
    hsd_status alloc(hsd_ctx *c, size_t n);
    void release();
    template <typename T> T *as() const { return static_cast<T *>(ptr); }
};

// Reusable scratch (grows, never shrinks) owned by a context or a slot.
struct Scratch {
    DevBuf buf;
    hsd_status ensure(hsd_ctx *c, size_t n);
};

// Device buffers of the NUFFT path, reused across calls (owned by a context
// or by a serving slot).
struct FftPlan;
struct NufftScratch {
    DevBuf pts, spts, keys, keys2, iota, offs, perm, sorttmp, grid1, fine, tri, ftq, hinv;
    DevBuf titems, tstart, itile, tilebuf, scantmp;   // spread work items per tile
    DevBuf heavy;     // [0] = count, then the tiles with more than one work item
    std::unique_ptr<FftPlan> plan;
    // stage timing of the last transform (recorded when the context asks):
    // events at the stage boundaries and each stage's algorithmic bytes
    hipEvent_t ev[6] = {};
    bool timed = false;
    std::vector<double> tab_key;          // parameters of the tables in tri, ftq, hinv
    int nq = 0, nftq = 0, nhinv = 0;      // their lengths
    double stage_bytes[5] = {};
    NufftScratch();
    ~NufftScratch();
    size_t bytes() const;    // device bytes held
    void release();          // free them all
};

} // namespace hsd

struct hsd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0;
    std::atomic<size_t> in_use{0};
    hipEvent_t ev0 = nullptr, ev1 = nullptr, evt0 = nullptr, evt1 = nullptr;
    hsd::Scratch partial;     // [K][N] complex partial transforms
    hsd::Scratch nodebuf;     // per-node residuals / finalize partials
    hsd::Scratch redbuf;      // reduction partials + result
    hsd::Scratch gradbuf;     // per-triangle and per-vertex gradients
    hsd::NufftScratch nufft;  // NUFFT grids, points, bins
    double *host_result = nullptr;   // pinned 8-byte readback
    std::mutex mu;
    int num_cu = 256;
    bool stage_timing = false;   // record NUFFT stage events (hsd_ctx_set_stage_timing)
    std::atomic<int> refs{1};
};

struct hsd_mesh {
    hsd_ctx *ctx = nullptr;
    int64_t nv = 0, nt = 0;
    hsd::DevBuf tris;         // TriRec[nt]
    hsd::DevBuf verts;        // double[nv*3]
    hsd::DevBuf idx;          // int32[nt*3]
    hsd::DevBuf csr_ptr;      // int32[nv+1]   vertex -> (triangle, slot)
    hsd::DevBuf csr_ent;      // int32[3*nt]   entries: 3*t + slot
    std::vector<double> host_verts;
    std::vector<int32_t> host_tris;
    double extent = 0.0;          // max |vertex coordinate|
    bool point_measure = false;   // built by hsd_create_point_measure
    std::atomic<int> refs{1};
    ~hsd_mesh();
};

namespace hsd {

// Spherical product rule in factored form plus a flattened copy on demand.
struct RuleSP {
    double r_max = 0, delta = 0, h = 0;       // panel width, half width
    int32_t P = 0, n = 0, n_cos = 0, n_phi = 0;
    std::vector<double> x;                    // GL nodes on [-1, 1], ascending
    std::vector<double> wx;                   // GL weights
    std::vector<double> radii, wr;            // [P*n]
    std::vector<double> mu, wmu;              // [n_cos]
    std::vector<double> dirs;                 // [n_dir*3]
    std::vector<double> wdir;                 // [n_dir]
};

} // namespace hsd

struct hsd_rule {
    hsd_ctx *ctx = nullptr;
    int32_t kind = 0;
    int64_t n_nodes = 0;
    int64_t n_dir = 0, n_rad = 0;             // factored sizes (SP)
    hsd::RuleSP sp;
    std::vector<double> host_nodes;           // [n*3] flattened (all kinds)
    std::vector<double> host_weights;         // [n]
    std::vector<double> host_radii;           // [n]
    double extent = 0.0;                      // max |node coordinate|
    hsd::DevBuf d_dirs;                       // SP: [n_dir*3]
    hsd::DevBuf d_wdir;                       // SP: [n_dir]
    hsd::DevBuf d_hx;                         // SP: h*x for the positive half [n/2]
    hsd::DevBuf d_radii;                      // SP: radial nodes [n_rad]; others: {1.0}
    hsd::DevBuf d_iradii;                     // SP: their reciprocals [n_rad]
    hsd::DevBuf d_nodes;                      // EXPLICIT/CUBE: [n*3]
    hsd::DevBuf d_wts;                        // SP: radial weights w_r [n_rad]; others: node
                                              // weights [n] (device-built weight tables)
    int32_t cube_M = 0;                       // CUBE: lattice indices -M/2..M/2 per axis
    double cube_h = 0.0;                      // CUBE: lattice spacing 2 xi_max / M
    // per-s tables, kept for the rule's lifetime (requests with different s
    // may run concurrently): SP -> radial [n_rad]; general -> per node [n]
    struct Tables {
        hsd::DevBuf w;                        // w (1+r^2)^-s (2pi)^-3 (SP: w_r r^2 ...)
        hsd::DevBuf nu;                       // sphere transform 4 pi sin r / r
    };
    std::map<std::pair<double, double>, std::unique_ptr<Tables>> tabs;   // by (s, freq_unit)
    // per-node 1 / Phi^(xi_k) of the type-3 NUFFT and the nodes' grouping by
    // interpolation tile, by (width, beta, h1, fine-grid size)
    struct NufftDeconv {
        int w = 0, n2 = 0;
        double beta = 0.0, h1 = 0.0;
        hsd::DevBuf inv;
        hsd::DevBuf order;   // nodes grouped by interpolation tile
        hsd::DevBuf items;   // int4 (tile, first, end, 0) work items over `order`
        int nitems = 0;
    };
    std::vector<std::unique_ptr<NufftDeconv>> nufft_deconv;
    std::mutex mu;
    std::atomic<int> refs{1};
    ~hsd_rule();
};

namespace hsd {

// Launch-level description of one direct-sum evaluation.
struct MeshPair {
    const TriRec *A = nullptr; int64_t nA = 0;   // +1
    const TriRec *B = nullptr; int64_t nB = 0;   // -1 (second mesh)
};

// Kernel launchers (hsd_direct.hip).
hsd_status launch_direct_sp(hipStream_t st, const MeshPair &mp, const hsd_rule *rule,
                            int form, double tau, int K, double2 *partial);
hsd_status launch_direct_gen(hipStream_t st, const MeshPair &mp, const double *nodes,
                             int64_t n, int form, double tau, int K, double2 *partial);
hsd_status launch_direct_sp_range(hipStream_t st, const MeshPair &mp, const hsd_rule *rule,
                                  int form, double tau, int K, int64_t d_begin, int64_t d_count,
                                  double2 *partial);
hsd_status launch_direct_gen_range(hipStream_t st, const MeshPair &mp, const double *nodes,
                                   int64_t n, int form, double tau, int K, int64_t i_begin,
                                   int64_t i_count, double2 *partial);
hsd_status create_mesh_on(hsd_ctx *ctx, hipStream_t st, const double *verts, int64_t nv, const int32_t *tris,
                          int64_t nt, int32_t mem_kind, hsd_mesh **out, const double *point_weights = nullptr);
hsd_status mesh_reload(hsd_ctx *ctx, hipStream_t st, hsd_mesh *m, const double *verts, int64_t nv,
                       const int32_t *tris, int64_t nt, std::vector<TriRec> &rec);
hsd_status launch_finalize(hipStream_t st, const hsd_rule *rule, const double *wtab,
                           const double *nutab, const double2 *partial, int K, int64_t n,
                           bool sphere_target, double2 *resid_out, double *block_out,
                           int64_t nblocks);
hsd_status launch_final_reduce(hipStream_t st, const double *block_in, int64_t nblocks,
                               double *out);
hsd_status launch_sum_partials(hipStream_t st, const double2 *partial, int K, int64_t n,
                               double2 *out);
int64_t finalize_blocks(int64_t n);
// wave-per-direction kernel (hsd_direct_wave.hip) for 16-node panels
bool wave_kernel_applies(const hsd_rule *rule);
int64_t wave_count(const hsd_rule *rule);
hsd_status launch_direct_wave(hipStream_t st, const MeshPair &mp, const hsd_rule *rule, int form,
                              double tau, int K, int64_t d_begin, int64_t d_count, double2 *partial);
int choose_k_splits_sp(const hsd_rule *rule, int64_t nt, int form, int num_cu, int req);
int choose_k_splits_gen(int64_t n, int64_t nt, int num_cu, int req);

// Adjoint (hsd_adjoint.hip).
int adjoint_splits(int64_t nt, int64_t n_dir, int num_cu);
hsd_status launch_adjoint_raw(hipStream_t st, const TriRec *tris, int64_t nt, const double *dirs, int64_t n_dir,
                              const double *radii, int n_rad, const double2 *resid, const double *wdir,
                              const double *wtab, double tau, int S, double *part, double *tri_grad, int P = 0,
                              int n = 0, double h = 0.0, const double *hx_tab = nullptr,
                              const double *iradii = nullptr);
hsd_status launch_gather(hipStream_t st, const hsd_mesh *m, const double *tri_grad,
                         double *grad);

// NUFFT (hsd_nufft.hip).
// Device bytes one transform of ntri triangles' points (sources within X of
// the origin per axis) on `rule` allocates, including the rule's cached
// per-node tables on first use; -1 if the grid is not supported.
int64_t nufft_footprint(double X, const hsd_rule *rule, const hsd_params *p, int64_t ntri);
hsd_status nufft_transform_rule(hsd_ctx *ctx, hipStream_t st, NufftScratch &sc,
                                const hsd_mesh *mu, const hsd_mesh *nu, const hsd_rule *rule,
                                const hsd_params *p, double2 *out, double *pairs);

// No-allocation entry point (hsd_noalloc.hip): takes the device address of
// its fixed scratch array once per device; called by hsd_init with the
// device current.
hsd_status noalloc_setup(int device);

// Shared host helpers (hsd_core.hip).
double freq_unit_of(const hsd_params *p);
hsd_status rule_tables(hsd_rule *rule, const hsd_params *p, hipStream_t st, const double **wtab,
                       const double **nutab);
hsd_status validate_params(const hsd_params *p);
double stated_rel_err(const hsd_params *p, int64_t nt);
hsd_status distance_core(hsd_ctx *ctx, hipStream_t st, const hsd_mesh *mu, const hsd_mesh *nu,
                         const hsd_rule *rule, const hsd_params *p, bool keep_resid,
                         Scratch &partial, Scratch &nodebuf, Scratch &redbuf,
                         NufftScratch &nsc, double **d_result, double *pairs,
                         hipEvent_t ev_tb = nullptr, hipEvent_t ev_te = nullptr);

} // namespace hsd
