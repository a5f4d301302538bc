// hsd_noalloc.hip -- hsd_distance_noalloc: the direct-sum distance of
// hsd_distance with every per-call device buffer placed in one fixed device
// array, so that a call allocates nothing.
//
// Layout of the array for one call (offsets rounded up to 256 bytes):
//   [W table | nu table]  per-(s, kappa) weights and sphere transform
//                         (radial for spherical-product rules, per node
//                         otherwise), built on the device from the rule's
//                         resident radii/nodes and weights
//   [block partials, result]  finalize output, then the final reduction's
//   [K][N] complex partial transforms of the direct sum
// The split count K is reduced until the partials fit.
#include <cmath>
#include <cstring>
#include <mutex>

#include "hsd_internal.hpp"

namespace hsd {

constexpr size_t kNoAllocBytes = HSD_NOALLOC_SCRATCH_BYTES;
constexpr int kNoAllocMaxDevices = 64;

// The array itself: one copy per GPU the library's code object is loaded on,
// held until the process ends.  Host code never uses this name as an address
// (in host code it is a stand-in, not device memory): the device address
// comes from hipGetSymbolAddress, once per device, in noalloc_setup.
static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];

namespace {
std::mutex g_mu;
void *g_ptr[kNoAllocMaxDevices] = {};
}

hsd_status noalloc_setup(int device)
{
    if (device < 0 || device >= kNoAllocMaxDevices) {
        set_error("device %d: the no-allocation scratch supports devices 0..%d", device, kNoAllocMaxDevices - 1);
        return HSD_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return HSD_OK;
    void *p = nullptr;
    HSD_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) {
        set_error("hipGetSymbolAddress returned NULL for the no-allocation scratch");
        return HSD_EDEVICE;
    }
    g_ptr[device] = p;
    return HSD_OK;
}

static void *scratch_of(int device)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return (device >= 0 && device < kNoAllocMaxDevices) ? g_ptr[device] : nullptr;
}

// W_i = w_i r_i^2 (1 + r_i^2 / kappa^2)^-s (2 pi)^-3 (spherical product:
// radial nodes r_i with radial weights w_i) or w_i (1 + r_i^2/kappa^2)^-s
// (2 pi)^-3 (other rules: node weights, r_i = |xi_i|); nu_i = 4 pi sin r / r
// (its Taylor polynomial below 1e-4).  The same expressions as the tables
// hsd_distance builds on the host, with the device's pow and sin.
__global__ void k_noalloc_tables(const double *__restrict__ radii, const double *__restrict__ nodes,
                                 const double *__restrict__ wts, int64_t n, double s, double ik2,
                                 double *__restrict__ W, double *__restrict__ nu)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double inv8pi3 = 1.0 / (8.0 * M_PI * M_PI * M_PI);
    double r, w;
    if (nodes) {
        const double x = nodes[3 * i], y = nodes[3 * i + 1], z = nodes[3 * i + 2];
        r = sqrt(x * x + y * y + z * z);
        w = wts[i];
    } else {
        r = radii[i];
        w = wts[i] * r * r;
    }
    W[i] = w * pow(1.0 + r * r * ik2, -s) * inv8pi3;
    nu[i] = r < 1e-4 ? 4.0 * M_PI * (1.0 - r * r / 6.0 + r * r * r * r / 120.0) : 4.0 * M_PI * sin(r) / r;
}

// The empty surface: zero partial transforms (a fill kernel, no memset).
__global__ void k_noalloc_zero(double2 *__restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_double2(0.0, 0.0);
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

} // namespace hsd

using namespace hsd;

extern "C" hsd_status hsd_distance_noalloc(hsd_ctx *ctx, const hsd_mesh *mu, const hsd_mesh *nu,
                                           const hsd_rule *rule, const hsd_params *p, hsd_result *out)
{
    if (!ctx) { set_error("context is NULL"); return HSD_EINVAL; }
    if (!mu || !rule || !out) { set_error("NULL argument"); return HSD_EINVAL; }
    hsd_status stt;
    if ((stt = validate_params(p)) != HSD_OK) return stt;
    if (p->method != HSD_METHOD_DIRECT) {
        set_error("hsd_distance_noalloc supports the direct method only");
        return HSD_EINVAL;
    }
    if (mu->ctx != ctx || (nu && nu->ctx != ctx) || rule->ctx != ctx) {
        set_error("mesh or rule belongs to another context");
        return HSD_EINVAL;
    }
    HSD_HIP_TRY(hipSetDevice(ctx->device));
    char *base = static_cast<char *>(scratch_of(ctx->device));
    if (!base) {
        set_error("no-allocation scratch not set up on device %d", ctx->device);
        return HSD_EDEVICE;
    }
    const bool sp = rule->kind == HSD_RULE_SPHERICAL_PRODUCT;
    const int64_t N = rule->n_nodes;
    const int64_t n_tab = sp ? rule->n_rad : N;
    const int64_t nb = finalize_blocks(N);
    const size_t tab_bytes = align256((size_t)n_tab * 8);
    const size_t red_bytes = align256((size_t)(nb + 1) * 8);
    const size_t unit = (size_t)N * sizeof(double2);
    const size_t fixed = 2 * tab_bytes + red_bytes;
    if (fixed > kNoAllocBytes || kNoAllocBytes - fixed < unit) {
        set_error("hsd_distance_noalloc: a rule of %lld nodes needs %zu bytes of scratch, more than the "
                  "%zu bytes the no-allocation entry point holds",
                  (long long)N, fixed + unit, kNoAllocBytes);
        return HSD_EINVAL;
    }
    MeshPair mp;
    mp.A = mu->tris.as<const TriRec>();
    mp.nA = mu->nt;
    if (nu) {
        mp.B = nu->tris.as<const TriRec>();
        mp.nB = nu->nt;
    }
    const int64_t ntot = mp.nA + mp.nB;
    int K = sp ? choose_k_splits_sp(rule, ntot, p->form, ctx->num_cu, p->k_splits)
               : choose_k_splits_gen(N, ntot, ctx->num_cu, p->k_splits);
    K = (int)std::min<int64_t>(K, (int64_t)((kNoAllocBytes - fixed) / unit));
    if (ntot == 0) K = 1;
    double *W = reinterpret_cast<double *>(base);
    double *nutab = reinterpret_cast<double *>(base + tab_bytes);
    double *red = reinterpret_cast<double *>(base + 2 * tab_bytes);
    double2 *partial = reinterpret_cast<double2 *>(base + fixed);

    std::lock_guard<std::mutex> lk(ctx->mu);
    hipStream_t st = ctx->stream;
    HSD_HIP_TRY(hipEventRecord(ctx->ev0, st));
    const double kappa = freq_unit_of(p);
    hipLaunchKernelGGL(k_noalloc_tables, dim3((unsigned)((n_tab + 255) / 256)), dim3(256), 0, st,
                       sp ? rule->d_radii.as<const double>() : nullptr,
                       sp ? nullptr : rule->d_nodes.as<const double>(), rule->d_wts.as<const double>(), n_tab,
                       p->s, 1.0 / (kappa * kappa), W, nutab);
    HSD_HIP_TRY(hipGetLastError());
    HSD_HIP_TRY(hipEventRecord(ctx->evt0, st));
    if (ntot == 0) {
        hipLaunchKernelGGL(k_noalloc_zero, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, partial, N);
        HSD_HIP_TRY(hipGetLastError());
    } else if (sp) {
        if ((stt = launch_direct_sp(st, mp, rule, p->form, p->taylor_tau, K, partial)) != HSD_OK) return stt;
    } else {
        if ((stt = launch_direct_gen(st, mp, rule->d_nodes.as<const double>(), N, p->form, p->taylor_tau, K,
                                     partial)) != HSD_OK)
            return stt;
    }
    HSD_HIP_TRY(hipEventRecord(ctx->evt1, st));
    if ((stt = launch_finalize(st, rule, W, nutab, partial, K, N, nu == nullptr, nullptr, red, nb)) != HSD_OK)
        return stt;
    if ((stt = launch_final_reduce(st, red, nb, red + nb)) != HSD_OK) return stt;
    HSD_HIP_TRY(hipEventRecord(ctx->ev1, st));
    HSD_HIP_TRY(hipMemcpyAsync(ctx->host_result, red + nb, sizeof(double), hipMemcpyDeviceToHost, st));
    HSD_HIP_TRY(hipStreamSynchronize(st));
    float ms = 0.0f, tms = 0.0f;
    HSD_HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    HSD_HIP_TRY(hipEventElapsedTime(&tms, ctx->evt0, ctx->evt1));
    std::memset(out, 0, sizeof *out);
    out->d2 = ctx->host_result[0];
    out->pairs = (double)ntot * (double)N;
    out->device_ms = ms;
    out->transform_ms = tms;
    out->rel_err_stated = stated_rel_err(p, ntot);
    out->status = HSD_OK;
    return HSD_OK;
}
