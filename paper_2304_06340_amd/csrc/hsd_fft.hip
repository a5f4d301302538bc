// hsd_fft.hip -- cubic 3-D complex FFT (FP64), sizes n = 2^a 3^b <= 2048,
// forward sign: X_m = sum_l x_l exp(-2 pi i l m / n), unnormalised.
//
// One kernel per axis.  A block loads Bt whole 1-D lines of the axis into
// LDS (for the strided axes the Bt lines are consecutive in the contiguous
// dimension, so every global access is a coalesced run of Bt complex
// values), runs a Stockham autosort FFT in LDS (radix 9, 4, 3 and 2 stages;
// each stage reads its inputs to registers, synchronises, and writes its
// outputs in place), and writes the lines back.  Twiddles come from a table
// exp(-2 pi i k / n), k < n, built on the host in FP64.
#include <vector>

#include "hsd_internal.hpp"
#include "hsd_math.hpp"
#include "hsd_fft.hpp"

namespace hsd {

constexpr int kFftThreads = 512;

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// a / d for 0 <= a < 2^22 and 1 <= d < 2^12, given rd = 1.0f / d: the FP32
// product is within a relative 2^-23 of a / d, so its truncation is the
// quotient or one off, which the two corrections remove.
__device__ __forceinline__ int qdiv(int a, int d, float rd)
{
    int q = (int)((float)a * rd);
    q += (q + 1) * d <= a ? 1 : 0;
    q -= q * d > a ? 1 : 0;
    return q;
}

constexpr int kFftMaxElems = 4374;   // complex values per block tile (68 KB of LDS: two blocks per CU)

// 3-point DFT, forward sign: y_q = sum_r x_r exp(-2 pi i r q / 3)
__device__ __forceinline__ void dft3(double2 x0, double2 x1, double2 x2, double2 &y0, double2 &y1, double2 &y2)
{
    // exp(-2 pi i / 3) = -1/2 - i sqrt(3)/2
    const double c = -0.5, s = 0.86602540378443864676;
    const double2 t = make_double2(x1.x + x2.x, x1.y + x2.y);
    const double2 d = make_double2(x1.x - x2.x, x1.y - x2.y);
    y0 = make_double2(x0.x + t.x, x0.y + t.y);
    const double2 m = make_double2(x0.x + c * t.x, x0.y + c * t.y);
    // -i s d = (s d.y, -s d.x)
    y1 = make_double2(m.x + s * d.y, m.y - s * d.x);
    y2 = make_double2(m.x - s * d.y, m.y + s * d.x);
}

// One Stockham stage of radix R on Bt lines of length n in LDS: every
// thread first gathers (and twiddles) the inputs of all its butterflies into
// registers, the block synchronises, then the outputs are written in place.
// A butterfly reads one twiddle w = exp(-2 pi i k / (Ns R)) from the table
// (all of a thread's reads issued before any is used) and forms its powers
// by products; indices are divided through FP32 reciprocals (qdiv).  Radix 9
// is a 3 x 3 decomposition in registers (inner 3-point DFTs over r2 of
// r = r1 + 3 r2, twiddles exp(-2 pi i r1 q1 / 9), outer 3-point DFTs over
// r1), so that a 729-point line takes three LDS passes instead of six.
template <int R>
__device__ void stockham_stage(double2 *buf, int n, int Bt, int Ns, const double2 *__restrict__ tw)
{
    constexpr int kMaxBf = (kFftMaxElems / R + kFftThreads - 1) / kFftThreads;
    const int nb = n / R;              // butterflies per line
    const int total = nb * Bt;
    const int twstep = n / (Ns * R);   // exp(-2 pi i / (Ns R)) = tw[twstep]
    const float rnb = 1.0f / (float)nb, rns = 1.0f / (float)Ns;
    int jj[kMaxBf], ll[kMaxBf], kk[kMaxBf];
    double2 w1[kMaxBf];
#pragma unroll
    for (int b = 0; b < kMaxBf; ++b) {
        const int idx = b * kFftThreads + (int)threadIdx.x;
        const int line = qdiv(idx, nb, rnb);
        const int j = idx - line * nb;
        const int k = j - qdiv(j, Ns, rns) * Ns;
        ll[b] = line;
        jj[b] = j;
        kk[b] = k;
        w1[b] = tw[idx < total ? k * twstep : 0];
    }
    double2 x[kMaxBf][R];
#pragma unroll
    for (int b = 0; b < kMaxBf; ++b) {
        const int idx = b * kFftThreads + (int)threadIdx.x;
        if (idx < total) {
            const double2 *L = buf + (size_t)ll[b] * n;
            double2 wp = w1[b];   // w^r
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double2 a = L[jj[b] + r * nb];
                if (r >= 1) a = cmul(a, wp);
                if (r >= 1 && r + 1 < R) wp = cmul(wp, w1[b]);
                x[b][r] = a;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < kMaxBf; ++b) {
        const int idx = b * kFftThreads + (int)threadIdx.x;
        if (idx < total) {
            const int line = ll[b];
            const int j = jj[b];
            const double2 *xi = x[b];
            double2 y[R];
            if (R == 2) {
                y[0] = make_double2(xi[0].x + xi[1].x, xi[0].y + xi[1].y);
                y[1] = make_double2(xi[0].x - xi[1].x, xi[0].y - xi[1].y);
            } else if (R == 3) {
                dft3(xi[0], xi[1], xi[2], y[0], y[1], y[2]);
            } else if (R == 9) {
                // exp(-2 pi i k / 9) for k = 1, 2, 4
                const double2 w9_1 = make_double2(0.766044443118978035202, -0.642787609686539326323);
                const double2 w9_2 = make_double2(0.173648177666930348852, -0.984807753012208059367);
                const double2 w9_4 = make_double2(-0.939692620785908384054, -0.342020143325668733044);
                double2 z[3][3];   // z[r1][q1]
#pragma unroll
                for (int r1 = 0; r1 < 3; ++r1) dft3(xi[r1], xi[r1 + 3], xi[r1 + 6], z[r1][0], z[r1][1], z[r1][2]);
                z[1][1] = cmul(z[1][1], w9_1);
                z[1][2] = cmul(z[1][2], w9_2);
                z[2][1] = cmul(z[2][1], w9_2);
                z[2][2] = cmul(z[2][2], w9_4);
#pragma unroll
                for (int q1 = 0; q1 < 3; ++q1) dft3(z[0][q1], z[1][q1], z[2][q1], y[q1], y[q1 + 3], y[q1 + 6]);
            } else {   // R == 4
                const double2 a0 = make_double2(xi[0].x + xi[2].x, xi[0].y + xi[2].y);
                const double2 a1 = make_double2(xi[0].x - xi[2].x, xi[0].y - xi[2].y);
                const double2 b0 = make_double2(xi[1].x + xi[3].x, xi[1].y + xi[3].y);
                const double2 b1 = make_double2(xi[1].x - xi[3].x, xi[1].y - xi[3].y);
                y[0] = make_double2(a0.x + b0.x, a0.y + b0.y);
                y[2] = make_double2(a0.x - b0.x, a0.y - b0.y);
                // -i b1 = (b1.y, -b1.x)
                y[1] = make_double2(a1.x + b1.y, a1.y - b1.x);
                y[3] = make_double2(a1.x - b1.y, a1.y + b1.x);
            }
            double2 *L = buf + (size_t)line * n;
            const int k = kk[b];
            const int obase = (j - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) L[obase + q * Ns] = y[q];
        }
    }
    __syncthreads();
}

// Index map of a pruned axis: compact index c < 2e covers m < e and
// m >= n - e (gap = n - 2e); gap = 0 is the identity.
__device__ __forceinline__ int64_t unprune(int64_t c, int e, int gap) { return c < e ? c : c + gap; }

// Batched 1-D FFTs along one axis.  Line (o, i) element e lives at
// data[o * so + i * si + e * se]; blockIdx.x covers Bt consecutive compact
// inner indices for one compact outer index blockIdx.y, each mapped by
// unprune (e_i, gap_i) and (e_o, gap_o).  Along the line only the elements
// of the input band (e_r, gap_r) are read (the others are zero and are
// filled in LDS) and only those of the output band (e_w, gap_w) written.
__global__ __launch_bounds__(kFftThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_fft_axis(
    double2 *__restrict__ data, int n, int Bt, int64_t se, int64_t si, int64_t so, int64_t n_inner,
    const double2 *__restrict__ tw, const int *__restrict__ plan, int n_stages, int e_i, int gap_i, int e_o,
    int gap_o, int e_r, int gap_r, int e_w, int gap_w)
{
    extern __shared__ double2 lds[];
    const int64_t i0 = (int64_t)blockIdx.x * Bt;
    const int64_t o = unprune(blockIdx.y, e_o, gap_o);
    const int nl = (int)((n_inner - i0) < Bt ? (n_inner - i0) : Bt);
    double2 *base = data + o * so;
    const int nr = n - gap_r, nw = n - gap_w;   // elements read / written per line
    const float rnr = 1.0f / (float)nr, rnw = 1.0f / (float)nw, rnl = 1.0f / (float)nl;
    // zeros of the input band's gap
    if (gap_r > 0) {
        const float rg = 1.0f / (float)gap_r;
        for (int idx = threadIdx.x; idx < nl * gap_r; idx += kFftThreads) {
            const int line = qdiv(idx, gap_r, rg);
            lds[line * n + e_r + (idx - line * gap_r)] = make_double2(0.0, 0.0);
        }
    }
    // load: batches of kLoadBatch independent global reads per thread, all
    // issued before their LDS writes, so that they overlap
    const int total = nl * nr;
    constexpr int kLoadBatch = 8;
    for (int idx0 = threadIdx.x; idx0 < total; idx0 += kLoadBatch * kFftThreads) {
        double2 v[kLoadBatch];
        int slot[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            // past the tile's end: read the tile's last element again (in
            // bounds) and write that same value back to its own LDS slot, so
            // that neither the reads nor the writes need a branch
            const int idx = min(idx0 + u * kFftThreads, total - 1);
            int line, c;
            if (se == 1) { line = qdiv(idx, nr, rnr); c = idx - line * nr; }
            else { c = qdiv(idx, nl, rnl); line = idx - c * nl; }
            const int e = (int)unprune(c, e_r, gap_r);
            slot[u] = line * n + e;
            v[u] = base[unprune(i0 + line, e_i, gap_i) * si + (int64_t)e * se];
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) lds[slot[u]] = v[u];
    }
    __syncthreads();
    int Ns = 1;
    for (int s = 0; s < n_stages; ++s) {
        const int R = plan[s];
        if (R == 9) stockham_stage<9>(lds, n, nl, Ns, tw);
        else if (R == 4) stockham_stage<4>(lds, n, nl, Ns, tw);
        else if (R == 3) stockham_stage<3>(lds, n, nl, Ns, tw);
        else stockham_stage<2>(lds, n, nl, Ns, tw);
        Ns *= R;
    }
    // store the output band
    for (int idx = threadIdx.x; idx < nl * nw; idx += kFftThreads) {
        int line, c;
        if (se == 1) { line = qdiv(idx, nw, rnw); c = idx - line * nw; }
        else { c = qdiv(idx, nl, rnl); line = idx - c * nl; }
        const int e = (int)unprune(c, e_w, gap_w);
        base[unprune(i0 + line, e_i, gap_i) * si + (int64_t)e * se] = lds[(size_t)line * n + e];
    }
}

bool fft_size_ok(int n)
{
    if (n < 1 || n > 2048) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

int fft_next_size(int n)
{
    for (int m = std::max(n, 1);; ++m)
        if (fft_size_ok(m)) return m;
}

hsd_status FftPlan::init(hsd_ctx *ctx, int n_)
{
    if (!fft_size_ok(n_)) {
        set_error("FFT size %d is not 2^a 3^b <= 2048", n_);
        return HSD_EINVAL;
    }
    n = n_;
    std::vector<int> st;
    int m = n;
    while (m % 9 == 0) { st.push_back(9); m /= 9; }
    while (m % 4 == 0) { st.push_back(4); m /= 4; }
    while (m % 3 == 0) { st.push_back(3); m /= 3; }
    while (m % 2 == 0) { st.push_back(2); m /= 2; }
    stages = st;
    std::vector<double2> t((size_t)n);
    for (int k = 0; k < n; ++k) {
        const long double a = 2.0L * 3.141592653589793238462643383279503L * (long double)k / (long double)n;
        t[k] = make_double2((double)std::cos(a), (double)-std::sin(a));
    }
    hsd_status stt;
    if ((stt = tw.alloc(ctx, (size_t)n * sizeof(double2))) != HSD_OK) return stt;
    if ((stt = plan.alloc(ctx, std::max<size_t>(st.size(), 1) * sizeof(int))) != HSD_OK) return stt;
    HSD_HIP_TRY(hipMemcpy(tw.ptr, t.data(), (size_t)n * sizeof(double2), hipMemcpyHostToDevice));
    if (!st.empty()) HSD_HIP_TRY(hipMemcpy(plan.ptr, st.data(), st.size() * sizeof(int), hipMemcpyHostToDevice));
    return HSD_OK;
}

// Lines per block: keep the LDS tile within kFftMaxElems complex values.
static int lines_per_block(int n)
{
    return std::max(1, std::min(kFftMaxElems / n, 16));
}

double fft3d_bytes(int n, int e_in, int e_out)
{
    const double i = (e_in > 0 && 2 * e_in < n) ? 2.0 * e_in : (double)n;
    const double o = (e_out > 0 && 2 * e_out < n) ? 2.0 * e_out : (double)n;
    // z: i x i lines, y: i x o lines, x: o x o lines; each reads i, writes o
    return 16.0 * (i + o) * (i * i + i * o + o * o);
}

hsd_status fft3d_forward(hipStream_t st, const FftPlan &p, double2 *data, int e_in, int e_out)
{
    const int n = p.n;
    const int bt = lines_per_block(n);
    const size_t lds = (size_t)bt * n * sizeof(double2);
    const int ns = (int)p.stages.size();
    struct Range { int cnt, e, gap; };   // compact count and unprune map of an axis
    auto range = [n](int e) {
        return (e > 0 && 2 * e < n) ? Range{2 * e, e, n - 2 * e} : Range{n, n, 0};
    };
    const Range in = range(e_in), out = range(e_out);
    // axis z (contiguous): outer = x, inner = y, both where the input lives
    {
        dim3 grid((unsigned)((in.cnt + bt - 1) / bt), (unsigned)in.cnt);
        hipLaunchKernelGGL(k_fft_axis, grid, dim3(kFftThreads), lds, st, data, n, bt, (int64_t)1, (int64_t)n,
                           (int64_t)n * n, (int64_t)in.cnt, p.tw.as<const double2>(), p.plan.as<const int>(), ns,
                           in.e, in.gap, in.e, in.gap, in.e, in.gap, out.e, out.gap);
        HSD_HIP_TRY(hipGetLastError());
    }
    // axis y: element stride n; inner = z (wanted outputs), outer = x (input)
    {
        dim3 grid((unsigned)((out.cnt + bt - 1) / bt), (unsigned)in.cnt);
        hipLaunchKernelGGL(k_fft_axis, grid, dim3(kFftThreads), lds, st, data, n, bt, (int64_t)n, (int64_t)1,
                           (int64_t)n * n, (int64_t)out.cnt, p.tw.as<const double2>(), p.plan.as<const int>(), ns,
                           out.e, out.gap, in.e, in.gap, in.e, in.gap, out.e, out.gap);
        HSD_HIP_TRY(hipGetLastError());
    }
    // axis x: element stride n^2; inner = z, outer = y (wanted outputs)
    {
        dim3 grid((unsigned)((out.cnt + bt - 1) / bt), (unsigned)out.cnt);
        hipLaunchKernelGGL(k_fft_axis, grid, dim3(kFftThreads), lds, st, data, n, bt, (int64_t)n * n, (int64_t)1,
                           (int64_t)n, (int64_t)out.cnt, p.tw.as<const double2>(), p.plan.as<const int>(), ns,
                           out.e, out.gap, out.e, out.gap, in.e, in.gap, out.e, out.gap);
        HSD_HIP_TRY(hipGetLastError());
    }
    return HSD_OK;
}

} // namespace hsd

#ifdef HSD_TEST_HOOKS
extern "C" {

// Test hook (not part of the public ABI): forward 3-D FFT of a host cube
// [n][n][n] of interleaved complex values, in place, on `ctx`'s device;
// e_in, e_out as for fft3d_forward (with e_out > 0 only outputs in the
// wrapped centred cube of half-extent e_out are defined).
int hsd__test_fft3d_pruned(hsd_ctx *ctx, double *host_data, int n, int e_in, int e_out)
{
    using namespace hsd;
    if (!ctx || !host_data) return HSD_EINVAL;
    FftPlan plan;
    hsd_status stt;
    if ((stt = plan.init(ctx, n)) != HSD_OK) return stt;
    DevBuf buf;
    const size_t bytes = (size_t)n * n * n * sizeof(double2);
    if ((stt = buf.alloc(ctx, bytes)) != HSD_OK) return stt;
    HSD_HIP_TRY(hipMemcpy(buf.ptr, host_data, bytes, hipMemcpyHostToDevice));
    if ((stt = fft3d_forward(nullptr, plan, buf.as<double2>(), e_in, e_out)) != HSD_OK) return stt;
    HSD_HIP_TRY(hipDeviceSynchronize());
    HSD_HIP_TRY(hipMemcpy(host_data, buf.ptr, bytes, hipMemcpyDeviceToHost));
    return HSD_OK;
}

int hsd__test_fft3d(hsd_ctx *ctx, double *host_data, int n) { return hsd__test_fft3d_pruned(ctx, host_data, n, 0, 0); }

} // extern "C"
#endif // HSD_TEST_HOOKS
