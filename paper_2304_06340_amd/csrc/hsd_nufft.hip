// hsd_nufft.hip -- type-3 NUFFT fast path for mu_h^ on the frequency rule.
//
// Every triangle is replaced by the weighted Dirac cloud of a triangle rule
// {(L(u_q), q_q * area)} (eqs. change_variable, change_variable_approx,
// Section 3.1), and the exponential sum
//     f(xi_k) = sum_j c_j exp(-i xi_k . x_j)
// is evaluated at the nonuniform nodes xi_k by a type-3 NUFFT (the general
// nonuniform-to-nonuniform case named at the end of Section 3.3), built from
// the exponential-of-semicircle kernel psi(z) = exp(beta (sqrt(1 - z^2) - 1)):
//
//  1. spread: b_l = sum_j c_j Phi(l h1 - x_j) on a grid of spacing
//     h1 = pi / (sigma S) (S = max |xi_d|), Phi a tensor product of
//     psi(2 y / (w h1)).  Then sum_j c_j exp(-i xi.x_j) Phi^(xi) =
//     int b(y) exp(-i xi.y) dy ~= h1^3 sum_l b_l exp(-i (xi h1).l).
//  2. type 2 on t = xi h1 in [-pi/sigma, pi/sigma]^3: pre-divide b_l by the
//     Fourier coefficients of the periodised fine-grid kernel, zero-pad to
//     n2 = sigma n1 (rounded to 2^a 3^b), 3-D FFT, interpolate with the same
//     kernel shape at t_k.
//  3. divide by Phi^(xi_k) (Gauss-Legendre quadrature of psi's transform).
//
// The spread is a gather (one thread per grid point, points visited in a
// fixed bin-sorted order), so it is deterministic without atomics on
// floating-point values; the points are ordered by a stable radix sort on
// their bin (rocPRIM), which keeps ascending point index inside each bin
// (bin sizes range from a few points to tens of thousands when a lattice
// rule packs a whole mesh into a few bins, so a per-bin sort would not do).
#include <algorithm>
#include <cmath>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "hsd_fft.hpp"
#include "hsd_internal.hpp"
#include "hsd_math.hpp"

namespace hsd {

constexpr int kBin = 8;            // grid cells per bin / spread tile edge
static_assert(kBin == 8, "the spread kernel splits value indices by shifts");
constexpr int kChunk = 64;         // points staged in LDS per spread step
constexpr double kKeepMargin = 1e-6; // grid units, see k_spread
constexpr int kMaxW = 16;          // largest kernel width supported

struct EsKernel {
    int w;
    double beta;
    double half;                   // w / 2
};

// psi(z) = exp(beta (sqrt(1 - z^2) - 1)) on |z| < 1, 0 elsewhere.  On the
// device, without branches or library calls: sqrt(a) from the hardware
// reciprocal square root refined by one Goldschmidt step and one Newton
// correction; exp(x) for x in [-beta, 0] by Cody-Waite reduction
// x = n ln 2 + r (ln 2 split in two), |r| <= ln 2 / 2, the Taylor series of
// e^r through r^11 (truncation below 7e-15 relative) and a scaling by 2^n.
constexpr double kLog2E = 1.4426950408889634;     // RN(1 / ln 2)
constexpr double kLn2Hi = 0.6931471805599453;     // RN(ln 2)
constexpr double kLn2Lo = 2.3190468138462996e-17; // RN(ln 2 - kLn2Hi)

// 1/k!, k = 0..11, in constant memory: read with scalar loads, so that the
// Horner steps take them from scalar registers instead of rebuilding 64-bit
// literals in vector registers on every evaluation.
__constant__ double kExpTaylor[12] = {inv_factorial(0), inv_factorial(1), inv_factorial(2),  inv_factorial(3),
                                      inv_factorial(4), inv_factorial(5), inv_factorial(6),  inv_factorial(7),
                                      inv_factorial(8), inv_factorial(9), inv_factorial(10), inv_factorial(11)};

HSD_HD double es_eval(double z, double beta)
{
    const double a = __builtin_fma(-z, z, 1.0);
#if defined(__HIP_DEVICE_COMPILE__)
    const double ac = a > 0.0 ? a : 1.0;   // keeps the arithmetic finite off the support
    const double y = __builtin_amdgcn_rsq(ac);
    double sq = ac * y, hy = 0.5 * y;
    const double e = __builtin_fma(-sq, hy, 0.5);
    sq = __builtin_fma(sq, e, sq);
    hy = __builtin_fma(hy, e, hy);
    sq = __builtin_fma(__builtin_fma(-sq, sq, ac), hy, sq);
    const double x = beta * (sq - 1.0);
    const double n = __builtin_rint(x * kLog2E);
    double r = __builtin_fma(-n, kLn2Hi, x);
    r = __builtin_fma(-n, kLn2Lo, r);
    double pe = kExpTaylor[11];
#pragma unroll
    for (int k = 10; k >= 0; --k) pe = __builtin_fma(pe, r, kExpTaylor[k]);
    const double v = ldexp(pe, (int)n);
    return a > 0.0 ? v : 0.0;
#else
    return a > 0.0 ? std::exp(beta * (std::sqrt(a) - 1.0)) : 0.0;
#endif
}

// --------------------------------------------------------------------------
// 1. points and bins
// --------------------------------------------------------------------------
__global__ void k_nufft_points(const TriRec *__restrict__ A, int64_t nA, const TriRec *__restrict__ B, int64_t nB,
                               const double4 *__restrict__ rule, int nq, double h1, int n1, int nbx,
                               double4 *__restrict__ pts, int *__restrict__ keys)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t np = (nA + nB) * nq;
    if (gid >= np) return;
    const int64_t t = gid / nq;
    const int q = (int)(gid - t * nq);
    const bool inA = t < nA;
    const TriRec T = inA ? A[t] : B[t - nA];
    const double4 bq = rule[q];   // barycentric (l0, l1, l2) and weight (sum 1)
    double4 p;
    p.x = T.p0[0] + bq.y * T.e1[0] + bq.z * T.e2[0];
    p.y = T.p0[1] + bq.y * T.e1[1] + bq.z * T.e2[1];
    p.z = T.p0[2] + bq.y * T.e1[2] + bq.z * T.e2[2];
    p.w = (inA ? 0.5 : -0.5) * T.J * bq.w;
    pts[gid] = p;
    const double half = 0.5 * n1;
    int b[3];
    const double c[3] = {p.x, p.y, p.z};
    for (int d = 0; d < 3; ++d) {
        int v = (int)floor((c[d] / h1 + half) / kBin);
        b[d] = v < 0 ? 0 : (v >= nbx ? nbx - 1 : v);
    }
    keys[gid] = (b[0] * nbx + b[1]) * nbx + b[2];
}

// Bin offsets from the sorted keys: offs[b] = first position whose key is
// >= b (offs[nbins] = np), one thread per bin by binary search (clustered
// points leave long runs of empty bins, which a thread per point would
// write one by one).
__global__ void k_bin_offsets(const int *__restrict__ skeys, int64_t np, int nbins, int *__restrict__ offs)
{
    const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b > nbins) return;
    int64_t lo = 0, hi = np;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (skeys[mid] < b) lo = mid + 1;
        else hi = mid;
    }
    offs[b] = (int)lo;
}

__global__ void k_iota(int *__restrict__ idx, int64_t np)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) idx[i] = (int)i;
}

__global__ void k_gather_points(const double4 *__restrict__ pts, const int *__restrict__ perm, int64_t np,
                                double4 *__restrict__ spts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) spts[i] = pts[perm[i]];
}

// --------------------------------------------------------------------------
// 2. spread (gather form): one wavefront per work item of one 8x8x8 tile of
//    grid points; lane (tx, ty) holds the tile's column of 8 z values in
//    registers.  The points of the 27 bins around the tile are staged in
//    chunks of 64; only those whose kernel support reaches the tile are kept
//    (ballot compaction, order preserved), so a point costs work only in the
//    tiles it touches.  Per kept point the wave evaluates the 24 kernel
//    values psi(x), psi(y), psi(z) of the tile into LDS; each lane then
//    forms psi(x) c psi(y) and, with the column psi(z) (the same for all
//    lanes), does 8 FMAs.
//
//    Work items: a tile whose neighbourhood holds more than kItemChunks
//    chunks gets several items, item s taking the chunks numbered
//    [s kItemChunks, (s + 1) kItemChunks) of the tile's sequence (bins in
//    order, chunks of 64 points); each writes a partial tile, summed by
//    k_tile_reduce (eighths of the item range in item order, then the eighths
//    in order).  Clustered points (a whole mesh in a few bins, as on the
//    cube lattice) then spread over many waves instead of a few long ones.
//    Sum order per grid point: fixed (items as above, then bin, then point
//    order).
// --------------------------------------------------------------------------
constexpr int kItemChunks = 64;   // candidate chunks per work item (at most)

__device__ __forceinline__ void tile_of(int t, int nbx, int &bx, int &by, int &bz)
{
    bz = t % nbx;
    by = (t / nbx) % nbx;
    bx = t / (nbx * nbx);
}

// titems[t] = number of work items of tile t (>= 1); titems[ntiles] = 0;
// heavy[0] (the count of tiles with several items) = 0
__global__ void k_tile_items(const int *__restrict__ offs, int nbx, int *__restrict__ titems, int *__restrict__ heavy)
{
    const int ntiles = nbx * nbx * nbx;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    if (t == ntiles) {
        titems[t] = 0;
        heavy[0] = 0;
        return;
    }
    int bx, by, bz;
    tile_of(t, nbx, bx, by, bz);
    int64_t chunks = 0;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                const int nx = bx + dx, ny = by + dy, nz = bz + dz;
                if (nx < 0 || ny < 0 || nz < 0 || nx >= nbx || ny >= nbx || nz >= nbx) continue;
                const int nb = (nx * nbx + ny) * nbx + nz;
                chunks += (offs[nb + 1] - offs[nb] + kChunk - 1) / kChunk;
            }
    titems[t] = (int)(chunks > 0 ? (chunks + kItemChunks - 1) / kItemChunks : 1);
}

// itile[item] = its tile, for the items of every tile (tstart = exclusive
// scan); the tiles with several items listed in heavy[1..heavy[0]] (in any
// order: each is reduced on its own, in a fixed order)
__global__ void k_item_map(const int *__restrict__ tstart, int ntiles, int *__restrict__ itile,
                           int *__restrict__ heavy)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    for (int i = tstart[t]; i < tstart[t + 1]; ++i) itile[i] = t;
    if (tstart[t + 1] - tstart[t] > 1) heavy[1 + atomicAdd(&heavy[0], 1)] = t;
}

__global__ __launch_bounds__(64) void k_spread(const double4 *__restrict__ spts, const int *__restrict__ offs,
                                               const int *__restrict__ tstart, const int *__restrict__ itile,
                                               int nbx, int n1, double h1, double half_w, double beta,
                                               double *__restrict__ grid, double *__restrict__ tilebuf)
{
    constexpr int kSub = 32;                    // kept points evaluated per pass
    __shared__ double kv[kSub][3 * kBin];       // psi at the tile's x, y and z lines
    __shared__ double gt[kChunk][3];            // (tile origin - point) / (w / 2) per axis
    __shared__ double cw[kChunk];
    const int ntiles = nbx * nbx * nbx;
    const int item = blockIdx.x;
    if (item >= tstart[ntiles]) return;         // beyond the items of this call
    const int tile = itile[item];
    const int split = item - tstart[tile], nsplit = tstart[tile + 1] - tstart[tile];
    const int lane = threadIdx.x;
    const int tx = lane & 7, ty = lane >> 3;
    int bx, by, bz;
    tile_of(tile, nbx, bx, by, bz);
    const int64_t cbeg = (int64_t)split * kItemChunks, cend = cbeg + kItemChunks;
    int64_t chunk_no = 0;   // first chunk of the current bin in the tile's sequence
    const int org[3] = {bx * kBin, by * kBin, bz * kBin};
    const double half = 0.5 * n1;
    const double ih1 = 1.0 / h1;
    const double iw = 1.0 / half_w;
    // this lane's first (point, value) slot of an evaluation pass: slot
    // v = lane + 64 j holds point v / 24, value v % 24
    const int p0 = lane / (3 * kBin), r0 = lane - p0 * (3 * kBin);
    double acc[kBin];
#pragma unroll
    for (int z = 0; z < kBin; ++z) acc[z] = 0.0;
    for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
                const int nx = bx + dx, ny = by + dy, nz = bz + dz;
                if (nx < 0 || ny < 0 || nz < 0 || nx >= nbx || ny >= nbx || nz >= nbx) continue;
                const int nb = (nx * nbx + ny) * nbx + nz;
                const int lo = offs[nb], hi = offs[nb + 1];
                const int nch = (hi - lo + kChunk - 1) / kChunk;
                const int64_t j0 = cbeg > chunk_no ? cbeg - chunk_no : 0;
                const int64_t j1 = cend - chunk_no < nch ? cend - chunk_no : nch;
                chunk_no += nch;
                for (int64_t jc = j0; jc < j1; ++jc) {            // block-uniform
                    const int c0 = lo + (int)jc * kChunk;
                    const int cnt = (hi - c0) < kChunk ? (hi - c0) : kChunk;
                    bool keep = false;
                    double g[3] = {0.0, 0.0, 0.0}, wv = 0.0;
                    if (lane < cnt) {
                        const double4 p = spts[c0 + lane];
                        g[0] = __builtin_fma(p.x, ih1, half);
                        g[1] = __builtin_fma(p.y, ih1, half);
                        g[2] = __builtin_fma(p.z, ih1, half);
                        wv = p.w;
                        // the point reaches a grid line org + i of the tile
                        // (|org + i - g| < w/2 on every axis) iff
                        // org - w/2 < g < org + kBin - 1 + w/2; beyond that its
                        // kernel values on the tile are exactly 0.  The margin
                        // (far above the rounding of g) only keeps points whose
                        // values there are 0 anyway.
                        keep = true;
                        for (int d = 0; d < 3; ++d)
                            keep = keep && g[d] > (double)org[d] - half_w - kKeepMargin &&
                                   g[d] < (double)(org[d] + kBin - 1) + half_w + kKeepMargin;
                    }
                    const unsigned long long m = __ballot(keep);
                    const int nk = __popcll(m);
                    if (nk == 0) continue;                        // wave-uniform
                    if (keep) {
                        const int pos = __popcll(m & ((1ull << lane) - 1ull));
#pragma unroll
                        for (int d = 0; d < 3; ++d) gt[pos][d] = ((double)org[d] - g[d]) * iw;
                        cw[pos] = wv;
                    }
                    for (int s0 = 0; s0 < nk; s0 += kSub) {
                        const int ns = (nk - s0) < kSub ? (nk - s0) : kSub;
                        __syncthreads();
                        int p = p0, r = r0;
                        for (int v = lane; v < ns * 3 * kBin; v += 64) {
                            // value r of point p: grid line i = r % 8 of axis d = r / 8
                            const int d = r >> 3, i = r & 7;      // kBin = 8
                            kv[p][r] = es_eval(__builtin_fma((double)i, iw, gt[s0 + p][d]), beta);
                            // v += 64 = 2 * 24 + 16
                            p += 2;
                            r += 16;
                            if (r >= 3 * kBin) { r -= 3 * kBin; ++p; }
                        }
                        __syncthreads();
                        int q = 0;
                        for (; q + 2 <= ns; q += 2) {
                            const double a0 = kv[q][tx] * cw[s0 + q] * kv[q][kBin + ty];
                            const double a1 = kv[q + 1][tx] * cw[s0 + q + 1] * kv[q + 1][kBin + ty];
                            double z0[kBin], z1[kBin];
#pragma unroll
                            for (int z = 0; z < kBin; ++z) { z0[z] = kv[q][2 * kBin + z]; z1[z] = kv[q + 1][2 * kBin + z]; }
#pragma unroll
                            for (int z = 0; z < kBin; ++z) acc[z] = __builtin_fma(a1, z1[z], __builtin_fma(a0, z0[z], acc[z]));
                        }
                        if (q < ns) {
                            const double a0 = kv[q][tx] * cw[s0 + q] * kv[q][kBin + ty];
#pragma unroll
                            for (int z = 0; z < kBin; ++z) acc[z] = __builtin_fma(a0, kv[q][2 * kBin + z], acc[z]);
                        }
                    }
                    __syncthreads();
                }
            }
    if (nsplit > 1) {
        double *dst = tilebuf + (int64_t)item * (kBin * kBin * kBin) + lane * kBin;
#pragma unroll
        for (int z = 0; z < kBin; ++z) dst[z] = acc[z];
        return;
    }
    const int lx = org[0] + tx, ly = org[1] + ty;
    if (lx < n1 && ly < n1) {
        double *col = grid + ((int64_t)lx * n1 + ly) * n1;
#pragma unroll
        for (int z = 0; z < kBin; ++z)
            if (org[2] + z < n1) col[org[2] + z] = acc[z];
    }
}

// Sum of the partial tiles of the tiles with several work items (the list
// in heavy): per tile with more than kReduceWaves items, the 8 waves of a
// block sum consecutive eighths of its items in item order, then wave 0 adds
// the eight partial sums in wave order (a tile in a cluster of points can
// have hundreds of items); fewer items are summed by wave 0 in item order.
// Either way the order is fixed.  Blocks stride over the list.
constexpr int kReduceWaves = 8;
__global__ __launch_bounds__(64 * kReduceWaves) void k_tile_reduce(const double *__restrict__ tilebuf,
                                                                   const int *__restrict__ tstart,
                                                                   const int *__restrict__ heavy, int nbx, int n1,
                                                                   double *__restrict__ grid)
{
    __shared__ double part[kReduceWaves][kBin][64];
    const int nh = heavy[0];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, tx = lane & 7, ty = lane >> 3;
    for (int hi = blockIdx.x; hi < nh; hi += gridDim.x) {   // block-uniform
        const int tile = heavy[1 + hi];
        const int i0 = tstart[tile];
        const int64_t n = tstart[tile + 1] - i0;
        int bx, by, bz;
        tile_of(tile, nbx, bx, by, bz);
        const int lx = bx * kBin + tx, ly = by * kBin + ty, z0 = bz * kBin;
        double acc[kBin];
        if (n <= kReduceWaves) {   // block-uniform
            if (w != 0) continue;
#pragma unroll
            for (int z = 0; z < kBin; ++z) acc[z] = 0.0;
            for (int i = i0; i < i0 + (int)n; ++i) {
                const double *src = tilebuf + (int64_t)i * (kBin * kBin * kBin) + lane * kBin;
#pragma unroll
                for (int z = 0; z < kBin; ++z) acc[z] += src[z];
            }
            if (lx < n1 && ly < n1) {
                double *col = grid + ((int64_t)lx * n1 + ly) * n1;
#pragma unroll
                for (int z = 0; z < kBin; ++z)
                    if (z0 + z < n1) col[z0 + z] = acc[z];
            }
            continue;
        }
        const int a = i0 + (int)(n * w / kReduceWaves), b = i0 + (int)(n * (w + 1) / kReduceWaves);
#pragma unroll
        for (int z = 0; z < kBin; ++z) acc[z] = 0.0;
        for (int i = a; i < b; ++i) {
            const double *src = tilebuf + (int64_t)i * (kBin * kBin * kBin) + lane * kBin;
#pragma unroll
            for (int z = 0; z < kBin; ++z) acc[z] += src[z];
        }
#pragma unroll
        for (int z = 0; z < kBin; ++z) part[w][z][lane] = acc[z];
        __syncthreads();
        if (w == 0) {
#pragma unroll
            for (int z = 0; z < kBin; ++z) {
                double t = part[0][z][lane];
                for (int ww = 1; ww < kReduceWaves; ++ww) t += part[ww][z][lane];
                acc[z] = t;
            }
            if (lx < n1 && ly < n1) {
                double *col = grid + ((int64_t)lx * n1 + ly) * n1;
#pragma unroll
                for (int z = 0; z < kBin; ++z)
                    if (z0 + z < n1) col[z0 + z] = acc[z];
            }
        }
        __syncthreads();   // part is rewritten by the next tile
    }
}

// --------------------------------------------------------------------------
// 3. pre-deconvolve into the fine grid (index m <-> l' = m or m - n2), over
//    the wrapped band m < e, m >= n2 - e of every axis only (cnt = 2 e
//    compact indices per axis, gap = n2 - 2 e; e <= n1 / 2): the fine grid is
//    zero outside it, and the FFT neither reads nor needs those values
// --------------------------------------------------------------------------
__global__ void k_predeconv(const double *__restrict__ grid, int n1, const double *__restrict__ hinv,
                            int n2, int cnt, int e, int gap, double2 *__restrict__ fine)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)cnt * cnt * cnt;
    if (g >= tot) return;
    const int c[3] = {(int)(g / ((int64_t)cnt * cnt)), (int)((g / cnt) % cnt), (int)(g % cnt)};
    int m[3], l[3];
    bool in = true;
    for (int d = 0; d < 3; ++d) {
        m[d] = c[d] < e ? c[d] : c[d] + gap;
        const int lp = m[d] < n2 / 2 ? m[d] : m[d] - n2;   // signed frequency index
        l[d] = lp + n1 / 2;
        in = in && (l[d] >= 0 && l[d] < n1);
    }
    double v = 0.0;
    if (in) {
        const int64_t cell = ((int64_t)l[0] * n1 + l[1]) * n1 + l[2];
        v = grid[cell] * (hinv[l[0]] * hinv[l[1]] * hinv[l[2]]);
    }
    fine[((int64_t)m[0] * n2 + m[1]) * n2 + m[2]] = make_double2(v, 0.0);
}

// --------------------------------------------------------------------------
// 4. interpolate at the targets and divide by Phi^
// --------------------------------------------------------------------------
// Targets are grouped by the tile of TS^3 grid points that holds the origin
// of their stencil (per axis lo = ceil(u - w/2), u the target in grid units,
// shifted by H = n2/2 + w to be non-negative); TS = 18 - w, so that the box
// of (TS + w - 1)^3 = 17^3 grid values covering every stencil of a tile
// fills 78.6 KB of LDS.  A block stages the box (periodic indices, rows along
// z), then its threads interpolate the tile's targets from LDS.  Tiles with
// many targets are cut into several work items, one block each.
//
// LDS banks: in 16-byte units a box element sits at x 17^2 + y 17 + z, which
// is x + y + z mod 16, so at every step of the stencil loop a lane reads the
// bank class of its stencil origin plus a step offset common to all lanes.
// Lanes whose origins share a class mod 16 (mod 8 for 128-byte LDS cycles)
// conflict, while lanes with the same origin read the same addresses (a
// broadcast).  Within a tile the targets are therefore ordered round-robin
// over the 16 classes (one target of each class in turn), each class in the
// order of its origins, so that 16 consecutive threads hold different
// classes or, where a tile has few classes, mostly the same origins.
template <int W> constexpr int interp_tile() { return 18 - W > 2 ? 18 - W : 2; }

__device__ __forceinline__ int wrap_index(int m, int n)
{
    m %= n;
    return m < 0 ? m + n : m;
}

// tile key of every target's stencil origin, with its index, and the
// origin's place in its tile (b_x TS^2 + b_y TS + b_z) times 16 plus its LDS
// bank class (lo_x + lo_y + lo_z) mod 16 (see k_interp)
__global__ __launch_bounds__(256) void k_target_tiles(const double *__restrict__ dirs, const double *__restrict__ radii,
                                                      int n_rad, int64_t N, double scale, int w, int H, int TS,
                                                      int nt1, int *__restrict__ keys, int *__restrict__ idx,
                                                      int *__restrict__ bank)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int64_t d = k / n_rad;
    const double r = radii[k - d * n_rad];
    int key = 0, sum = 0, place = 0;
    for (int a = 0; a < 3; ++a) {
        const double u = r * dirs[3 * d + a] * scale;
        const int lo = (int)ceil(u - 0.5 * w);
        int c = (lo + H) / TS;
        c = c < 0 ? 0 : (c >= nt1 ? nt1 - 1 : c);
        key = key * nt1 + c;
        sum += lo;
        const int b = lo + H - c * TS;
        place = place * TS + (b < 0 ? 0 : (b >= TS ? TS - 1 : b));
    }
    keys[k] = key;
    idx[k] = (int)k;
    bank[k] = (place << 4) | (sum & 15);
}

template <int W>
__global__ __launch_bounds__(256) void k_interp(const double2 *__restrict__ fine, int n2, const double *__restrict__ dirs,
                                                const double *__restrict__ radii, int n_rad, double h1, double beta,
                                                const double *__restrict__ phi_inv, const int *__restrict__ order,
                                                const int4 *__restrict__ items, int H, int nt1,
                                                double2 *__restrict__ out)
{
    constexpr int TS = interp_tile<W>(), B = TS + W - 1, B3 = B * B * B;
    __shared__ double2 box[B3];
    __shared__ int wrapped[3][B];        // periodic grid index of each box coordinate
    const int4 it = items[blockIdx.x];   // (tile, first target, end, 0) in the sorted order
    const int tile = it.x;
    const int o[3] = {(tile / (nt1 * nt1)) * TS - H, ((tile / nt1) % nt1) * TS - H, (tile % nt1) * TS - H};
    if (threadIdx.x < 3 * B) {
        const int a = threadIdx.x / B, bb = threadIdx.x - a * B;
        wrapped[a][bb] = wrap_index(o[a] + bb, n2);
    }
    __syncthreads();
    // stage the box: batches of 8 independent reads per thread issued before
    // their LDS writes; past the end a thread reads the box's last element
    // again and writes that same value back to its own slot (no branches)
    constexpr int kBatch = 8;
    for (int e0 = threadIdx.x; e0 < B3; e0 += kBatch * (int)blockDim.x) {
        double2 v[kBatch];
        int slot[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int e = min(e0 + u * (int)blockDim.x, B3 - 1);
            const int bz = e % B, by = (e / B) % B, bx = e / (B * B);
            slot[u] = e;
            v[u] = fine[((int64_t)wrapped[0][bx] * n2 + wrapped[1][by]) * n2 + wrapped[2][bz]];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) box[slot[u]] = v[u];
    }
    __syncthreads();
    const double half_w = 0.5 * W;
    const double iw = 1.0 / half_w;
    const double scale = (double)n2 * h1 / (2.0 * kPi);
    const double n2d = (double)n2;
    const double fscale = h1 * h1 * h1 / (n2d * n2d * n2d);
    for (int t = it.y + (int)threadIdx.x; t < it.z; t += blockDim.x) {
        const int k = order[t];
        const int d = k / n_rad;
        const double r = radii[k - d * n_rad];
        // kernel weights per axis in registers (all loops over them unrolled:
        // an array indexed by a loop counter would live in scratch memory)
        double wx[W], wy[W], wz[W];
        int b[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double u = r * dirs[3 * d + a] * scale;
            const int lo = (int)ceil(u - half_w);
            // in [0, TS) by the tile choice (|u| <= n2 / (2 sigma)); the clamp
            // only keeps every LDS read inside the box
            const int bb = lo - o[a];
            b[a] = bb < 0 ? 0 : (bb > TS - 1 ? TS - 1 : bb);
            double *wa = a == 0 ? wx : (a == 1 ? wy : wz);
#pragma unroll
            for (int i = 0; i < W; ++i) wa[i] = es_eval(((double)(lo + i) - u) * iw, beta);
        }
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
#pragma unroll
            for (int j = 0; j < W; ++j) {
                const double wxy = wx[i] * wy[j];
                const double2 *row = box + ((b[0] + i) * B + (b[1] + j)) * B + b[2];
                double sre = 0.0, sim = 0.0;
#pragma unroll
                for (int l = 0; l < W; ++l) {
                    const double2 v = row[l];
                    sre = __builtin_fma(v.x, wz[l], sre);
                    sim = __builtin_fma(v.y, wz[l], sim);
                }
                re = __builtin_fma(sre, wxy, re);
                im = __builtin_fma(sim, wxy, im);
            }
        }
        const double f = fscale * phi_inv[k];
        out[k] = make_double2(re * f, im * f);
    }
}

// 1 / Phi^(xi_k) per node, Phi^(xi) = prod_a (w h1 / 2) 2 sum_q wpsi_q
// cos(xi_a (w h1 / 2) z_q) (Gauss-Legendre quadrature of psi's transform).
__global__ __launch_bounds__(256) void k_phi_inv(const double *__restrict__ dirs, const double *__restrict__ radii,
                                                 int n_rad, int64_t N, double h1, int w,
                                                 const double2 *__restrict__ ftq, int nq, double *__restrict__ phi_inv)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int64_t d = k / n_rad;
    const int ir = (int)(k - d * n_rad);
    const double r = radii[ir];
    double phi = 1.0;
    const double hw = 0.5 * w * h1;
    for (int a = 0; a < 3; ++a) {
        const double xa = r * dirs[3 * d + a];
        double s = 0.0;
        for (int q = 0; q < nq; ++q) s += ftq[q].y * sincos64(xa * hw * ftq[q].x).c;
        phi *= hw * 2.0 * s;
    }
    phi_inv[k] = 1.0 / phi;
}

// --------------------------------------------------------------------------
// 4'. type 1 (lattice targets): read the transformed grid at the lattice
//     index of each node and divide by the kernel's transform
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_lattice_out(const double2 *__restrict__ fine, int n,
                                                     const double *__restrict__ nodes, int64_t N, double inv_h,
                                                     int M, const double *__restrict__ dec, double2 *__restrict__ out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    int64_t idx = 0;
    double f = 1.0;
    for (int a = 0; a < 3; ++a) {
        int k = (int)__builtin_rint(nodes[3 * q + a] * inv_h);
        k = k < -M / 2 ? -M / 2 : (k > M / 2 ? M / 2 : k);
        f *= dec[k + M / 2];
        idx = idx * n + (k < 0 ? k + n : k);
    }
    const double2 v = fine[idx];
    out[q] = make_double2(v.x * f, v.y * f);
}

// --------------------------------------------------------------------------
// host driver
// --------------------------------------------------------------------------
static void tri_rule_table(int kind, std::vector<double4> &tab)
{
    tab.clear();
    if (kind == HSD_TRI_GL8X8) {
        // 8 x 8 Gauss-Legendre applied twice (iterated integral): u1 = (1+x)/2,
        // u2 = (1 - u1)(1 + y)/2, weight w_x w_y (1 - u1)/4, times 2 so the
        // weights sum to 1 (the area ratio of the standard triangle is 1/2)
        double x[8], wx[8];
        const double pi = 3.14159265358979323846;
        for (int i = 0; i < 4; ++i) {
            double z = std::cos(pi * (i + 0.75) / 8.5);
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= 8; ++k) { double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k; p0 = p1; p1 = pk; }
                const double dp = 8.0 * (z * p1 - p0) / (z * z - 1.0);
                const double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-17) break;
            }
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= 8; ++k) { double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k; p0 = p1; p1 = pk; }
            const double dp = 8.0 * (z * p1 - p0) / (z * z - 1.0);
            x[7 - i] = z; x[i] = -z;
            wx[7 - i] = wx[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
        for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 8; ++j) {
                const double a = 0.5 * (x[i] + 1.0);
                const double b = (1.0 - a) * 0.5 * (x[j] + 1.0);
                tab.push_back(make_double4(1.0 - a - b, a, b, wx[i] * wx[j] * (1.0 - a) * 0.5));
            }
    } else {
        // seven-point degree-5 symmetric rule (Radon): centroid and two orbits
        const double s15 = std::sqrt(15.0);
        const double al = (6.0 - s15) / 21.0, be = (6.0 + s15) / 21.0;
        const double wa = (155.0 - s15) / 1200.0, wb = (155.0 + s15) / 1200.0;
        tab.push_back(make_double4(1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 9.0 / 40.0));
        const double o[2] = {al, be}, ow[2] = {wa, wb};
        for (int k = 0; k < 2; ++k) {
            const double a = o[k], c = 1.0 - 2.0 * o[k];
            tab.push_back(make_double4(a, a, c, ow[k]));
            tab.push_back(make_double4(a, c, a, ow[k]));
            tab.push_back(make_double4(c, a, a, ow[k]));
        }
    }
}

// psi^ quadrature nodes on [0, 1]: (z_q, w_q psi(z_q)).
static void es_ft_table(double beta, int q, std::vector<double2> &tab)
{
    std::vector<double> x(q), wx(q);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (q + 1) / 2; ++i) {
        double z = std::cos(pi * (i + 0.75) / (q + 0.5)), p0, p1, dp;
        for (int it = 0; it < 100; ++it) {
            p0 = 1.0; p1 = z;
            for (int k = 2; k <= q; ++k) { double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k; p0 = p1; p1 = pk; }
            dp = q * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        p0 = 1.0; p1 = z;
        for (int k = 2; k <= q; ++k) { double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k; p0 = p1; p1 = pk; }
        dp = q * (z * p1 - p0) / (z * z - 1.0);
        x[q - 1 - i] = z; x[i] = -z;
        wx[q - 1 - i] = wx[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    tab.resize(q);
    for (int i = 0; i < q; ++i) {
        const double z = 0.5 * (x[i] + 1.0);
        tab[i] = make_double2(z, 0.5 * wx[i] * es_eval(z, beta));
    }
}

static double es_ft_host(const std::vector<double2> &tab, double k)
{
    double s = 0.0;
    for (const auto &t : tab) s += t.y * std::cos(k * t.x);
    return 2.0 * s;
}

NufftScratch::NufftScratch() = default;
NufftScratch::~NufftScratch()
{
    for (hipEvent_t &e : ev)
        if (e) (void)hipEventDestroy(e);
}

size_t NufftScratch::bytes() const
{
    size_t b = 0;
    for (const DevBuf *x : {&pts, &spts, &keys, &keys2, &iota, &offs, &perm, &sorttmp, &grid1, &fine, &tri, &ftq,
                            &hinv, &titems, &tstart, &itile, &tilebuf, &scantmp, &heavy})
        b += x->bytes;
    if (plan) b += plan->tw.bytes + plan->plan.bytes;
    return b;
}

void NufftScratch::release()
{
    tab_key.clear();
    for (DevBuf *x : {&pts, &spts, &keys, &keys2, &iota, &offs, &perm, &sorttmp, &grid1, &fine, &tri, &ftq, &hinv,
                      &titems, &tstart, &itile, &tilebuf, &scantmp, &heavy})
        x->release();
    plan.reset();
}

// Grid sizes of one transform: kernel width and shape, source spacing,
// spread grid n1^3 and FFT grid n2^3 (type 3), or one grid of n1 = n2
// points per axis with the lattice read-out (type 1).
struct NufftSizes {
    bool lattice = false;
    int w = 0, n1 = 0, n2 = 0;
    double sigma = 2.0, beta = 0.0, h1 = 0.0;
};

static hsd_status nufft_sizes(double X, const hsd_rule *rule, const hsd_params *p, NufftSizes &z)
{
    const double sigma = p->nufft_sigma > 1.0 ? p->nufft_sigma : 2.0;
    int w = p->nufft_width;
    if (w <= 0) w = (int)std::ceil(std::log10(1.0 / std::max(p->nufft_tol, 1e-16))) + 1;
    w = std::max(2, std::min(w, kMaxW));
    const double beta = 0.97 * kPi * (1.0 - 0.5 / sigma) * w;
    X = std::max(X, 1e-3);
    const bool sp = rule->kind == HSD_RULE_SPHERICAL_PRODUCT;
    const double S = std::max(sp ? rule->sp.r_max : rule->extent, 1e-3);
    // Lattice targets (cube trapezoid rule, xi = h_xi k): type 1.  The sources
    // scaled to t = h_xi x must lie inside (-pi, pi) with the kernel's support
    // on a grid of n >= sigma (M+1) points per axis; then one grid serves as
    // spread grid and FFT grid, and the transform is read at the lattice
    // indices (no interpolation stage).  Otherwise (or if they do not fit):
    // type 3 as described above.
    bool lattice = false;
    int nl = 0;
    if (rule->kind == HSD_RULE_CUBE_TRAPEZOID && rule->cube_M > 0) {
        nl = 2 * fft_next_size((int)std::ceil(0.5 * sigma * (rule->cube_M + 1)));
        lattice = fft_size_ok(nl) && nl <= 2048 &&
                  X * nl * rule->cube_h / (2.0 * kPi) + 0.5 * w + 2.0 <= 0.5 * nl;
    }
    const double h1 = lattice ? 2.0 * kPi / (nl * rule->cube_h) : kPi / (sigma * S);
    int n1 = lattice ? nl : (int)std::ceil(2.0 * X / h1 + w + 2);
    n1 += n1 & 1;
    const int n2 = lattice ? nl : fft_next_size((int)std::ceil(sigma * n1));
    if (!fft_size_ok(n2) || n2 > 2048) {
        set_error("NUFFT grid %d^3 exceeds the supported FFT size (2048)", n2);
        return HSD_EINVAL;
    }
    z.lattice = lattice;
    z.w = w;
    z.n1 = n1;
    z.n2 = n2;
    z.sigma = sigma;
    z.beta = beta;
    z.h1 = h1;
    return HSD_OK;
}

static int64_t spread_items_bound(int64_t np, int nbins)
{
    return nbins + (27 * ((np + kChunk - 1) / kChunk + (int64_t)nbins) + kItemChunks - 1) / kItemChunks;
}

int64_t nufft_footprint(double X, const hsd_rule *rule, const hsd_params *p, int64_t ntri)
{
    NufftSizes z;
    if (nufft_sizes(X, rule, p, z) != HSD_OK) return -1;
    const int64_t nq = p->tri_rule == HSD_TRI_GL8X8 ? 64 : 7;
    const int64_t np = ntri * nq;
    const int64_t nbx = (z.n1 + kBin - 1) / kBin, nbins = nbx * nbx * nbx;
    const int64_t items = spread_items_bound(np, (int)nbins);
    const int64_t N = rule->n_nodes;
    int64_t b = np * (32 + 32 + 4 * 4)                        // points (raw, sorted), keys, iota, permutation
                + 2 * np * 4 + 2 * (nbins + 1) * 4 + (1 << 20)   // sort and scan temporaries (bounded)
                + (nbins + 1) * 4 * 4 + items * 4
                + items * (int64_t)kBin * kBin * kBin * 8        // partial tiles
                + (int64_t)z.n1 * z.n1 * z.n1 * 8                 // spread grid
                + (int64_t)z.n2 * z.n2 * z.n2 * 16                // FFT grid
                + (int64_t)z.n2 * 16 + 4096 + 64 * 32             // twiddles, stages, small tables
                + (z.lattice ? 0 : N * 40);                       // the rule's per-node tables (first use)
    return b;
}

hsd_status nufft_transform_rule(hsd_ctx *ctx, hipStream_t st, NufftScratch &sc, const hsd_mesh *mu,
                                const hsd_mesh *nu, const hsd_rule *rule, const hsd_params *p, double2 *out,
                                double *pairs)
{
    hsd_status stt;
    // extent of the sources (computed once, when the meshes were created)
    double X = 0.0;
    for (const hsd_mesh *m : {mu, nu})
        if (m) X = std::max(X, m->extent);
    X = std::max(X, 1e-3);
    NufftSizes z;
    if ((stt = nufft_sizes(X, rule, p, z)) != HSD_OK) return stt;
    const bool lattice = z.lattice;
    const int w = z.w, n1 = z.n1, n2 = z.n2;
    const double beta = z.beta, h1 = z.h1;
    const bool sp = rule->kind == HSD_RULE_SPHERICAL_PRODUCT;
    const double S = std::max(sp ? rule->sp.r_max : rule->extent, 1e-3);   // target extent per axis
    const int nbx = (n1 + kBin - 1) / kBin;
    const int nbins = nbx * nbx * nbx;
    const int64_t ntri = mu->nt + (nu ? nu->nt : 0);
    const int64_t N = rule->n_nodes;
    // grow-only scratch: a reallocation frees first, and hipFree waits for
    // the whole device (other serving slots included)
    auto ens = [&](DevBuf &b, size_t bytes) -> hsd_status {
        if (b.ptr && b.bytes >= bytes) return HSD_OK;
        return b.alloc(ctx, std::max<size_t>(bytes, 8));
    };
    // The small tables (triangle rule, kernel transform, deconvolution)
    // depend only on these parameters; they are rebuilt on the host and
    // uploaded only when the parameters change (the host work and the
    // pageable copies would otherwise hold up the stream on every call).
    const std::vector<double> key = {(double)p->tri_rule, (double)w, beta, (double)n1, (double)n2,
                                     lattice ? 1.0 : 0.0, lattice ? (double)rule->cube_M : 0.0};
    if (key != sc.tab_key || !sc.tri.ptr) {
        std::vector<double4> trule;
        tri_rule_table(p->tri_rule, trule);
        // kernel-transform tables
        std::vector<double2> ftq;
        es_ft_table(beta, 4 * w + 24, ftq);
        std::vector<double> hinv(n1, 1.0), dec;
        if (!lattice) {
            for (int l = 0; l < n1; ++l) {
                const int lp = l - n1 / 2;
                // H^_l = (1/2pi) int h(t) e^{-ilt} dt with h(t) = psi(t n2 / (pi w))
                const double Hl = (double)w / (2.0 * n2) * es_ft_host(ftq, lp * w * kPi / n2);
                hinv[l] = 1.0 / Hl;
            }
        } else {
            // spreading with phi(t) = psi(t n / (pi w)) on spacing 2 pi / n gives
            // sum_l b_l e^{-ik t_l} = (n / 2 pi)^3 prod phi^(k_a) sum_j c_j e^{-ik.t_j},
            // phi^(k) = (pi w / n) int_{-1}^{1} psi(z) e^{-i k (pi w / n) z} dz
            const int M = rule->cube_M;
            dec.resize((size_t)M + 1);
            for (int k = -M / 2; k <= M / 2; ++k)
                dec[(size_t)(k + M / 2)] = 2.0 / ((double)w * es_ft_host(ftq, k * kPi * w / n1));
        }
        if ((stt = ens(sc.tri, trule.size() * sizeof(double4))) != HSD_OK) return stt;
        if ((stt = ens(sc.ftq, ftq.size() * sizeof(double2))) != HSD_OK) return stt;
        if ((stt = ens(sc.hinv, (hinv.size() + dec.size()) * sizeof(double))) != HSD_OK) return stt;
        HSD_HIP_TRY(hipMemcpyAsync(sc.tri.ptr, trule.data(), trule.size() * sizeof(double4), hipMemcpyHostToDevice,
                                   st));
        HSD_HIP_TRY(hipMemcpyAsync(sc.ftq.ptr, ftq.data(), ftq.size() * sizeof(double2), hipMemcpyHostToDevice, st));
        HSD_HIP_TRY(hipMemcpyAsync(sc.hinv.ptr, hinv.data(), hinv.size() * sizeof(double), hipMemcpyHostToDevice,
                                   st));
        if (!dec.empty())
            HSD_HIP_TRY(hipMemcpyAsync(sc.hinv.as<double>() + hinv.size(), dec.data(), dec.size() * sizeof(double),
                                       hipMemcpyHostToDevice, st));
        sc.tab_key = key;
        sc.nq = (int)trule.size();
        sc.nftq = (int)ftq.size();
        sc.nhinv = (int)hinv.size();
    }
    const int nq = sc.nq;
    const int64_t np = ntri * nq;
    if ((stt = ens(sc.pts, (size_t)np * sizeof(double4))) != HSD_OK) return stt;
    if ((stt = ens(sc.spts, (size_t)np * sizeof(double4))) != HSD_OK) return stt;
    if ((stt = ens(sc.keys, (size_t)np * sizeof(int))) != HSD_OK) return stt;
    if ((stt = ens(sc.keys2, (size_t)np * sizeof(int))) != HSD_OK) return stt;
    if ((stt = ens(sc.iota, (size_t)np * sizeof(int))) != HSD_OK) return stt;
    if ((stt = ens(sc.perm, (size_t)np * sizeof(int))) != HSD_OK) return stt;
    int key_bits = 1;
    while ((1 << key_bits) < nbins) ++key_bits;
    size_t sort_bytes = 0;
    HSD_HIP_TRY(rocprim::radix_sort_pairs(nullptr, sort_bytes, sc.keys.as<int>(), sc.keys2.as<int>(),
                                          sc.iota.as<int>(), sc.perm.as<int>(), (unsigned int)np, 0, key_bits,
                                          st));
    if ((stt = ens(sc.sorttmp, sort_bytes)) != HSD_OK) return stt;
    if ((stt = ens(sc.offs, ((size_t)nbins + 1) * sizeof(int))) != HSD_OK) return stt;
    // spread work items: at most ntiles + 27 (np / 64 + nbins) / kItemChunks
    // (each tile scans 27 bins of ceil(count / 64) chunks), a bound known
    // without reading anything back
    const int ntiles = nbins;
    const int64_t max_items = spread_items_bound(np, nbins);
    if (max_items > INT32_MAX) {
        set_error("NUFFT: too many spread work items");
        return HSD_EINVAL;
    }
    size_t scan_bytes = 0;
    HSD_HIP_TRY(rocprim::exclusive_scan(nullptr, scan_bytes, sc.titems.as<const int>(), sc.tstart.as<int>(), 0,
                                        (size_t)ntiles + 1, rocprim::plus<int>(), st));
    if ((stt = ens(sc.scantmp, scan_bytes)) != HSD_OK) return stt;
    if ((stt = ens(sc.titems, ((size_t)ntiles + 1) * sizeof(int))) != HSD_OK) return stt;
    if ((stt = ens(sc.heavy, ((size_t)ntiles + 1) * sizeof(int))) != HSD_OK) return stt;
    if ((stt = ens(sc.tstart, ((size_t)ntiles + 1) * sizeof(int))) != HSD_OK) return stt;
    if ((stt = ens(sc.itile, (size_t)max_items * sizeof(int))) != HSD_OK) return stt;
    if ((stt = ens(sc.tilebuf, (size_t)max_items * kBin * kBin * kBin * sizeof(double))) != HSD_OK) return stt;
    if ((stt = ens(sc.grid1, (size_t)n1 * n1 * n1 * sizeof(double))) != HSD_OK) return stt;
    if ((stt = ens(sc.fine, (size_t)n2 * n2 * n2 * sizeof(double2))) != HSD_OK) return stt;
    if (!sc.plan || sc.plan->n != n2) {
        sc.plan.reset(new FftPlan());
        if ((stt = sc.plan->init(ctx, n2)) != HSD_OK) return stt;
    }
    const FftPlan &plan = *sc.plan;

    const TriRec *A = mu->tris.as<const TriRec>();
    const TriRec *B = nu ? nu->tris.as<const TriRec>() : nullptr;
    const int64_t nB = nu ? nu->nt : 0;
    // stage boundaries (events only when the context records stage times):
    // 0 points, sort and bins | 1 spread | 2 pre-deconvolution | 3 FFT |
    // 4 read-out
    sc.timed = ctx->stage_timing;
    auto mark = [&](int i) -> hsd_status {
        if (!sc.timed) return HSD_OK;
        if (!sc.ev[i]) HSD_HIP_TRY(hipEventCreate(&sc.ev[i]));
        HSD_HIP_TRY(hipEventRecord(sc.ev[i], st));
        return HSD_OK;
    };
    if ((stt = mark(0)) != HSD_OK) return stt;
    if (np > 0) {
        const unsigned g = (unsigned)((np + 255) / 256);
        hipLaunchKernelGGL(k_nufft_points, dim3(g), dim3(256), 0, st, A, mu->nt, B, nB, sc.tri.as<const double4>(), nq,
                           h1, n1, nbx, sc.pts.as<double4>(), sc.keys.as<int>());
        HSD_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_iota, dim3(g), dim3(256), 0, st, sc.iota.as<int>(), np);
        HSD_HIP_TRY(hipGetLastError());
        HSD_HIP_TRY(rocprim::radix_sort_pairs(sc.sorttmp.ptr, sort_bytes, sc.keys.as<int>(), sc.keys2.as<int>(),
                                              sc.iota.as<int>(), sc.perm.as<int>(), (unsigned int)np, 0, key_bits,
                                              st));
        hipLaunchKernelGGL(k_gather_points, dim3(g), dim3(256), 0, st, sc.pts.as<const double4>(),
                           sc.perm.as<const int>(), np, sc.spts.as<double4>());
        HSD_HIP_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_bin_offsets, dim3((unsigned)(((int64_t)nbins + 1 + 255) / 256)), dim3(256), 0, st,
                       sc.keys2.as<const int>(), np, nbins, sc.offs.as<int>());
    HSD_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_tile_items, dim3((unsigned)((ntiles + 1 + 255) / 256)), dim3(256), 0, st,
                       sc.offs.as<const int>(), nbx, sc.titems.as<int>(), sc.heavy.as<int>());
    HSD_HIP_TRY(hipGetLastError());
    HSD_HIP_TRY(rocprim::exclusive_scan(sc.scantmp.ptr, scan_bytes, sc.titems.as<const int>(), sc.tstart.as<int>(), 0,
                                        (size_t)ntiles + 1, rocprim::plus<int>(), st));
    hipLaunchKernelGGL(k_item_map, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, st,
                       sc.tstart.as<const int>(), ntiles, sc.itile.as<int>(), sc.heavy.as<int>());
    HSD_HIP_TRY(hipGetLastError());
    if ((stt = mark(1)) != HSD_OK) return stt;
    hipLaunchKernelGGL(k_spread, dim3((unsigned)max_items), dim3(64), 0, st, sc.spts.as<const double4>(),
                       sc.offs.as<const int>(), sc.tstart.as<const int>(), sc.itile.as<const int>(), nbx, n1, h1,
                       0.5 * w, beta, sc.grid1.as<double>(), sc.tilebuf.as<double>());
    HSD_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_tile_reduce, dim3((unsigned)std::min<int64_t>(ntiles, 2048)), dim3(64 * kReduceWaves), 0, st,
                       sc.tilebuf.as<const double>(), sc.tstart.as<const int>(), sc.heavy.as<const int>(), nbx, n1,
                       sc.grid1.as<double>());
    HSD_HIP_TRY(hipGetLastError());
    if ((stt = mark(2)) != HSD_OK) return stt;
    // the spread grid is zero beyond |l - n1/2| > X / h1 + w / 2 (all points
    // lie within X of the origin), so the fine grid is zero outside the
    // wrapped indices m < e, m >= n2 - e: only that band is written, and the
    // FFT skips the other lines and reads each line only in the band
    const int e_occ = std::min(n1 / 2, (int)std::floor(X / h1 + 0.5 * w) + 2);
    {
        // the band convention of fft3d_forward: e <= 0 or 2 e >= n2 is the whole axis
        const bool band = e_occ > 0 && 2 * e_occ < n2;
        const int cnt = band ? 2 * e_occ : n2;
        const int e = band ? e_occ : n2, gap = n2 - cnt;
        const int64_t tot = (int64_t)cnt * cnt * cnt;
        hipLaunchKernelGGL(k_predeconv, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                           sc.grid1.as<const double>(), n1, sc.hinv.as<const double>(), n2, cnt, e, gap,
                           sc.fine.as<double2>());
        HSD_HIP_TRY(hipGetLastError());
        sc.stage_bytes[2] = (double)tot * (8.0 + 16.0);
    }
    if ((stt = mark(3)) != HSD_OK) return stt;
    // and only the indices the read-out touches are wanted: the lattice
    // indices |k| <= M / 2, or the interpolation stencils around the scaled
    // targets |u| <= S n2 h1 / (2 pi) (w points from ceil(u - w/2))
    const int e_want = lattice ? rule->cube_M / 2 + 2
                               : std::min(n2 / 2, (int)std::floor(S * n2 * h1 / (2.0 * kPi) + 0.5 * w) + 2);
    if ((stt = fft3d_forward(st, plan, sc.fine.as<double2>(), e_occ, e_want)) != HSD_OK) return stt;
    if ((stt = mark(4)) != HSD_OK) return stt;
    // algorithmic bytes: triangle records read, points and keys written,
    // sorted (keys and values in and out) and gathered | sorted points read,
    // spread grid written | (above) | the FFT passes' band reads and writes |
    // the wanted band read once, one value written per target (plus its
    // node and deconvolution factor for the ball rules)
    sc.stage_bytes[0] = (double)(mu->nt + nB) * sizeof(TriRec) + (double)np * (32.0 + 8.0 + 16.0 + 68.0);
    sc.stage_bytes[1] = (double)np * 32.0 + (double)n1 * n1 * n1 * 8.0;
    sc.stage_bytes[3] = fft3d_bytes(n2, e_occ, e_want);
    {
        const double ew = (e_want > 0 && 2 * e_want < n2) ? 2.0 * e_want : (double)n2;
        sc.stage_bytes[4] = ew * ew * ew * 16.0 + (double)N * (lattice ? 16.0 + 16.0 : 16.0 + 8.0 + 4.0);
    }
    if (lattice) {
        hipLaunchKernelGGL(k_lattice_out, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                           sc.fine.as<const double2>(), n2, rule->d_nodes.as<const double>(), N, 1.0 / rule->cube_h,
                           rule->cube_M, sc.hinv.as<const double>() + sc.nhinv, out);
        HSD_HIP_TRY(hipGetLastError());
        if ((stt = mark(5)) != HSD_OK) return stt;
        if (pairs) *pairs = (double)np;
        return HSD_OK;
    }
    const double *dirs = sp ? rule->d_dirs.as<const double>() : rule->d_nodes.as<const double>();
    const int n_rad = sp ? (int)rule->n_rad : 1;
    // interpolation tiles: TS^3 stencil origins per tile, nt1 tiles per axis
    // over the shifted origins lo + H in [0, n2 + w + 2)
    const int TS = std::max(18 - w, 2);
    const int H = n2 / 2 + w;
    const int nt1 = (n2 + 2 * w + TS) / TS;
    if ((int64_t)nt1 * nt1 * nt1 > INT32_MAX || N > INT32_MAX) {
        set_error("NUFFT: too many nodes or interpolation tiles");
        return HSD_EINVAL;
    }
    const double *phi_inv = nullptr;
    const int *order = nullptr;
    const int4 *items = nullptr;
    int nitems = 0;
    {
        hsd_rule *rm = const_cast<hsd_rule *>(rule);
        std::lock_guard<std::mutex> lk(rm->mu);
        for (const auto &e : rm->nufft_deconv)
            if (e->w == w && e->beta == beta && e->h1 == h1 && e->n2 == n2) {
                phi_inv = e->inv.as<const double>();
                order = e->order.as<const int>();
                items = e->items.as<const int4>();
                nitems = e->nitems;
            }
        if (!phi_inv && N > 0) {
            std::unique_ptr<hsd_rule::NufftDeconv> e(new hsd_rule::NufftDeconv());
            e->w = w;
            e->beta = beta;
            e->h1 = h1;
            e->n2 = n2;
            const dim3 ng((unsigned)((N + 255) / 256)), nb(256);
            if ((stt = e->inv.alloc(ctx, (size_t)N * sizeof(double))) != HSD_OK) return stt;
            hipLaunchKernelGGL(k_phi_inv, ng, nb, 0, st, dirs, rule->d_radii.as<const double>(), n_rad, N, h1, w,
                               sc.ftq.as<const double2>(), sc.nftq, e->inv.as<double>());
            HSD_HIP_TRY(hipGetLastError());
            // targets grouped by interpolation tile (stable sort: ascending
            // node index within a tile), then cut into work items
            DevBuf keys, keys2, idx, tmp, bank;
            if ((stt = keys.alloc(ctx, (size_t)N * sizeof(int))) != HSD_OK) return stt;
            if ((stt = bank.alloc(ctx, (size_t)N * sizeof(int))) != HSD_OK) return stt;
            if ((stt = keys2.alloc(ctx, (size_t)N * sizeof(int))) != HSD_OK) return stt;
            if ((stt = idx.alloc(ctx, (size_t)N * sizeof(int))) != HSD_OK) return stt;
            if ((stt = e->order.alloc(ctx, (size_t)N * sizeof(int))) != HSD_OK) return stt;
            hipLaunchKernelGGL(k_target_tiles, ng, nb, 0, st, dirs, rule->d_radii.as<const double>(), n_rad, N,
                               (double)n2 * h1 / (2.0 * kPi), w, H, TS, nt1, keys.as<int>(), idx.as<int>(),
                               bank.as<int>());
            HSD_HIP_TRY(hipGetLastError());
            int key_bits = 1;
            while (((int64_t)1 << key_bits) < (int64_t)nt1 * nt1 * nt1) ++key_bits;
            size_t tmp_bytes = 0;
            HSD_HIP_TRY(rocprim::radix_sort_pairs(nullptr, tmp_bytes, keys.as<int>(), keys2.as<int>(), idx.as<int>(),
                                                  e->order.as<int>(), (unsigned int)N, 0, key_bits, st));
            if ((stt = tmp.alloc(ctx, std::max<size_t>(tmp_bytes, 8))) != HSD_OK) return stt;
            HSD_HIP_TRY(rocprim::radix_sort_pairs(tmp.ptr, tmp_bytes, keys.as<int>(), keys2.as<int>(), idx.as<int>(),
                                                  e->order.as<int>(), (unsigned int)N, 0, key_bits, st));
            std::vector<int> sk((size_t)N), ord((size_t)N), bk((size_t)N);
            HSD_HIP_TRY(hipMemcpyAsync(sk.data(), keys2.ptr, (size_t)N * sizeof(int), hipMemcpyDeviceToHost, st));
            HSD_HIP_TRY(hipMemcpyAsync(ord.data(), e->order.ptr, (size_t)N * sizeof(int), hipMemcpyDeviceToHost, st));
            HSD_HIP_TRY(hipMemcpyAsync(bk.data(), bank.ptr, (size_t)N * sizeof(int), hipMemcpyDeviceToHost, st));
            HSD_HIP_TRY(hipStreamSynchronize(st));
            // within each tile, targets round-robin over their LDS bank
            // classes, each class ordered by stencil origin (stable), see
            // k_interp
            {
                std::vector<int> seg;
                for (int64_t a = 0; a < N;) {
                    int64_t b = a + 1;
                    while (b < N && sk[(size_t)b] == sk[(size_t)a]) ++b;
                    if (b - a > 1) {
                        int cnt[16] = {}, start[17] = {};
                        for (int64_t q = a; q < b; ++q) ++cnt[bk[(size_t)ord[(size_t)q]] & 15];
                        int mx = 0;
                        for (int c = 0; c < 16; ++c) {
                            start[c + 1] = start[c] + cnt[c];
                            mx = std::max(mx, cnt[c]);
                        }
                        seg.assign((size_t)(b - a), 0);
                        int fill[16];
                        for (int c = 0; c < 16; ++c) fill[c] = start[c];
                        for (int64_t q = a; q < b; ++q) seg[(size_t)fill[bk[(size_t)ord[(size_t)q]] & 15]++] = ord[(size_t)q];
                        for (int c = 0; c < 16; ++c)
                            std::stable_sort(seg.begin() + start[c], seg.begin() + start[c + 1],
                                             [&](int x, int y) { return bk[(size_t)x] < bk[(size_t)y]; });
                        int64_t o = a;
                        for (int rr = 0; rr < mx; ++rr)
                            for (int c = 0; c < 16; ++c)
                                if (rr < cnt[c]) ord[(size_t)o++] = seg[(size_t)(start[c] + rr)];
                    }
                    a = b;
                }
            }
            HSD_HIP_TRY(hipMemcpyAsync(e->order.ptr, ord.data(), (size_t)N * sizeof(int), hipMemcpyHostToDevice, st));
            constexpr int kItemTargets = 1024;   // targets per interpolation work item (at most)
            std::vector<int4> it;
            for (int64_t a = 0; a < N;) {
                int64_t b = a + 1;
                while (b < N && sk[(size_t)b] == sk[(size_t)a]) ++b;
                for (int64_t c = a; c < b; c += kItemTargets)
                    it.push_back(make_int4(sk[(size_t)a], (int)c, (int)std::min<int64_t>(b, c + kItemTargets), 0));
                a = b;
            }
            // largest items first (blocks start roughly in launch order, so
            // the long ones do not form the tail of the launch)
            std::stable_sort(it.begin(), it.end(), [](const int4 &x, const int4 &y) { return x.z - x.y > y.z - y.y; });
            e->nitems = (int)it.size();
            if ((stt = e->items.alloc(ctx, std::max<size_t>(it.size(), 1) * sizeof(int4))) != HSD_OK) return stt;
            if (!it.empty())
                HSD_HIP_TRY(hipMemcpyAsync(e->items.ptr, it.data(), it.size() * sizeof(int4), hipMemcpyHostToDevice, st));
            // complete before other streams (serving slots) may read them and
            // before the temporaries are freed
            HSD_HIP_TRY(hipStreamSynchronize(st));
            phi_inv = e->inv.as<const double>();
            order = e->order.as<const int>();
            items = e->items.as<const int4>();
            nitems = e->nitems;
            rm->nufft_deconv.push_back(std::move(e));
        }
    }
    if (nitems > 0) {
        const dim3 ig((unsigned)nitems), ib(256);
        const double2 *fg = sc.fine.as<const double2>();
        const double *rr = rule->d_radii.as<const double>();
        switch (w) {
#define HSD_INTERP_W(WW)                                                                                     \
    case WW: hipLaunchKernelGGL(k_interp<WW>, ig, ib, 0, st, fg, n2, dirs, rr, n_rad, h1, beta, phi_inv, order, \
                                items, H, nt1, out);                                                       \
        break;
            HSD_INTERP_W(2) HSD_INTERP_W(3) HSD_INTERP_W(4) HSD_INTERP_W(5) HSD_INTERP_W(6) HSD_INTERP_W(7)
            HSD_INTERP_W(8) HSD_INTERP_W(9) HSD_INTERP_W(10) HSD_INTERP_W(11) HSD_INTERP_W(12) HSD_INTERP_W(13)
            HSD_INTERP_W(14) HSD_INTERP_W(15) HSD_INTERP_W(16)
#undef HSD_INTERP_W
        default: set_error("NUFFT width %d unsupported", w); return HSD_EINVAL;
        }
    }
    HSD_HIP_TRY(hipGetLastError());
    if ((stt = mark(5)) != HSD_OK) return stt;
    if (pairs) *pairs = (double)np;
    return HSD_OK;
}

} // namespace hsd
