// Covariance of measurements over a suite of mock catalogues (arXiv:2408.03036,
// Sec. 4.3):
//   C_ij = 1/(N_m - 1) sum_k (d_i^k - dbar_i)(d_j^k - dbar_j)          eq. (covariance)
//   C^-1 = (N_m - N_d - 2)/(N_m - 1) C_hat^-1                           eq. (Hartlap)
//
//  k_cov_gather   X[k][i] = src[k * stride + offset[i]] (the data vector of mock k)
//  k_cov_colsum / k_cov_mean / k_cov_center
//                 mean over the mocks (chunks of 64 mocks, then the chunks,
//                 in a fixed order), then X -= mean
//  k_cov_syrk     X^T X on FP64 16x16x4 MFMA, one wavefront per (upper-
//                 triangle 16x16 tile, slice of the mocks)
//  k_cov_reduce   sum of the slices in a fixed order, / (N_m - 1), mirrored
//  k_cov_pivot    one launch per pivot of the Gauss-Jordan sweep of the
//                 symmetric positive definite matrix (positive pivots, no
//                 pivoting), ping-pong between two buffers; k_cov_scale
//                 applies the Hartlap factor. A non-positive pivot sets a flag.
#include <algorithm>
#include <mutex>

#include "tpcf_internal.h"

namespace tpcf {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// An offset outside a row (possible only for offsets given in device memory,
// which the host cannot check) reads nothing and gives NaN.
__global__ void k_cov_gather(const double* __restrict__ src, int64_t stride, const int64_t* __restrict__ off,
                             int nm, int nd, double* __restrict__ X) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nm * nd) return;
    const int k = (int)(t / nd), i = (int)(t % nd);
    const int64_t o = off ? off[i] : (int64_t)i;
    X[t] = (o >= 0 && o < stride) ? src[(int64_t)k * stride + o] : __builtin_nan("");
}

// Column sums over chunks of kMeanChunk mocks (one thread per (chunk, entry)),
// then the chunks in order, then the centring: a fixed summation order.
constexpr int kMeanChunk = 64;

__global__ void k_cov_colsum(const double* __restrict__ X, int nm, int nd, double* __restrict__ psum) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    const int k0 = blockIdx.y * kMeanChunk, k1 = min(nm, k0 + kMeanChunk);
    double s = 0.0;
    for (int k = k0; k < k1; ++k) s += X[(int64_t)k * nd + i];
    psum[(int64_t)blockIdx.y * nd + i] = s;
}

__global__ void k_cov_mean(const double* __restrict__ psum, int nchunk, int nm, int nd, double* __restrict__ mean) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nd) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += psum[(int64_t)c * nd + i];
    mean[i] = s / nm;
}

__global__ void k_cov_center(double* __restrict__ X, int nm, int nd, const double* __restrict__ mean) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nm * nd) return;
    X[t] -= mean[t % nd];
}

constexpr int kCovWaves = 4;

// One wavefront per (upper-triangle 16x16 tile, slice of the mocks): the
// slice's sum of products goes to its own partial, summed over the slices in
// a fixed order by k_cov_reduce.
__global__ void __launch_bounds__(64 * kCovWaves) k_cov_syrk(const double* __restrict__ X, int nm, int nd,
                                                               int kslice, double* __restrict__ part) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nt = (nd + 15) / 16;
    int t = blockIdx.x * kCovWaves + wave;
    if (t >= nt * (nt + 1) / 2) return;
    int ti = 0;
    while (t >= nt - ti) {  // t-th upper-triangle tile, row-major
        t -= nt - ti;
        ++ti;
    }
    const int tj = ti + t;
    const int i = lane & 15, g = lane >> 4;
    const int ca = 16 * ti + i, cb = 16 * tj + i;
    const int k_lo = blockIdx.y * kslice, k_hi = min(nm, k_lo + kslice);
    f64x4 acc = (f64x4)0.0;
    for (int k0 = k_lo; k0 < k_hi; k0 += 4) {
        const int k = k0 + g;
        const double a = (k < k_hi && ca < nd) ? X[(int64_t)k * nd + ca] : 0.0;
        const double b = (k < k_hi && cb < nd) ? X[(int64_t)k * nd + cb] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    double* P = part + (int64_t)blockIdx.y * nd * nd;
    const int j = 16 * tj + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * ti + (lane >> 4) + 4 * r;
        if (row < nd && j < nd && row <= j) P[(int64_t)row * nd + j] = acc[r];
    }
}

// C[i][j] = C[j][i] = (sum over slices, in order) / (N_m - 1), i <= j
__global__ void k_cov_reduce(const double* __restrict__ part, int nslice, int nd, int nm, double* __restrict__ C) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nd * nd) return;
    const int i = (int)(e / nd), j = (int)(e % nd);
    if (i > j) return;
    double s = 0.0;
    for (int q = 0; q < nslice; ++q) s += part[(int64_t)q * nd * nd + e];
    s /= (double)(nm - 1);
    C[e] = s;
    C[(int64_t)j * nd + i] = s;
}

// One Gauss-Jordan pivot of the symmetric positive definite matrix, from A to
// B (ping-pong, so every thread reads the pivot row and column unchanged):
// with p = A[k][k],
//   B[i][j] = A[i][j] - A[i][k] A[k][j] / p  (i, j != k),  B[k][j] = A[k][j] / p,
//   B[i][k] = -A[i][k] / p,  B[k][k] = 1 / p.
// After the pivots 0 .. n-1 the matrix holds the inverse (no pivoting: the
// pivots of a positive definite matrix stay positive). A non-positive pivot
// sets *bad.
__global__ void k_cov_pivot(const double* __restrict__ A, double* __restrict__ B, int n, int k,
                            int* __restrict__ bad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int i = e / n, j = e - i * n;
    const double p = A[k * n + k];
    if (e == 0 && !(p > 0.0)) atomicOr(bad, 1);
    const double ip = 1.0 / p;
    double v;
    if (i == k && j == k) v = ip;
    else if (i == k) v = A[k * n + j] * ip;
    else if (j == k) v = -A[i * n + k] * ip;
    else v = A[e] - A[i * n + k] * A[k * n + j] * ip;
    B[e] = v;
}

__global__ void k_cov_scale(const double* __restrict__ A, double* __restrict__ B, int64_t nn, double scale) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nn) B[e] = A[e] * scale;
}

}  // namespace

// Scratch of the allocation-free covariance (tpcf_covariance_noalloc): the
// gathered data vectors and the partial products, kCovScratchBytes on every
// device the library runs on, held until the process ends. Host code never
// passes the array's name to a kernel or a copy: it is a host-side stand-in
// there. It uses the device address that cov_scratch_init looks up once per
// device.
__device__ __align__(256) static unsigned char scratch[kCovScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

hipError_t cov_scratch_init(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        // the caller has made `device` current
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

int64_t cov_scratch_need(int nm, int nd) {
    return (int64_t)sizeof(double) * ((int64_t)nm * nd + cov_part_doubles(nm, nd));
}

int64_t cov_part_doubles(int nm, int nd) {
    const int64_t prod = (int64_t)cov_slices(nm, nd) * nd * nd;
    const int64_t sums = ((int64_t)(nm + kMeanChunk - 1) / kMeanChunk + 1) * nd;
    return std::max(prod, sums);
}

int cov_slices(int nm, int nd) {
    // enough (tile, slice) wavefronts to fill the chip, slices of at least 64 mocks
    const int nt = (nd + 15) / 16;
    const int ntiles = nt * (nt + 1) / 2;
    int ns = (4096 + ntiles - 1) / ntiles;
    ns = std::min(ns, std::max(1, nm / 64));
    return std::max(1, std::min(ns, 64));
}

hipError_t launch_cov(const double* src, int64_t stride, const int64_t* off, int nm, int nd, double* X,
                      double* part, double* mean, double* C, hipStream_t s) {
    const int64_t ne = (int64_t)nm * nd;
    if (ne <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cov_gather, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, src, stride, off, nm, nd, X);
    // the column sums use the start of `part` (nchunk x nd <= slices x nd x nd) before the products
    const int nchunk = (nm + kMeanChunk - 1) / kMeanChunk;
    double* msum = part;
    double* mu = part + (int64_t)nchunk * nd;
    hipLaunchKernelGGL(k_cov_colsum, dim3((nd + 63) / 64, nchunk), dim3(64), 0, s, X, nm, nd, msum);
    hipLaunchKernelGGL(k_cov_mean, dim3((nd + 255) / 256), dim3(256), 0, s, msum, nchunk, nm, nd, mu);
    if (mean) {
        hipError_t e = hipMemcpyAsync(mean, mu, sizeof(double) * nd, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_cov_center, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, X, nm, nd, mu);
    const int nt = (nd + 15) / 16;
    const int ntiles = nt * (nt + 1) / 2;
    const int ns = cov_slices(nm, nd);
    const int kslice = (nm + ns - 1) / ns;
    hipLaunchKernelGGL(k_cov_syrk, dim3((ntiles + kCovWaves - 1) / kCovWaves, ns), dim3(64 * kCovWaves), 0, s, X,
                       nm, nd, kslice, part);
    const int64_t nn = (int64_t)nd * nd;
    hipLaunchKernelGGL(k_cov_reduce, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, part, ns, nd, nm, C);
    return hipGetLastError();
}

hipError_t launch_cov_invert(double* A, double* W, int n, double scale, int* bad, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t nn = (int64_t)n * n;
    const unsigned nblk = (unsigned)((nn + 255) / 256);
    double* src = A;
    double* dst = W;
    for (int k = 0; k < n; ++k) {
        hipLaunchKernelGGL(k_cov_pivot, dim3(nblk), dim3(256), 0, s, src, dst, n, k, bad);
        std::swap(src, dst);
    }
    hipLaunchKernelGGL(k_cov_scale, dim3(nblk), dim3(256), 0, s, src, A, nn, scale);
    return hipGetLastError();
}

}  // namespace tpcf
