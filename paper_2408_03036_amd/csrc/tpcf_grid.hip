// Neighbour grid: a counting sort of the points by cell (the linked-list
// spatial partition of Sec. 4.1, laid out as contiguous per-cell ranges so
// the pair pass reads neighbour cells with coalesced loads).
//
// Steps: assign (wrap, cell id, histogram) -> scan (cell starts) ->
// scatter (atomic slots) -> order (rank by z, then input index, inside a
// cell, so the layout is deterministic) -> fill (sorted SoA copies).
#include "tpcf_internal.h"

namespace tpcf {

namespace {

__device__ inline double wrap_coord(double x, double L) {
    double y = fmod(x, L);
    if (y < 0.0) y += L;
    if (y >= L) y -= L;
    return y;
}

__device__ inline int cell_of(double x, const Grid& g) {
    int c = (int)(x * g.inv_h);
    c = c < 0 ? 0 : c;
    return c >= g.nc ? g.nc - 1 : c;
}

__device__ inline int find_cat(const int64_t* off, int ncat, int64_t i) {
    int lo = 0, hi = ncat;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_grid_assign(const double* __restrict__ pos, int64_t n,
                              const int64_t* __restrict__ pt_off, int ncat, Grid g,
                              int* __restrict__ cellid, int* __restrict__ count,
                              int* __restrict__ nonfinite, int* __restrict__ catbad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    int c = find_cat(pt_off, ncat, i);
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
        atomicAdd(nonfinite, 1);
        atomicAdd(&catbad[c], 1);
        x = y = z = 0.0;
    }
    x = wrap_coord(x, g.box);
    y = wrap_coord(y, g.box);
    z = wrap_coord(z, g.box);
    int id = c * g.ncell + (cell_of(x, g) * g.nc + cell_of(y, g)) * g.nc + cell_of(z, g);
    cellid[i] = id;
    atomicAdd(&count[id], 1);
}

// Single-workgroup exclusive scan: each thread scans a contiguous segment.
__global__ void __launch_bounds__(1024) k_grid_scan(const int* __restrict__ count, int64_t m,
                                                    int* __restrict__ start) {
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int64_t seg = (m + 1023) / 1024;
    const int64_t a = t * seg;
    const int64_t b = a + seg < m ? a + seg : m;
    int s = 0;
    for (int64_t i = a; i < b; ++i) s += count[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;
    for (int64_t i = a; i < b; ++i) {
        start[i] = run;
        run += count[i];
    }
    if (t == 1023) start[m] = part[1023];
}

// Three-phase exclusive scan of m counts: per-block sums of kScanBlock
// elements, a scan of the block sums (k_grid_scan), then each block's scan
// plus its offset.
constexpr int kScanBlock = 4096;  // 256 threads x 16 elements

__global__ void __launch_bounds__(256) k_scan_sums(const int* __restrict__ count, int64_t m,
                                                   int* __restrict__ sums) {
    __shared__ int red[256];
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    int s = 0;
    for (int i = threadIdx.x; i < kScanBlock; i += 256) {
        const int64_t e = b0 + i;
        if (e < m) s += count[e];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_scan_apply(const int* __restrict__ count, int64_t m,
                                                    const int* __restrict__ boff, int* __restrict__ start) {
    __shared__ int part[256];
    const int64_t b0 = (int64_t)blockIdx.x * kScanBlock;
    const int t = threadIdx.x;
    // thread t owns elements [b0 + 16 t, b0 + 16 t + 16)
    int v[16];
    int s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int64_t e = b0 + 16 * t + k;
        v[k] = e < m ? count[e] : 0;
        s += v[k];
    }
    part[t] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int x = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    int run = boff[blockIdx.x] + part[t] - s;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int64_t e = b0 + 16 * t + k;
        if (e < m) start[e] = run;
        if (e == m - 1) start[m] = run + v[k];
        run += v[k];
    }
}

__global__ void k_grid_scatter(const int* __restrict__ cellid, int64_t n,
                               const int* __restrict__ start, int* __restrict__ cursor,
                               const double* __restrict__ pos, double box,
                               int* __restrict__ tmp_idx, double* __restrict__ tmp_key) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cellid[i];
    int slot = atomicAdd(&cursor[c], 1);
    // the order key: the wrapped z the fill stores (0 for a non-finite point)
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    const bool fin = isfinite(x) && isfinite(y) && isfinite(z);
    tmp_idx[start[c] + slot] = (int)i;
    tmp_key[start[c] + slot] = wrap_coord(fin ? z : 0.0, box);
}

// Placement inside a cell by z, ties by input index: a point's rank is the
// number of points of its cell that come before it in that order. Along
// every run of cells consecutive in z the points are then in increasing z,
// which lets the pair pass cut a run to the z range a work item can reach.
// The layout is deterministic.
__global__ void k_grid_order(const int* __restrict__ cellid, int64_t n,
                             const int* __restrict__ start, const int* __restrict__ tmp_idx,
                             const double* __restrict__ tmp_key, int* __restrict__ orig) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = tmp_idx[s];
    const double zi = tmp_key[s];
    const int c = cellid[i];
    const int a = start[c], b = start[c + 1];
    int rank = 0;
    for (int t = a; t < b; ++t) {
        const double zt = tmp_key[t];
        rank += zt < zi || (zt == zi && tmp_idx[t] < i);
    }
    orig[a + rank] = i;
}

__global__ void k_grid_fill(const double* __restrict__ pos, const double* __restrict__ w,
                            int64_t n, const int* __restrict__ orig,
                            const int* __restrict__ cellid, Grid g, float4* __restrict__ pf,
                            float* __restrict__ pw, float4* __restrict__ pa, double4* __restrict__ pd,
                            int* __restrict__ perm, int* __restrict__ catid) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int i = orig[s];
    double x = pos[3 * (int64_t)i], y = pos[3 * (int64_t)i + 1], z = pos[3 * (int64_t)i + 2];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) x = y = z = 0.0;
    x = wrap_coord(x, g.box);
    y = wrap_coord(y, g.box);
    z = wrap_coord(z, g.box);
    double wi = w ? w[i] : 1.0;
    int id = cellid[i];
    int cat = id / g.ncell;
    int loc = id - cat * g.ncell;
    int cz = loc % g.nc;
    int cy = (loc / g.nc) % g.nc;
    int cx = loc / (g.nc * g.nc);
    // Offsets from the cell's lower corner; exact in FP64, rounded once to FP32.
    float4 q;
    q.x = (float)(x - cx * g.h);
    q.y = (float)(y - cy * g.h);
    q.z = (float)(z - cz * g.h);
    q.w = (float)cz;
    pf[s] = q;
    pw[s] = (float)wi;
    pa[s] = make_float4(q.x, q.y, q.z, (float)wi);
    pd[s] = make_double4(x, y, z, wi);
    perm[i] = (int)s;
    catid[s] = cat;
}

__global__ void k_fill_i32(int* p, int64_t n, int v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Work items of the binning pass: cell c holds ceil(count / kItemPrims) items.
__global__ void k_items_count(const int* __restrict__ cell_start, int64_t m, int* __restrict__ nitems) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    const int n = cell_start[c + 1] - cell_start[c];
    nitems[c] = (n + kItemPrims - 1) / kItemPrims;
}

__global__ void k_items_fill(const int* __restrict__ item_start, int64_t m, int* __restrict__ item_cell) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    for (int i = item_start[c]; i < item_start[c + 1]; ++i) item_cell[i] = (int)c;
}

__global__ void k_items_cat(const int* __restrict__ item_start, int ncat, int ncell, int* __restrict__ item_cat) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c <= ncat) item_cat[c] = item_start[(int64_t)c * ncell];
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_items_count(const int* cell_start, int64_t m, int* nitems, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_items_count, dim3(nblk(m, 256)), dim3(256), 0, s, cell_start, m, nitems);
    return hipGetLastError();
}

hipError_t launch_items_fill(const int* item_start, int64_t m, int* item_cell, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_items_fill, dim3(nblk(m, 256)), dim3(256), 0, s, item_start, m, item_cell);
    return hipGetLastError();
}

hipError_t launch_items_cat(const int* item_start, int ncat, int ncell, int* item_cat, hipStream_t s) {
    hipLaunchKernelGGL(k_items_cat, dim3(nblk(ncat + 1, 256)), dim3(256), 0, s, item_start, ncat, ncell,
                       item_cat);
    return hipGetLastError();
}

hipError_t launch_grid_assign(const double* pos, const double*, int64_t n, const int64_t* pt_off,
                              int ncat, Grid g, int* cellid, int* count, int* nonfinite, int* catbad,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grid_assign, dim3(nblk(n, 256)), dim3(256), 0, s, pos, n, pt_off, ncat, g,
                       cellid, count, nonfinite, catbad);
    return hipGetLastError();
}

hipError_t launch_grid_scan(const int* count, int64_t m, int* start, int* work, hipStream_t s) {
    const int64_t nb = (m + kScanBlock - 1) / kScanBlock;
    if (nb <= 1) {
        hipLaunchKernelGGL(k_grid_scan, dim3(1), dim3(1024), 0, s, count, m, start);
        return hipGetLastError();
    }
    // work: nb block sums, then nb + 1 block offsets
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(256), 0, s, count, m, work);
    hipLaunchKernelGGL(k_grid_scan, dim3(1), dim3(1024), 0, s, work, nb, work + nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, s, count, m, work + nb, start);
    return hipGetLastError();
}

int64_t grid_scan_work_ints(int64_t m) { return 2 * ((m + kScanBlock - 1) / kScanBlock) + 1; }

hipError_t launch_grid_scatter(const int* cellid, int64_t n, const int* start, int* cursor,
                               const double* pos, double box, int* tmp_idx, double* tmp_key, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grid_scatter, dim3(nblk(n, 256)), dim3(256), 0, s, cellid, n, start,
                       cursor, pos, box, tmp_idx, tmp_key);
    return hipGetLastError();
}

hipError_t launch_grid_order(const int* cellid, int64_t n, const int* start, const int* tmp_idx,
                             const double* tmp_key, int* orig, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grid_order, dim3(nblk(n, 256)), dim3(256), 0, s, cellid, n, start,
                       tmp_idx, tmp_key, orig);
    return hipGetLastError();
}

hipError_t launch_grid_fill(const double* pos, const double* w, int64_t n, const int* orig,
                            const int* cellid, Grid g, float4* pf, float* pw, float4* pa, double4* pd,
                            int* perm, int* catid, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grid_fill, dim3(nblk(n, 256)), dim3(256), 0, s, pos, w, n, orig, cellid,
                       g, pf, pw, pa, pd, perm, catid);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int64_t n, int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(nblk(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace tpcf
