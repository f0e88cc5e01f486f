// Internal declarations shared by the host runtime and the HIP kernels of
// libtpcf. Not part of the public ABI (include/tpcf.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpcf {

constexpr int kMaxBins = 32;
constexpr int kMaxLmax = 16;
constexpr int kMaxRuns = 2 * 81;   // stencil column runs after z-wrap splitting (grid_refine <= 4)
constexpr int kMaxCodes = 729;     // (2k+1)^3 stencil offsets for grid_refine <= 4
constexpr int kWave = 64;

// Number of real accumulator values per (primary, bin): a_lm for m = 0 (real,
// l = 0..lmax), m >= 1 (re and im, l = m..lmax), then the 2 lmax + 1 moments
// of the squared weights sum_j w_j^2 R^0_L(z) for L = 0..2 lmax.
__host__ __device__ constexpr int n_alm_values(int lmax) { return (lmax + 1) * (lmax + 1); }
__host__ __device__ constexpr int n_values(int lmax) { return (lmax + 1) * (lmax + 1) + 2 * lmax + 1; }
// Offset of the first value of order m inside a bin's value vector.
// m = 0 occupies [0, lmax]; m >= 1 occupies 2 (lmax - m + 1) values: re for
// l = m..lmax, then im for l = m..lmax.
__host__ __device__ constexpr int value_offset(int lmax, int m) {
    return m == 0 ? 0 : (lmax + 1) + (m - 1) * (2 * lmax + 2 - m);
}

// Neighbour grid of one build (all catalogues of a group share it).
struct Grid {
    double box;        // L
    double h;          // cell side L / nc
    double inv_h;      // nc / L
    float hf;          // (float)h
    float boxf;        // (float)L
    int nc;            // cells per side
    int ncell;         // nc^3
    int k;             // stencil half-width in cells (0 in single-cell mode)
    int single;        // 1: one cell, minimum image per pair
    int code_bits;     // bits of the stencil-offset code in a list entry
    uint32_t idx_mask; // mask of the catalogue-relative point index in a list entry
};

struct StencilRun { int ox, oy, oz_lo, oz_hi; };

// Per-catalogue bookkeeping of a group (device arrays).
struct CatArrays {
    const int64_t* pt_off;   // [ncat+1] first point of each catalogue (input = sorted order ranges)
    int ncat;
};

// ---------------------------------------------------------------- launchers
// Grid build (tpcf_grid.hip)
// nonfinite counts points with a non-finite coordinate, catbad[c] those of catalogue c
hipError_t launch_grid_assign(const double* pos, const double* w, int64_t n, const int64_t* pt_off,
                              int ncat, Grid g, int* cellid, int* count, int* nonfinite, int* catbad,
                              hipStream_t s);
// Exclusive scan of m counts into start[0..m]; work holds grid_scan_work_ints(m) ints.
hipError_t launch_grid_scan(const int* count, int64_t m, int* start, int* work, hipStream_t s);
int64_t grid_scan_work_ints(int64_t m);
hipError_t launch_grid_scatter(const int* cellid, int64_t n, const int* start, int* cursor,
                               const double* pos, double box, int* tmp_idx, double* tmp_key, hipStream_t s);
hipError_t launch_grid_order(const int* cellid, int64_t n, const int* start, const int* tmp_idx,
                             const double* tmp_key, int* orig, hipStream_t s);
hipError_t launch_grid_fill(const double* pos, const double* w, int64_t n, const int* orig,
                            const int* cellid, Grid g, float4* pf, float* pw, float4* pa, double4* pd,
                            int* perm, int* catid, hipStream_t s);
hipError_t launch_fill_i32(int* p, int64_t n, int v, hipStream_t s);
// Work items of the binning pass: each cell's primaries in blocks of kItemPrims.
constexpr int kItemPrims = 16;
hipError_t launch_items_count(const int* cell_start, int64_t m, int* nitems, hipStream_t s);
hipError_t launch_items_fill(const int* item_start, int64_t m, int* item_cell, hipStream_t s);
hipError_t launch_items_cat(const int* item_start, int ncat, int ncell, int* item_cat, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);

// Pair pass (tpcf_pairs.hip)
struct BinArgs {
    const float4* pf;        // sorted (xr, yr, zr, iz) cell-relative FP32
    const float* pw;         // sorted FP32 weights (null: all weights are 1)
    const double4* pd;       // sorted (x, y, z, w) FP64 wrapped
    const int* catid;        // sorted catalogue id
    const int* cell_start;   // [ncat*ncell+1]
    const int64_t* pt_off;   // [ncat+1]
    const StencilRun* runs;  // stencil runs
    int nruns;
    Grid g;
    int nb;
    const double* e2;        // [nb+1] squared edges (FP64)
    const float* e2f;        // [nb+1] squared edges (FP32)
    const float* guard;      // [nb+1] FP32 guard band around each squared edge
    int64_t p_begin, p_end;  // primaries (sorted indices) of this chunk
    uint32_t* list;          // hit lists of the chunk (list entries), or
    float4* rec;             // hit records (dx, dy, dz, w_j) when not null (FP32 paths)
    int rec_oct;             // 8-byte records, the octahedral code of the direction: unit weights, read by the whole-m FP32 kernels
    unsigned long long* cursor; // [kSlots*16] bump allocators, one region of `list` each (in blocks of four entries)
    unsigned long long capacity;  // room of `list` in blocks of four entries or records
    int nslots;              // regions the room is split into, one cursor each (<= kSlots)
    uint32_t* boff;          // [(p_end-p_begin)*nb] offsets of (p, b) lists, in blocks of four entries (every list starts at a multiple of four)
    uint32_t* cnt;           // [(p_end-p_begin)*nb] lengths
    int* overflow;           // [1] set when `list` is too small
    int2* fix;               // fix-up list: (cell, chunk-relative primary) whose predicted bin regions overflowed
    int* nfix;               // [1] its length
    int* nfix_total;         // [1] the fix-up launches add the lengths they processed
    const double* vol;       // [nb] shell volumes
    float inv_vst;           // 1 / stencil volume (the box in one-cell mode)
    float reach2;            // squared reach of a work item's candidate cut (outer edge, with a margin)
    int npmax;               // capacity of the piece table (>= 2 nruns)
    int uniform;             // bins equally spaced in r: bin = floor((r - e0) / dr)
    float e0f, inv_dr;       // FP32 first edge and 1 / bin width (uniform bins)
    float delta;             // guard band in units of the bin width (uniform bins)
    float inv_boxf;          // 1 / L (single-cell mode)
    const int* item_start;   // [ncat*ncell+1] first work item of each cell
    const int* item_cell;    // [items] cell of each work item
    int64_t item_lo, item_hi;// work items of the catalogues holding the chunk's primaries
};
constexpr int kSlots = 256;  // list allocation cursors (each on its own 128-byte line)
hipError_t launch_pair_bin(const BinArgs& a, hipStream_t s);
// Fix-up launch: a fixed grid walks the list whose length the binning launch
// left at *nfix, so the two launches need no host round trip between them.
constexpr int kFixGrid = 2048;
hipError_t launch_pair_fix(const BinArgs& a, hipStream_t s);
size_t pair_bin_lds_bytes(int npmax);

struct AlmArgs {
    const float4* pf;        // sorted (xr, yr, zr, iz) cell-relative FP32
    const float4* pa;        // sorted (xr, yr, zr, w): one 16-byte gather per neighbour
    const double4* pd;
    const int* catid;
    const int64_t* pt_off;
    Grid g;
    int nb;
    int lmax;
    int64_t p_begin, p_end;
    const uint32_t* list;    // list entries (FP64 path)
    const float4* rec;       // hit records (dx, dy, dz, w_j) (FP32 paths)
    int unit_w;              // all weights are 1
    int wave_per_list;       // long lists: one wavefront per (p, b) list (FP32, lmax <= 6)
    int self_lo;             // FP32 whole-m lanes: self moments only to order lmax (run asks for L <= lmax)
    const uint32_t* boff;
    const uint32_t* cnt;
    void* A;                 // [nb][nvalues][ldA] float or double
    int64_t ldA;             // leading dimension (primaries of the chunk, padded)
    const float* shift_f;    // [ncodes*3] stencil offset in length units (FP32)
    const int* shift_i;      // [ncodes*3] stencil offset in cells
    int ncodes;
};
hipError_t launch_pair_alm(const AlmArgs& a, int fp64, hipStream_t s);

// Lets a kernel take up to a CU's 160 KiB of LDS. The limit belongs to the
// device current at the call, so launchers set it before every launch (a
// host-side call of a few microseconds) rather than once per process.
inline hipError_t allow_full_lds(const void* kernel) {
    return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

// 2PCF pair counts (tpcf_xi.hip)
constexpr int kXiMaxBins = 16384;  // nb * nmu: one uint32 LDS counter per (r, mu) bin
struct XiArgs {
    const float4* pf;        // sorted (xr, yr, zr, iz) cell-relative FP32
    const double4* pd;       // sorted (x, y, z, w) FP64 wrapped
    const int* cell_start;   // [ncell+1]
    const StencilRun* runs;  // half stencil: offsets positive in (x, y, z) order and the home cell
    int nruns;
    int home_code;           // stencil code of the home cell
    Grid g;
    int nb;
    const double* e2;        // [nb+1] squared edges (FP64)
    const float* e2f;        // [nb+1] squared edges (FP32)
    const float* guard;      // [nb+1] FP32 guard band around each squared edge
    int uniform;             // bins equally spaced in r
    float e0f, inv_dr, delta;// uniform bins: first edge, 1 / width, guard band in bin units
    float inv_boxf;          // 1 / L (single-cell mode)
    float reach2;            // squared reach of a work item's candidate cut (outer edge, with a margin)
    int nmu;                 // mu bins over [-1, 1]
    float hmu_f;             // nmu / 2
    double hmu;
    float gmu_a, gmu_b;      // FP32 guard band of t = (mu + 1) nmu / 2: gmu_a / r + gmu_b
    const int* item_start;   // [ncell+1] first work item of each cell
    const int* item_cell;    // [items] cell of each work item
    int64_t nitems;
    int npmax;
    unsigned long long* counts; // [nb * nmu] (zeroed before the launch)
    int* queue;              // [8 * 32] work cursors, one per XCD range (zeroed)
};
hipError_t launch_xi_count(const XiArgs& a, hipStream_t s);
size_t xi_lds_bytes(int nb, int nmu, int npmax);

struct XiFinalArgs {
    const long long* counts; // [nb * nmu]
    int nb, nmu, n_ell;
    const double* coef;      // [n_ell * nmu] (2l+1)/2 * integral of P_l over mu bin k
    const double* rr;        // [nb] analytic random pairs per (r, mu) bin
    double* out;             // [n_ell * nb]
};
hipError_t launch_xi_finalize(const XiFinalArgs& a, hipStream_t s);

// Covariance over mock catalogues (tpcf_cov.hip)
// X (nm x nd workspace) <- gathered data vectors, centred; C (nd x nd) <- X^T X / (nm - 1),
// through cov_slices(nm, nd) partial products of nd x nd (workspace `part`).
int cov_slices(int nm, int nd);
int64_t cov_part_doubles(int nm, int nd);  // size of `part`: the slices' products and the mean's sums
hipError_t launch_cov(const double* src, int64_t stride, const int64_t* off, int nm, int nd, double* X,
                      double* part, double* mean, double* C, hipStream_t s);
// Allocation-free covariance: a static device array of kCovScratchBytes per
// device. cov_scratch_init (with `device` current) returns its device address,
// looked up once per device; cov_scratch_need gives the bytes launch_cov uses
// for X followed by `part`.
constexpr int64_t kCovScratchBytes = 32ll << 20;
hipError_t cov_scratch_init(int device, void** out);
int64_t cov_scratch_need(int nm, int nd);
// A (n x n, symmetric positive definite) <- scale * A^-1 in place, W (n x n) as workspace;
// *bad |= 1 on a non-positive pivot.
hipError_t launch_cov_invert(double* A, double* W, int n, double scale, int* bad, hipStream_t s);

// Contraction (tpcf_contract.hip)
struct ContractArgs {
    const void* A;           // [nb][nvalues][ldA]
    int64_t ldA;
    const double4* pd;       // weights of the primaries (w in .w), sorted order
    int64_t p_begin;         // first primary of the chunk (sorted index)
    int nb, lmax;
    const int* sub_start;    // [nsub+1] chunk-relative first primary of each subchunk
    int nsub;
    int sub_base;            // global index of the first subchunk of this chunk
    float* part32;           // partial sums (FP32 modes): [nsub_total][gsize]
    double* part64;          // partial sums (FP64 mode)
    int64_t gsize;           // sum_m K_m^2
    const int64_t* goff;     // [lmax+1] offset of G_m inside a partial
    int mode;                // 0 fp64, 1 fp32, 2 bf16x3, 3 bf16x6
    int unit_weights;        // all weights 1: skip the weight multiply
    const float* pw;         // FP32 weights, sorted order (split-BF16 modes)
    int ks_max;              // split-BF16: longest step in primaries (0: the longest that fits)
    int lcouple;             // split-BF16: blocks with |l1 - l2| > lcouple may be skipped (>= lmax: none)
};
hipError_t launch_contract(const ContractArgs& a, hipStream_t s);
// Isotropic schedule: only the l1 = l2 blocks of every G_m (nb <= 32); the
// other entries of the partials must be zero beforehand.
hipError_t launch_contract_iso(const ContractArgs& a, hipStream_t s);

struct SelfArgs {
    const void* A;
    int64_t ldA;
    const double4* pd;
    const uint32_t* cnt;
    int64_t p_begin;
    int nb, lmax;
    const int* sub_start;
    int nsub;
    int sub_base;
    double* part;            // [nsub_total][nb*(2lmax+2)]: moments then pair count per bin
    int fp64;
    int unit_w;              // all weights 1 (pd[].w not read)
    int self_lo;             // orders above lmax neither written by the harmonic pass nor read: zero
};
hipError_t launch_self_moments(const SelfArgs& a, hipStream_t s);

// Fixed-order sums of subchunk partials per catalogue.
hipError_t launch_reduce_partials(const float* p32, const double* p64, int64_t width,
                                  const int* cat_sub, int ncat, double* out, hipStream_t s);

struct FinalArgs {
    const double* G;         // [ncat][gsize] (FP64, upper-triangle-complete symmetric)
    int64_t gsize;
    const int64_t* goff;     // [lmax+1]
    const double* S;         // [ncat][nb*(2lmax+2)] self moments and pair counts
    const double* nd;        // [ncat] N_D
    int nb, lmax;
    int n_mult;
    const int* mult;         // [n_mult*3]
    const double* coefG;     // [n_mult][lmax+1] coefficient of s s G_m
    const double* coefS;     // [n_mult][lmax+1][2lmax+1] coefficient of the self moments
    const double* vol;       // [nb] shell volumes
    double inv_box6;
    int subtract_self;
    double* out;             // [ncat][n_mult][nb][nb]
    int ncat;
};
hipError_t launch_finalize(const FinalArgs& a, hipStream_t s);

// Edge correction of isotropic multipoles: out[l][q] solves sum_l' M_{l l'} out[l'][q] = N[l][q],
// M_{l l'} = sum_l'' T[(l nl + l') nl + l''] R[l''][q], q < nbb (= nb^2); *bad |= 1 if singular.
hipError_t launch_edge_iso(const double* N, const double* R, const double* T, int nl, int nbb, double* out, int* bad,
                           hipStream_t s);

// Anisotropic edge correction (tpcf_edge.hip): one n x n real system per
// (b1, b2), n = number of (l1, l2, m) with 0 <= m <= l1, l2 <= lmax.
constexpr int kMaxEdgeLmax = 10;
constexpr int kMaxEdgeUnknowns = 506;  // n at lmax = 10
struct EdgeArgs {
    const double* N;         // [(lmax+1)^3][nsys] NNN^m export of the data-minus-randoms run
    const double* R;         // the same of the randoms run
    const double* inv_rrr_N; // [nsys] 1 / RRR of each run
    const double* inv_rrr_R;
    const double* gaunt;     // [S][S][S][2S-1][S] g(l, m; l', m'; l'') (S = lmax + 1, m >= 0, |m'| <= lmax)
    const int4* units;       // [n] (l1, l2, m) of each unknown
    int n, lmax, nsys;       // nsys = nbins^2, system q = b1 nbins + b2
    double* M;               // [nsys][n][n] workspace
    double* rhs;             // [nsys][n] workspace: right-hand sides, then solutions
    double* zeta;            // [(lmax+1)^3][nsys] corrected coefficients (zero-filled beforehand)
    int* bad;                // set when a system is singular
    int n_mult;
    const int* mult;         // [n_mult * 3]
    const double* coef;      // [n_mult][S] TripoSH weight of zeta^m
    double* out;             // [n_mult][nsys]
};
hipError_t launch_edge_aniso(const EdgeArgs& a, hipStream_t s);

struct NnnArgs {
    const double* G;         // [gsize] one catalogue
    const int64_t* goff;
    const double* S;         // [nb*(2lmax+2)]
    int nb, lmax;
    const double* scale;     // [(lmax+1)^2] s_lm at l*(lmax+1)+m
    const double* gaunt;     // [(lmax+1)^3 (2lmax+1)] g_L(l1,l2,m) * gamma0_L at ((m*s1+l1)*s1+l2)*(2lmax+1)+L
    int subtract_self;
    int isotropic;           // only l1 = l2 blocks exist (others are exported as zero)
    double* out;             // [(lmax+1)^3][nb][nb]
};
hipError_t launch_export_nnn(const NnnArgs& a, hipStream_t s);

struct AlmExportArgs {
    const void* A;
    int64_t ldA;
    const int* perm;         // original index -> sorted index
    int64_t p_begin;         // sorted index of the chunk's first primary
    int64_t first, count;    // original indices
    int nb, lmax;
    const double* sign_scale;// [(lmax+1)^2] (-1)^m s_lm
    int fp64;
    double* out;
};
hipError_t launch_export_alm(const AlmExportArgs& a, hipStream_t s);

}  // namespace tpcf
