// Host runtime of libtpcf: the C ABI of include/tpcf.h.
//
// It validates arguments, plans the neighbour grid and the work split,
// derives the constant tables of the estimator (spherical-harmonic scale
// factors and the Legendre-product integrals that give both the tripolar
// weights of eq. (slep2sugy) and the degenerate-triangle correction), owns the
// device workspace and enqueues the kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/tpcf.h"
#include "tpcf_internal.h"

namespace tpcf {
size_t contract_lds_bytes(int mode, int nb, int lmax);
}

using namespace tpcf;

namespace {

constexpr int kStages = 6;                // timed stages (tpcf_stage_times)
constexpr int kPlanCandidates = 16;       // refinement x list mode x contraction step
const double kPi = 3.14159265358979323846;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct Timer {
    hipEvent_t a, b;
    int stage;
};

struct Chunk {
    int64_t p_begin, p_end;  // sorted indices
    int sub_begin, sub_end;  // global subchunk range
    int sub_off;             // offset of the chunk's relative subchunk table in d_subs
    int64_t item_lo = -1, item_hi = -1;  // exact work items of the chunk (one catalogue), or -1
};

}  // namespace

struct tpcf_handle_s {
    tpcf_config cfg{};
    std::vector<double> edges;
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int nb = 0, lmax = 0, NV = 0, mode = 0, fp64 = 0;
    int refine = 0;
    int list_mode = -1;    // harmonic pass: -1 by predicted list length, 0 a lane per list, 1 a wavefront per list
    int contract_step = 0; // split-BF16 contraction step (primaries), 0 = the longest that fits
    int64_t limit = 0;
    int64_t used = 0;
    std::vector<DevBuf*> bufs;

    // constants
    std::vector<double> e2, vol, scale, sign_scale, gamma0;
    std::vector<float> e2f, guard;
    std::vector<double> q;  // q[((l1*s1+l2)*s1+m)*(2lmax+1)+L]
    std::vector<int64_t> goff;
    int64_t gsize = 0;
    DevBuf d_e2, d_e2f, d_guard, d_runs, d_shift_f, d_goff, d_vol, d_scale, d_sign_scale,
        d_gaunt;

    // grid of the current group
    Grid g{};
    std::vector<StencilRun> runs;
    int ncodes = 0;
    int ncat = 0;
    int64_t npts = 0;
    std::vector<int64_t> pt_off;
    std::vector<double> n_data;
    bool unit_w = true;
    bool self_lo = false;  // tpcf_run_catalogs with multipoles of L <= lmax only (no per-m export)
    bool self_cut = false;  // the summed self moments stop at order lmax (set by such a run)
    int couple = -1;        // this pass's contraction may skip blocks with |l1 - l2| > couple (-1: none)
    int couple_cut = -1;    // the summed blocks stop at |l1 - l2| <= couple_cut (set by tpcf_run_catalogs)
    DevBuf d_pt_off, d_cellid, d_count, d_start, d_cursor, d_tmp, d_tmpz, d_orig, d_pf, d_pw, d_pa, d_pd, d_perm,
        d_catid, d_flag, d_istart, d_icell, d_icat, d_scanw, d_catbad;
    std::vector<int32_t> cat_status;  // per catalogue of the last tpcf_run_catalogs
    std::vector<int> item_cat;       // [ncat+1] first work item of each catalogue

    // pair pass
    std::vector<int64_t> sub_start;  // global subchunks (sorted index of first primary), + end
    std::vector<int> cat_sub;        // [ncat+1]
    std::vector<Chunk> chunks;
    int64_t kc = 4096;  // primaries per subchunk (the self-moment kernel stages at most 4096 weights)
    int uniform = 0;      // bins equally spaced in r
    float inv_dr = 0.f;   // 1 / bin width (uniform bins)
    float delta = 0.f;    // FP32 guard band in units of the bin width
    int64_t chunk_cap = 0;
    double hits_per_list = 0.0;  // predicted mean length of a (p, b) list
    double list_grow = 1.0;      // list room found needed beyond the prediction (doubles per overflow)
    unsigned long long list_cap = 0;
    DevBuf d_fix;
    int64_t nfix_total = 0;   // primaries rebinned with exact counts (all chunks since creation)
    double inv_vst = 0.0;     // 1 / stencil volume
    DevBuf d_list, d_lcursor, d_boff, d_cnt, d_A, d_subs, d_catsub, d_part, d_pself, d_G, d_S, d_nd,
        d_mult, d_coefG, d_coefS, d_lflag;
    int64_t ldA = 0;
    int stage = 0;         // 0 nothing, 1 grid, 2 a_lm, 3 contracted
    bool alm_kept = false; // A of the whole catalogue is resident (single chunk)
    bool contracted_in_pass = false;
    int64_t pairs = 0;
    bool pairs_valid = false;

    // 2PCF
    DevBuf d_xiq, d_xicoef, d_xirr, d_xiruns;
    // covariance
    DevBuf d_covx, d_covoff, d_covflag, d_covpart;
    // edge correction
    DevBuf d_edgeT, d_egaunt, d_eunits, d_errr, d_ecoef, d_eM, d_erhs, d_ezeta, d_emult;
    int egaunt_lmax = -1;  // lmax of the Gaunt table held in d_egaunt
    // device address of the static scratch of the allocation-free covariance
    void* cov_scratch = nullptr;

    // timing
    bool timing = false;
    std::vector<Timer> timers;
    double ms[kStages] = {0, 0, 0, 0, 0, 0};
    int64_t nl[kStages] = {0, 0, 0, 0, 0, 0};
};

namespace {

tpcf_status fail(tpcf_handle h, tpcf_status st, const std::string& msg) {
    if (h) h->err = msg;
    return st;
}

// Live handles. A handle is checked by looking its address up here, never by
// reading through it, so a destroyed (freed) or foreign pointer is refused
// without touching its memory. The set is never destroyed: handles may still
// be released by static destructors at process exit.
std::mutex g_live_mu;
std::unordered_set<const void*>& live_handles() {
    static auto* s = new std::unordered_set<const void*>();
    return *s;
}

bool alive(tpcf_handle h) {
    if (!h) return false;
    std::lock_guard<std::mutex> lock(g_live_mu);
    return live_handles().count(h) != 0;
}

tpcf_status hip_fail(tpcf_handle h, hipError_t e, const char* what) {
    return fail(h, TPCF_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr)                                            \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) return hip_fail(h, _e, #expr);    \
    } while (0)

// Grows a device buffer to at least `bytes` (contents are not preserved).
tpcf_status ensure(tpcf_handle h, DevBuf& b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return TPCF_OK;
    if (b.p) {
        hipFree(b.p);
        h->used -= (int64_t)b.bytes;
        b.p = nullptr;
        b.bytes = 0;
    }
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) / 256 * 256;
    if (h->used + (int64_t)bytes > h->limit)
        return fail(h, TPCF_ERR_ALLOC, "workspace limit exceeded (" + std::to_string(h->used + bytes) +
                                           " > " + std::to_string(h->limit) + " bytes)");
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        return fail(h, TPCF_ERR_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    b.bytes = bytes;
    h->used += (int64_t)bytes;
    return TPCF_OK;
}

// Stream-ordered copy of a small host table; waits for it so that the host
// memory may be released and the table is never overwritten under a kernel.
tpcf_status upload(tpcf_handle h, DevBuf& b, const void* src, size_t bytes) {
    tpcf_status st = ensure(h, b, bytes);
    if (st != TPCF_OK) return st;
    HIPCHK(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return TPCF_OK;
}

void release(tpcf_handle h, DevBuf& b) {
    if (b.p) {
        hipFree(b.p);
        h->used -= (int64_t)b.bytes;
    }
    b.p = nullptr;
    b.bytes = 0;
}

template <class T> T* P(DevBuf& b) { return reinterpret_cast<T*>(b.p); }

// ---------------------------------------------------------------- timing

void t_begin(tpcf_handle h, int stage, Timer& t) {
    if (!h->timing) return;
    t.stage = stage;
    hipEventCreate(&t.a);
    hipEventCreate(&t.b);
    hipEventRecord(t.a, h->stream);
}
void t_end(tpcf_handle h, Timer& t) {
    if (!h->timing) return;
    hipEventRecord(t.b, h->stream);
    h->timers.push_back(t);
}

// ---------------------------------------------------------------- constants

// R_lm(z) for l = m..lmax at one z (R_mm = 1, R_{m+1,m} = z,
// R_lm = z R_{l-1,m} - beta_lm R_{l-2,m}).
void r_chain(int lmax, int m, double z, std::vector<double>& out) {
    out.assign(lmax + 1, 0.0);
    if (m > lmax) return;
    out[m] = 1.0;
    if (m + 1 <= lmax) out[m + 1] = z;
    for (int l = m + 2; l <= lmax; ++l) {
        const double beta = (double)((l + m - 1) * (l - m - 1)) / (double)((2 * l - 1) * (2 * l - 3));
        out[l] = z * out[l - 1] - beta * out[l - 2];
    }
}

double gamma_lm(int l, int m) {
    double g = 1.0;
    for (int k = 1; k <= 2 * m - 1; k += 2) g *= k;  // (2m-1)!!
    for (int ll = m + 1; ll <= l; ++ll) g *= (double)(2 * ll - 1) / (double)(ll - m);
    return g;
}

double norm_lm(int l, int m) {
    double r = 1.0;
    for (int k = l - m + 1; k <= l + m; ++k) r /= (double)k;
    return std::sqrt((2.0 * l + 1.0) / (4.0 * kPi) * r);
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        const double dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// q(l1,l2,m,L) = int_{-1}^{1} Nbar_l1m(z) Nbar_l2m(z) P_L(z) dz, where
// Nbar_lm(z) = N_lm |P_l^m(z)| sign-free: the polar part shared by Y_l1m and
// Y_l2m, so that conj(Y_l1m) Y_l2m = sum_L (2L+1)/2 q P_L(z) and the Gaunt
// integral gives H (l1 l2 L; m -m 0) = (-1)^m 2 pi q / sqrt((2l1+1)(2l2+1)).
void build_q(tpcf_handle h) {
    const int lmax = h->lmax, s1 = lmax + 1, nL = 2 * lmax + 1;
    std::vector<double> x, w;
    gauss_legendre(64, x, w);
    h->q.assign((size_t)s1 * s1 * s1 * nL, 0.0);
    std::vector<std::vector<double>> Pm(s1), R;
    std::vector<double> tmp, P0;
    for (size_t i = 0; i < x.size(); ++i) {
        const double z = x[i];
        // Nbar_lm(z) for all l, m
        std::vector<double> nb((size_t)s1 * s1, 0.0);
        for (int m = 0; m <= lmax; ++m) {
            r_chain(lmax, m, z, tmp);
            const double sm = std::pow(std::max(0.0, 1.0 - z * z), 0.5 * m);
            for (int l = m; l <= lmax; ++l) nb[l * s1 + m] = norm_lm(l, m) * gamma_lm(l, m) * tmp[l] * sm;
        }
        r_chain(2 * lmax, 0, z, P0);
        for (int L = 0; L <= 2 * lmax; ++L) P0[L] *= gamma_lm(L, 0);  // Legendre P_L
        for (int l1 = 0; l1 <= lmax; ++l1)
            for (int l2 = 0; l2 <= lmax; ++l2)
                for (int m = 0; m <= std::min(l1, l2); ++m) {
                    const double f = w[i] * nb[l1 * s1 + m] * nb[l2 * s1 + m];
                    double* qq = &h->q[(((size_t)l1 * s1 + l2) * s1 + m) * nL];
                    for (int L = 0; L < nL; ++L) qq[L] += f * P0[L];
                }
    }
    // exact zeros where parity or the triangle rule forbid the coupling
    for (int l1 = 0; l1 <= lmax; ++l1)
        for (int l2 = 0; l2 <= lmax; ++l2)
            for (int m = 0; m <= std::min(l1, l2); ++m)
                for (int L = 0; L < nL; ++L)
                    if (((l1 + l2 + L) & 1) || L < std::abs(l1 - l2) || L > l1 + l2)
                        h->q[(((size_t)l1 * s1 + l2) * s1 + m) * nL + L] = 0.0;
}

double qv(tpcf_handle h, int l1, int l2, int m, int L) {
    const int s1 = h->lmax + 1, nL = 2 * h->lmax + 1;
    return h->q[(((size_t)l1 * s1 + l2) * s1 + m) * nL + L];
}

double ulp32(double x) {
    if (x <= 0) return std::ldexp(1.0, -149);
    int e;
    std::frexp(x, &e);  // x = f * 2^e, f in [0.5, 1)
    return std::ldexp(1.0, e - 24);
}

tpcf_status setup_constants(tpcf_handle h) {
    const int nb = h->nb, lmax = h->lmax, s1 = lmax + 1;
    h->e2.resize(nb + 1);
    h->e2f.resize(nb + 1);
    for (int b = 0; b <= nb; ++b) {
        h->e2[b] = h->edges[b] * h->edges[b];
        h->e2f[b] = (float)h->e2[b];
    }
    h->vol.resize(nb);
    for (int b = 0; b < nb; ++b)
        h->vol[b] = 4.0 * kPi / 3.0 *
                    (h->edges[b + 1] * h->edges[b + 1] * h->edges[b + 1] - h->edges[b] * h->edges[b] * h->edges[b]);
    h->scale.assign((size_t)s1 * s1, 0.0);
    h->sign_scale.assign((size_t)s1 * s1, 0.0);
    for (int l = 0; l <= lmax; ++l)
        for (int m = 0; m <= l; ++m) {
            h->scale[l * s1 + m] = norm_lm(l, m) * gamma_lm(l, m);
            h->sign_scale[l * s1 + m] = ((m & 1) ? -1.0 : 1.0) * h->scale[l * s1 + m];
        }
    h->gamma0.resize(2 * lmax + 1);
    for (int L = 0; L <= 2 * lmax; ++L) h->gamma0[L] = gamma_lm(L, 0);
    build_q(h);
    h->goff.resize(lmax + 2);
    int64_t off = 0;
    for (int m = 0; m <= lmax; ++m) {
        h->goff[m] = off;
        const int64_t K = (int64_t)nb * (lmax - m + 1);
        off += K * K;
    }
    h->goff[lmax + 1] = off;
    h->gsize = off;
    // gaunt table for the NNN export: (2L+1)/2 q gamma0_L
    const int nL = 2 * lmax + 1;
    std::vector<double> gaunt((size_t)s1 * s1 * s1 * nL, 0.0);
    for (int m = 0; m <= lmax; ++m)
        for (int l1 = m; l1 <= lmax; ++l1)
            for (int l2 = m; l2 <= lmax; ++l2)
                for (int L = 0; L < nL; ++L)
                    gaunt[(((size_t)m * s1 + l1) * s1 + l2) * nL + L] =
                        0.5 * (2.0 * L + 1.0) * qv(h, l1, l2, m, L) * h->gamma0[L];
    tpcf_status st;
    if ((st = upload(h, h->d_e2, h->e2.data(), sizeof(double) * (nb + 1))) != TPCF_OK) return st;
    if ((st = upload(h, h->d_e2f, h->e2f.data(), sizeof(float) * (nb + 1))) != TPCF_OK) return st;
    if ((st = upload(h, h->d_goff, h->goff.data(), sizeof(int64_t) * (lmax + 2))) != TPCF_OK) return st;
    if ((st = upload(h, h->d_vol, h->vol.data(), sizeof(double) * nb)) != TPCF_OK) return st;
    if ((st = upload(h, h->d_scale, h->scale.data(), sizeof(double) * s1 * s1)) != TPCF_OK) return st;
    if ((st = upload(h, h->d_sign_scale, h->sign_scale.data(), sizeof(double) * s1 * s1)) != TPCF_OK)
        return st;
    if ((st = upload(h, h->d_gaunt, gaunt.data(), sizeof(double) * gaunt.size())) != TPCF_OK) return st;
    HIPCHK(hipStreamSynchronize(h->stream));
    return TPCF_OK;
}

// ---------------------------------------------------------------- grid plan

// Stencil of cells that can hold a neighbour in [e0, rmax) of some point of
// the home cell, as runs of consecutive oz for each (ox, oy).
std::vector<StencilRun> make_stencil(int k, double hcell, double e0, double rmax) {
    std::vector<StencilRun> runs;
    for (int ox = -k; ox <= k; ++ox)
        for (int oy = -k; oy <= k; ++oy) {
            int cur_lo = 0;
            bool open = false;
            for (int oz = -k; oz <= k + 1; ++oz) {
                bool keep = false;
                if (oz <= k) {
                    auto gap = [](int o) { return std::max(std::abs(o) - 1, 0); };
                    auto far = [](int o) { return std::abs(o) + 1; };
                    const double dmin = hcell * std::sqrt((double)(gap(ox) * gap(ox) + gap(oy) * gap(oy) + gap(oz) * gap(oz)));
                    const double dmax = hcell * std::sqrt((double)(far(ox) * far(ox) + far(oy) * far(oy) + far(oz) * far(oz)));
                    keep = dmin < rmax * (1.0 + 1e-9) && dmax > e0 * (1.0 - 1e-9);
                }
                if (keep && !open) { cur_lo = oz; open = true; }
                if (!keep && open) {
                    runs.push_back({ox, oy, cur_lo, oz - 1});
                    open = false;
                }
            }
        }
    return runs;
}

int bits_for(int n) {
    int b = 1;
    while ((1 << b) < n) ++b;
    return b;
}

tpcf_status plan_grid(tpcf_handle h, int64_t max_cat) {
    const double L = h->cfg.box, rmax = h->edges[h->nb], e0 = h->edges[0];
    int kmax = h->refine > 0 ? h->refine : 3;
    for (int k = kmax; k >= 1; --k) {
        const int nc = (int)std::floor(k * L / rmax);
        if (nc < 2 * k + 1) continue;
        if ((int64_t)nc * nc * nc * h->ncat > (1LL << 30)) continue;
        const int K2 = 2 * k + 1;
        const int cb = bits_for(K2 * K2 * K2);
        if (max_cat >= (1LL << (32 - cb))) continue;
        const double hc = L / nc;
        std::vector<StencilRun> runs = make_stencil(k, hc, e0, rmax);
        if (2 * (int)runs.size() > kMaxRuns) continue;
        h->g.box = L;
        h->g.nc = nc;
        h->g.ncell = nc * nc * nc;
        h->g.h = hc;
        h->g.inv_h = nc / L;
        h->g.hf = (float)hc;
        h->g.boxf = (float)L;
        h->g.k = k;
        h->g.single = 0;
        h->g.code_bits = cb;
        h->g.idx_mask = (uint32_t)((1ULL << (32 - cb)) - 1);
        h->runs = runs;
        int64_t cells = 0;
        for (const StencilRun& r : runs) cells += r.oz_hi - r.oz_lo + 1;
        h->inv_vst = 1.0 / ((double)cells * hc * hc * hc);
        h->ncodes = K2 * K2 * K2;
        break;
    }
    if (h->g.nc == 0) {
        // one cell: every point is a candidate, minimum image per pair
        if (max_cat >= (1LL << 31)) return fail(h, TPCF_ERR_RANGE, "catalogue too large");
        h->g.box = L;
        h->g.nc = 1;
        h->g.ncell = 1;
        h->g.h = L;
        h->g.inv_h = 1.0 / L;
        h->g.hf = (float)L;
        h->g.boxf = (float)L;
        h->g.k = 0;
        h->g.single = 1;
        h->g.code_bits = 1;
        h->g.idx_mask = 0x7fffffffu;
        h->runs = {{0, 0, 0, 0}};
        h->inv_vst = 1.0 / (L * L * L);
        h->ncodes = 1;
    }
    // shift table
    const int k = h->g.k, K2 = 2 * k + 1;
    std::vector<float> sh((size_t)h->ncodes * 3);
    for (int c = 0; c < h->ncodes; ++c) {
        const int ox = c / (K2 * K2) - k, oy = (c / K2) % K2 - k, oz = c % K2 - k;
        sh[3 * c] = (float)(ox * h->g.h);
        sh[3 * c + 1] = (float)(oy * h->g.h);
        sh[3 * c + 2] = (float)(oz * h->g.h);
    }
    // guard bands of the FP32 binning: bound of the single-precision error of
    // r^2 for pairs inside the stencil: rounding of the cell-relative inputs,
    // of the separations and of r^2 itself, with a factor 4 of margin
    const double span = h->g.single ? L : (k + 1) * h->g.h;
    const double dd = 4.0 * ulp32(span);
    h->guard.resize(h->nb + 1);
    for (int b = 0; b <= h->nb; ++b) {
        const double e = h->edges[b];
        const double gb = 4.0 * (2.0 * std::sqrt(3.0) * std::max(e, dd) * dd + 4.0 * std::ldexp(e * e, -24) + 3.0 * dd * dd);
        h->guard[b] = (float)gb;
    }
    // Equally spaced bins are found as floor((r - e0) / dr) in FP32; the
    // guard band becomes a band of width delta (in bin units) around each
    // integer, covering the error of r^2 above plus that of the square root,
    // of e0 and 1/dr in FP32.
    {
        const int nb = h->nb;
        const double e0 = h->edges[0], dr = (h->edges[nb] - e0) / nb;
        bool uni = true;
        for (int b = 0; b <= nb; ++b)
            if (std::fabs(h->edges[b] - (e0 + b * dr)) > 1e-12 * h->edges[nb]) uni = false;
        double gmax = 0.0;
        for (int b = 0; b <= nb; ++b) {
            const double g2 = h->guard[b];
            gmax = std::max(gmax, g2 / (h->edges[b] + std::sqrt(g2)));
        }
        const double eps = 2.0 * gmax / dr + 4.0 * (ulp32(h->edges[nb]) + ulp32(std::max(e0, 1e-30))) / dr +
                           8.0 * ulp32((double)nb + 1.0);
        h->uniform = uni && eps < 0.05 ? 1 : 0;
        h->inv_dr = (float)(1.0 / dr);
        h->delta = (float)eps;
    }
    tpcf_status st;
    if ((st = upload(h, h->d_runs, h->runs.data(), sizeof(StencilRun) * h->runs.size())) != TPCF_OK) return st;
    if ((st = upload(h, h->d_shift_f, sh.data(), sizeof(float) * sh.size())) != TPCF_OK) return st;
    if ((st = upload(h, h->d_guard, h->guard.data(), sizeof(float) * (h->nb + 1))) != TPCF_OK) return st;
    return TPCF_OK;
}

// ---------------------------------------------------------------- stages

tpcf_status build_grid_group(tpcf_handle h, const double* d_pos, const double* d_w,
                             const std::vector<int64_t>& n, const std::vector<int64_t>& n_data) {
    h->ncat = (int)n.size();
    h->pt_off.assign(h->ncat + 1, 0);
    int64_t max_cat = 0;
    for (int c = 0; c < h->ncat; ++c) {
        h->pt_off[c + 1] = h->pt_off[c] + n[c];
        max_cat = std::max(max_cat, n[c]);
    }
    h->npts = h->pt_off[h->ncat];
    h->n_data.assign(n_data.begin(), n_data.end());
    h->unit_w = d_w == nullptr;
    h->g = Grid{};
    tpcf_status st = plan_grid(h, max_cat);
    if (st != TPCF_OK) return st;
    const int64_t N = h->npts;
    const int64_t M = (int64_t)h->ncat * h->g.ncell;
    if ((st = upload(h, h->d_pt_off, h->pt_off.data(), sizeof(int64_t) * (h->ncat + 1))) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_cellid, sizeof(int) * N)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_count, sizeof(int) * (M + 1))) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_start, sizeof(int) * (M + 1))) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_scanw, sizeof(int) * grid_scan_work_ints(M))) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_cursor, sizeof(int) * (M + 1))) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_tmp, sizeof(int) * N)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_tmpz, sizeof(double) * N)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_orig, sizeof(int) * N)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_pf, sizeof(float4) * N)) != TPCF_OK) return st;
    // 16 floats of padding: the contractions stage 8- and 16-wide windows
    if ((st = ensure(h, h->d_pw, sizeof(float) * (N + 16))) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_pa, sizeof(float4) * N)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_pd, sizeof(double4) * N)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_perm, sizeof(int) * N)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_catid, sizeof(int) * N)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_flag, sizeof(int) * 4)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_catbad, sizeof(int) * h->ncat)) != TPCF_OK) return st;
    Timer t;
    t_begin(h, 0, t);
    HIPCHK(launch_fill_i32(P<int>(h->d_count), M + 1, 0, h->stream));
    HIPCHK(launch_fill_i32(P<int>(h->d_cursor), M + 1, 0, h->stream));
    HIPCHK(launch_fill_i32(P<int>(h->d_flag), 4, 0, h->stream));
    HIPCHK(launch_fill_i32(P<int>(h->d_catbad), h->ncat, 0, h->stream));
    HIPCHK(launch_grid_assign(d_pos, d_w, N, P<int64_t>(h->d_pt_off), h->ncat, h->g, P<int>(h->d_cellid),
                              P<int>(h->d_count), P<int>(h->d_flag), P<int>(h->d_catbad), h->stream));
    HIPCHK(launch_grid_scan(P<int>(h->d_count), M, P<int>(h->d_start), P<int>(h->d_scanw), h->stream));
    HIPCHK(launch_grid_scatter(P<int>(h->d_cellid), N, P<int>(h->d_start), P<int>(h->d_cursor), d_pos, h->g.box,
                               P<int>(h->d_tmp), P<double>(h->d_tmpz), h->stream));
    HIPCHK(launch_grid_order(P<int>(h->d_cellid), N, P<int>(h->d_start), P<int>(h->d_tmp), P<double>(h->d_tmpz),
                             P<int>(h->d_orig), h->stream));
    HIPCHK(launch_grid_fill(d_pos, d_w, N, P<int>(h->d_orig), P<int>(h->d_cellid), h->g, P<float4>(h->d_pf),
                            P<float>(h->d_pw), P<float4>(h->d_pa), P<double4>(h->d_pd), P<int>(h->d_perm), P<int>(h->d_catid),
                            h->stream));
    // work items of the binning pass: blocks of up to kItemPrims primaries of one cell
    const int64_t nitems_max = M + N / kItemPrims + 1;
    if ((st = ensure(h, h->d_istart, sizeof(int) * (M + 1))) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_icell, sizeof(int) * nitems_max)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_icat, sizeof(int) * (h->ncat + 1))) != TPCF_OK) return st;
    HIPCHK(launch_items_count(P<int>(h->d_start), M, P<int>(h->d_cursor), h->stream));
    HIPCHK(launch_grid_scan(P<int>(h->d_cursor), M, P<int>(h->d_istart), P<int>(h->d_scanw), h->stream));
    HIPCHK(launch_items_fill(P<int>(h->d_istart), M, P<int>(h->d_icell), h->stream));
    HIPCHK(launch_items_cat(P<int>(h->d_istart), h->ncat, h->g.ncell, P<int>(h->d_icat), h->stream));
    t_end(h, t);
    h->item_cat.assign(h->ncat + 1, 0);
    HIPCHK(hipMemcpyAsync(h->item_cat.data(), P<int>(h->d_icat), sizeof(int) * (h->ncat + 1),
                          hipMemcpyDeviceToHost, h->stream));
    return TPCF_OK;
}

// Bytes per hit in the neighbour lists: 4-byte list entries (FP64 path),
// 16-byte records (FP32), or 8-byte direction codes with unit weights at
// lmax <= 10 (as the binning writes them).
size_t list_elem_bytes(tpcf_handle h) {
    if (h->fp64) return sizeof(uint32_t);
    return (h->unit_w && h->lmax <= 10) ? 2 * sizeof(float) : sizeof(float4);
}

// Splits every catalogue into subchunks of kc primaries and groups whole
// subchunks into chunks whose a_lm operand and hit lists fit the workspace share.
tpcf_status plan_chunks(tpcf_handle h) {
    const int64_t N = h->npts;
    const size_t elem = h->fp64 ? 8 : 4;
    const int64_t per_prim = (int64_t)h->nb * h->NV * (int64_t)elem;
    // expected in-shell hits per primary (uniform density), for the list size
    const double L3 = h->cfg.box * h->cfg.box * h->cfg.box;
    const double rmax = h->edges[h->nb], e0 = h->edges[0];
    const double shell = 4.0 * kPi / 3.0 * (rmax * rmax * rmax - e0 * e0 * e0);
    int64_t maxn = 0;
    for (int c = 0; c < h->ncat; ++c) maxn = std::max(maxn, h->pt_off[c + 1] - h->pt_off[c]);
    const double hits = std::min((double)maxn, maxn / L3 * shell);
    // hit lists: 4-byte entries (FP64 path) or 12/16-byte records (FP32 paths);
    // room for the predicted bin regions of each primary at its catalogue's
    // mean density (the binning kernel's margin), plus the rare exact rebins (a
    // pass that runs out of room runs again with twice the room, and the
    // handle keeps the factor for the list room of its later passes)
    const double lelem = list_elem_bytes(h);
    // list room per primary of a catalogue of n points
    auto room_of = [&](int64_t n) {
        double r = 64.0;
        for (int b = 0; b < h->nb; ++b) {
            const double pred = std::min((double)n, n / L3 * h->vol[b]);
            r += 1.15 * pred + 4.0 * std::sqrt(pred) + 11.0;
        }
        return r;
    };
    std::vector<double> room(h->ncat);
    for (int c = 0; c < h->ncat; ++c) room[c] = room_of(h->pt_off[c + 1] - h->pt_off[c]);
    h->hits_per_list = hits / h->nb;
    const double budget = (double)(h->limit / 2);
    // A chunk takes whole subchunks while its primaries stay within 2^23,
    // its operand and predicted list room within the budget, and its list
    // room within 12.8e9 entries (list offsets are 32-bit counts of blocks of
    // four entries: the list regions then get 15 % of slack within 16e9). The room of a subchunk is
    // that of its own catalogue's density, so that a batch of uneven
    // catalogues is not budgeted at the densest one.
    const int64_t cap = 1 << 23;
    h->chunk_cap = cap;
    h->sub_start.clear();
    h->cat_sub.assign(h->ncat + 1, 0);
    for (int c = 0; c < h->ncat; ++c) {
        h->cat_sub[c] = (int)h->sub_start.size();
        for (int64_t p = h->pt_off[c]; p < h->pt_off[c + 1]; p += h->kc) h->sub_start.push_back(p);
    }
    h->cat_sub[h->ncat] = (int)h->sub_start.size();
    h->sub_start.push_back(N);
    h->chunks.clear();
    const int nsub = (int)h->sub_start.size() - 1;
    int s = 0, cat = 0;
    double max_room = 0.0;
    while (s < nsub) {
        Chunk ch;
        ch.sub_begin = s;
        ch.p_begin = h->sub_start[s];
        int64_t n_acc = 0;
        double r_acc = 0.0, b_acc = 0.0;
        while (s < nsub) {
            while (h->cat_sub[cat + 1] <= s) ++cat;
            const int64_t n_s = h->sub_start[s + 1] - h->sub_start[s];
            const double r_s = (double)n_s * room[cat];
            const double b_s = (double)n_s * per_prim + lelem * r_s;
            if (s > ch.sub_begin && (n_acc + n_s > cap || r_acc + r_s > 12.8e9 || b_acc + b_s > budget)) break;
            n_acc += n_s;
            r_acc += r_s;
            b_acc += b_s;
            ++s;
        }
        ch.sub_end = s;
        ch.p_end = h->sub_start[s];
        max_room = std::max(max_room, r_acc);
        h->chunks.push_back(ch);
    }
    int64_t maxch = 0;
    for (auto& ch : h->chunks) maxch = std::max(maxch, ch.p_end - ch.p_begin);
    // One catalogue split over several chunks: launch only the work items
    // holding each chunk's primaries (from host copies of the cell and item
    // starts) rather than every item of the catalogue.
    if (h->ncat == 1 && h->chunks.size() > 1) {
        const int64_t M = h->g.ncell;
        std::vector<int> cs(M + 1), is(M + 1);
        HIPCHK(hipMemcpyAsync(cs.data(), h->d_start.p, sizeof(int) * (M + 1), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipMemcpyAsync(is.data(), h->d_istart.p, sizeof(int) * (M + 1), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        auto item_of = [&](int64_t p) {
            // the cell holding sorted point p, then its block of kItemPrims
            const int64_t c = std::upper_bound(cs.begin(), cs.end(), (int)p) - cs.begin() - 1;
            return (int64_t)is[c] + (p - cs[c]) / kItemPrims;
        };
        for (auto& ch : h->chunks) {
            ch.item_lo = item_of(ch.p_begin);
            ch.item_hi = item_of(ch.p_end - 1) + 1;
        }
    }
    h->ldA = (maxch + 63) / 64 * 64;
    // 15 % above the predicted room: a catalogue of even density fills its
    // regions to their prediction on average, and the 256 regions differ
    // times the growth earlier passes of this handle needed (strong
    // clustering); the chunk sizes keep the prediction
    h->list_cap = (unsigned long long)std::min(16.0e9, std::max(1.0e6, 1.15 * max_room * h->list_grow));
    tpcf_status st;
    if ((st = ensure(h, h->d_boff, sizeof(uint32_t) * maxch * h->nb)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_fix, sizeof(int) * 2 * maxch)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_cnt, sizeof(uint32_t) * maxch * h->nb)) != TPCF_OK) return st;
    // 8 elements of padding: the contraction's staging reads 8-wide windows
    if ((st = ensure(h, h->d_A, ((size_t)h->nb * h->NV * h->ldA + 8) * elem)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_list, (size_t)list_elem_bytes(h) * h->list_cap)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_lcursor, sizeof(unsigned long long) * kSlots * 16)) != TPCF_OK) return st;
    // subchunk tables: chunk-relative starts of every chunk, one upload
    std::vector<int> rel;
    for (Chunk& ch : h->chunks) {
        ch.sub_off = (int)rel.size();
        for (int q = ch.sub_begin; q <= ch.sub_end; ++q) rel.push_back((int)(h->sub_start[q] - ch.p_begin));
    }
    if ((st = ensure(h, h->d_subs, sizeof(int) * rel.size() + 64)) != TPCF_OK) return st;
    if ((st = upload(h, h->d_subs, rel.data(), sizeof(int) * rel.size())) != TPCF_OK) return st;
    if ((st = upload(h, h->d_catsub, h->cat_sub.data(), sizeof(int) * (h->ncat + 1))) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_part, (size_t)nsub * h->gsize * sizeof(double))) != TPCF_OK) return st;
    const int sw = h->nb * (2 * h->lmax + 2);
    if ((st = ensure(h, h->d_pself, sizeof(double) * nsub * sw)) != TPCF_OK) return st;
    return TPCF_OK;
}

// Pair pass of one chunk: binning, fix-up of the primaries whose predicted
// regions overflowed, harmonics. Nothing is read back: a list that ran out of
// room raises the flag that pair_pass reads after the last chunk.
tpcf_status pair_chunk(tpcf_handle h, const Chunk& ch) {
    HIPCHK(launch_fill_u64(P<unsigned long long>(h->d_lcursor), kSlots * 16, 0ull, h->stream));
    HIPCHK(launch_fill_i32(P<int>(h->d_flag) + 2, 1, 0, h->stream));  // fix-up list length
    BinArgs b{};
    b.pf = P<float4>(h->d_pf);
    b.pd = P<double4>(h->d_pd);
    b.catid = P<int>(h->d_catid);
    b.cell_start = P<int>(h->d_start);
    b.pt_off = P<int64_t>(h->d_pt_off);
    b.runs = P<StencilRun>(h->d_runs);
    b.nruns = (int)h->runs.size();
    b.g = h->g;
    b.nb = h->nb;
    b.e2 = P<double>(h->d_e2);
    b.e2f = P<float>(h->d_e2f);
    b.guard = P<float>(h->d_guard);
    b.p_begin = ch.p_begin;
    b.p_end = ch.p_end;
    b.list = h->fp64 ? P<uint32_t>(h->d_list) : nullptr;
    b.rec = h->fp64 ? nullptr : P<float4>(h->d_list);
    // unit weights with the whole m range in one FP32 lane (lmax <= 10):
    // the harmonic kernels that read the records (their UNIT forms) take
    // no weight, and only the direction: a record is its octahedral code
    b.rec_oct = (!h->fp64 && h->unit_w && h->lmax <= 10) ? 1 : 0;
    b.pw = h->unit_w ? nullptr : P<float>(h->d_pw);  // null: all weights 1
    b.cursor = P<unsigned long long>(h->d_lcursor);
    b.capacity = h->list_cap / 4;  // in blocks of four entries, the unit of the list offsets
    // at least ~64 work items (of at most 16 primaries) per region, so that
    // the regions, taken by the items in turn, fill evenly within the slack
    b.nslots = (int)std::min<int64_t>(kSlots, std::max<int64_t>(1, (ch.p_end - ch.p_begin) / 1024));
    b.boff = P<uint32_t>(h->d_boff);
    b.cnt = P<uint32_t>(h->d_cnt);
    b.overflow = P<int>(h->d_flag) + 1;
    b.fix = P<int2>(h->d_fix);
    b.nfix = P<int>(h->d_flag) + 2;
    b.nfix_total = P<int>(h->d_flag) + 3;
    b.vol = P<double>(h->d_vol);
    b.inv_vst = (float)h->inv_vst;
    // the reach of the per-item candidate cut: the outer edge with a margin
    // of 1e-4 (relative), far above the FP32 rounding of the coordinates
    b.reach2 = (float)(h->edges[h->nb] * h->edges[h->nb] * (1.0 + 2e-4));
    b.npmax = 2 * (int)h->runs.size();
    b.uniform = h->uniform;
    b.e0f = (float)h->edges[0];
    b.inv_dr = h->inv_dr;
    b.delta = h->delta;
    b.inv_boxf = (float)(1.0 / h->g.box);
    b.item_start = P<int>(h->d_istart);
    b.item_cell = P<int>(h->d_icell);
    {
        // work items of the catalogues holding the chunk's primaries
        int c0 = 0, c1 = 0;
        while (c0 + 1 < h->ncat && h->pt_off[c0 + 1] <= ch.p_begin) ++c0;
        c1 = c0;
        while (c1 + 1 < h->ncat && h->pt_off[c1 + 1] < ch.p_end) ++c1;
        b.item_lo = h->item_cat[c0];
        b.item_hi = h->item_cat[c1 + 1];
        if (ch.item_lo >= 0) {
            b.item_lo = ch.item_lo;
            b.item_hi = ch.item_hi;
        }
    }
    Timer tb;
    t_begin(h, 1, tb);
    HIPCHK(launch_pair_bin(b, h->stream));
    // primaries whose predicted bin regions overflowed: exact counts
    HIPCHK(launch_pair_fix(b, h->stream));
    t_end(h, tb);
    AlmArgs a{};
    a.pf = P<float4>(h->d_pf);
    a.pa = P<float4>(h->d_pa);
    a.pd = P<double4>(h->d_pd);
    a.catid = P<int>(h->d_catid);
    a.pt_off = P<int64_t>(h->d_pt_off);
    a.g = h->g;
    a.nb = h->nb;
    a.lmax = h->lmax;
    a.p_begin = ch.p_begin;
    a.p_end = ch.p_end;
    a.list = h->fp64 ? P<uint32_t>(h->d_list) : nullptr;
    a.rec = h->fp64 ? nullptr : P<float4>(h->d_list);
    a.unit_w = h->unit_w ? 1 : 0;
    // a wavefront per list once lists average 256 records or more (the
    // predicted hits of a primary of the densest catalogue, over the bins)
    // (or as the plan sets it)
    const bool wave_ok = !h->fp64 && h->lmax <= 6;
    a.wave_per_list = (wave_ok && (h->list_mode == 1 || (h->list_mode < 0 && h->hits_per_list >= 256.0))) ? 1 : 0;
    a.self_lo = h->self_lo ? 1 : 0;
    a.boff = P<uint32_t>(h->d_boff);
    a.cnt = P<uint32_t>(h->d_cnt);
    a.A = h->d_A.p;
    a.ldA = h->ldA;
    a.shift_f = P<float>(h->d_shift_f);
    a.ncodes = h->ncodes;
    Timer t;
    t_begin(h, 2, t);
    HIPCHK(launch_pair_alm(a, h->fp64, h->stream));
    t_end(h, t);
    return TPCF_OK;
}

tpcf_status contract_chunk(tpcf_handle h, const Chunk& ch) {
    const int nsub = ch.sub_end - ch.sub_begin;
    Timer t;
    t_begin(h, 3, t);
    ContractArgs c{};
    c.A = h->d_A.p;
    c.ldA = h->ldA;
    c.pd = P<double4>(h->d_pd);
    c.p_begin = ch.p_begin;
    c.nb = h->nb;
    c.lmax = h->lmax;
    c.sub_start = P<int>(h->d_subs) + ch.sub_off;
    c.nsub = nsub;
    c.sub_base = ch.sub_begin;
    c.part32 = nullptr;
    c.part64 = P<double>(h->d_part);
    c.gsize = h->gsize;
    c.goff = P<int64_t>(h->d_goff);
    // weighted catalogues (data minus randoms) need the six-product split
    c.mode = (h->mode == TPCF_PREC_MIXED_BF16X3 && !h->unit_w) ? TPCF_PREC_MIXED_BF16X6 : h->mode;
    c.unit_weights = h->unit_w ? 1 : 0;
    c.pw = P<float>(h->d_pw);
    c.ks_max = h->contract_step;
    c.lcouple = h->couple >= 0 ? h->couple : h->lmax;
    if (h->cfg.flags & TPCF_F_ISOTROPIC) {
        // only the l1 = l2 blocks are formed; the rest of the partials is zero
        HIPCHK(launch_fill_u64(reinterpret_cast<unsigned long long*>(P<double>(h->d_part) + (int64_t)ch.sub_begin * h->gsize),
                               (int64_t)nsub * h->gsize, 0ull, h->stream));
        HIPCHK(launch_contract_iso(c, h->stream));
    } else {
        HIPCHK(launch_contract(c, h->stream));
    }
    SelfArgs s{};
    s.A = h->d_A.p;
    s.ldA = h->ldA;
    s.pd = P<double4>(h->d_pd);
    s.cnt = P<uint32_t>(h->d_cnt);
    s.p_begin = ch.p_begin;
    s.nb = h->nb;
    s.lmax = h->lmax;
    s.sub_start = P<int>(h->d_subs) + ch.sub_off;
    s.nsub = nsub;
    s.sub_base = ch.sub_begin;
    s.part = P<double>(h->d_pself);
    s.fp64 = h->fp64;
    s.unit_w = h->unit_w ? 1 : 0;
    s.self_lo = h->self_lo ? 1 : 0;
    HIPCHK(launch_self_moments(s, h->stream));
    t_end(h, t);
    return TPCF_OK;
}

tpcf_status reduce_group(tpcf_handle h) {
    tpcf_status st;
    const int sw = h->nb * (2 * h->lmax + 2);
    if ((st = ensure(h, h->d_G, sizeof(double) * h->ncat * h->gsize)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_S, sizeof(double) * h->ncat * sw)) != TPCF_OK) return st;
    Timer t;
    t_begin(h, 3, t);
    HIPCHK(launch_reduce_partials(nullptr, P<double>(h->d_part), h->gsize,
                                  P<int>(h->d_catsub), h->ncat, P<double>(h->d_G), h->stream));
    HIPCHK(launch_reduce_partials(nullptr, P<double>(h->d_pself), sw, P<int>(h->d_catsub), h->ncat,
                                  P<double>(h->d_S), h->stream));
    t_end(h, t);
    return TPCF_OK;
}

tpcf_status check_mults(tpcf_handle h, int32_t n_mult, const int32_t* m) {
    if (n_mult < 1 || !m) return fail(h, TPCF_ERR_ARG, "n_mult must be >= 1 with a host triple array");
    for (int t = 0; t < n_mult; ++t) {
        const int l1 = m[3 * t], l2 = m[3 * t + 1], L = m[3 * t + 2];
        if (l1 < 0 || l2 < 0 || L < 0 || l1 > h->lmax || l2 > h->lmax || L < std::abs(l1 - l2) ||
            L > l1 + l2 || ((l1 + l2 + L) & 1))
            return fail(h, TPCF_ERR_ARG, "invalid multipole triple (" + std::to_string(l1) + "," +
                                             std::to_string(l2) + "," + std::to_string(L) + ")");
        if ((h->cfg.flags & TPCF_F_ISOTROPIC) && L != 0)
            return fail(h, TPCF_ERR_ARG, "an isotropic handle gives only (l, l, 0) multipoles");
    }
    return TPCF_OK;
}

tpcf_status finalize_group(tpcf_handle h, int32_t n_mult, const int32_t* mult, double* d_out) {
    const int lmax = h->lmax, s1 = lmax + 1, nL = 2 * lmax + 1;
    std::vector<double> cg((size_t)n_mult * s1, 0.0), cs((size_t)n_mult * s1 * nL, 0.0);
    const bool lit = (h->cfg.flags & TPCF_F_PAPER_LITERAL) != 0;
    for (int t = 0; t < n_mult; ++t) {
        const int l1 = mult[3 * t], l2 = mult[3 * t + 1], L = mult[3 * t + 2];
        const double f = lit ? 4.0 * kPi / std::sqrt((2.0 * l1 + 1.0) * (2.0 * l2 + 1.0)) : 1.0;
        for (int m = 0; m <= std::min(l1, l2); ++m) {
            const double base = 8.0 * kPi * kPi * (2.0 * L + 1.0) * qv(h, l1, l2, m, L) * (m > 0 ? 2.0 : 1.0) * f;
            cg[t * s1 + m] = base * h->scale[l1 * s1 + m] * h->scale[l2 * s1 + m];
            // Degenerate triangles: the product of the two harmonics at one
            // point expands into self moments of every order L2, but summed
            // over m (with the 3j weights of this multipole) the coefficient
            // of each order L2 != L vanishes (orthogonality of the 3j symbols
            // (l1 l2 L; m -m 0) over m). Only the order-L term is kept, so the
            // result needs no self moment above L and carries no rounding
            // residue of the cancelling orders.
            cs[((size_t)t * s1 + m) * nL + L] = base * 0.5 * (2.0 * L + 1.0) * qv(h, l1, l2, m, L) * h->gamma0[L];
        }
    }
    tpcf_status st;
    if ((st = upload(h, h->d_mult, mult, sizeof(int) * 3 * n_mult)) != TPCF_OK) return st;
    if ((st = upload(h, h->d_coefG, cg.data(), sizeof(double) * cg.size())) != TPCF_OK) return st;
    if ((st = upload(h, h->d_coefS, cs.data(), sizeof(double) * cs.size())) != TPCF_OK) return st;
    if ((st = upload(h, h->d_nd, h->n_data.data(), sizeof(double) * h->ncat)) != TPCF_OK) return st;
    FinalArgs a{};
    a.G = P<double>(h->d_G);
    a.gsize = h->gsize;
    a.goff = P<int64_t>(h->d_goff);
    a.S = P<double>(h->d_S);
    a.nd = P<double>(h->d_nd);
    a.nb = h->nb;
    a.lmax = lmax;
    a.n_mult = n_mult;
    a.mult = P<int>(h->d_mult);
    a.coefG = P<double>(h->d_coefG);
    a.coefS = P<double>(h->d_coefS);
    a.vol = P<double>(h->d_vol);
    const double L = h->cfg.box;
    a.inv_box6 = 1.0 / (L * L * L * L * L * L);
    a.subtract_self = (h->cfg.flags & TPCF_F_KEEP_DEGENERATE) ? 0 : 1;
    a.out = d_out;
    a.ncat = h->ncat;
    Timer t;
    t_begin(h, 4, t);
    HIPCHK(launch_finalize(a, h->stream));
    t_end(h, t);
    return TPCF_OK;
}

tpcf_status check_nonfinite(tpcf_handle h) {
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, P<int>(h->d_flag), sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (flag) return fail(h, TPCF_ERR_DEVICE, std::to_string(flag) + " non-finite input position(s)");
    return TPCF_OK;
}

// pair pass over every chunk; contracts each chunk right away when the
// operand cannot be kept for the whole group. The chunks run without a host
// round trip; the list-overflow flag and the fix-up count are read once at
// the end, and a pass whose lists ran out of room is run again with twice the
// room (its partial sums are overwritten, not accumulated).
tpcf_status pair_pass(tpcf_handle h, bool contract_now) {
    tpcf_status st;
    for (int attempt = 0;; ++attempt) {
        HIPCHK(launch_fill_i32(P<int>(h->d_flag) + 1, 3, 0, h->stream));  // overflow, fix-up length and total
        for (const Chunk& ch : h->chunks) {
            if ((st = pair_chunk(h, ch)) != TPCF_OK) return st;
            if (contract_now && (st = contract_chunk(h, ch)) != TPCF_OK) return st;
        }
        int flag[3] = {0, 0, 0};
        HIPCHK(hipMemcpyAsync(flag, P<int>(h->d_flag) + 1, sizeof(flag), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        h->nfix_total += flag[2];
        if (!flag[0]) return TPCF_OK;
        const unsigned long long ncap = std::min<unsigned long long>(16000000000ull, h->list_cap * 2);
        if (attempt == 5 || ncap == h->list_cap) return fail(h, TPCF_ERR_ALLOC, "neighbour list capacity exhausted");
        h->list_cap = ncap;
        h->list_grow = std::min(h->list_grow * 2.0, 64.0);  // kept for the next groups and calls
        if ((st = ensure(h, h->d_list, (size_t)list_elem_bytes(h) * h->list_cap)) != TPCF_OK) return st;
    }
}

// Polar part of Y_lm for any sign of m: Y_lm = Theta_lm(cos t) e^{i m phi},
// Theta_lm = (-1)^m N_lm (1-z^2)^{m/2} d^m P_l/dz^m for m >= 0 (Condon-Shortley)
// and Theta_l,-m = (-1)^m Theta_lm (from Y_l,-m = (-1)^m conj(Y_lm)).
// th[(l * (2 lmax + 1)) + m + lmax] at one z.
void polar_parts(int lmax, double z, std::vector<double>& th) {
    const int S2 = 2 * lmax + 1;
    th.assign((size_t)(lmax + 1) * S2, 0.0);
    std::vector<double> R;
    for (int m = 0; m <= lmax; ++m) {
        r_chain(lmax, m, z, R);
        const double sm = std::pow(std::max(0.0, 1.0 - z * z), 0.5 * m);
        for (int l = m; l <= lmax; ++l) {
            const double nbar = norm_lm(l, m) * gamma_lm(l, m) * R[l] * sm;
            th[(size_t)l * S2 + m + lmax] = (m & 1) ? -nbar : nbar;
            th[(size_t)l * S2 - m + lmax] = nbar;
        }
    }
}

// g(l, m; l', m'; l'') = integral of conj(Y_lm) Y_l'm' Y_l'',m-m' over the
// sphere = 2 pi integral of Theta_lm Theta_l'm' Theta_l'',m-m' dz, by 64-point
// Gauss-Legendre quadrature (the integrand is a polynomial of degree at most
// 3 lmax). Layout [l][m >= 0][l'][m' + lmax][l''], exact zeros where the
// triangle rule, parity or |m - m'| > l'' forbid the coupling.
void build_edge_gaunt(int lmax, std::vector<double>& g) {
    const int S = lmax + 1, S2 = 2 * lmax + 1;
    g.assign((size_t)S * S * S * S2 * S, 0.0);
    std::vector<double> x, w, th;
    gauss_legendre(64, x, w);
    std::vector<std::vector<double>> T(x.size());
    for (size_t i = 0; i < x.size(); ++i) polar_parts(lmax, x[i], T[i]);
    for (int l = 0; l <= lmax; ++l)
        for (int m = 0; m <= l; ++m)
            for (int lp = 0; lp <= lmax; ++lp)
                for (int mp = -lp; mp <= lp; ++mp)
                    for (int lpp = 0; lpp <= lmax; ++lpp) {
                        const int mpp = m - mp;
                        if (std::abs(mpp) > lpp || lpp < std::abs(l - lp) || lpp > l + lp || ((l + lp + lpp) & 1))
                            continue;
                        double v = 0.0;
                        for (size_t i = 0; i < x.size(); ++i)
                            v += w[i] * T[i][(size_t)l * S2 + m + lmax] * T[i][(size_t)lp * S2 + mp + lmax] *
                                 T[i][(size_t)lpp * S2 + mpp + lmax];
                        g[((((size_t)l * S + m) * S + lp) * S2 + mp + lmax) * S + lpp] = 2.0 * kPi * v;
                    }
}

tpcf_status validate_config(const tpcf_config* c) {
    if (!c) return TPCF_ERR_ARG;
    if (!(c->box > 0.0) || !std::isfinite(c->box)) return TPCF_ERR_ARG;
    if (c->nbins < 1 || c->nbins > kMaxBins || !c->h_edges) return c->h_edges ? TPCF_ERR_RANGE : TPCF_ERR_ARG;
    for (int b = 0; b <= c->nbins; ++b)
        if (!std::isfinite(c->h_edges[b])) return TPCF_ERR_RANGE;
    for (int b = 0; b < c->nbins; ++b)
        if (!(c->h_edges[b + 1] > c->h_edges[b])) return TPCF_ERR_RANGE;
    if (c->h_edges[0] < 0.0 || c->h_edges[c->nbins] > 0.5 * c->box) return TPCF_ERR_RANGE;
    if (c->lmax < 0 || c->lmax > kMaxLmax) return TPCF_ERR_RANGE;
    if (c->precision < 0 || c->precision > 3) return TPCF_ERR_ARG;
    if (c->grid_refine < 0 || c->grid_refine > 4) return TPCF_ERR_RANGE;
    if (c->workspace_limit < 0) return TPCF_ERR_ARG;
    if (c->flags & ~(uint32_t)(TPCF_F_KEEP_DEGENERATE | TPCF_F_PAPER_LITERAL | TPCF_F_ISOTROPIC))
        return TPCF_ERR_ARG;
    const int mode = c->precision;
    if (contract_lds_bytes(mode, c->nbins, c->lmax) > 160 * 1024) return TPCF_ERR_RANGE;
    if (mode == TPCF_PREC_MIXED_BF16X3 &&
        contract_lds_bytes(TPCF_PREC_MIXED_BF16X6, c->nbins, c->lmax) > 160 * 1024)
        return TPCF_ERR_RANGE;
    return TPCF_OK;
}

// Steps 1-3 (and with d_out step 4) of ncat catalogues, in groups of whole
// catalogues whose points fit a quarter of the workspace. self_lo: every
// multipole asked for has L <= lmax.
// A catalogue with non-finite positions (status != nullptr): its status
// becomes TPCF_ERR_DEVICE, its output NaN, and the other catalogues of its
// group are run again without it.
tpcf_status run_groups(tpcf_handle h, int32_t ncat, const int64_t* h_n, const int64_t* h_n_data,
                       const double* d_pos, const double* d_w, bool self_lo, int32_t n_mult,
                       const int32_t* h_l1l2L, double* d_out, int32_t* status) {
    tpcf_status st;
    const int64_t per_point = 104;  // grid arrays per point (bytes)
    const int64_t max_pts = std::max<int64_t>(1, std::min<int64_t>((h->limit / 4) / per_point, (1LL << 31) - 1));
    int c0 = 0;
    int64_t pos_off = 0;
    const int64_t per_out = (int64_t)n_mult * h->nb * h->nb;
    while (c0 < ncat) {
        int c1 = c0;
        int64_t pts = 0;
        while (c1 < ncat && (c1 == c0 || pts + h_n[c1] <= max_pts)) pts += h_n[c1++];
        std::vector<int64_t> n(h_n + c0, h_n + c1), nd(h_n_data + c0, h_n_data + c1);
        h->stage = 0;
        if ((st = build_grid_group(h, d_pos + 3 * pos_off, d_w ? d_w + pos_off : nullptr, n, nd)) != TPCF_OK)
            return st;
        if ((st = check_nonfinite(h)) != TPCF_OK) {
            if (!status || st != TPCF_ERR_DEVICE) return st;
            // which catalogues: mark them, NaN their outputs, rerun the runs of good ones
            std::vector<int> bad(c1 - c0, 0);
            HIPCHK(hipMemcpyAsync(bad.data(), h->d_catbad.p, sizeof(int) * bad.size(), hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
            int r0 = c0;
            for (int c = c0; c <= c1; ++c) {
                const bool is_bad = c < c1 && bad[c - c0] > 0;
                if (c == c1 || is_bad) {
                    if (c > r0) {
                        // the good catalogues r0 .. c-1
                        int64_t o = pos_off;
                        for (int q = c0; q < r0; ++q) o += h_n[q];
                        if ((st = run_groups(h, c - r0, h_n + r0, h_n_data + r0, d_pos + 3 * o, d_w ? d_w + o : nullptr,
                                             self_lo, n_mult, h_l1l2L, d_out ? d_out + per_out * r0 : nullptr,
                                             status + r0)) != TPCF_OK)
                            return st;
                    }
                    if (is_bad) {
                        status[c] = TPCF_ERR_DEVICE;
                        if (d_out && per_out > 0)
                            HIPCHK(launch_fill_u64(reinterpret_cast<unsigned long long*>(d_out + per_out * c), per_out,
                                                   0x7ff8000000000000ull, h->stream));
                    }
                    r0 = c + 1;
                }
            }
            pos_off += pts;
            c0 = c1;
            continue;
        }
        if ((st = plan_chunks(h)) != TPCF_OK) return st;
        // The self moments of order above lmax cancel from every multipole
        // of L <= lmax (their coefficients sum to zero over m), and this run
        // keeps no per-m sums: the harmonic pass may stop them at lmax.
        h->self_lo = self_lo;
        h->self_cut = h->self_lo;
        // The multipoles use only the blocks with |l1 - l2| <= L: the
        // contraction may skip the others.
        int lc = 0;
        for (int t = 0; t < n_mult; ++t) lc = std::max(lc, std::abs(h_l1l2L[3 * t] - h_l1l2L[3 * t + 1]));
        h->couple = n_mult > 0 && lc < h->lmax ? lc : -1;
        h->couple_cut = h->couple;
        st = pair_pass(h, true);
        h->self_lo = false;
        h->couple = -1;
        if (st != TPCF_OK) return st;
        if ((st = reduce_group(h)) != TPCF_OK) return st;
        h->stage = 3;
        if (d_out && (st = finalize_group(h, n_mult, h_l1l2L, d_out + per_out * c0)) != TPCF_OK) return st;
        pos_off += pts;
        c0 = c1;
    }
    h->alm_kept = false;
    return TPCF_OK;
}

}  // namespace

// ================================================================ C ABI

extern "C" {

tpcf_status tpcf_create(const tpcf_config* cfg, int device, void* hip_stream, tpcf_handle* out) {
    if (!out) return TPCF_ERR_ARG;
    *out = nullptr;
    tpcf_status st = validate_config(cfg);
    if (st != TPCF_OK) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TPCF_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return TPCF_ERR_DEVICE;
    tpcf_handle h = new tpcf_handle_s();
    {
        std::lock_guard<std::mutex> lock(g_live_mu);
        live_handles().insert(h);
    }
    h->cfg = *cfg;
    h->edges.assign(cfg->h_edges, cfg->h_edges + cfg->nbins + 1);
    h->cfg.h_edges = h->edges.data();
    h->device = device;
    h->stream = (hipStream_t)hip_stream;
    h->nb = cfg->nbins;
    h->lmax = cfg->lmax;
    h->NV = n_values(cfg->lmax);
    h->mode = cfg->precision;  // contraction mode: 0 fp64, 1 fp32, 2 bf16x3, 3 bf16x6
    h->fp64 = cfg->precision == TPCF_PREC_FP64 ? 1 : 0;
    h->refine = cfg->grid_refine;
    h->limit = cfg->workspace_limit > 0 ? cfg->workspace_limit : (64LL << 30);
    // the device's address of the allocation-free covariance's scratch (looked
    // up once per device, with the device current)
    if (cov_scratch_init(device, &h->cov_scratch) != hipSuccess) {
        tpcf_destroy(h);
        return TPCF_ERR_DEVICE;
    }
    st = setup_constants(h);
    if (st != TPCF_OK) {
        tpcf_destroy(h);
        return st;
    }
    *out = h;
    return TPCF_OK;
}

void tpcf_destroy(tpcf_handle h) {
    {
        // unregister first: a second destroy, or a call racing this one, sees
        // a dead handle without reading it
        std::lock_guard<std::mutex> lock(g_live_mu);
        if (!h || live_handles().erase(h) == 0) return;
    }
    hipSetDevice(h->device);
    hipStreamSynchronize(h->stream);
    for (Timer& t : h->timers) {
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    DevBuf* all[] = {&h->d_e2, &h->d_e2f, &h->d_guard, &h->d_runs, &h->d_shift_f, &h->d_goff,
                     &h->d_vol, &h->d_scale, &h->d_sign_scale, &h->d_gaunt, &h->d_pt_off, &h->d_cellid,
                     &h->d_count, &h->d_start, &h->d_cursor, &h->d_tmp, &h->d_tmpz, &h->d_orig, &h->d_pf, &h->d_pw,
                     &h->d_pa, &h->d_istart, &h->d_icell, &h->d_icat, &h->d_scanw, &h->d_catbad, &h->d_pd, &h->d_perm, &h->d_catid, &h->d_flag, &h->d_list, &h->d_fix, &h->d_lcursor, &h->d_boff,
                     &h->d_cnt, &h->d_A, &h->d_subs, &h->d_catsub, &h->d_part, &h->d_pself, &h->d_G,
                     &h->d_S, &h->d_nd, &h->d_mult, &h->d_coefG, &h->d_coefS, &h->d_lflag,
                     &h->d_xiq, &h->d_xicoef, &h->d_xirr, &h->d_xiruns, &h->d_covx, &h->d_covoff,
                     &h->d_covflag, &h->d_covpart, &h->d_edgeT, &h->d_egaunt, &h->d_eunits, &h->d_errr,
                     &h->d_ecoef, &h->d_eM, &h->d_erhs, &h->d_ezeta, &h->d_emult};
    for (DevBuf* b : all) release(h, *b);
    delete h;
}

const char* tpcf_last_error(tpcf_handle h) {
    if (!alive(h)) return "invalid or destroyed tpcf handle";
    return h->err.c_str();
}

tpcf_status tpcf_build_grid(tpcf_handle h, const double* d_pos, const double* d_w, int64_t n,
                            int64_t n_data) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!d_pos) return fail(h, TPCF_ERR_ARG, "d_pos is NULL");
    if (n < 1 || n > (1LL << 27)) return fail(h, TPCF_ERR_ARG, "n must be in 1 .. 2^27");
    if (n_data < 3) return fail(h, TPCF_ERR_ARG, "n_data must be >= 3");
    HIPCHK(hipSetDevice(h->device));
    h->stage = 0;
    h->pairs_valid = false;
    h->self_cut = false;
    h->couple_cut = -1;
    tpcf_status st = build_grid_group(h, d_pos, d_w, {n}, {n_data});
    if (st != TPCF_OK) return st;
    h->stage = 1;
    return TPCF_OK;
}

tpcf_status tpcf_alm_accumulate(tpcf_handle h) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (h->stage < 1) return fail(h, TPCF_ERR_STATE, "tpcf_build_grid must come first");
    HIPCHK(hipSetDevice(h->device));
    tpcf_status st = check_nonfinite(h);
    if (st != TPCF_OK) return st;
    if ((st = plan_chunks(h)) != TPCF_OK) return st;
    const bool single = h->chunks.size() == 1;
    // the step calls keep every self-moment order and every block (h->self_lo
    // is false and h->couple is -1 here)
    h->self_cut = h->self_lo;
    h->couple_cut = h->couple;
    if ((st = pair_pass(h, !single)) != TPCF_OK) return st;
    h->alm_kept = single;
    h->contracted_in_pass = !single;
    h->pairs_valid = false;
    h->stage = 2;
    return TPCF_OK;
}

tpcf_status tpcf_get_alm(tpcf_handle h, int64_t first, int64_t count, double* d_out) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (h->stage < 2) return fail(h, TPCF_ERR_STATE, "tpcf_alm_accumulate must come first");
    if (!h->alm_kept) return fail(h, TPCF_ERR_STATE, "a_lm of this catalogue is not resident (several chunks)");
    if (!d_out || first < 0 || count < 0 || first + count > h->npts)
        return fail(h, TPCF_ERR_ARG, "bad primary range or NULL output");
    HIPCHK(hipSetDevice(h->device));
    AlmExportArgs a{};
    a.A = h->d_A.p;
    a.ldA = h->ldA;
    a.perm = P<int>(h->d_perm);
    a.p_begin = h->chunks[0].p_begin;
    a.first = first;
    a.count = count;
    a.nb = h->nb;
    a.lmax = h->lmax;
    a.sign_scale = P<double>(h->d_sign_scale);
    a.fp64 = h->fp64;
    a.out = d_out;
    HIPCHK(launch_export_alm(a, h->stream));
    return TPCF_OK;
}

tpcf_status tpcf_contract(tpcf_handle h, double* d_nnn_out) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (h->stage < 2) return fail(h, TPCF_ERR_STATE, "tpcf_alm_accumulate must come first");
    HIPCHK(hipSetDevice(h->device));
    tpcf_status st;
    if (h->stage == 2) {
        if (!h->contracted_in_pass)
            for (const Chunk& ch : h->chunks)
                if ((st = contract_chunk(h, ch)) != TPCF_OK) return st;
        if ((st = reduce_group(h)) != TPCF_OK) return st;
        h->stage = 3;
    }
    if (d_nnn_out) {
        if (h->self_cut || h->couple_cut >= 0 || h->ncat != 1)
            return fail(h, TPCF_ERR_STATE, "tpcf_run_catalogs keeps no per-m sums; use the step calls");
        NnnArgs a{};
        a.G = P<double>(h->d_G);
        a.goff = P<int64_t>(h->d_goff);
        a.S = P<double>(h->d_S);
        a.nb = h->nb;
        a.lmax = h->lmax;
        a.scale = P<double>(h->d_scale);
        a.gaunt = P<double>(h->d_gaunt);
        a.subtract_self = (h->cfg.flags & TPCF_F_KEEP_DEGENERATE) ? 0 : 1;
        a.isotropic = (h->cfg.flags & TPCF_F_ISOTROPIC) ? 1 : 0;
        a.out = d_nnn_out;
        HIPCHK(launch_export_nnn(a, h->stream));
    }
    return TPCF_OK;
}

tpcf_status tpcf_multipoles(tpcf_handle h, int32_t n_mult, const int32_t* h_l1l2L, double* d_out) {
    if (!alive(h)) return TPCF_ERR_ARG;
    tpcf_status st = check_mults(h, n_mult, h_l1l2L);
    if (st != TPCF_OK) return st;
    if (!d_out) return fail(h, TPCF_ERR_ARG, "d_out is NULL");
    if (h->stage < 3) return fail(h, TPCF_ERR_STATE, "tpcf_contract must come first");
    // d_out holds one catalogue's multipoles
    if (h->ncat != 1)
        return fail(h, TPCF_ERR_STATE, "the handle holds the sums of " + std::to_string(h->ncat) +
                                           " catalogues; tpcf_run_catalogs returns their multipoles");
    if (h->self_cut)
        for (int t = 0; t < n_mult; ++t)
            if (h_l1l2L[3 * t + 2] > h->lmax)
                return fail(h, TPCF_ERR_STATE, "the self moments of the last tpcf_run_catalogs stop at order lmax");
    if (h->couple_cut >= 0)
        for (int t = 0; t < n_mult; ++t)
            if (std::abs(h_l1l2L[3 * t] - h_l1l2L[3 * t + 1]) > h->couple_cut)
                return fail(h, TPCF_ERR_STATE, "the last tpcf_run_catalogs summed only the blocks with |l1 - l2| <= " +
                                                   std::to_string(h->couple_cut));
    HIPCHK(hipSetDevice(h->device));
    return finalize_group(h, n_mult, h_l1l2L, d_out);
}

tpcf_status tpcf_run_catalogs(tpcf_handle h, int32_t ncat, const int64_t* h_n, const int64_t* h_n_data,
                              const double* d_pos, const double* d_w, int32_t n_mult,
                              const int32_t* h_l1l2L, double* d_out) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (ncat < 1 || !h_n || !h_n_data || !d_pos || !d_out)
        return fail(h, TPCF_ERR_ARG, "ncat >= 1 and non-NULL h_n, h_n_data, d_pos, d_out required");
    tpcf_status st = check_mults(h, n_mult, h_l1l2L);
    if (st != TPCF_OK) return st;
    int max_L = 0;
    for (int t = 0; t < n_mult; ++t) max_L = std::max(max_L, (int)h_l1l2L[3 * t + 2]);
    for (int c = 0; c < ncat; ++c) {
        if (h_n[c] < 1 || h_n[c] > (1LL << 27)) return fail(h, TPCF_ERR_ARG, "catalogue size out of range");
        if (h_n_data[c] < 3) return fail(h, TPCF_ERR_ARG, "n_data must be >= 3");
    }
    HIPCHK(hipSetDevice(h->device));
    h->cat_status.assign(ncat, TPCF_OK);
    if ((st = run_groups(h, ncat, h_n, h_n_data, d_pos, d_w, max_L <= h->lmax, n_mult, h_l1l2L, d_out,
                         h->cat_status.data())) != TPCF_OK)
        return st;
    std::string badlist;
    int nbad = 0;
    for (int c = 0; c < ncat; ++c)
        if (h->cat_status[c] != TPCF_OK) {
            if (nbad < 8) badlist += (nbad ? ", " : "") + std::to_string(c);
            ++nbad;
        }
    if (nbad)
        return fail(h, TPCF_ERR_DEVICE, std::to_string(nbad) + " catalogue(s) with non-finite positions (" + badlist +
                                            (nbad > 8 ? ", ..." : "") +
                                            "): their outputs are NaN, the others are complete (tpcf_catalog_status)");
    return TPCF_OK;
}

tpcf_status tpcf_catalog_status(tpcf_handle h, int32_t ncat, int32_t* h_status) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!h_status || ncat != (int32_t)h->cat_status.size())
        return fail(h, TPCF_ERR_ARG, "h_status is NULL or ncat differs from the last tpcf_run_catalogs");
    std::copy(h->cat_status.begin(), h->cat_status.end(), h_status);
    return TPCF_OK;
}

tpcf_status tpcf_xi_count(tpcf_handle h, int32_t nmu, int64_t* d_counts) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!d_counts) return fail(h, TPCF_ERR_ARG, "d_counts is NULL");
    if (nmu < 1 || nmu > 4096) return fail(h, TPCF_ERR_RANGE, "nmu must be in 1 .. 4096");
    if ((int64_t)h->nb * nmu > kXiMaxBins) return fail(h, TPCF_ERR_RANGE, "nbins * nmu exceeds 16384");
    if (h->stage < 1) return fail(h, TPCF_ERR_STATE, "tpcf_build_grid must come first");
    if (h->ncat != 1) return fail(h, TPCF_ERR_STATE, "the 2PCF counts the catalogue of tpcf_build_grid");
    if (!h->unit_w) return fail(h, TPCF_ERR_ARG, "the 2PCF pair counts take unit weights (d_w = NULL)");
    // half stencil: every unordered pair of distinct cells once, and the home cell
    std::vector<StencilRun> half;
    for (const StencilRun& r : h->runs) {
        if (h->g.single || r.ox > 0 || (r.ox == 0 && r.oy > 0)) {
            half.push_back(r);
        } else if (r.ox == 0 && r.oy == 0) {
            if (r.oz_lo <= 0 && r.oz_hi >= 0) half.push_back({0, 0, 0, 0});
            if (r.oz_hi >= 1) half.push_back({0, 0, std::max(r.oz_lo, 1), r.oz_hi});
        }
    }
    const int npmax = 2 * (int)half.size();
    if (xi_lds_bytes(h->nb, nmu, npmax) > 160 * 1024)
        return fail(h, TPCF_ERR_RANGE, "the (r, mu) histogram does not fit the LDS");
    HIPCHK(hipSetDevice(h->device));
    tpcf_status st = check_nonfinite(h);  // also completes the copy of item_cat
    if (st != TPCF_OK) return st;
    if ((st = upload(h, h->d_xiruns, half.data(), sizeof(StencilRun) * std::max<size_t>(half.size(), 1))) != TPCF_OK)
        return st;
    if ((st = ensure(h, h->d_xiq, sizeof(int) * 8 * 32)) != TPCF_OK) return st;
    HIPCHK(launch_fill_i32(P<int>(h->d_xiq), 8 * 32, 0, h->stream));
    HIPCHK(launch_fill_u64(reinterpret_cast<unsigned long long*>(d_counts), (int64_t)h->nb * nmu, 0ull,
                           h->stream));
    XiArgs a{};
    a.pf = P<float4>(h->d_pf);
    a.pd = P<double4>(h->d_pd);
    a.cell_start = P<int>(h->d_start);
    a.runs = P<StencilRun>(h->d_xiruns);
    a.nruns = (int)half.size();
    {
        const int k = h->g.k, K2 = 2 * k + 1;
        a.home_code = (k * K2 + k) * K2 + k;
    }
    a.g = h->g;
    a.nb = h->nb;
    a.e2 = P<double>(h->d_e2);
    a.e2f = P<float>(h->d_e2f);
    a.guard = P<float>(h->d_guard);
    a.uniform = h->uniform;
    a.e0f = (float)h->edges[0];
    a.inv_dr = h->inv_dr;
    a.delta = h->delta;
    a.inv_boxf = (float)(1.0 / h->cfg.box);
    a.reach2 = (float)(h->edges[h->nb] * h->edges[h->nb] * (1.0 + 2e-4));
    a.nmu = nmu;
    a.hmu = nmu / 2.0;
    a.hmu_f = (float)a.hmu;
    // Error bound of t = (mu + 1) nmu / 2 in FP32. Each separation component
    // is within dd of its exact value (the bound of the radial guard bands),
    // so mu = dz / r is within (1 + sqrt 3) dd / r, plus a few ulp of the
    // square root, reciprocal and product; the fused t adds half an ulp.
    {
        const double span = h->g.single ? h->cfg.box : (h->g.k + 1) * h->g.h;
        const double dd = 4.0 * ulp32(span);
        a.gmu_a = (float)(a.hmu * (1.0 + std::sqrt(3.0)) * dd);
        a.gmu_b = (float)(2.0 * (a.hmu * 4.0 * std::ldexp(1.0, -23) + nmu * std::ldexp(1.0, -24)));
    }
    a.item_start = P<int>(h->d_istart);
    a.item_cell = P<int>(h->d_icell);
    a.nitems = h->item_cat[1] - h->item_cat[0];
    a.npmax = npmax;
    a.counts = reinterpret_cast<unsigned long long*>(d_counts);
    a.queue = P<int>(h->d_xiq);
    Timer t;
    t_begin(h, 5, t);
    HIPCHK(launch_xi_count(a, h->stream));
    t_end(h, t);
    return TPCF_OK;
}

tpcf_status tpcf_xi_multipoles(tpcf_handle h, int32_t nmu, const int64_t* d_counts, int64_t n_data,
                               int32_t n_ell, const int32_t* h_ells, double* d_out) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!d_counts || !d_out || !h_ells) return fail(h, TPCF_ERR_ARG, "NULL counts, ells or output");
    if (nmu < 1 || nmu > 4096) return fail(h, TPCF_ERR_RANGE, "nmu must be in 1 .. 4096");
    if (n_data < 2) return fail(h, TPCF_ERR_ARG, "n_data must be >= 2");
    if (n_ell < 1 || n_ell > 64) return fail(h, TPCF_ERR_ARG, "n_ell must be in 1 .. 64");
    for (int i = 0; i < n_ell; ++i)
        if (h_ells[i] < 0 || h_ells[i] > 60) return fail(h, TPCF_ERR_ARG, "multipole orders must be in 0 .. 60");
    HIPCHK(hipSetDevice(h->device));
    // c_lk = (2l+1)/2 times the integral of P_l over mu bin k, by 32-point
    // Gauss-Legendre quadrature on the bin (exact for the degrees allowed)
    std::vector<double> gx, gw;
    gauss_legendre(32, gx, gw);
    std::vector<double> coef((size_t)n_ell * nmu);
    for (int i = 0; i < n_ell; ++i) {
        const int l = h_ells[i];
        for (int k = 0; k < nmu; ++k) {
            const double lo = -1.0 + 2.0 * k / nmu, hi = -1.0 + 2.0 * (k + 1) / nmu;
            const double c = 0.5 * (lo + hi), hw = 0.5 * (hi - lo);
            double s = 0.0;
            for (size_t q = 0; q < gx.size(); ++q) {
                const double x = c + hw * gx[q];
                double p0 = 1.0, p1 = x;
                double pl = l == 0 ? 1.0 : x;
                for (int n = 1; n < l; ++n) {
                    pl = ((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0);
                    p0 = p1;
                    p1 = pl;
                }
                s += gw[q] * pl;
            }
            coef[(size_t)i * nmu + k] = 0.5 * (2.0 * l + 1.0) * hw * s;
        }
    }
    // analytic random pairs of one (r, mu) bin in a periodic box
    std::vector<double> rr(h->nb);
    const double nd = (double)n_data, L3 = h->cfg.box * h->cfg.box * h->cfg.box;
    for (int b = 0; b < h->nb; ++b) rr[b] = nd * (nd - 1.0) * h->vol[b] / (nmu * L3);
    tpcf_status st;
    if ((st = upload(h, h->d_xicoef, coef.data(), sizeof(double) * coef.size())) != TPCF_OK) return st;
    if ((st = upload(h, h->d_xirr, rr.data(), sizeof(double) * rr.size())) != TPCF_OK) return st;
    XiFinalArgs a{};
    a.counts = reinterpret_cast<const long long*>(d_counts);
    a.nb = h->nb;
    a.nmu = nmu;
    a.n_ell = n_ell;
    a.coef = P<double>(h->d_xicoef);
    a.rr = P<double>(h->d_xirr);
    a.out = d_out;
    Timer t;
    t_begin(h, 4, t);
    HIPCHK(launch_xi_finalize(a, h->stream));
    t_end(h, t);
    return TPCF_OK;
}

tpcf_status tpcf_triangle_index(int32_t nbins, const double* h_edges, double eta, double r_min, int32_t n_rows,
                                const int32_t* h_rows, int64_t capacity, int64_t* h_offsets, int64_t* h_count) {
    if (nbins < 1 || nbins > kMaxBins || !h_edges || n_rows < 0 || (n_rows > 0 && !h_rows) || !h_count ||
        capacity < 0 || (capacity > 0 && !h_offsets) || !(eta >= 0.0) || !std::isfinite(r_min))
        return TPCF_ERR_ARG;
    const double e0 = h_edges[0], dr = (h_edges[nbins] - e0) / nbins;
    if (!(dr > 0.0)) return TPCF_ERR_RANGE;
    for (int b = 0; b <= nbins; ++b)
        if (std::fabs(h_edges[b] - (e0 + b * dr)) > 1e-9 * dr) return TPCF_ERR_RANGE;  // equal-width bins
    for (int t = 0; t < n_rows; ++t)
        if (h_rows[t] < 0) return TPCF_ERR_ARG;
    int64_t n = 0;
    for (int t = 0; t < n_rows; ++t)
        for (int b1 = 0; b1 < nbins; ++b1)
            for (int b2 = b1 + 1; b2 < nbins; ++b2) {
                const double r1 = e0 + (b1 + 0.5) * dr, r2 = e0 + (b2 + 0.5) * dr;
                if (r2 - r1 < (eta - 1e-9) * dr || r1 < r_min - 1e-9 * dr) continue;
                if (n < capacity) h_offsets[n] = ((int64_t)h_rows[t] * nbins + b1) * nbins + b2;
                ++n;
            }
    *h_count = n;
    return n > capacity && capacity > 0 ? TPCF_ERR_RANGE : TPCF_OK;
}

tpcf_status tpcf_covariance(tpcf_handle h, int32_t n_mocks, int64_t stride, const double* d_src, int32_t n_d,
                            const int64_t* h_offsets, double* d_mean, double* d_cov) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!d_src || !d_cov) return fail(h, TPCF_ERR_ARG, "NULL source or covariance");
    if (n_mocks < 2) return fail(h, TPCF_ERR_ARG, "n_mocks must be >= 2");
    if (n_d < 1 || stride < 1) return fail(h, TPCF_ERR_ARG, "n_d and stride must be >= 1");
    if (!h_offsets && n_d > stride) return fail(h, TPCF_ERR_ARG, "n_d > stride without offsets");
    if (h_offsets)
        for (int i = 0; i < n_d; ++i)
            if (h_offsets[i] < 0 || h_offsets[i] >= stride) return fail(h, TPCF_ERR_ARG, "offset outside a mock's row");
    HIPCHK(hipSetDevice(h->device));
    tpcf_status st;
    if ((st = ensure(h, h->d_covx, sizeof(double) * (size_t)n_mocks * n_d)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_covpart, sizeof(double) * (size_t)cov_part_doubles(n_mocks, n_d))) != TPCF_OK)
        return st;
    const int64_t* doff = nullptr;
    if (h_offsets) {
        if ((st = upload(h, h->d_covoff, h_offsets, sizeof(int64_t) * n_d)) != TPCF_OK) return st;
        doff = P<int64_t>(h->d_covoff);
    }
    HIPCHK(launch_cov(d_src, stride, doff, n_mocks, n_d, P<double>(h->d_covx), P<double>(h->d_covpart), d_mean, d_cov,
                      h->stream));
    return TPCF_OK;
}

tpcf_status tpcf_covariance_noalloc(tpcf_handle h, int32_t n_mocks, int64_t stride, const double* d_src, int32_t n_d,
                                    const int64_t* d_offsets, double* d_mean, double* d_cov) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!d_src || !d_cov) return fail(h, TPCF_ERR_ARG, "NULL source or covariance");
    if (n_mocks < 2) return fail(h, TPCF_ERR_ARG, "n_mocks must be >= 2");
    if (n_d < 1 || stride < 1) return fail(h, TPCF_ERR_ARG, "n_d and stride must be >= 1");
    if (!d_offsets && n_d > stride) return fail(h, TPCF_ERR_ARG, "n_d > stride without offsets");
    const int64_t need = cov_scratch_need(n_mocks, n_d);
    if (need > kCovScratchBytes)
        return fail(h, TPCF_ERR_RANGE, "n_mocks x n_d needs " + std::to_string(need) + " bytes of scratch, over the " +
                                           std::to_string(kCovScratchBytes) + " of the allocation-free covariance");
    if (!h->cov_scratch) return fail(h, TPCF_ERR_STATE, "no scratch address for this device");
    HIPCHK(hipSetDevice(h->device));
    double* X = static_cast<double*>(h->cov_scratch);
    double* part = X + (int64_t)n_mocks * n_d;
    HIPCHK(launch_cov(d_src, stride, d_offsets, n_mocks, n_d, X, part, d_mean, d_cov, h->stream));
    return TPCF_OK;
}

tpcf_status tpcf_precision_matrix(tpcf_handle h, int32_t n_d, const double* d_cov, int32_t n_mocks, double* d_prec) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!d_cov || !d_prec) return fail(h, TPCF_ERR_ARG, "NULL covariance or output");
    if (n_d < 1 || n_d > 4096) return fail(h, TPCF_ERR_RANGE, "n_d must be in 1 .. 4096");
    if (n_mocks < n_d + 3) return fail(h, TPCF_ERR_RANGE, "the Hartlap factor needs n_mocks >= n_d + 3");
    HIPCHK(hipSetDevice(h->device));
    tpcf_status st;
    if ((st = ensure(h, h->d_covflag, sizeof(int))) != TPCF_OK) return st;
    HIPCHK(launch_fill_i32(P<int>(h->d_covflag), 1, 0, h->stream));
    if (d_prec != d_cov)
        HIPCHK(hipMemcpyAsync(d_prec, d_cov, sizeof(double) * (size_t)n_d * n_d, hipMemcpyDeviceToDevice, h->stream));
    const double hartlap = (n_mocks - n_d - 2.0) / (n_mocks - 1.0);
    if ((st = ensure(h, h->d_covpart, sizeof(double) * (size_t)n_d * n_d)) != TPCF_OK) return st;
    HIPCHK(launch_cov_invert(d_prec, P<double>(h->d_covpart), n_d, hartlap, P<int>(h->d_covflag), h->stream));
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, h->d_covflag.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (bad) return fail(h, TPCF_ERR_RANGE, "the covariance is not positive definite");
    return TPCF_OK;
}

tpcf_status tpcf_percival_m1(int32_t n_mocks, int32_t n_d, int32_t n_params, double* h_m1) {
    if (!h_m1 || n_params < 0 || n_d < 1 || n_mocks < n_d + 5) return TPCF_ERR_ARG;
    const double nm = n_mocks, nd = n_d, np = n_params;
    const double den = (nm - nd - 1.0) * (nm - nd - 4.0);
    const double A = 2.0 / den, B = (nm - nd - 2.0) / den;
    *h_m1 = (1.0 + B * (nd - np)) / (1.0 + A + B * (np + 1.0));
    return TPCF_OK;
}

tpcf_status tpcf_autotune(tpcf_handle h, const double* d_pos, const double* d_w, int64_t n, int64_t n_data,
                          int32_t nmu, int32_t* h_refine, double* h_ms) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!d_pos || !h_refine) return fail(h, TPCF_ERR_ARG, "d_pos and h_refine are required");
    if (n < 1 || n > (1LL << 27)) return fail(h, TPCF_ERR_ARG, "n must be in 1 .. 2^27");
    if (n_data < 3) return fail(h, TPCF_ERR_ARG, "n_data must be >= 3");
    if (nmu < 0) return fail(h, TPCF_ERR_ARG, "nmu must be >= 0");
    if (nmu > 0 && d_w) return fail(h, TPCF_ERR_ARG, "the 2PCF pair counts take unit weights (d_w = NULL)");
    HIPCHK(hipSetDevice(h->device));
    tpcf_status st;
    int64_t* d_counts = nullptr;
    DevBuf counts;
    if (nmu > 0) {
        if ((st = ensure(h, counts, sizeof(int64_t) * (size_t)h->nb * nmu)) != TPCF_OK) return st;
        d_counts = P<int64_t>(counts);
    }
    const bool timing = h->timing;
    h->timing = false;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int best = 0, last_k = -1;
    double best_ms = 0.0;
    st = TPCF_OK;
    for (int k = 1; k <= 4 && st == TPCF_OK; ++k) {
        if (h_ms) h_ms[k - 1] = -1.0;
        h->refine = k;
        h->stage = 0;
        if ((st = build_grid_group(h, d_pos, d_w, {n}, {n_data})) != TPCF_OK) break;
        h->stage = 1;
        if (h->g.k == last_k || (h->g.k != k && !h->g.single)) continue;  // not admissible: fell back
        last_k = h->g.k;
        if ((st = check_nonfinite(h)) != TPCF_OK) break;
        if (nmu == 0 && (st = plan_chunks(h)) != TPCF_OK) break;
        // one untimed pass, then the timed one
        double ms = 0.0;
        for (int rep = 0; rep < 2 && st == TPCF_OK; ++rep) {
            if (hipEventRecord(e0, h->stream) != hipSuccess) { st = fail(h, TPCF_ERR_DEVICE, "hipEventRecord"); break; }
            st = nmu > 0 ? tpcf_xi_count(h, nmu, d_counts) : pair_pass(h, false);
            if (st != TPCF_OK) break;
            if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                st = fail(h, TPCF_ERR_DEVICE, "hipEvent");
                break;
            }
            float f = 0.f;
            hipEventElapsedTime(&f, e0, e1);
            ms = f;
        }
        if (st != TPCF_OK) break;
        if (h_ms) h_ms[k - 1] = ms;
        if (best == 0 || ms < best_ms) {
            best = h->g.single ? k : h->g.k;
            best_ms = ms;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    release(h, counts);
    h->timing = timing;
    h->stage = 0;  // the grid of the sample is not kept
    h->pairs_valid = false;
    if (st != TPCF_OK) {
        h->refine = h->cfg.grid_refine;
        return st;
    }
    h->refine = best;
    *h_refine = best;
    return TPCF_OK;
}

tpcf_status tpcf_set_plan(tpcf_handle h, const tpcf_plan* p) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!p) return fail(h, TPCF_ERR_ARG, "NULL plan");
    if (p->grid_refine < 0 || p->grid_refine > 4) return fail(h, TPCF_ERR_RANGE, "grid_refine must be in 0 .. 4");
    if (p->list_mode < -1 || p->list_mode > 1) return fail(h, TPCF_ERR_RANGE, "list_mode must be -1, 0 or 1");
    if (p->contract_step != 0 && p->contract_step != 16 && p->contract_step != 32 && p->contract_step != 64 &&
        p->contract_step != 128)
        return fail(h, TPCF_ERR_RANGE, "contract_step must be 0, 16, 32, 64 or 128");
    h->refine = p->grid_refine;
    h->list_mode = p->list_mode;
    h->contract_step = p->contract_step;
    h->stage = 0;  // a new plan applies from the next grid build
    return TPCF_OK;
}

tpcf_status tpcf_get_plan(tpcf_handle h, tpcf_plan* p) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!p) return fail(h, TPCF_ERR_ARG, "NULL plan");
    p->grid_refine = h->refine;
    p->list_mode = h->list_mode;
    p->contract_step = h->contract_step;
    p->reserved = 0;
    p->ms = 0.0;
    return TPCF_OK;
}

tpcf_status tpcf_autotune_plan(tpcf_handle h, int32_t ncat, const int64_t* h_n, const int64_t* h_n_data,
                               const double* d_pos, const double* d_w, tpcf_plan* h_plan, double* h_ms) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (ncat < 1 || !h_n || !h_n_data || !d_pos || !h_plan)
        return fail(h, TPCF_ERR_ARG, "ncat >= 1 and non-NULL h_n, h_n_data, d_pos, h_plan required");
    for (int c = 0; c < ncat; ++c) {
        if (h_n[c] < 1 || h_n[c] > (1LL << 27)) return fail(h, TPCF_ERR_ARG, "catalogue size out of range");
        if (h_n_data[c] < 3) return fail(h, TPCF_ERR_ARG, "n_data must be >= 3");
    }
    HIPCHK(hipSetDevice(h->device));
    if (h_ms)
        for (int i = 0; i < kPlanCandidates; ++i) h_ms[i] = -1.0;
    const bool timing = h->timing;
    h->timing = false;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // the candidates: every admissible refinement; both list modes where the
    // wavefront kernel exists (FP32, lmax <= 6); for the split-BF16
    // contraction (not the isotropic one) the longest step and 64
    const bool wave_ok = !h->fp64 && h->lmax <= 6;
    const bool bf = (h->mode == TPCF_PREC_MIXED_BF16X3 || h->mode == TPCF_PREC_MIXED_BF16X6) &&
                    !(h->cfg.flags & TPCF_F_ISOTROPIC);
    const int steps[2] = {0, 64};
    tpcf_plan best{};
    best.ms = -1.0;
    tpcf_status st = TPCF_OK;
    int last_k = -1;
    for (int k = 1; k <= 4 && st == TPCF_OK; ++k) {
        // admissibility from the grid the first catalogue gets (a refinement
        // that does not fit falls back to a coarser one, or the one-cell grid)
        h->refine = k;
        h->stage = 0;
        if ((st = build_grid_group(h, d_pos, d_w, {h_n[0]}, {h_n_data[0]})) != TPCF_OK) break;
        if (h->g.k == last_k || (h->g.k != k && !h->g.single)) continue;
        last_k = h->g.k;
        for (int mode = 0; mode <= (wave_ok ? 1 : 0) && st == TPCF_OK; ++mode)
            for (int si = 0; si <= (bf ? 1 : 0) && st == TPCF_OK; ++si) {
                h->list_mode = mode;
                h->contract_step = steps[si];
                double ms = 0.0;
                // one untimed pass, then the timed one: grid build, pair pass, contraction
                bool fits = true;
                for (int rep = 0; rep < 2 && st == TPCF_OK; ++rep) {
                    if (hipEventRecord(e0, h->stream) != hipSuccess) { st = fail(h, TPCF_ERR_DEVICE, "hipEventRecord"); break; }
                    if ((st = run_groups(h, ncat, h_n, h_n_data, d_pos, d_w, true, 0, nullptr, nullptr, nullptr)) !=
                        TPCF_OK) {
                        // a candidate whose lists do not fit the workspace is not admissible
                        if (st == TPCF_ERR_ALLOC) {
                            HIPCHK(hipStreamSynchronize(h->stream));
                            st = TPCF_OK;
                            fits = false;
                        }
                        break;
                    }
                    if (hipEventRecord(e1, h->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                        st = fail(h, TPCF_ERR_DEVICE, "hipEvent");
                        break;
                    }
                    float f = 0.f;
                    hipEventElapsedTime(&f, e0, e1);
                    ms = f;
                }
                if (st != TPCF_OK) break;
                if (!fits) continue;
                if (h_ms) h_ms[((k - 1) * 2 + mode) * 2 + si] = ms;
                if (best.ms < 0.0 || ms < best.ms) {
                    best.grid_refine = h->g.single ? k : h->g.k;
                    best.list_mode = mode;
                    best.contract_step = steps[si];
                    best.ms = ms;
                }
            }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    h->timing = timing;
    h->stage = 0;  // the sample's grid and sums are not kept
    h->self_cut = false;
    h->couple_cut = -1;
    h->pairs_valid = false;
    if (st == TPCF_OK && best.ms < 0.0) st = fail(h, TPCF_ERR_ALLOC, "no plan fits the workspace");
    if (st != TPCF_OK) {
        h->refine = h->cfg.grid_refine;
        h->list_mode = -1;
        h->contract_step = 0;
        return st;
    }
    h->refine = best.grid_refine;
    h->list_mode = best.list_mode;
    h->contract_step = best.contract_step;
    *h_plan = best;
    return TPCF_OK;
}

tpcf_status tpcf_edge_correct_isotropic(tpcf_handle h, int32_t n_ell, const double* d_N, const double* d_R,
                                        double* d_out) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!d_N || !d_R || !d_out) return fail(h, TPCF_ERR_ARG, "NULL multipoles or output");
    if (n_ell < 1 || n_ell > 25) return fail(h, TPCF_ERR_RANGE, "n_ell must be in 1 .. 25");
    HIPCHK(hipSetDevice(h->device));
    // T[l][l'][l''] = (2l+1)/2 int_{-1}^{1} P_l P_l' P_l'' dx, by Gauss-Legendre quadrature
    // (exact: the integrand has degree <= 3 (n_ell - 1) <= 72 < 2 * 40)
    const int nl = n_ell;
    std::vector<double> gx, gw;
    gauss_legendre(40, gx, gw);
    std::vector<double> Pq(gx.size() * nl);
    for (size_t q = 0; q < gx.size(); ++q) {
        double p0 = 1.0, p1 = gx[q];
        for (int l = 0; l < nl; ++l) {
            double v;
            if (l == 0) v = 1.0;
            else if (l == 1) v = gx[q];
            else {
                v = ((2.0 * l - 1.0) * gx[q] * p1 - (l - 1.0) * p0) / l;
                p0 = p1;
                p1 = v;
            }
            Pq[q * nl + l] = v;
        }
    }
    std::vector<double> T((size_t)nl * nl * nl, 0.0);
    for (int l = 0; l < nl; ++l)
        for (int lp = 0; lp < nl; ++lp)
            for (int lpp = 0; lpp < nl; ++lpp) {
                double s = 0.0;
                for (size_t q = 0; q < gx.size(); ++q) s += gw[q] * Pq[q * nl + l] * Pq[q * nl + lp] * Pq[q * nl + lpp];
                T[((size_t)l * nl + lp) * nl + lpp] = 0.5 * (2.0 * l + 1.0) * s;
            }
    tpcf_status st;
    if ((st = upload(h, h->d_edgeT, T.data(), sizeof(double) * T.size())) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_covflag, sizeof(int))) != TPCF_OK) return st;
    HIPCHK(launch_fill_i32(P<int>(h->d_covflag), 1, 0, h->stream));
    HIPCHK(launch_edge_iso(d_N, d_R, P<double>(h->d_edgeT), nl, h->nb * h->nb, d_out, P<int>(h->d_covflag), h->stream));
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, h->d_covflag.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (bad) return fail(h, TPCF_ERR_RANGE, "singular coupling matrix (random multipoles)");
    return TPCF_OK;
}

tpcf_status tpcf_edge_correct(tpcf_handle h, const double* d_nnn_N, int64_t n_data_N, const double* d_nnn_R,
                              int64_t n_data_R, int32_t n_mult, const int32_t* h_l1l2L, double* d_out,
                              double* d_zeta) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!d_nnn_N || !d_nnn_R) return fail(h, TPCF_ERR_ARG, "NULL triplet-count coefficients");
    if (!d_out && !d_zeta) return fail(h, TPCF_ERR_ARG, "neither multipoles nor coefficients requested");
    if (n_data_N < 3 || n_data_R < 3) return fail(h, TPCF_ERR_ARG, "n_data must be >= 3 for both runs");
    if (h->lmax > kMaxEdgeLmax) return fail(h, TPCF_ERR_RANGE, "the anisotropic edge correction needs lmax <= 10");
    tpcf_status st;
    if (d_out) {
        if ((st = check_mults(h, n_mult, h_l1l2L)) != TPCF_OK) return st;
    } else {
        n_mult = 0;
    }
    HIPCHK(hipSetDevice(h->device));
    const int lmax = h->lmax, S = lmax + 1, nb = h->nb, nsys = nb * nb;
    std::vector<int4> units;
    for (int m = 0; m <= lmax; ++m)
        for (int l1 = m; l1 <= lmax; ++l1)
            for (int l2 = m; l2 <= lmax; ++l2) units.push_back(make_int4(l1, l2, m, 0));
    const int n = (int)units.size();
    if (h->egaunt_lmax != lmax) {
        std::vector<double> g;
        build_edge_gaunt(lmax, g);
        if ((st = upload(h, h->d_egaunt, g.data(), sizeof(double) * g.size())) != TPCF_OK) return st;
        h->egaunt_lmax = lmax;
    }
    // 1 / RRR of both runs (analytic periodic-box counts), [run][b1 nb + b2]
    std::vector<double> irrr(2 * (size_t)nsys);
    const double L = h->cfg.box, L6 = L * L * L * L * L * L;
    for (int r = 0; r < 2; ++r) {
        const double nd = (double)(r == 0 ? n_data_N : n_data_R);
        for (int b1 = 0; b1 < nb; ++b1)
            for (int b2 = 0; b2 < nb; ++b2)
                irrr[(size_t)r * nsys + b1 * nb + b2] = L6 / (nd * (nd - 1.0) * (nd - 2.0) * h->vol[b1] * h->vol[b2]);
    }
    // TripoSH weight of zeta^m in c_{l1 l2 L}: 8 pi^2 (2L+1) q(l1, l2, m, L), doubled for m > 0
    // (zeta^-m = zeta^m), as in the multipoles of the contraction
    std::vector<double> coef((size_t)std::max(n_mult, 1) * S, 0.0);
    const bool lit = (h->cfg.flags & TPCF_F_PAPER_LITERAL) != 0;
    for (int t = 0; t < n_mult; ++t) {
        const int l1 = h_l1l2L[3 * t], l2 = h_l1l2L[3 * t + 1], LL = h_l1l2L[3 * t + 2];
        const double f = lit ? 4.0 * kPi / std::sqrt((2.0 * l1 + 1.0) * (2.0 * l2 + 1.0)) : 1.0;
        for (int m = 0; m <= std::min(l1, l2); ++m)
            coef[(size_t)t * S + m] = 8.0 * kPi * kPi * (2.0 * LL + 1.0) * qv(h, l1, l2, m, LL) * (m > 0 ? 2.0 : 1.0) * f;
    }
    if ((st = upload(h, h->d_eunits, units.data(), sizeof(int4) * units.size())) != TPCF_OK) return st;
    if ((st = upload(h, h->d_errr, irrr.data(), sizeof(double) * irrr.size())) != TPCF_OK) return st;
    if ((st = upload(h, h->d_ecoef, coef.data(), sizeof(double) * coef.size())) != TPCF_OK) return st;
    if (n_mult > 0 && (st = upload(h, h->d_emult, h_l1l2L, sizeof(int) * 3 * n_mult)) != TPCF_OK) return st;
    const int64_t nz = (int64_t)S * S * S * nsys;
    if ((st = ensure(h, h->d_eM, sizeof(double) * (size_t)nsys * n * n)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_erhs, sizeof(double) * (size_t)nsys * n)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_ezeta, sizeof(double) * (size_t)nz)) != TPCF_OK) return st;
    if ((st = ensure(h, h->d_covflag, sizeof(int))) != TPCF_OK) return st;
    HIPCHK(launch_fill_i32(P<int>(h->d_covflag), 1, 0, h->stream));
    HIPCHK(launch_fill_u64(P<unsigned long long>(h->d_ezeta), nz, 0ull, h->stream));
    EdgeArgs a{};
    a.N = d_nnn_N;
    a.R = d_nnn_R;
    a.inv_rrr_N = P<double>(h->d_errr);
    a.inv_rrr_R = P<double>(h->d_errr) + nsys;
    a.gaunt = P<double>(h->d_egaunt);
    a.units = P<int4>(h->d_eunits);
    a.n = n;
    a.lmax = lmax;
    a.nsys = nsys;
    a.M = P<double>(h->d_eM);
    a.rhs = P<double>(h->d_erhs);
    a.zeta = P<double>(h->d_ezeta);
    a.bad = P<int>(h->d_covflag);
    a.n_mult = n_mult;
    a.mult = n_mult > 0 ? P<int>(h->d_emult) : nullptr;
    a.coef = P<double>(h->d_ecoef);
    a.out = d_out;
    Timer t;
    t_begin(h, 4, t);
    HIPCHK(launch_edge_aniso(a, h->stream));
    t_end(h, t);
    if (d_zeta)
        HIPCHK(hipMemcpyAsync(d_zeta, h->d_ezeta.p, sizeof(double) * (size_t)nz, hipMemcpyDeviceToDevice, h->stream));
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, h->d_covflag.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (bad) return fail(h, TPCF_ERR_RANGE, "singular coupling matrix (random triplet counts)");
    return TPCF_OK;
}

tpcf_status tpcf_sync(tpcf_handle h) {
    if (!alive(h)) return TPCF_ERR_ARG;
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipStreamSynchronize(h->stream));
    return TPCF_OK;
}

tpcf_status tpcf_rebinned_count(tpcf_handle h, int64_t* h_out) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!h_out) return fail(h, TPCF_ERR_ARG, "h_out is NULL");
    *h_out = h->nfix_total;
    return TPCF_OK;
}

tpcf_status tpcf_pair_count(tpcf_handle h, int64_t* h_out) {
    if (!alive(h)) return TPCF_ERR_ARG;
    if (!h_out) return fail(h, TPCF_ERR_ARG, "h_out is NULL");
    if (h->stage < 3) return fail(h, TPCF_ERR_STATE, "pair counts are available after tpcf_contract");
    HIPCHK(hipSetDevice(h->device));
    const int sw = h->nb * (2 * h->lmax + 2);
    std::vector<double> S((size_t)h->ncat * sw);
    HIPCHK(hipMemcpyAsync(S.data(), h->d_S.p, sizeof(double) * S.size(), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    double tot = 0.0;
    for (int c = 0; c < h->ncat; ++c)
        for (int b = 0; b < h->nb; ++b) tot += S[(size_t)c * sw + b * (2 * h->lmax + 2) + 2 * h->lmax + 1];
    *h_out = (int64_t)std::llround(tot);
    return TPCF_OK;
}

tpcf_status tpcf_set_timing(tpcf_handle h, int enable) {
    if (!alive(h)) return TPCF_ERR_ARG;
    h->timing = enable != 0;
    return TPCF_OK;
}

tpcf_status tpcf_stage_times(tpcf_handle h, int32_t n, double* h_ms, int64_t* h_launches) {
    if (!alive(h)) return TPCF_ERR_ARG;
    HIPCHK(hipSetDevice(h->device));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (Timer& t : h->timers) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, t.a, t.b);
        h->ms[t.stage] += ms;
        h->nl[t.stage] += 1;
        hipEventDestroy(t.a);
        hipEventDestroy(t.b);
    }
    h->timers.clear();
    for (int i = 0; i < kStages && i < n; ++i) {
        if (h_ms) h_ms[i] = h->ms[i];
        if (h_launches) h_launches[i] = h->nl[i];
    }
    for (int i = 0; i < kStages; ++i) {
        h->ms[i] = 0.0;
        h->nl[i] = 0;
    }
    return TPCF_OK;
}

}  // extern "C"
