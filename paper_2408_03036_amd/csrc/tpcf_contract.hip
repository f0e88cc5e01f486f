// Contraction of the per-primary harmonic coefficients into the global
// moments (arXiv:2408.03036, eq. (measured_mult) averaged over positions, with
// m = m' for the common line of sight):
//
//   G_m[(b1,l1),(b2,l2)] = sum_p w_p Re(A_l1m(p,b1) conj(A_l2m(p,b2)))
//                        = sum over rows (p, re|im) of w_p X[row][c1] X[row][c2]
//
// i.e. a symmetric rank-K update (K = primaries, two rows per primary for
// m >= 1) of a K_m x K_m matrix, K_m = nbins (lmax - m + 1). It runs on MFMA:
//   mode 0: FP64 16x16x4 (plain double path)
//   mode 1: FP32 32x32x2
//   mode 2: split-BF16: x = hi + lo with hi = bf16(x), lo = bf16(x - hi);
//           G ~ hi hi' + hi lo' + lo hi' on 32x32x16 BF16 MFMA, FP32 accumulate.
//   mode 3: x = hi + mid + lo (three BF16 pieces) and the six products whose
//           size is above 2^-24 |x y|: FP32-level accuracy.
// A workgroup owns one subchunk of primaries (a fixed slice of one catalogue)
// and a group of upper-triangle output tiles; it writes its partial sums, and
// the partials are reduced per catalogue in a fixed order in FP64, so the
// result does not depend on scheduling.
//
// The same file holds the isotropic schedule (the l1 = l2 blocks only), the
// degenerate-triangle moments, the fixed-order partial reduction, the final
// conversion to the tripolar multipoles (eq. (slep2sugy)) and the edge
// correction of isotropic multipoles by explicit random triplet counts.
#include <algorithm>
#include <type_traits>

#include "tpcf_internal.h"

namespace tpcf {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ inline unsigned short bf16_bits_rn(float x) {
    uint32_t u = __float_as_uint(x);
    // round to nearest even (inputs are finite)
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_float(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

template <int MODE> struct Cfg;
template <> struct Cfg<0> { static constexpr int TS = 16, KS = 32, TPW = 8, KSTEP = 4; };
template <> struct Cfg<1> { static constexpr int TS = 32, KS = 32, TPW = 4, KSTEP = 2; };
template <> struct Cfg<2> { static constexpr int TS = 32, KS = 64, TPW = 4, KSTEP = 16; };
template <> struct Cfg<3> { static constexpr int TS = 32, KS = 32, TPW = 4, KSTEP = 16; };

__device__ inline void tile_of(int t, int nt, int& ti, int& tj) {
    // t-th upper-triangle tile in row-major order
    int r = 0, rem = t;
    while (rem >= nt - r) { rem -= nt - r; ++r; }
    ti = r;
    tj = r + rem;
}

template <int MODE>
__global__ void __launch_bounds__(256) k_contract(ContractArgs a) {
    using C = Cfg<MODE>;
    constexpr int TS = C::TS, KS = C::KS, TPW = C::TPW;
    extern __shared__ unsigned char smem[];
    const int s = blockIdx.x;
    const int m = blockIdx.y;
    const int lmax = a.lmax, nb = a.nb;
    const int nl = lmax - m + 1;
    const int K = nb * nl;
    const int nt = (K + TS - 1) / TS;
    const int ntiles = nt * (nt + 1) / 2;
    const int t0 = blockIdx.z * 4 * TPW;
    if (t0 >= ntiles) return;
    const int parts = m == 0 ? 1 : 2;
    const int NV = n_values(lmax);
    const int voff = value_offset(lmax, m);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t pa = a.sub_start[s], pb = a.sub_start[s + 1];
    const int ncol = nt * TS;

    int ti[TPW], tj[TPW];
    bool tv[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int t = t0 + wave + 4 * q;
        tv[q] = t < ntiles;
        tile_of(tv[q] ? t : 0, nt, ti[q], tj[q]);
    }

    // LDS: X[col][k] (and weighted copy), stride KSP elements
    constexpr int KSP = MODE >= 2 ? KS + 8 : KS + 1;
    constexpr int NPC = MODE == 3 ? 3 : 2;  // BF16 pieces per value
    typedef typename std::conditional<MODE == 0, double, float>::type TA;
    // FP32 MFMA accumulators are emptied into FP64 registers after every
    // K-step (KS primaries), so single precision only ever sums a few dozen
    // products before the FP64 sum takes over.
    f32x16 acc32[TPW];
    f64x4 acc64[TPW];
    double accd[TPW][MODE == 0 ? 1 : 16];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        acc32[q] = (f32x16)0.0f;
        acc64[q] = (f64x4)0.0;
#pragma unroll
        for (int r = 0; r < (MODE == 0 ? 1 : 16); ++r) accd[q][r] = 0.0;
    }
    double* wts = reinterpret_cast<double*>(smem);  // KS weights
    unsigned char* xbase = smem + KS * sizeof(double);

    for (int64_t p0 = pa; p0 < pb; p0 += KS) {
        const int kk_valid = (int)min((int64_t)KS, pb - p0);
        for (int part = 0; part < parts; ++part) {
            __syncthreads();
            if (threadIdx.x < KS) {
                const int k = threadIdx.x;
                wts[k] = (k < kk_valid) ? a.pd[a.p_begin + p0 + k].w : 0.0;
            }
            __syncthreads();
            // stage columns
            for (int idx = threadIdx.x; idx < ncol * KS; idx += 256) {
                const int c = idx / KS, k = idx - c * KS;
                TA v = (TA)0;
                if (c < K && k < kk_valid) {
                    const int b = c / nl, lp = c - b * nl;
                    const int64_t row = (int64_t)b * NV + voff + part * nl + lp;
                    v = reinterpret_cast<const TA*>(a.A)[row * a.ldA + p0 + k];
                }
                if constexpr (MODE >= 2) {
                    // pieces of x in planes 0..NPC-1, pieces of w x in planes NPC..2NPC-1
                    unsigned short* xp = reinterpret_cast<unsigned short*>(xbase);
                    const int plane = ncol * KSP;
                    float r = (float)v;
#pragma unroll
                    for (int q = 0; q < NPC; ++q) {
                        const unsigned short hq = bf16_bits_rn(r);
                        xp[q * plane + c * KSP + k] = hq;
                        r -= bf16_to_float(hq);
                    }
                    if (!a.unit_weights) {
                        float rw = (float)((double)v * wts[k]);
#pragma unroll
                        for (int q = 0; q < NPC; ++q) {
                            const unsigned short hq = bf16_bits_rn(rw);
                            xp[(NPC + q) * plane + c * KSP + k] = hq;
                            rw -= bf16_to_float(hq);
                        }
                    }
                } else {
                    TA* X = reinterpret_cast<TA*>(xbase);
                    X[c * KSP + k] = v;
                }
            }
            __syncthreads();
            if constexpr (MODE == 0) {
                const double* X = reinterpret_cast<const double*>(xbase);
                const int i = lane & 15, kg = lane >> 4;
                for (int k0 = 0; k0 < KS; k0 += 4) {
                    const double wv = a.unit_weights ? 1.0 : wts[k0 + kg];
#pragma unroll
                    for (int q = 0; q < TPW; ++q) {
                        if (!tv[q]) continue;
                        const double av = X[(ti[q] * TS + i) * KSP + k0 + kg] * wv;
                        const double bv = X[(tj[q] * TS + i) * KSP + k0 + kg];
                        acc64[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc64[q], 0, 0, 0);
                    }
                }
            } else if constexpr (MODE == 1) {
                const float* X = reinterpret_cast<const float*>(xbase);
                const int i = lane & 31, kg = lane >> 5;
                for (int k0 = 0; k0 < KS; k0 += 2) {
                    const float wv = a.unit_weights ? 1.0f : (float)wts[k0 + kg];
#pragma unroll
                    for (int q = 0; q < TPW; ++q) {
                        if (!tv[q]) continue;
                        const float av = X[(ti[q] * TS + i) * KSP + k0 + kg] * wv;
                        const float bv = X[(tj[q] * TS + i) * KSP + k0 + kg];
                        acc32[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc32[q], 0, 0, 0);
                    }
                }
            } else {
                const unsigned short* xp = reinterpret_cast<const unsigned short*>(xbase);
                const int plane = ncol * KSP;
                const unsigned short* wp = a.unit_weights ? xp : xp + NPC * plane;
                const int i = lane & 31, kg = lane >> 5;
                for (int k0 = 0; k0 < KS; k0 += 16) {
#pragma unroll
                    for (int q = 0; q < TPW; ++q) {
                        if (!tv[q]) continue;
                        const int ra = (ti[q] * TS + i) * KSP + k0 + 8 * kg;
                        const int rb = (tj[q] * TS + i) * KSP + k0 + 8 * kg;
                        bf16x8 ap[NPC], bp[NPC];
#pragma unroll
                        for (int u = 0; u < NPC; ++u) {
                            ap[u] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(wp + u * plane + ra));
                            bp[u] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(xp + u * plane + rb));
                        }
                        // products of pieces u, v with u + v <= NPC - 1: hi.hi, hi.lo, lo.hi
                        // for two pieces; hi.hi, hi.mid, mid.hi, mid.mid, hi.lo, lo.hi for three
#pragma unroll
                        for (int u = 0; u < NPC; ++u)
#pragma unroll
                            for (int v2 = 0; v2 < NPC; ++v2)
                                if (u + v2 <= NPC - 1)
                                    acc32[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ap[u], bp[v2], acc32[q], 0, 0, 0);
                    }
                }
            }
        }
        if constexpr (MODE != 0) {
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
#pragma unroll
                for (int r = 0; r < 16; ++r) accd[q][r] += (double)acc32[q][r];
                acc32[q] = (f32x16)0.0f;
            }
        }
    }
    // write the partial tiles
    const int64_t sg = (int64_t)(a.sub_base + s);
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        if (!tv[q]) continue;
        if constexpr (MODE == 0) {
            const int j = lane & 15;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = (lane >> 4) + 4 * r;
                const int ci = ti[q] * TS + i, cj = tj[q] * TS + j;
                if (ci < K && cj < K)
                    a.part64[sg * a.gsize + a.goff[m] + (int64_t)ci * K + cj] = acc64[q][r];
            }
        } else {
            const int j = lane & 31;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int ci = ti[q] * TS + i, cj = tj[q] * TS + j;
                if (ci < K && cj < K)
                    a.part64[sg * a.gsize + a.goff[m] + (int64_t)ci * K + cj] = accd[q][r];
            }
        }
    }
}

// ---------------------------------------------------------------- FP64, double-buffered
// The FP64 contraction of k_contract<0> (16x16 tiles, eight per wavefront,
// 16x16x4 FP64 MFMA, the same LDS layout) with the staging of the
// split-BF16 kernel. Per step (KS primaries of one part) every thread owns up
// to kF64IPT items of four consecutive primaries of one column. Their loads
// for step st + 1 (two 16-byte loads per item, unconditional and in bounds:
// the operand buffer ends with 8 elements of padding, and an idle item or one
// past the step's primaries reads the start of the buffer or of its row) are
// issued before the MFMAs of step st and stored into the other LDS buffer
// after them, with the elements that are not the step's primaries zeroed.
// Used when the items of the widest m fit the workgroup and two buffers fit
// LDS; k_contract<0> covers the other shapes.
constexpr int kF64IPT = 4;

__host__ __device__ constexpr size_t f64db_lds(int ncol) {
    return 2 * (size_t)(Cfg<0>::KS + ncol * (Cfg<0>::KS + 1)) * sizeof(double);
}

template <bool W>
__global__ void __launch_bounds__(256) k_contract_f64(ContractArgs a) {
    using C = Cfg<0>;
    constexpr int TS = C::TS, KS = C::KS, TPW = C::TPW, KSP = KS + 1;
    extern __shared__ unsigned char smem[];
    const int s = blockIdx.x;
    const int m = blockIdx.y;
    const int lmax = a.lmax, nb = a.nb;
    const int nl = lmax - m + 1;
    const int K = nb * nl;
    const int nt = (K + TS - 1) / TS;
    const int ntiles = nt * (nt + 1) / 2;
    const int t0 = blockIdx.z * 4 * TPW;
    if (t0 >= ntiles) return;
    const int parts = m == 0 ? 1 : 2;
    const int NV = n_values(lmax);
    const int voff = value_offset(lmax, m);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t pa = a.sub_start[s], pb = a.sub_start[s + 1];
    const int ncol = nt * TS;

    int ti[TPW], tj[TPW];
    bool tv[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int t = t0 + wave + 4 * q;
        tv[q] = t < ntiles;
        tile_of(tv[q] ? t : 0, nt, ti[q], tj[q]);
    }
    f64x4 acc64[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc64[q] = (f64x4)0.0;

    // per buffer: KS weights, then X[col][k] with stride KSP
    const int bufd = KS + ncol * KSP;
    double* lds = reinterpret_cast<double*>(smem);
    const double* A = reinterpret_cast<const double*>(a.A);
    constexpr int groups = KS / 4;
    const int nitems = ncol * groups;
    const int nkst = (int)((pb - pa + KS - 1) / KS);
    const int nsteps = nkst * parts;

    // the thread's items: column c, primaries k4 .. k4+3 of the step
    int64_t irow[kF64IPT];
    int ioff[kF64IPT], ik4[kF64IPT];
    bool iok[kF64IPT], istore[kF64IPT];
#pragma unroll
    for (int u = 0; u < kF64IPT; ++u) {
        const int it = threadIdx.x + u * 256;
        const int c = it / groups, k4 = (it - c * groups) * 4;
        const int b = c / nl, lp = c - b * nl;
        istore[u] = it < nitems;
        iok[u] = it < nitems && c < K;
        ik4[u] = k4;
        ioff[u] = c * KSP + k4;
        irow[u] = ((int64_t)b * NV + voff + lp) * a.ldA;
    }
    const int64_t part_stride = (int64_t)nl * a.ldA;

    struct Stage {
        double x[kF64IPT][4];
        double w;
    };
    auto load = [&](int st, Stage& R) {
        const int part = st % parts;
        const int64_t p0 = pa + (int64_t)(st / parts) * KS;
        const int kv = (int)min((int64_t)KS, pb - p0);
#pragma unroll
        for (int u = 0; u < kF64IPT; ++u) {
            const int kk = ik4[u] < kv ? ik4[u] : 0;
            const double* src = A + (iok[u] ? irow[u] + part * part_stride + p0 + kk : 0);
            double2 v0, v1;
            __builtin_memcpy(&v0, src, 16);
            __builtin_memcpy(&v1, src + 2, 16);
            R.x[u][0] = v0.x;
            R.x[u][1] = v0.y;
            R.x[u][2] = v1.x;
            R.x[u][3] = v1.y;
        }
        if constexpr (W) {
            // thread k (< KS) stages the weight of primary k of the step
            const int k = threadIdx.x % KS;
            R.w = a.pd[a.p_begin + p0 + (k < kv ? k : 0)].w;
        }
    };
    auto store = [&](int st, int buf, const Stage& R) {
        double* base = lds + buf * bufd;
        const int64_t p0 = pa + (int64_t)(st / parts) * KS;
        const int kv = (int)min((int64_t)KS, pb - p0);
        if constexpr (W) {
            if (threadIdx.x < KS) base[threadIdx.x] = (int)threadIdx.x < kv ? R.w : 0.0;
        }
        double* X = base + KS;
#pragma unroll
        for (int u = 0; u < kF64IPT; ++u) {
            if (!istore[u]) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const bool ok = iok[u] && ik4[u] + e < kv;
                X[ioff[u] + e] = ok ? R.x[u][e] : 0.0;
            }
        }
    };
    const int i = lane & 15, kg = lane >> 4;
    auto compute = [&](int buf) {
        const double* base = lds + buf * bufd;
        const double* X = base + KS;
        for (int k0 = 0; k0 < KS; k0 += 4) {
            const double wv = W ? base[k0 + kg] : 1.0;
#pragma unroll
            for (int q = 0; q < TPW; ++q) {
                if (!tv[q]) continue;
                const double av = X[(ti[q] * TS + i) * KSP + k0 + kg] * wv;
                const double bv = X[(tj[q] * TS + i) * KSP + k0 + kg];
                acc64[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc64[q], 0, 0, 0);
            }
        }
    };

    Stage R;
    load(0, R);
    store(0, 0, R);
    __syncthreads();
    for (int st = 0; st < nsteps; ++st) {
        if (st + 1 < nsteps) load(st + 1, R);
        compute(st & 1);
        if (st + 1 < nsteps) store(st + 1, (st + 1) & 1, R);
        __syncthreads();
    }
    const int64_t sg = (int64_t)(a.sub_base + s);
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        if (!tv[q]) continue;
        const int j = lane & 15;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ii = (lane >> 4) + 4 * r;
            const int ci = ti[q] * TS + ii, cj = tj[q] * TS + j;
            if (ci < K && cj < K) a.part64[sg * a.gsize + a.goff[m] + (int64_t)ci * K + cj] = acc64[q][r];
        }
    }
}

// ---------------------------------------------------------------- isotropic schedule
// The isotropic multipoles are the L = 0 case of eq. (slep2sugy) (Sec. 2.3:
// the tripolar basis with L = 0 reduces to Legendre polynomials of the angle
// between r1 and r2), and they read only the l1 = l2 blocks of G_m:
//   G_m[(b1,l),(b2,l)] = sum_p w_p Re(A_lm(p,b1) conj(A_lm(p,b2))).
// One wavefront per (subchunk, (l, m)) forms that nb x nb block on 16x16x4
// MFMA in 16 x 16 tiles over (b1, b2) (up to 32 bins). A step covers 64
// primaries from a 16-aligned start: lane (i, g) = (lane % 16, lane / 16)
// loads 16 consecutive values of bin i (vector loads, masked to the subchunk)
// and feeds 16 MFMAs, each summing four primaries, one per lane group. FP64
// operands use FP64 MFMA; FP32 operands use FP32 MFMA, and the FP32 sums of
// one step (16 products per entry and chain) go into FP64 registers.
constexpr int kIsoWaves = 4;

// 16 consecutive values of one row (16-aligned), kept in their storage type
// until used: the next step's values are loaded while the current step's
// MFMAs run.
template <typename TA> struct Raw16;
typedef float fvec4 __attribute__((ext_vector_type(4)));
template <> struct Raw16<float> {
    fvec4 v[4];
    __device__ __forceinline__ void load(const float* src) {
        const fvec4* p = reinterpret_cast<const fvec4*>(src);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = p[q];
    }
    __device__ __forceinline__ double get(int k) const { return (double)v[k >> 2][k & 3]; }
};
template <> struct Raw16<double> {
    double2 v[8];
    __device__ __forceinline__ void load(const double* src) {
        const double2* p = reinterpret_cast<const double2*>(src);
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = p[q];
    }
    __device__ __forceinline__ double get(int k) const { return (k & 1) ? v[k >> 1].y : v[k >> 1].x; }
};

template <typename TA, bool W>
__global__ void __launch_bounds__(64 * kIsoWaves) k_contract_iso(ContractArgs a) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lmax = a.lmax, nb = a.nb;
    int u = blockIdx.y * kIsoWaves + wave;
    const int nlm = (lmax + 1) * (lmax + 2) / 2;
    if (u >= nlm) return;
    int m = 0;
    while (u >= lmax - m + 1) {  // units ordered m-major, l = m..lmax
        u -= lmax - m + 1;
        ++m;
    }
    const int l = m + u;
    const int nl = lmax - m + 1, K = nb * nl;
    const int parts = m == 0 ? 1 : 2;
    const int NV = n_values(lmax);
    const int v0 = value_offset(lmax, m) + (l - m);
    const int s = blockIdx.x;
    const int64_t pa = a.sub_start[s], pb = a.sub_start[s + 1];
    const int i = lane & 15, g = lane >> 4;
    const int nt = (nb + 15) / 16;  // 1 or 2 tiles of bins
    const TA* A = reinterpret_cast<const TA*>(a.A);
    // rows of bins i and 16 + i (clamped in range; their values are zeroed)
    const bool ok0 = i < nb, ok1 = nt > 1 && 16 + i < nb;
    const int64_t row0 = ((int64_t)min(i, nb - 1) * NV + v0) * a.ldA;
    const int64_t row1 = ((int64_t)min(16 + i, nb - 1) * NV + v0) * a.ldA;
    const int64_t pstep = (int64_t)nl * a.ldA;  // re -> im rows
    f64x4 acc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[q] = (f64x4)0.0;

    // steps of 64 primaries from a 16-aligned start; rows are padded to ldA
    // (a multiple of 64), so every 16-aligned group starting below pb is
    // inside its row
    const int64_t p00 = pa & ~(int64_t)15;
    const int nsteps = (int)((pb - p00 + 63) / 64);
    const int nit = nsteps * parts;
    auto group = [&](int it) { return p00 + (int64_t)(it / parts) * 64 + 16 * g; };
    // FP32 weights of a group are prefetched with its values (the weight
    // buffer ends with 16 floats of padding); FP64 reads them from the points
    constexpr bool F32 = std::is_same<TA, float>::value;
    constexpr bool WPRE = W && F32;
    struct Set {
        Raw16<TA> r0, r1;
        Raw16<float> w;
    };
    // Loads of iteration it into set S: unconditional, a group past the
    // subchunk reads the first group instead (its values are masked), so the
    // loads in flight are the same on every path and the wait before a set is
    // used covers only that set (a two-set ping-pong, no register rotation).
    auto fetch = [&](int it, Set& S) {
        int64_t q0 = group(it);
        if (q0 >= pb) q0 = p00;
        const int64_t off = (it % parts) * pstep + q0;
        S.r0.load(A + row0 + off);
        if (nt > 1) S.r1.load(A + row1 + off);
        if constexpr (WPRE) {
            // not 16-byte aligned in general
            const float* wsrc = a.pw + a.p_begin + q0;
#pragma unroll
            for (int q = 0; q < 4; ++q) __builtin_memcpy(&S.w.v[q], wsrc + 4 * q, 16);
        }
    };
    // FP32 operands: FP32 16x16x4 MFMA in two chains, emptied into FP64
    // after every step of 64 primaries (16 products per chain and entry)
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    double accd[3][4];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) accd[q][r] = 0.0;
    auto step = [&](int it, const Set& S) {
        const Raw16<TA>& c0 = S.r0;
        const Raw16<TA>& c1 = S.r1;
        const int64_t q0 = group(it);
        const int lo = (int)max<int64_t>(pa - q0, -1), hi = (int)min<int64_t>(pb - q0, 17);
        if constexpr (F32) {
            f32x4 sa[3], sb[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) sa[q] = sb[q] = (f32x4)0.0f;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const bool in = k >= lo && k < hi;
                const float x0 = (in && ok0) ? c0.v[k >> 2][k & 3] : 0.0f;
                const float wk = W ? (in ? S.w.v[k >> 2][k & 3] : 0.0f) : 1.0f;
                const float wa0 = W ? x0 * wk : x0;
                f32x4* acc = (k & 1) ? sb : sa;
                acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa0, x0, acc[0], 0, 0, 0);
                if (nt > 1) {
                    const float x1 = (in && ok1) ? c1.v[k >> 2][k & 3] : 0.0f;
                    acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa0, x1, acc[1], 0, 0, 0);
                    acc[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(W ? x1 * wk : x1, x1, acc[2], 0, 0, 0);
                }
            }
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) accd[q][r] += (double)sa[q][r] + (double)sb[q][r];
        } else {
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const bool in = k >= lo && k < hi;
                const double x0 = (in && ok0) ? c0.get(k) : 0.0;
                const double wk = W ? (in ? a.pd[a.p_begin + q0 + k].w : 0.0) : 1.0;
                const double wa0 = W ? x0 * wk : x0;
                acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa0, x0, acc[0], 0, 0, 0);
                if (nt > 1) {
                    const double x1 = (in && ok1) ? c1.get(k) : 0.0;
                    acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa0, x1, acc[1], 0, 0, 0);
                    acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(W ? x1 * wk : x1, x1, acc[2], 0, 0, 0);
                }
            }
        }
    };
    Set sA, sB;
    if (nit > 0) fetch(0, sA);
    for (int it = 0; it < nit; it += 2) {
        fetch(it + 1, sB);
        step(it, sA);
        fetch(it + 2, sA);
        if (it + 1 < nit) step(it + 1, sB);
    }
    // upper triangle of the block: tiles (0,0), (0,1), (1,1)
    const int64_t base = (int64_t)(a.sub_base + s) * a.gsize + a.goff[m];
    const int j = lane & 15;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        if (q > 0 && nt < 2) break;
        const int ti = q == 2 ? 1 : 0, tj = q == 0 ? 0 : 1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // output rows of a 16x16 MFMA: FP64 lane / 16 + 4 r, FP32 4 (lane / 16) + r
            const int c1r = 16 * ti + (F32 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r), c2 = 16 * tj + j;
            if (c1r < nb && c2 < nb && c1r <= c2)
                a.part64[base + (int64_t)(c1r * nl + (l - m)) * K + c2 * nl + (l - m)] =
                    F32 ? accd[q][r] : acc[q][r];
        }
    }
}

// ---------------------------------------------------------------- split-BF16 contraction
// One workgroup per (subchunk, m): eight wavefronts, up to two 32x32 output
// tiles each. Per step (KS primaries of one part, KS chosen per m), every
// thread stages 8 consecutive primaries of one column: two vector loads,
// packed round-to-nearest BF16 conversion of the pieces, one 16-byte LDS
// store per plane. Two LDS buffers: the loads of the next step are in flight
// while the MFMAs of the current one run. Columns are l-major, and a batched
// run forms only the tiles its multipoles couple (lcouple).
constexpr int kBfWaves = 8;
constexpr int kBfTPW = 2;
// staged 8-element groups per thread and step: four without weights, two with
// (the weighted staging also holds the weights)
template <bool W> constexpr int bf_ipt() { return W ? 2 : 4; }

// Step length (primaries) of each m, passed by value to the kernel.
struct BfSteps { int ks[kMaxLmax + 1]; };

// Step length of one m: the longest power of two from cap down to 16 whose
// staging fits the threads' registers (ncol * KS / 8 items of 8 primaries,
// ipt per thread) and whose nbuf LDS buffers fit in lds bytes; 0 if none.
// The narrow high-m operands thus take long steps, and their workgroups
// fewer of them: every step waits for its loads and a barrier.
inline int bf_step(int ncol, int nplanes, int ipt, int nbuf, int cap, size_t lds) {
    for (int ks = cap; ks >= 16; ks /= 2) {
        if ((int64_t)ncol * (ks / 8) > (int64_t)64 * kBfWaves * ipt) continue;
        if ((size_t)nbuf * nplanes * ncol * (ks + 8) * sizeof(uint16_t) > lds) continue;
        return ks;
    }
    return 0;
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

__device__ inline uint32_t cvt_pk_bf16(float a, float b) {
    bf16x2_t v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}

// Splits 8 floats into NPC BF16 pieces, piece q as 4 packed dwords.
template <int NPC>
__device__ inline void split8(float (&x)[8], uint4 (&out)[NPC]) {
#pragma unroll
    for (int q = 0; q < NPC; ++q) {
        uint32_t w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            w[j] = cvt_pk_bf16(x[2 * j], x[2 * j + 1]);
            if (q + 1 < NPC) {
                x[2 * j] -= __uint_as_float(w[j] << 16);
                x[2 * j + 1] -= __uint_as_float(w[j] & 0xffff0000u);
            }
        }
        out[q] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

template <bool W>
struct BfStage {
    float x[bf_ipt<W>()][8];
    float w[W ? bf_ipt<W>() : 1][8];
};

template <int NPC, bool W>
__global__ void __launch_bounds__(64 * kBfWaves) k_contract_bf16(ContractArgs a, BfSteps steps, int nbuf) {
    constexpr int TS = 32;
    extern __shared__ unsigned char smem[];
    const int s = blockIdx.x;
    const int m = blockIdx.y;
    const int lmax = a.lmax, nb = a.nb;
    const int nl = lmax - m + 1;
    const int K = nb * nl;
    const int nt = (K + TS - 1) / TS;
    const int t0 = blockIdx.z * kBfWaves * kBfTPW;
    const int parts = m == 0 ? 1 : 2;
    const int NV = n_values(lmax);
    const int voff = value_offset(lmax, m);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t pa = a.sub_start[s], pb = a.sub_start[s + 1];
    const int ncol = nt * TS;
    constexpr bool weighted = W;
    constexpr int IPT = bf_ipt<W>();
    const int nplanes = weighted ? 2 * NPC : NPC;
    const int KS = steps.ks[m];
    const int KSP = KS + 8;
    const int plane = ncol * KSP;                 // elements per plane
    const int bufsz = nplanes * plane;            // elements per buffer
    uint16_t* lds = reinterpret_cast<uint16_t*>(smem);
    const float* A = reinterpret_cast<const float*>(a.A);

    // Columns are l-major (column c holds l - m = c / nb of bin c % nb), so
    // the l of a 32-column tile spans a few consecutive values. The tiles of
    // the upper triangle whose columns couple some l1, l2 with |l1 - l2| <=
    // lcouple are the needed ones; this wave takes the (t0 + wave + 8 q)-th
    // of them in row-major order. (Along a row of tiles the smallest l
    // distance only grows, so a row ends at its first tile past the limit.)
    int ti[kBfTPW], tj[kBfTPW];
    bool tv[kBfTPW];
#pragma unroll
    for (int q = 0; q < kBfTPW; ++q) {
        ti[q] = tj[q] = 0;
        tv[q] = false;
    }
    int nneed = 0;
    for (int r = 0; r < nt; ++r) {
        const int lhi = (min(K, r * TS + TS) - 1) / nb;
        for (int c2 = r; c2 < nt; ++c2) {
            if (c2 * TS / nb - lhi > a.lcouple) break;
#pragma unroll
            for (int q = 0; q < kBfTPW; ++q)
                if (nneed == t0 + wave + kBfWaves * q) {
                    ti[q] = r;
                    tj[q] = c2;
                    tv[q] = true;
                }
            ++nneed;
        }
    }
    if (t0 >= nneed) return;
    f32x16 acc32[kBfTPW];
    double accd[kBfTPW][16];
#pragma unroll
    for (int q = 0; q < kBfTPW; ++q) {
        acc32[q] = (f32x16)0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) accd[q][r] = 0.0;
    }

    const int groups = KS / 8;
    const int nitems = ncol * groups;
    const int nkst = (int)((pb - pa + KS - 1) / KS);
    const int nsteps = nkst * parts;

    // The thread's staging items do not change from step to step: column c
    // and primaries k8..k8+7 of the step. Their A row (part 0), LDS offset and
    // validity are computed once.
    int64_t irow[IPT];
    int ioff[IPT], ik8[IPT];
    bool iok[IPT], istore[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
        const int it = threadIdx.x + u * 64 * kBfWaves;
        const int c = it / groups, k8 = (it - c * groups) * 8;
        const int lp = c / nb, b = c - lp * nb;
        istore[u] = it < nitems;
        iok[u] = it < nitems && c < K;
        ik8[u] = k8;
        ioff[u] = c * KSP + k8;
        irow[u] = ((int64_t)b * NV + voff + lp) * a.ldA;
    }
    const int64_t part_stride = (int64_t)nl * a.ldA;

    // Loads of step st into registers: two unconditional 16-byte loads per
    // item (and two of weights), all in bounds (the operand and the weight
    // buffers end with 8 elements of padding; an idle item, or one past the
    // step's primaries, reads the start of its row or of the buffer). The
    // elements that are not the step's primaries are zeroed when the step is
    // stored. Unconditional loads keep the count of loads in flight the same
    // on every path, so that waiting for one step never waits for the next.
    auto load = [&](int st, BfStage<W>& R) {
        const int part = st % parts;
        const int64_t p0 = pa + (int64_t)(st / parts) * KS;
        const int kv = (int)min((int64_t)KS, pb - p0);
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
            const int kk = ik8[u] < kv ? ik8[u] : 0;
            const float* src = A + (iok[u] ? irow[u] + part * part_stride + p0 + kk : 0);
            float4 v0, v1;
            __builtin_memcpy(&v0, src, 16);
            __builtin_memcpy(&v1, src + 4, 16);
            R.x[u][0] = v0.x; R.x[u][1] = v0.y; R.x[u][2] = v0.z; R.x[u][3] = v0.w;
            R.x[u][4] = v1.x; R.x[u][5] = v1.y; R.x[u][6] = v1.z; R.x[u][7] = v1.w;
            if constexpr (W) {
                const float* wsrc = a.pw + a.p_begin + p0 + kk;
                __builtin_memcpy(&v0, wsrc, 16);
                __builtin_memcpy(&v1, wsrc + 4, 16);
                R.w[u][0] = v0.x; R.w[u][1] = v0.y; R.w[u][2] = v0.z; R.w[u][3] = v0.w;
                R.w[u][4] = v1.x; R.w[u][5] = v1.y; R.w[u][6] = v1.z; R.w[u][7] = v1.w;
            }
        }
    };
    // converts the registers of step st into BF16 planes of buffer `buf`
    auto store = [&](int st, int buf, BfStage<W>& R) {
        uint16_t* base = lds + buf * bufsz;
        const int64_t p0 = pa + (int64_t)(st / parts) * KS;
        const int kv = (int)min((int64_t)KS, pb - p0);
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
            if (!istore[u]) continue;
            const int off = ioff[u];
            float x[8], y[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const bool ok = iok[u] && ik8[u] + e < kv;
                x[e] = ok ? R.x[u][e] : 0.f;
                if constexpr (W) y[e] = ok ? R.x[u][e] * R.w[u][e] : 0.f;
            }
            uint4 pc[NPC];
            split8<NPC>(x, pc);
#pragma unroll
            for (int q = 0; q < NPC; ++q) *reinterpret_cast<uint4*>(base + q * plane + off) = pc[q];
            if constexpr (W) {
                split8<NPC>(y, pc);
#pragma unroll
                for (int q = 0; q < NPC; ++q) *reinterpret_cast<uint4*>(base + (NPC + q) * plane + off) = pc[q];
            }
        }
    };

    // FP32 accumulation spans at most 128 primaries of one part, or one step
    // of both parts where a step is shorter: then the sums go to FP64
    auto flush = [&]() {
#pragma unroll
        for (int q = 0; q < kBfTPW; ++q) {
#pragma unroll
            for (int r = 0; r < 16; ++r) accd[q][r] += (double)acc32[q][r];
            acc32[q] = (f32x16)0.0f;
        }
    };
    const int i = lane & 31, kg = lane >> 5;
    // MFMAs of NQ valid tiles over one step: no branch inside, so that the
    // LDS reads of one tile or slice overlap the MFMAs of the previous one
    auto mma = [&](auto nq, const uint16_t* xp, const uint16_t* wp) {
        constexpr int NQ = decltype(nq)::value;
        int ra[NQ], rb[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            ra[q] = (ti[q] * TS + i) * KSP + 8 * kg;
            rb[q] = (tj[q] * TS + i) * KSP + 8 * kg;
        }
        const int kc = KS > 128 ? 128 : KS;
        for (int kb = 0; kb < KS; kb += kc) {
#pragma unroll 2
            for (int k0 = kb; k0 < kb + kc; k0 += 16) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    bf16x8 ap[NPC], bp[NPC];
#pragma unroll
                    for (int u = 0; u < NPC; ++u) {
                        ap[u] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(wp + u * plane + ra[q] + k0));
                        bp[u] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(xp + u * plane + rb[q] + k0));
                    }
                    // products of pieces u, v with u + v <= NPC - 1
#pragma unroll
                    for (int u = 0; u < NPC; ++u)
#pragma unroll
                        for (int v2 = 0; v2 < NPC; ++v2)
                            if (u + v2 <= NPC - 1)
                                acc32[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ap[u], bp[v2], acc32[q], 0, 0, 0);
                }
            }
            if (KS > 128) flush();
        }
    };
    // MFMAs of step st from LDS buffer buf, then the FP64 flushes (a second
    // tile of a wave is valid only if its first is)
    auto compute = [&](int st, int buf) {
        const uint16_t* xp = lds + buf * bufsz;
        const uint16_t* wp = weighted ? xp + NPC * plane : xp;
        if (tv[1]) mma(std::integral_constant<int, 2>{}, xp, wp);
        else if (tv[0]) mma(std::integral_constant<int, 1>{}, xp, wp);
        if (KS <= 128 && st % parts == parts - 1) flush();
    };

    if (nbuf == 2) {
        // two LDS buffers and one register stage: the loads of step st + 1
        // are issued before the MFMAs of step st and converted into the
        // other buffer after them (a second register stage, loading two
        // steps ahead, spilled registers and measured slower)
        BfStage<W> R;
        load(0, R);
        store(0, 0, R);
        __syncthreads();
        for (int st = 0; st < nsteps; ++st) {
            if (st + 1 < nsteps) load(st + 1, R);
            compute(st, st & 1);
            if (st + 1 < nsteps) store(st + 1, (st + 1) & 1, R);
            __syncthreads();
        }
    } else {
        BfStage<W> R;
        load(0, R);
        store(0, 0, R);
        __syncthreads();
        for (int st = 0; st < nsteps; ++st) {
            compute(st, 0);
            if (st + 1 < nsteps) {
                __syncthreads();
                load(st + 1, R);
                store(st + 1, 0, R);
            }
            __syncthreads();
        }
    }
    // Each unordered column pair is written once (in a diagonal tile, the
    // entry with the smaller l-major column first), at the upper-triangle
    // position of the bin-major order c = b (lmax - m + 1) + l - m that the
    // reduction, finalize and export read.
    const int64_t sg = (int64_t)(a.sub_base + s);
#pragma unroll
    for (int q = 0; q < kBfTPW; ++q) {
        if (!tv[q]) continue;
        const int j = lane & 31;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int ii = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int ci = ti[q] * TS + ii, cj = tj[q] * TS + j;
            if (ci < K && cj < K && (ti[q] < tj[q] || ci <= cj)) {
                const int oi = (ci % nb) * nl + ci / nb, oj = (cj % nb) * nl + cj / nb;
                a.part64[sg * a.gsize + a.goff[m] + (int64_t)min(oi, oj) * K + max(oi, oj)] = accd[q][r];
            }
        }
    }
}

// Degenerate-triangle moments sum_p w_p sum_j w_j^2 R^0_L(z_pj) and pair
// counts per bin. One workgroup per (subchunk, group of kSelfTasks tasks); the
// subchunk's primary weights are staged in LDS once (not with unit weights),
// and every wavefront sums its tasks with four independent FP64 partial sums
// in a fixed order. A row is streamed kSelfUnroll loads per lane at a time, so
// that enough loads are in flight to cover the memory latency. With unit
// weights the pair count of a bin is its L = 0 moment (an exact integer sum),
// written by that task.
constexpr int kSelfTasks = 16;
constexpr int kSelfMaxSub = 4096;  // primaries per subchunk
constexpr int kSelfUnroll = 16;

template <bool UNIT>
__global__ void __launch_bounds__(256) k_self_moments(SelfArgs a) {
    __shared__ double wsh[UNIT ? 1 : kSelfMaxSub];
    const int s = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nL = 2 * a.lmax + 1;
    const int width = nL + 1;
    const int ntask = a.nb * width;
    const int NV = n_values(a.lmax);
    const int na = n_alm_values(a.lmax);
    const int64_t pa = a.sub_start[s], pb = a.sub_start[s + 1];
    const int n = (int)(pb - pa);
    if constexpr (!UNIT) {
        for (int i = threadIdx.x; i < n; i += 256) wsh[i] = a.pd[a.p_begin + pa + i].w;
        __syncthreads();
    }
    const int nfull = n / (64 * kSelfUnroll) * (64 * kSelfUnroll);
    for (int q = 0; q < kSelfTasks / 4; ++q) {
        const int task = blockIdx.y * kSelfTasks + wave * (kSelfTasks / 4) + q;
        if (task >= ntask) break;
        const int b = task / width, L = task - b * width;
        if (UNIT && L == nL) continue;  // written by the L = 0 task
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (a.self_lo && L > a.lmax && L < nL) {
            // not written by the harmonic pass of such a run: the moment is zero
        } else if (L < nL) {
            const int64_t row = ((int64_t)b * NV + na + L) * a.ldA + pa;
            auto val = [&](int p) {
                return a.fp64 ? reinterpret_cast<const double*>(a.A)[row + p]
                              : (double)reinterpret_cast<const float*>(a.A)[row + p];
            };
            for (int p0 = 0; p0 < nfull; p0 += 64 * kSelfUnroll) {
                double v[kSelfUnroll];
#pragma unroll
                for (int u = 0; u < kSelfUnroll; ++u) v[u] = val(p0 + 64 * u + lane);
#pragma unroll
                for (int u = 0; u < kSelfUnroll; ++u) {
                    const int p = p0 + 64 * u + lane;
                    acc[u & 3] += UNIT ? v[u] : wsh[p] * v[u];
                }
            }
            for (int p = nfull + lane; p < n; p += 64) acc[0] += UNIT ? val(p) : wsh[p] * val(p);
        } else {
            for (int p0 = 0; p0 < n; p0 += 256) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int p = p0 + 64 * u + lane;
                    if (p < n) acc[u] += (double)a.cnt[(pa + p) * a.nb + b];
                }
            }
        }
        double sum = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
        if (lane == 0) {
            double* out = a.part + (int64_t)(a.sub_base + s) * a.nb * width;
            out[task] = sum;
            if (UNIT && L == 0) out[b * width + nL] = sum;
        }
    }
}

__global__ void k_reduce_partials(const float* __restrict__ p32, const double* __restrict__ p64,
                                  int64_t width, const int* __restrict__ cat_sub, int ncat,
                                  double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (e >= width || c >= ncat) return;
    double s = 0.0;
    for (int q = cat_sub[c]; q < cat_sub[c + 1]; ++q)
        s += p32 ? (double)p32[(int64_t)q * width + e] : p64[(int64_t)q * width + e];
    out[(int64_t)c * width + e] = s;
}

__global__ void k_finalize(FinalArgs a) {
    const int nb = a.nb;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)a.n_mult * nb * nb;
    const int c = blockIdx.y;
    if (idx >= per || c >= a.ncat) return;
    const int t = (int)(idx / (nb * nb));
    const int b1 = (int)((idx / nb) % nb), b2 = (int)(idx % nb);
    const int l1 = a.mult[3 * t], l2 = a.mult[3 * t + 1];
    const int mm = min(l1, l2);
    const int nL = 2 * a.lmax + 1;
    const int sw = nb * (nL + 1);
    const double* G = a.G + (int64_t)c * a.gsize;
    double sum = 0.0;
    for (int m = 0; m <= mm; ++m) {
        const int nl = a.lmax - m + 1;
        const int K = nb * nl;
        const int ci = b1 * nl + (l1 - m), cj = b2 * nl + (l2 - m);
        const double g = G[a.goff[m] + (int64_t)min(ci, cj) * K + max(ci, cj)];
        sum += a.coefG[t * (a.lmax + 1) + m] * g;
        if (b1 == b2 && a.subtract_self) {
            const double* cs = a.coefS + ((int64_t)t * (a.lmax + 1) + m) * nL;
            const double* S = a.S + (int64_t)c * sw + b1 * (nL + 1);
            for (int L = 0; L < nL; ++L) sum -= cs[L] * S[L];
        }
    }
    const double nd = a.nd[c];
    const double rrr = nd * (nd - 1.0) * (nd - 2.0) * a.vol[b1] * a.vol[b2] * a.inv_box6;
    a.out[(int64_t)c * per + idx] = sum / rrr;
}

// Edge correction of the isotropic multipoles for the Szapudi-Szalay estimator
// with explicit randoms (eq. (ssest)): the triplet counts of the data-minus-
// randoms field and of the randoms are related as functions of the opening
// angle by N = zeta R, which for Legendre coefficients reads
//   N_l = sum_{l'} M_{l l'} zeta_{l'},  M_{l l'} = sum_{l''} T[l][l'][l''] R_{l''},
// with T[l][l'][l''] = (2l+1)/2 int P_l P_l' P_l'' (the relation of Slepian &
// Eisenstein 2015). One thread per (b1, b2) forms M in LDS and solves by
// Gaussian elimination with partial pivoting in FP64; a singular M sets *bad.
__global__ void k_edge_iso(const double* __restrict__ N, const double* __restrict__ R, const double* __restrict__ T,
                           int nl, int nbb, double* __restrict__ out, int* __restrict__ bad) {
    extern __shared__ double esh[];
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nbb) return;
    double* M = esh + (size_t)threadIdx.x * (nl * nl + nl);
    double* x = M + nl * nl;
    for (int l = 0; l < nl; ++l) {
        x[l] = N[(int64_t)l * nbb + q];
        for (int lp = 0; lp < nl; ++lp) {
            double v = 0.0;
            for (int lpp = 0; lpp < nl; ++lpp) v += T[(l * nl + lp) * nl + lpp] * R[(int64_t)lpp * nbb + q];
            M[l * nl + lp] = v;
        }
    }
    for (int c = 0; c < nl; ++c) {
        int piv = c;
        for (int r = c + 1; r < nl; ++r)
            if (fabs(M[r * nl + c]) > fabs(M[piv * nl + c])) piv = r;
        if (!(fabs(M[piv * nl + c]) > 0.0)) {
            atomicOr(bad, 1);
            return;
        }
        if (piv != c) {
            for (int k = 0; k < nl; ++k) {
                const double t = M[c * nl + k];
                M[c * nl + k] = M[piv * nl + k];
                M[piv * nl + k] = t;
            }
            const double t = x[c];
            x[c] = x[piv];
            x[piv] = t;
        }
        const double ip = 1.0 / M[c * nl + c];
        for (int r = c + 1; r < nl; ++r) {
            const double f = M[r * nl + c] * ip;
            for (int k = c; k < nl; ++k) M[r * nl + k] -= f * M[c * nl + k];
            x[r] -= f * x[c];
        }
    }
    for (int c = nl - 1; c >= 0; --c) {
        double v = x[c];
        for (int k = c + 1; k < nl; ++k) v -= M[c * nl + k] * x[k];
        x[c] = v / M[c * nl + c];
    }
    for (int l = 0; l < nl; ++l) out[(int64_t)l * nbb + q] = x[l];
}

__global__ void k_export_nnn(NnnArgs a) {
    const int nb = a.nb, s1 = a.lmax + 1, nL = 2 * a.lmax + 1;
    const int64_t n = (int64_t)s1 * s1 * s1 * nb * nb;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int b2 = (int)(idx % nb), b1 = (int)((idx / nb) % nb);
    const int64_t t = idx / ((int64_t)nb * nb);
    const int l2 = (int)(t % s1), l1 = (int)((t / s1) % s1), m = (int)(t / ((int64_t)s1 * s1));
    double v = 0.0;
    if (l1 >= m && l2 >= m && (!a.isotropic || l1 == l2)) {
        const int nl = a.lmax - m + 1, K = nb * nl;
        const int ci = b1 * nl + (l1 - m), cj = b2 * nl + (l2 - m);
        v = a.scale[l1 * s1 + m] * a.scale[l2 * s1 + m] *
            a.G[a.goff[m] + (int64_t)min(ci, cj) * K + max(ci, cj)];
        if (b1 == b2 && a.subtract_self) {
            const double* g = a.gaunt + ((int64_t)(m * s1 + l1) * s1 + l2) * nL;
            const double* S = a.S + b1 * (nL + 1);
            for (int L = 0; L < nL; ++L) v -= g[L] * S[L];
        }
    }
    a.out[idx] = v;
}

__global__ void k_export_alm(AlmExportArgs a) {
    const int nb = a.nb, s1 = a.lmax + 1;
    const int NV = n_values(a.lmax);
    const int64_t n = a.count * nb * s1 * s1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int m = (int)(idx % s1), l = (int)((idx / s1) % s1), b = (int)((idx / (s1 * s1)) % nb);
    const int64_t i = idx / ((int64_t)s1 * s1 * nb);
    double re = 0.0, im = 0.0;
    if (m <= l) {
        const int64_t p = a.perm[a.first + i] - a.p_begin;
        const int nl = a.lmax - m + 1;
        const int v0 = value_offset(a.lmax, m) + (l - m);
        const int64_t r0 = ((int64_t)b * NV + v0) * a.ldA + p;
        if (a.fp64) {
            const double* A = reinterpret_cast<const double*>(a.A);
            re = A[r0];
            if (m > 0) im = A[r0 + (int64_t)nl * a.ldA];
        } else {
            const float* A = reinterpret_cast<const float*>(a.A);
            re = A[r0];
            if (m > 0) im = A[r0 + (int64_t)nl * a.ldA];
        }
        const double f = a.sign_scale[l * s1 + m];
        re *= f;
        im *= f;
    }
    a.out[2 * idx] = re;
    a.out[2 * idx + 1] = im;
}

template <int MODE>
size_t contract_lds(int ncol) {
    using C = Cfg<MODE>;
    constexpr int KSP = MODE >= 2 ? C::KS + 8 : C::KS + 1;
    // bytes per staged element: value (fp64/fp32) or 2 x pieces x 2 bytes (BF16 planes of
    // x and of w x)
    size_t x = MODE == 0 ? sizeof(double) : (MODE == 1 ? sizeof(float) : (MODE == 2 ? 8 : 12));
    return C::KS * sizeof(double) + (size_t)ncol * KSP * x;
}

template <int MODE>
hipError_t launch_contract_mode(const ContractArgs& a, hipStream_t s) {
    using C = Cfg<MODE>;
    const int K0 = a.nb * (a.lmax + 1);
    const int nt0 = (K0 + C::TS - 1) / C::TS;
    const int ntiles0 = nt0 * (nt0 + 1) / 2;
    const int ngroups = (ntiles0 + 4 * C::TPW - 1) / (4 * C::TPW);
    if constexpr (MODE == 0) {
        // the double-buffered kernel when its items and buffers fit
        const int ncol = nt0 * C::TS;
        const size_t lds2 = f64db_lds(ncol);
        if (ncol * (C::KS / 4) <= 256 * kF64IPT && lds2 <= 160 * 1024) {
            const hipError_t e = a.unit_weights ? allow_full_lds((const void*)k_contract_f64<false>)
                                                : allow_full_lds((const void*)k_contract_f64<true>);
            if (e != hipSuccess) return e;
            const dim3 grid(a.nsub, a.lmax + 1, ngroups);
            if (a.unit_weights)
                hipLaunchKernelGGL(k_contract_f64<false>, grid, dim3(256), lds2, s, a);
            else
                hipLaunchKernelGGL(k_contract_f64<true>, grid, dim3(256), lds2, s, a);
            return hipGetLastError();
        }
    }
    const size_t lds = contract_lds<MODE>(nt0 * C::TS);
    const hipError_t e = allow_full_lds((const void*)k_contract<MODE>);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_contract<MODE>, dim3(a.nsub, a.lmax + 1, ngroups), dim3(256), lds, s, a);
    return hipGetLastError();
}

}  // namespace

// Step cap and buffer count of the split-BF16 contraction. Every m takes
// its own step (bf_step): the longest up to cap (512, or ks_max when given)
// that fits the registers and LDS for its columns; m = 0, the widest, needs
// at least 16. Double-buffered when every m's buffers fit in LDS. lds is the
// largest need over the m (the allocation of each workgroup).
struct BfPlan { BfSteps steps; int nbuf; size_t lds; };
BfPlan bf_plan(int npc, int nb, int lmax, bool weighted, int ks_max = 0) {
    const int nplanes = weighted ? 2 * npc : npc;
    const int ipt = weighted ? bf_ipt<true>() : bf_ipt<false>();
    const int cap = ks_max >= 16 ? std::min(ks_max, 512) : 512;
    BfPlan pl{};
    for (int nbuf = 2; nbuf >= 1; --nbuf) {
        size_t need = 0;
        bool ok = lmax <= kMaxLmax;
        for (int m = 0; m <= lmax && ok; ++m) {
            const int ncol = (nb * (lmax - m + 1) + 31) / 32 * 32;
            const int ks = bf_step(ncol, nplanes, ipt, nbuf, cap, 160 * 1024);
            ok = ks > 0;
            pl.steps.ks[m] = ks;
            need = std::max(need, (size_t)nbuf * nplanes * ncol * (ks + 8) * sizeof(uint16_t));
        }
        if (ok) {
            pl.nbuf = nbuf;
            pl.lds = need;
            return pl;
        }
    }
    return BfPlan{};
}

template <int NPC, bool W>
hipError_t launch_contract_bf16_w(const ContractArgs& a, hipStream_t s) {
    const int K0 = a.nb * (a.lmax + 1);
    const int nt0 = (K0 + 31) / 32;
    const int ntiles0 = nt0 * (nt0 + 1) / 2;
    const int ngroups = (ntiles0 + kBfWaves * kBfTPW - 1) / (kBfWaves * kBfTPW);
    const BfPlan pl = bf_plan(NPC, a.nb, a.lmax, !a.unit_weights, a.ks_max);
    if (pl.nbuf == 0) return hipErrorInvalidValue;
    const hipError_t e = allow_full_lds((const void*)k_contract_bf16<NPC, W>);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_contract_bf16<NPC, W>), dim3(a.nsub, a.lmax + 1, ngroups), dim3(64 * kBfWaves),
                       pl.lds, s, a, pl.steps, pl.nbuf);
    return hipGetLastError();
}

template <int NPC>
hipError_t launch_contract_bf16(const ContractArgs& a, hipStream_t s) {
    return a.unit_weights ? launch_contract_bf16_w<NPC, false>(a, s) : launch_contract_bf16_w<NPC, true>(a, s);
}

hipError_t launch_contract_iso(const ContractArgs& a, hipStream_t s) {
    if (a.nsub <= 0) return hipSuccess;
    if (a.nb > 32) return hipErrorInvalidValue;
    const int nlm = (a.lmax + 1) * (a.lmax + 2) / 2;
    const dim3 grid(a.nsub, (nlm + kIsoWaves - 1) / kIsoWaves);
    const bool f64 = a.mode == 0;
    if (a.unit_weights) {
        if (f64) hipLaunchKernelGGL((k_contract_iso<double, false>), grid, dim3(64 * kIsoWaves), 0, s, a);
        else hipLaunchKernelGGL((k_contract_iso<float, false>), grid, dim3(64 * kIsoWaves), 0, s, a);
    } else {
        if (f64) hipLaunchKernelGGL((k_contract_iso<double, true>), grid, dim3(64 * kIsoWaves), 0, s, a);
        else hipLaunchKernelGGL((k_contract_iso<float, true>), grid, dim3(64 * kIsoWaves), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_contract(const ContractArgs& a, hipStream_t s) {
    if (a.nsub <= 0) return hipSuccess;
    switch (a.mode) {
        case 0: return launch_contract_mode<0>(a, s);
        case 1: return launch_contract_mode<1>(a, s);
        case 2:
        case 3: {
            // a split-BF16 step must stage at least 16 primaries of every
            // column in the threads' registers (nbins (lmax + 1) <= 512 with
            // weights); beyond that the FP32 MFMA contraction runs instead
            if (bf_plan(a.mode == 2 ? 2 : 3, a.nb, a.lmax, !a.unit_weights, a.ks_max).nbuf == 0)
                return launch_contract_mode<1>(a, s);
            return a.mode == 2 ? launch_contract_bf16<2>(a, s) : launch_contract_bf16<3>(a, s);
        }
        default: return hipErrorInvalidValue;
    }
}

size_t contract_lds_bytes(int mode, int nb, int lmax) {
    const int K0 = nb * (lmax + 1);
    switch (mode) {
        case 0: return contract_lds<0>((K0 + 15) / 16 * 16);
        case 1: return contract_lds<1>((K0 + 31) / 32 * 32);
        default: {
            const BfPlan pl = bf_plan(mode == 2 ? 2 : 3, nb, lmax, true);
            return pl.nbuf ? pl.lds : contract_lds<1>((K0 + 31) / 32 * 32);
        }
    }
}

hipError_t launch_self_moments(const SelfArgs& a, hipStream_t s) {
    if (a.nsub <= 0) return hipSuccess;
    const int ntask = a.nb * (2 * a.lmax + 2);
    const dim3 grid(a.nsub, (ntask + kSelfTasks - 1) / kSelfTasks);
    if (a.unit_w)
        hipLaunchKernelGGL(k_self_moments<true>, grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_self_moments<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(const float* p32, const double* p64, int64_t width,
                                  const int* cat_sub, int ncat, double* out, hipStream_t s) {
    if (ncat <= 0 || width <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)((width + 255) / 256), ncat), dim3(256), 0,
                       s, p32, p64, width, cat_sub, ncat, out);
    return hipGetLastError();
}

hipError_t launch_finalize(const FinalArgs& a, hipStream_t s) {
    const int64_t per = (int64_t)a.n_mult * a.nb * a.nb;
    if (per <= 0 || a.ncat <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((per + 255) / 256), a.ncat), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_edge_iso(const double* N, const double* R, const double* T, int nl, int nbb, double* out, int* bad,
                           hipStream_t s) {
    if (nbb <= 0 || nl <= 0) return hipSuccess;
    // one system (nl^2 + nl doubles) per thread in LDS: up to 32 threads, within 160 KiB
    const size_t per = (size_t)(nl * nl + nl) * sizeof(double);
    const int kThreads = (int)std::max<size_t>(1, std::min<size_t>(32, (size_t)160 * 1024 / per));
    const size_t lds = (size_t)kThreads * per;
    if (lds > 64 * 1024) {
        hipError_t e = allow_full_lds((const void*)k_edge_iso);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_edge_iso, dim3((nbb + kThreads - 1) / kThreads), dim3(kThreads), lds, s, N, R, T, nl, nbb,
                       out, bad);
    return hipGetLastError();
}

hipError_t launch_export_nnn(const NnnArgs& a, hipStream_t s) {
    const int64_t n = (int64_t)(a.lmax + 1) * (a.lmax + 1) * (a.lmax + 1) * a.nb * a.nb;
    hipLaunchKernelGGL(k_export_nnn, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_export_alm(const AlmExportArgs& a, hipStream_t s) {
    const int64_t n = a.count * a.nb * (a.lmax + 1) * (a.lmax + 1);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_export_alm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace tpcf
