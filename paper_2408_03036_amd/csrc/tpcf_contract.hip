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
// The same file holds the degenerate-triangle moments, the fixed-order partial
// reduction, and the final conversion to the tripolar multipoles
// (eq. (slep2sugy)).
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

// Degenerate-triangle moments sum_p w_p sum_j w_j^2 R^0_L(z_pj) and pair
// counts per bin, one workgroup per subchunk, one wavefront per task.
__global__ void __launch_bounds__(256) k_self_moments(SelfArgs a) {
    const int s = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nL = 2 * a.lmax + 1;
    const int width = nL + 1;
    const int ntask = a.nb * width;
    const int NV = n_values(a.lmax);
    const int na = n_alm_values(a.lmax);
    const int64_t pa = a.sub_start[s], pb = a.sub_start[s + 1];
    for (int task = wave; task < ntask; task += 4) {
        const int b = task / width, L = task - b * width;
        double sum = 0.0;
        for (int64_t p = pa + lane; p < pb; p += 64) {
            if (L < nL) {
                const int64_t idx = ((int64_t)b * NV + na + L) * a.ldA + p;
                const double v = a.fp64 ? reinterpret_cast<const double*>(a.A)[idx]
                                        : (double)reinterpret_cast<const float*>(a.A)[idx];
                sum += a.pd[a.p_begin + p].w * v;
            } else {
                sum += (double)a.cnt[p * a.nb + b];
            }
        }
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
        if (lane == 0) a.part[(int64_t)(a.sub_base + s) * a.nb * width + task] = sum;
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

__global__ void k_export_nnn(NnnArgs a) {
    const int nb = a.nb, s1 = a.lmax + 1, nL = 2 * a.lmax + 1;
    const int64_t n = (int64_t)s1 * s1 * s1 * nb * nb;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int b2 = (int)(idx % nb), b1 = (int)((idx / nb) % nb);
    const int64_t t = idx / ((int64_t)nb * nb);
    const int l2 = (int)(t % s1), l1 = (int)((t / s1) % s1), m = (int)(t / ((int64_t)s1 * s1));
    double v = 0.0;
    if (l1 >= m && l2 >= m) {
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
    const size_t lds = contract_lds<MODE>(nt0 * C::TS);
    static bool attr = false;
    if (!attr) {
        hipFuncSetAttribute((const void*)k_contract<MODE>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
        attr = true;
    }
    hipLaunchKernelGGL(k_contract<MODE>, dim3(a.nsub, a.lmax + 1, ngroups), dim3(256), lds, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_contract(const ContractArgs& a, hipStream_t s) {
    if (a.nsub <= 0) return hipSuccess;
    switch (a.mode) {
        case 0: return launch_contract_mode<0>(a, s);
        case 1: return launch_contract_mode<1>(a, s);
        case 2: return launch_contract_mode<2>(a, s);
        case 3: return launch_contract_mode<3>(a, s);
        default: return hipErrorInvalidValue;
    }
}

size_t contract_lds_bytes(int mode, int nb, int lmax) {
    const int K0 = nb * (lmax + 1);
    switch (mode) {
        case 0: return contract_lds<0>((K0 + 15) / 16 * 16);
        case 1: return contract_lds<1>((K0 + 31) / 32 * 32);
        case 2: return contract_lds<2>((K0 + 31) / 32 * 32);
        default: return contract_lds<3>((K0 + 31) / 32 * 32);
    }
}

hipError_t launch_self_moments(const SelfArgs& a, hipStream_t s) {
    if (a.nsub <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_self_moments, dim3(a.nsub), dim3(256), 0, s, a);
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
