// Pair pass of the anisotropic 3PCF estimator (arXiv:2408.03036, Sec. 4.2,
// eq. (alm)): for every primary p and every neighbour j with |x_j - x_p| in
// radial bin b, accumulate w_j conj(Y_lm(rhat_pj)) into a_lm(p, b).
//
// Two kernels:
//  k_pair_bin  one wavefront per primary. Lanes walk the primary's stencil of
//              neighbour cells as one flattened candidate range (coalesced
//              loads of the cell-sorted points), test the separation, find the
//              bin and collect the hits in LDS. The hits are then written to a
//              per-primary list sorted by bin (stable, so the accumulation
//              order is deterministic), with (offset, count) per (p, b).
//  k_pair_alm  lane = one (primary, bin) list. A wavefront holds 64
//              consecutive primaries of one bin; each lane walks its list and
//              accumulates every harmonic in registers, so no cross-lane
//              reduction is needed. The result goes to the contraction operand
//              A[b][v][p] (primaries contiguous).
//
// The harmonics use the Cartesian form conj(Y_lm) = (-1)^m N_lm gamma_lm
// R_lm(z) (x - i y)^m, where R_lm = (d^m P_l / dz^m) / gamma_lm obeys
// R_lm = z R_{l-1,m} - beta_lm R_{l-2,m}, R_mm = 1, R_{m+1,m} = z, with
// beta_lm = (l+m-1)(l-m-1)/((2l-1)(2l-3)) and gamma_lm = (2l-1) gamma_{l-1,m}/(l-m),
// gamma_mm = (2m-1)!!. The constant (-1)^m N_lm gamma_lm is applied when the
// multipoles are formed. The same chain for m = 0 up to 2 lmax gives the
// Legendre moments sum_j w_j^2 P_L(z) of the degenerate (j == k) triangles.
//
// Binning must agree with an exact double-precision evaluation of
// r^2 = dx*dx + dy*dy + dz*dz against the squared edges. The FP32 path bins in
// single precision from cell-relative coordinates and re-evaluates in FP64 the
// rare pairs that fall inside a guard band around an edge.
#include "tpcf_internal.h"

namespace tpcf {

namespace {

constexpr int kHB = 2048;  // hits a wavefront can sort in LDS per pass

__device__ inline int lane_id() { return threadIdx.x & 63; }

__device__ inline int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// XCD-aware block remap: the hardware hands consecutive workgroups to the 8
// XCDs in turn; this gives every XCD a contiguous range of logical blocks so
// that neighbouring primaries share that XCD's L2.
__device__ inline int64_t xcd_block(int64_t bid, int64_t nblocks) {
    int64_t per = (nblocks + 7) / 8;
    return (bid % 8) * per + bid / 8;
}

struct RunLds {
    int start[kMaxRuns];
    int pref[kMaxRuns + 1];
    float sx[kMaxRuns], sy[kMaxRuns], zo[kMaxRuns];
    int code[kMaxRuns];   // (ox+k)*(2k+1)+(oy+k): z offset is added per candidate
    int wrap[kMaxRuns];   // wrap signs, 2 bits per axis (x: bits 0-1, y: 2-3, z: 4-5), value+1
    int n;
};

struct BinLds {
    RunLds r;
    uint32_t buf[kHB];
    unsigned char bbuf[kHB];
    int cnt[kMaxBins];
    int pre[kMaxBins];
};

__device__ inline double wrap_shift(int bits, int axis, double L) {
    return (double)(((bits >> (2 * axis)) & 3) - 1) * L;
}

// Exact FP64 bin of a pair (the reference evaluation), -1 if outside the
// shells or at zero separation. Shifts come from the cell geometry (equal to
// the minimum image for any pair inside the shells) or, in single-cell mode,
// from rint.
__device__ inline int exact_bin(const double4& P, const double4& Q, int wbits, const BinArgs& a) {
#pragma clang fp contract(off)
    double dx = Q.x - P.x, dy = Q.y - P.y, dz = Q.z - P.z;
    if (a.g.single) {
        dx -= a.g.box * rint(dx / a.g.box);
        dy -= a.g.box * rint(dy / a.g.box);
        dz -= a.g.box * rint(dz / a.g.box);
    } else {
        dx += wrap_shift(wbits, 0, a.g.box);
        dy += wrap_shift(wbits, 1, a.g.box);
        dz += wrap_shift(wbits, 2, a.g.box);
    }
    double r2 = dx * dx;
    r2 += dy * dy;
    r2 += dz * dz;
    if (r2 == 0.0 || r2 < a.e2[0] || r2 >= a.e2[a.nb]) return -1;
    int b = a.lut[min(kLut - 1, max(0, (int)((float)(r2 - a.e2[0]) * a.lut_scale)))];
    while (b + 1 < a.nb && r2 >= a.e2[b + 1]) ++b;
    while (b > 0 && r2 < a.e2[b]) --b;
    return b;
}

// Builds the flattened candidate ranges of primary p (cell cx,cy,cz) in LDS.
// Every stencil run (fixed ox, oy; oz in [oz_lo, oz_hi]) becomes at most two
// pieces of consecutive cells: the part that wraps through the z boundary and
// the part that does not.
__device__ void build_runs(RunLds& R, const BinArgs& a, int cat, int cx, int cy, int cz) {
    const int lane = lane_id();
    const int nc = a.g.nc, k = a.g.k;
    const int base = cat * a.g.ncell;
    int total_pieces = 0;
    for (int r0 = 0; r0 < a.nruns; r0 += 64) {
        const int r = r0 + lane;
        int np = 0;
        int s0 = 0, e0 = 0, s1 = 0, e1 = 0, w0 = 0, w1 = 0, cb = 0;
        bool has_wrap = false, has_in = false;
        float sxv = 0.f, syv = 0.f, zo0 = 0.f, zo1 = 0.f;
        if (r < a.nruns) {
            const StencilRun st = a.runs[r];
            int qx = cx + st.ox, qy = cy + st.oy;
            int wx = 0, wy = 0;
            if (qx < 0) { qx += nc; wx = -1; } else if (qx >= nc) { qx -= nc; wx = 1; }
            if (qy < 0) { qy += nc; wy = -1; } else if (qy >= nc) { qy -= nc; wy = 1; }
            const int col = base + (qx * nc + qy) * nc;
            const int zlo = cz + st.oz_lo, zhi = cz + st.oz_hi;
            cb = (st.ox + k) * (2 * k + 1) + (st.oy + k);
            sxv = (float)(st.ox * a.g.h);
            syv = (float)(st.oy * a.g.h);
            const int wxy = (wx + 1) | ((wy + 1) << 2);
            if (zlo < 0) {
                // cells zlo..min(zhi,-1) are nc+zlo..nc+min(zhi,-1); z offset = izf - nc - cz
                const int za = zlo + nc, zb = min(zhi, -1) + nc;
                s0 = a.cell_start[col + za];
                e0 = a.cell_start[col + zb + 1];
                zo0 = (float)(-nc - cz);
                w0 = wxy | (0 << 4);
                has_wrap = true;
            } else if (zhi > nc - 1) {
                // cells max(zlo,nc)..zhi are those minus nc; z offset = izf + nc - cz
                const int za = max(zlo, nc) - nc, zb = zhi - nc;
                s0 = a.cell_start[col + za];
                e0 = a.cell_start[col + zb + 1];
                zo0 = (float)(nc - cz);
                w0 = wxy | (2 << 4);
                has_wrap = true;
            }
            const int lo_in = max(zlo, 0), hi_in = min(zhi, nc - 1);
            if (hi_in >= lo_in) {
                s1 = a.cell_start[col + lo_in];
                e1 = a.cell_start[col + hi_in + 1];
                zo1 = (float)(-cz);
                w1 = wxy | (1 << 4);
                has_in = true;
            }
            np = (int)has_wrap + (int)has_in;
        }
        int incl = np;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off, 64);
            if (lane >= off) incl += t;
        }
        int q = total_pieces + incl - np;
        if (has_wrap) {
            R.start[q] = s0;
            R.pref[q] = e0 - s0;
            R.sx[q] = sxv; R.sy[q] = syv; R.zo[q] = zo0;
            R.code[q] = cb;
            R.wrap[q] = w0;
            ++q;
        }
        if (has_in) {
            R.start[q] = s1;
            R.pref[q] = e1 - s1;
            R.sx[q] = sxv; R.sy[q] = syv; R.zo[q] = zo1;
            R.code[q] = cb;
            R.wrap[q] = w1;
        }
        total_pieces += __shfl(incl, 63, 64);
    }
    wave_sync();
    // exclusive prefix of the piece lengths (held in pref) -> pref
    int carry = 0;
    for (int q0 = 0; q0 < total_pieces; q0 += 64) {
        const int q = q0 + lane;
        const int len = q < total_pieces ? R.pref[q] : 0;
        int incl = len;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off, 64);
            if (lane >= off) incl += t;
        }
        wave_sync();
        if (q < total_pieces) R.pref[q] = carry + incl - len;
        carry += __shfl(incl, 63, 64);
        wave_sync();
    }
    if (lane == 0) {
        R.pref[total_pieces] = carry;
        R.n = total_pieces;
    }
    wave_sync();
}

// Classifies candidate g of the flattened range: returns its bin (or -1) and
// its list entry. r is the piece holding g.
template <bool FP64>
__device__ __forceinline__ int classify(const BinLds& L, const BinArgs& a, int64_t p,
                                        const float4& P32, const double4& P64, int r, int g,
                                        int64_t cstart, int k, uint32_t& entry) {
    const int64_t j = L.r.start[r] + (g - L.r.pref[r]);
    const float4 q = a.pf[j];
    const int oz = (int)(q.w + L.r.zo[r]);
    const int wb = L.r.wrap[r];
    int b = -1;
    if (j != p) {
        if (FP64) {
            b = exact_bin(P64, a.pd[j], wb, a);
        } else {
            float dx, dy, dz;
            if (a.g.single) {
                dx = q.x - P32.x;
                dy = q.y - P32.y;
                dz = q.z - P32.z;
                dx -= a.g.boxf * rintf(dx / a.g.boxf);
                dy -= a.g.boxf * rintf(dy / a.g.boxf);
                dz -= a.g.boxf * rintf(dz / a.g.boxf);
            } else {
                dx = (q.x - P32.x) + L.r.sx[r];
                dy = (q.y - P32.y) + L.r.sy[r];
                dz = fmaf((float)oz, a.g.hf, q.z - P32.z);
            }
            const float r2 = dx * dx + dy * dy + dz * dz;
            if (r2 >= a.e2f[0] - a.guard[0] && r2 < a.e2f[a.nb] + a.guard[a.nb]) {
                int bb = a.lut[min(kLut - 1, max(0, (int)((r2 - a.e2f[0]) * a.lut_scale)))];
                while (bb + 1 < a.nb && r2 >= a.e2f[bb + 1]) ++bb;
                while (bb > 0 && r2 < a.e2f[bb]) --bb;
                const bool near = fabsf(r2 - a.e2f[bb]) < a.guard[bb] ||
                                  fabsf(a.e2f[bb + 1] - r2) < a.guard[bb + 1] ||
                                  r2 < a.e2f[0] || r2 >= a.e2f[a.nb];
                b = near ? exact_bin(P64, a.pd[j], wb, a) : bb;
            }
        }
    }
    if (b >= 0) {
        const int code = a.g.single ? 0 : L.r.code[r] * (2 * k + 1) + (oz + k);
        entry = (uint32_t)(j - cstart) | ((uint32_t)code << (32 - a.g.code_bits));
    }
    return b;
}

// One scan over the candidates. Hits with bin in [blo, bhi) are appended to
// the LDS buffer (up to kHB); with COUNT the per-bin totals of all hits are
// accumulated in L.cnt.
template <bool FP64, bool COUNT>
__device__ int scan_candidates(BinLds& L, const BinArgs& a, int64_t p, const float4& P32,
                               const double4& P64, int blo, int bhi, int64_t cstart, int k) {
    const int lane = lane_id();
    const int total = L.r.pref[L.r.n];
    int tot = 0;
    int rcur = 0;
    for (int t = 0; t < total; t += 64) {
        while (L.r.pref[rcur + 1] <= t) ++rcur;
        const int g = t + lane;
        int b = -1;
        uint32_t entry = 0;
        if (g < total) {
            int r = rcur;
            while (L.r.pref[r + 1] <= g) ++r;
            b = classify<FP64>(L, a, p, P32, P64, r, g, cstart, k, entry);
            if (COUNT && b >= 0) atomicAdd(&L.cnt[b], 1);
        }
        const bool keep = b >= blo && b < bhi;
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int pos = tot + lanes_below(m);
            if (pos < kHB) {
                L.buf[pos] = entry;
                L.bbuf[pos] = (unsigned char)b;
            }
        }
        tot += __popcll(m);
    }
    wave_sync();
    return tot;
}

// Writes the LDS hits (bins [blo,bhi)) to global memory, each bin's hits in
// candidate order at base + pre[b].
__device__ void write_hits(BinLds& L, const BinArgs& a, int tot, uint32_t base_off, int blo,
                           int bhi) {
    const int lane = lane_id();
    int runv = 0;  // lane bb holds the hits of bin bb written so far
    for (int e0 = 0; e0 < tot; e0 += 64) {
        const int e = e0 + lane;
        const int b = e < tot ? (int)L.bbuf[e] : -1;
        const uint32_t v = e < tot ? L.buf[e] : 0u;
        int rank = 0;
        for (int bb = blo; bb < bhi; ++bb) {
            const uint64_t m = __ballot(b == bb);
            if (m == 0) continue;
            const int basebb = __shfl(runv, bb, 64);
            if (b == bb) rank = basebb + lanes_below(m);
            if (lane == bb) runv += __popcll(m);
        }
        if (b >= 0) a.list[base_off + (uint32_t)L.pre[b] + (uint32_t)rank] = v;
    }
    wave_sync();
}

template <bool FP64>
__global__ void __launch_bounds__(256) k_pair_bin(BinArgs a) {
    extern __shared__ unsigned char smem[];
    BinLds& L = reinterpret_cast<BinLds*>(smem)[threadIdx.x >> 6];
    const int lane = lane_id();
    const int64_t nprim = a.p_end - a.p_begin;
    const int64_t nblk = (nprim + 3) / 4;
    const int64_t blk = xcd_block(blockIdx.x, (int64_t)gridDim.x);
    if (blk >= nblk) return;
    const int64_t p = a.p_begin + blk * 4 + (threadIdx.x >> 6);
    if (p >= a.p_end) return;
    const int64_t pl = p - a.p_begin;

    const float4 P32 = a.pf[p];
    const double4 P64 = a.pd[p];
    const int cat = a.catid[p];
    const int64_t cstart = a.pt_off[cat];
    int cx = 0, cy = 0, cz = 0;
    if (!a.g.single) {
        cz = (int)P32.w;
        // x and y cells from the FP64 position, with the same rule as the grid build
        cx = min(a.g.nc - 1, max(0, (int)(P64.x * a.g.inv_h)));
        cy = min(a.g.nc - 1, max(0, (int)(P64.y * a.g.inv_h)));
    }
    if (lane < kMaxBins) L.cnt[lane] = 0;
    wave_sync();
    build_runs(L.r, a, cat, cx, cy, cz);

    const int k = a.g.k;
    const int tot = scan_candidates<FP64, true>(L, a, p, P32, P64, 0, a.nb, cstart, k);
    // per-bin counts and offsets
    const int c = lane < a.nb ? L.cnt[lane] : 0;
    int incl = c;
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    const int total_hits = __shfl(incl, 63, 64);
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(a.cursor, (unsigned long long)total_hits);
    base = __shfl(base, 0, 64);
    if (base + (unsigned long long)total_hits > a.capacity) {
        if (lane == 0) atomicOr(a.overflow, 1);
        if (lane < a.nb) {
            a.cnt[pl * a.nb + lane] = 0;
            a.boff[pl * a.nb + lane] = 0;
        }
        return;
    }
    if (lane < a.nb) {
        L.pre[lane] = incl - c;
        a.cnt[pl * a.nb + lane] = (uint32_t)c;
        a.boff[pl * a.nb + lane] = (uint32_t)(base + (unsigned long long)(incl - c));
    }
    wave_sync();
    if (tot <= kHB) {
        write_hits(L, a, tot, (uint32_t)base, 0, a.nb);
        return;
    }
    // More hits than the LDS buffer: rescan in passes over runs of bins that
    // fit. A bin larger than the buffer is streamed to global memory in
    // candidate order.
    int blo = 0;
    while (blo < a.nb) {
        int bhi = blo, sum = 0;
        while (bhi < a.nb && sum + L.cnt[bhi] <= kHB) { sum += L.cnt[bhi]; ++bhi; }
        if (bhi > blo) {
            const int got = scan_candidates<FP64, false>(L, a, p, P32, P64, blo, bhi, cstart, k);
            write_hits(L, a, got, (uint32_t)base, blo, bhi);
            blo = bhi;
            continue;
        }
        const int b1 = blo;
        const int total = L.r.pref[L.r.n];
        int written = 0;
        int rcur = 0;
        for (int t = 0; t < total; t += 64) {
            while (L.r.pref[rcur + 1] <= t) ++rcur;
            const int g = t + lane;
            int b = -1;
            uint32_t entry = 0;
            if (g < total) {
                int r = rcur;
                while (L.r.pref[r + 1] <= g) ++r;
                b = classify<FP64>(L, a, p, P32, P64, r, g, cstart, k, entry);
            }
            const bool keep = b == b1;
            const uint64_t m = __ballot(keep);
            if (keep) a.list[(uint32_t)base + (uint32_t)L.pre[b1] + (uint32_t)(written + lanes_below(m))] = entry;
            written += __popcll(m);
        }
        blo = b1 + 1;
    }
}

// ---------------------------------------------------------------- harmonics

template <typename T>
__device__ constexpr T beta(int l, int m) {
    return (T)((l + m - 1) * (l - m - 1)) / (T)((2 * l - 1) * (2 * l - 3));
}

// Split point of the m range when the values of one bin do not fit one lane.
__host__ __device__ constexpr int m_split(int lmax) {
    // largest M such that values(m <= M) + self stay within half of all values
    const int total = n_values(lmax);
    int acc = 2 * lmax + 1 + (lmax + 1);
    int M = 0;
    while (M < lmax && 2 * (acc + 2 * (lmax - M)) <= total) {
        ++M;
        acc += 2 * (lmax - M + 1);
    }
    return M;
}

template <typename T, int LMAX, int G>
struct Acc {
    static constexpr int MLO = G == 2 ? m_split(LMAX) + 1 : 0;
    static constexpr int MHI = G == 1 ? m_split(LMAX) : LMAX;
    static constexpr bool SELF = G != 2;
    static constexpr int V0 = value_offset(LMAX, MLO);
    static constexpr int V1 = value_offset(LMAX, MHI + 1);
    static constexpr int NA = V1 - V0;            // a_lm values held
    static constexpr int NS = SELF ? 2 * LMAX + 1 : 0;
    T a[NA > 0 ? NA : 1];
    T s[NS > 0 ? NS : 1];
};

// Accumulates one neighbour (unit vector x,y,z; weight w).
template <typename T, int LMAX, int G>
__device__ __forceinline__ void add_hit(Acc<T, LMAX, G>& A, T x, T y, T z, T w) {
    using AC = Acc<T, LMAX, G>;
    constexpr int MLO = AC::MLO, MHI = AC::MHI, V0 = AC::V0;
    if constexpr (MLO == 0 || AC::SELF) {
        // m = 0 chain, up to 2 lmax when the self moments are held
        constexpr int LTOP = AC::SELF ? 2 * LMAX : LMAX;
        const T w2 = w * w;
        T r0 = (T)1, r1 = z;
        if constexpr (MLO == 0) A.a[0 - V0] += w;
        if constexpr (AC::SELF) A.s[0] += w2;
        if constexpr (LTOP >= 1) {
            if constexpr (MLO == 0 && LMAX >= 1) A.a[1 - V0] = fma(w, r1, A.a[1 - V0]);
            if constexpr (AC::SELF) A.s[1] = fma(w2, r1, A.s[1]);
        }
#pragma unroll
        for (int l = 2; l <= LTOP; ++l) {
            const T r2 = fma(z, r1, -beta<T>(l, 0) * r0);
            if (MLO == 0 && l <= LMAX) A.a[l - V0] = fma(w, r2, A.a[l - V0]);
            if (AC::SELF) A.s[l] = fma(w2, r2, A.s[l]);
            r0 = r1;
            r1 = r2;
        }
    }
    if constexpr (MHI >= 1) {
        // c_m = w (x - i y)^m
        T cr = w * x, ci = -(w * y);
#pragma unroll
        for (int m = 1; m <= MHI; ++m) {
            if (m > 1) {
                const T t = fma(cr, x, ci * y);
                ci = fma(ci, x, -(cr * y));
                cr = t;
            }
            if (m >= MLO) {
                const int vo = value_offset(LMAX, m) - V0;
                const int nl = LMAX - m + 1;
                A.a[vo] += cr;
                A.a[vo + nl] += ci;
                if (m + 1 <= LMAX) {
                    T q0 = (T)1, q1 = z;
                    A.a[vo + 1] = fma(q1, cr, A.a[vo + 1]);
                    A.a[vo + nl + 1] = fma(q1, ci, A.a[vo + nl + 1]);
#pragma unroll
                    for (int l = m + 2; l <= LMAX; ++l) {
                        const T q2 = fma(z, q1, -beta<T>(l, m) * q0);
                        A.a[vo + l - m] = fma(q2, cr, A.a[vo + l - m]);
                        A.a[vo + nl + l - m] = fma(q2, ci, A.a[vo + nl + l - m]);
                        q0 = q1;
                        q1 = q2;
                    }
                }
            }
        }
    }
}

template <typename T, int LMAX, int G>
__global__ void __launch_bounds__(256) k_pair_alm(AlmArgs a) {
    using AC = Acc<T, LMAX, G>;
    constexpr int NV = n_values(LMAX);
    __shared__ float sh[kMaxCodes * 3];
    for (int i = threadIdx.x; i < a.ncodes * 3; i += blockDim.x) sh[i] = a.shift_f[i];
    __syncthreads();

    const int lane = lane_id();
    const int64_t nprim = a.p_end - a.p_begin;
    const int64_t nblk64 = (nprim + 63) / 64;
    const int64_t nwaves = nblk64 * a.nb;
    const int64_t nwg = (nwaves + 3) / 4;
    const int64_t wg = xcd_block(blockIdx.x, (int64_t)gridDim.x);
    if (wg >= nwg) return;
    const int64_t wv = wg * 4 + (threadIdx.x >> 6);
    if (wv >= nwaves) return;
    const int64_t blk = wv / a.nb;
    const int b = (int)(wv - blk * a.nb);
    const int64_t pl = blk * 64 + lane;
    const int64_t p = a.p_begin + pl;
    const bool active = pl < nprim;

    AC acc;
#pragma unroll
    for (int i = 0; i < (AC::NA > 0 ? AC::NA : 1); ++i) acc.a[i] = (T)0;
#pragma unroll
    for (int i = 0; i < (AC::NS > 0 ? AC::NS : 1); ++i) acc.s[i] = (T)0;

    uint32_t n = 0, off = 0;
    int64_t cstart = 0;
    float4 P32 = make_float4(0.f, 0.f, 0.f, 0.f);
    double4 P64 = make_double4(0.0, 0.0, 0.0, 0.0);
    if (active) {
        n = a.cnt[pl * a.nb + b];
        off = a.boff[pl * a.nb + b];
        cstart = a.pt_off[a.catid[p]];
        if (sizeof(T) == 4) P32 = a.pf[p]; else P64 = a.pd[p];
    }
    const uint32_t mask = a.g.idx_mask;
    const int cshift = 32 - a.g.code_bits;
    for (uint32_t t = 0; t < n; ++t) {
        const uint32_t e = a.list[off + t];
        const int64_t j = cstart + (int64_t)(e & mask);
        T x, y, z, w;
        if constexpr (sizeof(T) == 4) {
            const float4 q = a.pf[j];
            w = a.pw[j];
            float dx = q.x - P32.x, dy = q.y - P32.y, dz = q.z - P32.z;
            if (a.g.single) {
                dx -= a.g.boxf * rintf(dx / a.g.boxf);
                dy -= a.g.boxf * rintf(dy / a.g.boxf);
                dz -= a.g.boxf * rintf(dz / a.g.boxf);
            } else {
                const int code = (int)(e >> cshift);
                dx += sh[3 * code];
                dy += sh[3 * code + 1];
                dz += sh[3 * code + 2];
            }
            const float r2 = dx * dx + dy * dy + dz * dz;
            const float inv = __builtin_amdgcn_rsqf(r2);
            x = dx * inv; y = dy * inv; z = dz * inv;
        } else {
            const double4 q = a.pd[j];
            w = q.w;
            double dx = q.x - P64.x, dy = q.y - P64.y, dz = q.z - P64.z;
            const double L = a.g.box, hL = 0.5 * a.g.box;
            dx = dx > hL ? dx - L : (dx < -hL ? dx + L : dx);
            dy = dy > hL ? dy - L : (dy < -hL ? dy + L : dy);
            dz = dz > hL ? dz - L : (dz < -hL ? dz + L : dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            double inv = __builtin_amdgcn_rsq(r2);
            inv = inv * fma(-0.5 * r2 * inv, inv, 1.5);
            inv = inv * fma(-0.5 * r2 * inv, inv, 1.5);
            x = dx * inv; y = dy * inv; z = dz * inv;
        }
        add_hit<T, LMAX, G>(acc, x, y, z, w);
    }
    if (!active) return;
    T* A = reinterpret_cast<T*>(a.A);
    const int64_t ld = a.ldA;
#pragma unroll
    for (int i = 0; i < AC::NA; ++i) A[((int64_t)b * NV + AC::V0 + i) * ld + pl] = acc.a[i];
    if constexpr (AC::SELF) {
#pragma unroll
        for (int i = 0; i < AC::NS; ++i)
            A[((int64_t)b * NV + n_alm_values(LMAX) + i) * ld + pl] = acc.s[i];
    }
}

template <typename T, int LMAX, int G>
hipError_t launch_alm_one(const AlmArgs& a, hipStream_t s) {
    const int64_t nprim = a.p_end - a.p_begin;
    const int64_t nwaves = ((nprim + 63) / 64) * a.nb;
    int64_t nwg = (nwaves + 3) / 4;
    nwg = (nwg + 7) / 8 * 8;
    hipLaunchKernelGGL((k_pair_alm<T, LMAX, G>), dim3((unsigned)nwg), dim3(256), 0, s, a);
    return hipGetLastError();
}

// FP32 keeps every value of a bin in one lane up to lmax 10; FP64 splits the
// m range over two launches from lmax 7 on (register budget).
template <int LMAX>
hipError_t launch_alm_lmax(const AlmArgs& a, int fp64, hipStream_t s) {
    if (!fp64) {
        if constexpr (LMAX <= 10) {
            return launch_alm_one<float, LMAX, 0>(a, s);
        } else {
            hipError_t e = launch_alm_one<float, LMAX, 1>(a, s);
            if (e != hipSuccess) return e;
            return launch_alm_one<float, LMAX, 2>(a, s);
        }
    } else {
        if constexpr (LMAX <= 6) {
            return launch_alm_one<double, LMAX, 0>(a, s);
        } else {
            hipError_t e = launch_alm_one<double, LMAX, 1>(a, s);
            if (e != hipSuccess) return e;
            return launch_alm_one<double, LMAX, 2>(a, s);
        }
    }
}

}  // namespace

hipError_t launch_pair_bin(const BinArgs& a, hipStream_t s) {
    const int64_t nprim = a.p_end - a.p_begin;
    if (nprim <= 0) return hipSuccess;
    int64_t nblk = (nprim + 3) / 4;
    nblk = (nblk + 7) / 8 * 8;
    const size_t lds = 4 * sizeof(BinLds);
    if (a.fp64)
        hipLaunchKernelGGL(k_pair_bin<true>, dim3((unsigned)nblk), dim3(256), lds, s, a);
    else
        hipLaunchKernelGGL(k_pair_bin<false>, dim3((unsigned)nblk), dim3(256), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_pair_alm(const AlmArgs& a, int fp64, hipStream_t s) {
    if (a.p_end <= a.p_begin) return hipSuccess;
    switch (a.lmax) {
        case 0: return launch_alm_lmax<0>(a, fp64, s);
        case 1: return launch_alm_lmax<1>(a, fp64, s);
        case 2: return launch_alm_lmax<2>(a, fp64, s);
        case 3: return launch_alm_lmax<3>(a, fp64, s);
        case 4: return launch_alm_lmax<4>(a, fp64, s);
        case 5: return launch_alm_lmax<5>(a, fp64, s);
        case 6: return launch_alm_lmax<6>(a, fp64, s);
        case 7: return launch_alm_lmax<7>(a, fp64, s);
        case 8: return launch_alm_lmax<8>(a, fp64, s);
        case 9: return launch_alm_lmax<9>(a, fp64, s);
        case 10: return launch_alm_lmax<10>(a, fp64, s);
        case 11: return launch_alm_lmax<11>(a, fp64, s);
        case 12: return launch_alm_lmax<12>(a, fp64, s);
        default: return hipErrorInvalidValue;
    }
}

size_t pair_bin_lds_bytes() { return 4 * sizeof(BinLds); }

}  // namespace tpcf
