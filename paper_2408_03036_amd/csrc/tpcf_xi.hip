// Pair counts of the anisotropic 2PCF (arXiv:2408.03036, Sec. 4.1): DD(r, mu)
// over ordered pairs, r the minimum-image separation and mu = dz / r the
// cosine to the line of sight z, and the Legendre multipoles of the natural
// estimator DD / RR - 1 with analytic periodic RR (eq. (xi_natest),
// (xi_meas_leg)).
//
//  k_xi_count     persistent workgroups over the work items of the neighbour
//                 grid (up to 16 primaries of one cell). Every unordered pair
//                 is tested once: the stencil is halved (cell offsets that are
//                 positive in (x, y, z) order, plus the home cell), and a pair
//                 with its neighbour outside the home cell adds both ordered
//                 pairs, (p, j) at mu and (j, p) at -mu, whose separation is
//                 exactly the negated one. Home-cell pairs are seen from both
//                 ends and add one each. The half stencil is staged tile by
//                 tile in LDS in the home cell's frame and tested against the
//                 primaries; each hit increments uint32 counters of a
//                 workgroup histogram in LDS, flushed to the 64-bit global
//                 counts once at the end (or earlier when a counter could
//                 overflow). Items are taken from eight queues, one per
//                 contiguous eighth of the cells, so that the workgroups of
//                 one XCD share neighbours in that XCD's L2; a workgroup
//                 whose queue is empty moves on to the next one. In
//                 single-cell mode (small boxes) the stencil is the whole box
//                 and every ordered pair is tested.
//  k_xi_finalize  xi_l(r_b) = sum_k c_lk (DD(b, k) / RR_b - 1).
//
// Bin decisions equal those of an exact double-precision evaluation:
// r^2 = dx*dx + dy*dy + dz*dz against the squared edges, and
// k = floor((dz / sqrt(r^2) + 1) * nmu / 2) clamped to [0, nmu - 1], every
// operation rounded in double. The FP32 test sends every pair within a
// rounding-error bound of an r or mu edge to that exact evaluation.
#include <algorithm>

#include "tpcf_cells.h"

namespace tpcf {

namespace {

constexpr int kXW = 4;                     // wavefronts per workgroup
constexpr int kXG = kItemPrims / kXW;      // primaries per wavefront
constexpr int kXTile = 128;                // candidates per LDS tile
constexpr int kXUT = kXTile / 64;          // tile candidates per lane
constexpr int kXStage = (kXTile + 64 * kXW - 1) / (64 * kXW);  // candidates each thread stages
constexpr int kQueues = 8;
constexpr int kQueueStride = 32;           // ints between queue cursors (128 bytes)
static_assert(kXG * kXW == kItemPrims, "item size");

// Exact bin indices b * nmu + k of the pair (p, j) and of the reversed pair
// (j, p), or -1 (outside the shells, or zero separation). The reversed pair's
// separation is exactly the negated one (rounding and rint are odd), so its
// mu is exactly -mu. Periodic shifts come from the stencil code (equal to the
// minimum image inside the shells) or, in single-cell mode, from rint.
template <bool SINGLE>
__device__ __forceinline__ int2 exact_xi_t(const double4 P, const double4 Q, int wbits, double box, int nb,
                                        const double* e2, int nmu, double hmu) {
#pragma clang fp contract(off)
    double dx = Q.x - P.x, dy = Q.y - P.y, dz = Q.z - P.z;
    if constexpr (SINGLE) {
        dx -= box * rint(dx / box);
        dy -= box * rint(dy / box);
        dz -= box * rint(dz / box);
    } else {
        dx += wrap_shift(wbits, 0, box);
        dy += wrap_shift(wbits, 1, box);
        dz += wrap_shift(wbits, 2, box);
    }
    double r2 = dx * dx;
    r2 += dy * dy;
    r2 += dz * dz;
    if (r2 == 0.0 || r2 < e2[0] || r2 >= e2[nb]) return make_int2(-1, -1);
    int b = 0;
    while (b + 1 < nb && r2 >= e2[b + 1]) ++b;
    const double r = sqrt(r2);
    const double mu = dz / r;
    auto kbin = [&](double m) {
        const int k = (int)floor((m + 1.0) * hmu);
        return k < 0 ? 0 : (k > nmu - 1 ? nmu - 1 : k);
    };
    return make_int2(b * nmu + kbin(mu), b * nmu + kbin(-mu));
}

// Inlined, and evaluated after a tile's tests for the pairs they marked: as
// a call inside the test loop it would cost the kernel the callee-saved
// registers and make every tile wait for its pending loads.
template <bool SINGLE>
__device__ __forceinline__ int2 exact_xi_pair(const double4* pd, int64_t p, uint32_t entry, uint32_t mask,
                                           int cshift, int cx, int cy, int cz, int k, int nc, double box,
                                           int nb, const double* e2, int nmu, double hmu) {
    const int64_t j = (int64_t)(entry & mask);
    const int wb = SINGLE ? 0 : wrap_bits_of((int)(entry >> cshift), cx, cy, cz, k, nc);
    return exact_xi_t<SINGLE>(pd[p], pd[j], wb, box, nb, e2, nmu, hmu);
}

// One candidate being staged: its point, its piece's shift and its index.
struct XStaged {
    int r;
    float4 q;
    float sx, sy, zo;
    int code;
    uint32_t j;
    bool ok;
};

__device__ __forceinline__ void xstage_load(XStaged& st, const Pieces& S, int total, int g, const float4* pf) {
    st.ok = g < total;
    if (st.ok) {
        int r = st.r;
        while (S.pref[r + 1] <= g) ++r;
        st.r = r;
        const float4 rc = S.rec[r];
        st.j = (uint32_t)(g + __float_as_int(rc.x));
        st.sx = rc.y;
        st.sy = rc.z;
        st.zo = rc.w;
        st.code = S.code[r] & 0xffff;
        st.q = pf[st.j];
    }
}

// Also called for an empty slot (past the last candidate, never tested): the
// write is then harmless, and being unconditional it keeps the wait for the
// slot's load on every path.
template <bool SINGLE>
__device__ __forceinline__ void xstage_store(const XStaged& st, float4* dst, uint32_t* dent, int cshift,
                                             float hf) {
    if constexpr (SINGLE) {
        *dst = make_float4(st.q.x, st.q.y, st.q.z, 0.f);
        *dent = st.j;
    } else {
        const int oz = (int)(st.q.w + st.zo);
        *dst = make_float4(st.q.x + st.sx, st.q.y + st.sy, fmaf((float)oz, hf, st.q.z), 0.f);
        *dent = st.j | ((uint32_t)(st.code + oz) << cshift);
    }
}

struct XiLds {
    double e2[kMaxBins + 1];
    float e2f[kMaxBins + 1];
    float guard[kMaxBins + 1];
    int item;
    int pad[3];
};

__host__ __device__ inline size_t xi_hist_offset() { return (sizeof(XiLds) + 15) / 16 * 16; }

template <bool SINGLE, bool UNIFORM>
__global__ void __launch_bounds__(64 * kXW) k_xi_count(XiArgs a) {
    extern __shared__ unsigned char smem[];
    XiLds& X = *reinterpret_cast<XiLds*>(smem);
    const int nh = a.nb * a.nmu;
    size_t off = xi_hist_offset();
    uint32_t* hist = reinterpret_cast<uint32_t*>(smem + off);
    off += ((size_t)nh * sizeof(uint32_t) + 15) / 16 * 16;
    float4* tiles = reinterpret_cast<float4*>(smem + off);
    off += sizeof(float4) * 2 * kXTile;
    uint32_t* tent = reinterpret_cast<uint32_t*>(smem + off);
    off += sizeof(uint32_t) * 2 * kXTile;
    Pieces S = pieces_view(smem + off, a.npmax);

    for (int i = threadIdx.x; i <= a.nb; i += blockDim.x) {
        X.e2[i] = a.e2[i];
        X.e2f[i] = a.e2f[i];
        X.guard[i] = a.guard[i];
    }
    for (int i = threadIdx.x; i < nh; i += blockDim.x) hist[i] = 0u;

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = lane_id();
    const int cshift = 32 - a.g.code_bits;
    const uint32_t mask = a.g.idx_mask;
    const uint32_t home_code = (uint32_t)a.home_code;
    const unsigned nbu = (unsigned)a.nb;
    const float ne0 = -a.e0f * a.inv_dr;
    const int64_t per = (a.nitems + kQueues - 1) / kQueues;
    int qi = 0;                       // queues visited (thread 0)
    const int home = blockIdx.x % kQueues;
    unsigned long long bound = 0;     // upper bound of the hits since the last flush

    auto flush = [&]() {
        for (int i = threadIdx.x; i < nh; i += blockDim.x) {
            const uint32_t v = hist[i];
            if (v) {
                atomicAdd(a.counts + i, (unsigned long long)v);
                hist[i] = 0u;
            }
        }
    };

    for (;;) {
        if (threadIdx.x == 0) {
            int item = -1;
            while (qi < kQueues) {
                const int q = (home + qi) % kQueues;
                const int64_t lo = (int64_t)q * per, hi = min(lo + per, a.nitems);
                if (lo < hi) {
                    const int v = atomicAdd(a.queue + q * kQueueStride, 1);
                    if (lo + v < hi) {
                        item = (int)(lo + v);
                        break;
                    }
                }
                ++qi;
            }
            X.item = item;
        }
        __syncthreads();
        const int item = X.item;
        if (item < 0) break;

        const int gc = a.item_cell[item];
        const int64_t first = (int64_t)a.cell_start[gc] + (int64_t)(item - a.item_start[gc]) * kItemPrims;
        const int64_t last = min(first + kItemPrims, (int64_t)a.cell_start[gc + 1]);
        const int cz = gc % a.g.nc, cy = (gc / a.g.nc) % a.g.nc, cx = gc / (a.g.nc * a.g.nc);
        if (wave == 0) {
            // candidates cut to the reach of the item's primaries, as in the
            // 3PCF binning (a pair within the outer edge keeps its candidate)
            if constexpr (SINGLE) build_pieces(S, a, 0, 0, 0, 0);
            else build_pieces<true>(S, a, 0, cx, cy, cz, item_box(a.pf, first, last, a.reach2));
        }
        __syncthreads();
        const int total = S.pref[*S.n];
        const int rem = (int)(last - first);
        const int ng = rem > wave ? (rem - wave + kXW - 1) / kXW : 0;

        // a counter may reach at most twice the tests of the items since the last flush
        bound += 2ull * (unsigned long long)rem * (unsigned long long)total;
        if (bound > 0x7fffffffull) {
            flush();
            __syncthreads();
            bound = 2ull * (unsigned long long)rem * (unsigned long long)total;
        }

        float px[kXG], py[kXG], pz[kXG];
#pragma unroll
        for (int g = 0; g < kXG; ++g) {
            px[g] = py[g] = pz[g] = 0.f;
            if (g < ng) {
                // uniform over the wavefront: scalar registers
                const float4 P = a.pf[first + wave + kXW * g];
                px[g] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(P.x)));
                py[g] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(P.y)));
                pz[g] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(P.z)));
            }
        }

        // the first kXTile / 64 wavefronts stage, thread x tile slot x: its
        // load is issued before the tests and its LDS write follows them
        static_assert(kXStage == 1 && kXTile % 64 == 0, "one staging slot per staging thread");
        XStaged st;
        st.r = 0;
        const bool stager = wave < kXTile / 64;
        if (stager) {
            xstage_load(st, S, total, (int)threadIdx.x, a.pf);
            xstage_store<SINGLE>(st, tiles + threadIdx.x, tent + threadIdx.x, cshift, a.g.hf);
        }
        __syncthreads();
        int buf = 0;
        for (int t = 0; t < total; t += kXTile) {
            const float4* cur = tiles + buf * kXTile;
            const uint32_t* cure = tent + buf * kXTile;
            const bool more = t + kXTile < total;
            if (more && stager) xstage_load(st, S, total, t + kXTile + (int)threadIdx.x, a.pf);
            const int nt = min(kXTile, total - t);
            uint32_t nearbits = 0;
            static_assert(kXUT * kXG <= 32, "near-edge marks");
#pragma unroll 2
            for (int u = 0; u < kXUT; ++u) {
                const int i = u * 64 + lane;
                if (i >= nt) break;
                const float4 q = cur[i];
                const uint32_t entry = cure[i];
                // neighbours outside the home cell stand for both ordered pairs
                const bool both = !SINGLE && (entry >> cshift) != home_code;
#pragma unroll
                for (int g = 0; g < kXG; ++g) {
                    if (g >= ng) break;
                    float dx = q.x - px[g], dy = q.y - py[g], dz = q.z - pz[g];
                    if constexpr (SINGLE) {
                        dx -= a.g.boxf * rintf(dx * a.inv_boxf);
                        dy -= a.g.boxf * rintf(dy * a.inv_boxf);
                        dz -= a.g.boxf * rintf(dz * a.inv_boxf);
                    }
                    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    const float r = __builtin_amdgcn_sqrtf(r2);
                    int bb;
                    bool near;
                    if constexpr (UNIFORM) {
                        const float uu = fmaf(r, a.inv_dr, ne0);
                        const float fl = floorf(uu);
                        bb = (int)fl;
                        const float fr = uu - fl;
                        near = (fr < a.delta || fr > 1.0f - a.delta) && (unsigned)(bb + 1) <= nbu + 1u;
                    } else {
                        bb = -1;
                        near = false;
                        if (r2 >= X.e2f[0] - X.guard[0] && r2 < X.e2f[a.nb] + X.guard[a.nb]) {
                            for (int e = 0; e <= a.nb; ++e) {
                                bb += r2 >= X.e2f[e];
                                near |= fabsf(r2 - X.e2f[e]) < X.guard[e];
                            }
                        }
                    }
                    if (!near && (unsigned)bb >= nbu) continue;
                    // mu bins: t = (+-mu + 1) nmu / 2 in FP32 with its error bound
                    const float rinv = __builtin_amdgcn_rcpf(r);
                    const float mu = dz * rinv;
                    const float tt = fmaf(mu, a.hmu_f, a.hmu_f);
                    const float tr = fmaf(-mu, a.hmu_f, a.hmu_f);
                    const float fk = floorf(tt), fkr = floorf(tr);
                    const float ft = tt - fk, ftr = tr - fkr;
                    const float gt = fmaf(a.gmu_a, rinv, a.gmu_b);
                    near |= !(ft >= gt && ft <= 1.0f - gt);  // also catches r = 0 (inf / nan)
                    near |= both && !(ftr >= gt && ftr <= 1.0f - gt);
                    // a pair near an edge is only marked here
                    if (__ballot(near) != 0ull) {
                        if (near) nearbits |= 1u << (u * kXG + g);
                    }
                    if (!near) {
                        const int row = bb * a.nmu, top = a.nmu - 1;
                        atomicAdd(hist + row + min(max((int)fk, 0), top), 1u);
                        if (both) atomicAdd(hist + row + min(max((int)fkr, 0), top), 1u);
                    }
                }
            }
            // the next tile's slot (written also after the last tile: the
            // other buffer is then unused)
            if (stager)
                xstage_store<SINGLE>(st, tiles + (buf ^ 1) * kXTile + threadIdx.x,
                                     tent + (buf ^ 1) * kXTile + threadIdx.x, cshift, a.g.hf);
            // the marked pairs, binned exactly (rare)
            if (__ballot(nearbits != 0u) != 0ull) {
#pragma unroll
                for (int g = 0; g < kXG; ++g) {
                    uint32_t m = nearbits & (0x11111111u << g);  // bits u kXG + g
                    while (m != 0u) {
                        const int bit = __builtin_ctz(m);
                        m &= m - 1u;
                        const uint32_t entry = cure[(bit / kXG) * 64 + lane];
                        const bool both = !SINGLE && (entry >> cshift) != home_code;
                        const int2 idx = exact_xi_pair<SINGLE>(a.pd, first + wave + kXW * g, entry, mask, cshift, cx,
                                                               cy, cz, a.g.k, a.g.nc, a.g.box, a.nb, X.e2, a.nmu,
                                                               a.hmu);
                        if (idx.x >= 0) {
                            atomicAdd(hist + idx.x, 1u);
                            if (both) atomicAdd(hist + idx.y, 1u);
                        }
                    }
                }
            }
            __syncthreads();
            buf ^= 1;
        }
    }
    flush();
}

__global__ void k_xi_finalize(XiFinalArgs a) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n_ell * a.nb) return;
    const int i = t / a.nb, b = t % a.nb;
    const double inv = 1.0 / a.rr[b];
    double s = 0.0;
    for (int k = 0; k < a.nmu; ++k) {
        const double xi = (double)a.counts[(size_t)b * a.nmu + k] * inv - 1.0;
        s = fma(a.coef[(size_t)i * a.nmu + k], xi, s);
    }
    a.out[t] = s;
}

template <bool SINGLE, bool UNIFORM>
hipError_t launch_xi_variant(const XiArgs& a, hipStream_t s) {
    const size_t lds = xi_lds_bytes(a.nb, a.nmu, a.npmax);
    if (lds > 64 * 1024) {
        hipError_t e = allow_full_lds((const void*)k_xi_count<SINGLE, UNIFORM>);
        if (e != hipSuccess) return e;
    }
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_xi_count<SINGLE, UNIFORM>, 64 * kXW,
                                                          lds)) != hipSuccess)
        return e;
    int64_t grid = (int64_t)std::max(per_cu, 1) * std::max(ncu, 1);
    grid = std::min<int64_t>(grid, (a.nitems + 1) / 2 * 2);
    grid = std::max<int64_t>((grid + kQueues - 1) / kQueues * kQueues, kQueues);
    hipLaunchKernelGGL((k_xi_count<SINGLE, UNIFORM>), dim3((unsigned)grid), dim3(64 * kXW), lds, s, a);
    return hipGetLastError();
}

}  // namespace

size_t xi_lds_bytes(int nb, int nmu, int npmax) {
    return xi_hist_offset() + ((size_t)nb * nmu * sizeof(uint32_t) + 15) / 16 * 16 +
           (sizeof(float4) + sizeof(uint32_t)) * 2 * kXTile + pieces_lds_bytes(npmax);
}

hipError_t launch_xi_count(const XiArgs& a, hipStream_t s) {
    if (a.nitems <= 0) return hipSuccess;
    if (a.g.single) return a.uniform ? launch_xi_variant<true, true>(a, s) : launch_xi_variant<true, false>(a, s);
    return a.uniform ? launch_xi_variant<false, true>(a, s) : launch_xi_variant<false, false>(a, s);
}

hipError_t launch_xi_finalize(const XiFinalArgs& a, hipStream_t s) {
    const int n = a.n_ell * a.nb;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_xi_finalize, dim3((n + 127) / 128), dim3(128), 0, s, a);
    return hipGetLastError();
}

}  // namespace tpcf
