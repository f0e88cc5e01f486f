// Pair pass of the anisotropic 3PCF estimator (arXiv:2408.03036, Sec. 4.2,
// eq. (alm)): for every primary p and every neighbour j with |x_j - x_p| in
// radial bin b, accumulate w_j conj(Y_lm(rhat_pj)) into a_lm(p, b).
//
// Two kernels:
//  k_pair_bin  one workgroup per work item (up to 16 primaries of one cell of
//              the neighbour grid). The cell's stencil of neighbour cells is
//              one flattened candidate range, staged tile by tile in LDS in the
//              home cell's frame; every wavefront tests the tile against its
//              primaries and writes each hit into its primary's list, laid out
//              bin by bin in regions predicted from the local density, with
//              (offset, count) per (p, b). Primaries that overflow a region
//              are redone by a second launch with exact counts.
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
#include <type_traits>

#include "tpcf_cells.h"

namespace tpcf {

namespace {

// Exact FP64 bin of a pair (the reference evaluation: r^2 = dx*dx + dy*dy +
// dz*dz in that order, no fused multiply-add), -1 outside the shells or at
// zero separation. Periodic shifts come from the cell geometry (equal to the
// minimum image for any pair inside the shells) or, in single-cell mode,
// from rint.
template <bool SINGLE>
__device__ __forceinline__ int exact_bin_t(const double4 P, const double4 Q, int wbits, double box, int nb,
                                           const double* e2) {
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
    if (r2 == 0.0 || r2 < e2[0] || r2 >= e2[nb]) return -1;
    int b = 0;
    while (b + 1 < nb && r2 >= e2[b + 1]) ++b;
    return b;
}

// Exact bin of the pair (primary p, candidate with list entry `entry`) for a
// pair inside an FP32 guard band (rare). Inlined: it is evaluated once per
// tile, after the tests, where its registers are free; as a call it would
// cost the kernel the callee-saved registers and make every tile wait for
// its pending loads before the tests.
template <bool SINGLE>
__device__ __forceinline__ int exact_pair(const double4* pd, int64_t p, int64_t cstart, uint32_t entry,
                                          uint32_t mask, int cshift, int cx, int cy, int cz, int k, int nc,
                                          double box, int nb, const double* e2) {
    const int64_t j = cstart + (int64_t)(entry & mask);
    const int wb = SINGLE ? 0 : wrap_bits_of((int)(entry >> cshift), cx, cy, cz, k, nc);
    return exact_bin_t<SINGLE>(pd[p], pd[j], wb, box, nb, e2);
}

constexpr int kNW = 4;                     // wavefronts per workgroup
constexpr int kGM = kItemPrims / kNW;      // primaries per wavefront
constexpr int kTile = 256;                 // candidates per LDS tile
constexpr int kUT = kTile / 64;            // tile candidates per lane
// staging: a thread stages kStage slots of each tile (all threads when the
// tile holds at least one slot per thread, else the first kTile / 64 waves)
constexpr int kStage = kTile >= 64 * kNW ? kTile / (64 * kNW) : 1;
static_assert(kTile % 64 == 0 && (kTile < 64 * kNW || kTile % (64 * kNW) == 0), "tile shape");
// near-edge marks of a lane: bit u kGM + g for (tile slot u, primary g);
// kNearPrimary has the bits of primary 0
using NearMask = std::conditional_t<(kUT * kGM > 32), uint64_t, uint32_t>;
static_assert(kUT * kGM <= 64, "near-edge marks");
constexpr NearMask near_primary_bits() {
    NearMask m = 0;
    for (int u = 0; u < kUT; ++u) m |= (NearMask)1 << (u * kGM);
    return m;
}
constexpr NearMask kNearPrimary = near_primary_bits();
constexpr uint32_t kNoBase = 0xffffffffu;

// Octahedral code of a direction, the 8-byte record of a hit with unit
// weights: the point d / (|dx| + |dy| + |dz|) of the octahedron |x| + |y| +
// |z| = 1, whose lower half (z < 0) is folded onto the square's corners,
// (x, y) -> ((1 - |y|) sgn x, (1 - |x|) sgn y), kept as (p, q). The harmonic
// pass needs only the direction of a hit (its list is its bin). Decoding
// is z = 1 - |p| - |q|, unfolding where z < 0; both steps are well
// conditioned, so the direction comes back within a few FP32 rounding
// errors in absolute terms, also near the fold (an encoding by x, y and
// the sign of z would lose accuracy near z = 0, where z = sqrt(1 - x^2 - y^2)).
// The approximate reciprocal scales p and q together, and the decoded point
// is normalised by the reader, so its error does not change the direction
// beyond that bound.
__device__ __forceinline__ float2 oct_encode(float dx, float dy, float dz) {
    const float is = __builtin_amdgcn_rcpf(fabsf(dx) + fabsf(dy) + fabsf(dz));
    float p = dx * is, q = dy * is;
    if (dz < 0.f) {
        const float p0 = p;
        p = copysignf(1.f - fabsf(q), p0);
        q = copysignf(1.f - fabsf(p0), q);
    }
    return make_float2(p, q);
}
// The octahedron point (x, y, z) of a code (a direction, not normalised).
__device__ __forceinline__ float3 oct_decode(float p, float q) {
    const float z = 1.f - fabsf(p) - fabsf(q);
    const float x = z < 0.f ? copysignf(1.f - fabsf(q), p) : p;
    const float y = z < 0.f ? copysignf(1.f - fabsf(p), q) : q;
    return make_float3(x, y, z);
}
static_assert(kGM * kNW == kItemPrims, "item size");

// A candidate being staged: the point (cell-relative FP32), its piece's shift
// and its index, held in registers while the previous tile is tested.
struct Staged {
    int r;      // piece of the slot's last candidate (advances monotonically)
    float4 q;
    float w;
    float sx, sy, zo;
    int code;
    uint32_t j;
    bool ok;
};

template <bool SINGLE, int REC>
__device__ __forceinline__ void stage_load(Staged& st, const Pieces& S, int np, int total, int g,
                                           const float4* pf, const float* pw) {
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
        // unit weights are applied when the candidate is stored: the weight
        // register is only ever written by its load
        if (REC == 4 && pw) st.w = pw[st.j];
    }
}

// Writes a staged candidate in the home cell's frame, (x, y, z, w), and its
// list entry = catalogue-relative index | stencil code << cshift. Also called
// for an empty slot (past the last candidate, never tested): the write is
// then harmless, and being unconditional it keeps the wait for the slot's
// load on every path.
template <bool SINGLE, int REC>
__device__ __forceinline__ void stage_store(const Staged& st, float4* dst, uint32_t* dent, uint32_t cst,
                                            int cshift, float hf, bool weighted) {
    const float w = REC == 4 ? (weighted ? st.w : 1.f) : 0.f;
    float4 v;
    uint32_t e;
    if constexpr (SINGLE) {
        v = make_float4(st.q.x, st.q.y, st.q.z, w);
        e = st.j - cst;
    } else {
        const int oz = (int)(st.q.w + st.zo);
        v.x = st.q.x + st.sx;
        v.y = st.q.y + st.sy;
        v.z = fmaf((float)oz, hf, st.q.z);
        v.w = w;
        e = (st.j - cst) | ((uint32_t)(st.code + oz) << cshift);
    }
    *dst = v;
    *dent = e;
}

// State of one work item shared by its two sweeps.
struct ItemCtx {
    const Pieces* S;
    float4* tiles;          // [2][kTile] candidates (x, y, z, w) in the home cell's frame
    uint32_t* tent;         // [2][kTile] their list entries
    const BinTables* T;
    uint32_t* cnt;          // this wavefront's [kGM][kMaxBins] counters / write cursors
    uint32_t* end;          // this wavefront's [kGM][kMaxBins] ends of the predicted regions
    int np, total;          // pieces and candidates after the cut to the item
    int total_full;         // candidates of the whole stencil (density estimate)
    int64_t cs, cstart;     // first primary of this wavefront's group, catalogue start
    uint32_t cst, mask;
    int cshift, cx, cy, cz, wave, lane, ng;
    int slot;               // allocation region of this wavefront
};

// Separation of a staged candidate from a primary, in the FP32 frame of the
// tests and the records.
template <bool SINGLE>
__device__ __forceinline__ void separation(const BinArgs& a, const float4 q, float px, float py, float pz,
                                           float& dx, float& dy, float& dz) {
    dx = q.x - px;
    dy = q.y - py;
    dz = q.z - pz;
    if constexpr (SINGLE) {
        dx -= a.g.boxf * rintf(dx * a.inv_boxf);
        dy -= a.g.boxf * rintf(dy * a.inv_boxf);
        dz -= a.g.boxf * rintf(dz * a.inv_boxf);
    }
}

// Records a hit of primary g in bin b (b < 0: none): SWEEP 0 counts it;
// SWEEP 1 and 2 take the next slot of the bin and write what REC selects:
// 0 the list entry (FP64 path), 2 the octahedral code of the direction
// (p, q) (unit weights), 4 the record (dx, dy, dz, w_j); SWEEP 2 drops (but
// still counts) a hit beyond the end of the bin's predicted region.
template <int SWEEP, int REC>
__device__ __forceinline__ void put_hit(const BinArgs& a, const ItemCtx& c, int g, bool hit, int b, uint32_t base_g,
                                        float dx, float dy, float dz, float w, uint32_t entry) {
    if constexpr (SWEEP == 0) {
        if (hit) atomicAdd(&c.cnt[g * kMaxBins + b], 1u);
    } else if (hit && base_g != kNoBase) {
        // the LDS unit serves the lanes of one atomic in a fixed order, so
        // the lists are the same on every run
        const uint32_t pos = atomicAdd(&c.cnt[g * kMaxBins + b], 1u);
        if (SWEEP == 2 && pos >= c.end[g * kMaxBins + b]) return;
        // base_g counts blocks of four slots (the unit of the list offsets)
        const size_t at = 4 * (size_t)base_g + pos;
        if constexpr (REC == 2) {
            reinterpret_cast<float2*>(a.rec)[at] = oct_encode(dx, dy, dz);
        } else if constexpr (REC == 4) {
            a.rec[at] = make_float4(dx, dy, dz, w);
        } else {
            a.list[at] = entry;
        }
    }
}

// One sweep over the item's candidates. SWEEP 0 counts the hits of every
// (primary, bin); SWEEP 1 writes each hit at base[g] + (running offset of its
// bin), the offsets having been prepared in cnt; SWEEP 2 does the same inside
// the predicted regions (their ends in end), and drops (but still counts) the hits
// beyond a region's end. A hit is written as a list entry, or (REC 2 or 4) as
// the record that the FP32 harmonic pass streams.
//
// Each thread stages one slot of the next tile: its load is issued before the
// tests and its LDS write follows them, so the tile's loads are covered by
// the tests and the only wait of a tile is the one of that write (loads and
// stores complete in order, so it also drains the tile's hit stores).
//
// A pair inside the guard band of an edge is only marked during the tests
// (one bit per (tile slot, primary) of the lane) and binned exactly after
// them, outside the test loop.
template <int SWEEP, bool SINGLE, bool UNIFORM, int REC>
__device__ __forceinline__ void bin_sweep(const BinArgs& a, const ItemCtx& c, const float (&px)[kGM],
                                          const float (&py)[kGM], const float (&pz)[kGM],
                                          const uint32_t (&base)[kGM]) {
    const BinTables& T = *c.T;
    const float ne0 = -a.e0f * a.inv_dr;
    const float lo2 = T.e2f[0] - T.guard[0];
    const float hi2 = T.e2f[a.nb] + T.guard[a.nb];
    const unsigned nbu = (unsigned)a.nb;
    // thread x stages tile slots x + 64 kNW s (s < kStage); the staging
    // waves are uniform, so their branches are scalar
    const bool stager = kTile >= 64 * kNW || c.wave < kTile / 64;
    Staged st[kStage];
#pragma unroll
    for (int s = 0; s < kStage; ++s) st[s].r = 0;
    if (stager) {
#pragma unroll
        for (int s = 0; s < kStage; ++s)
            stage_load<SINGLE, REC>(st[s], *c.S, c.np, c.total, (int)threadIdx.x + 64 * kNW * s, a.pf, a.pw);
#pragma unroll
        for (int s = 0; s < kStage; ++s)
            stage_store<SINGLE, REC>(st[s], c.tiles + threadIdx.x + 64 * kNW * s, c.tent + threadIdx.x + 64 * kNW * s,
                                     c.cst, c.cshift, a.g.hf, a.pw != nullptr);
    }
    __syncthreads();
    int buf = 0;
    for (int t = 0; t < c.total; t += kTile) {
        const float4* cur = c.tiles + buf * kTile;
        const uint32_t* cure = c.tent + buf * kTile;
        const bool more = t + kTile < c.total;
        if (more && stager) {
#pragma unroll
            for (int s = 0; s < kStage; ++s)
                stage_load<SINGLE, REC>(st[s], *c.S, c.np, c.total, t + kTile + (int)threadIdx.x + 64 * kNW * s, a.pf,
                                        a.pw);
        }
        const int nt = min(kTile, c.total - t);
        NearMask nearbits = 0;
        // fully unrolled: every guard-band bit is a constant (66 VGPRs, seven
        // waves per SIMD, measured faster than the loop unrolled twice)
#pragma unroll
        for (int u = 0; u < kUT; ++u) {
            const int i = u * 64 + c.lane;
            const float4 q = cur[i];
            const bool valid = i < nt;
            const uint32_t entry = cure[i];
#pragma unroll
            for (int g = 0; g < kGM; ++g) {
                if (g >= c.ng) break;
                float dx, dy, dz;
                separation<SINGLE>(a, q, px[g], py[g], pz[g], dx, dy, dz);
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                int bb;
                bool near;
                if constexpr (UNIFORM) {
                    const float uu = fmaf(__builtin_amdgcn_sqrtf(r2), a.inv_dr, ne0);
                    const float fl = floorf(uu);
                    bb = (int)fl;
                    const float fr = uu - fl;
                    // guard bands of the edges e_0 .. e_nb: bb in [-1, nb]
                    near = (fr < a.delta || fr > 1.0f - a.delta) && (unsigned)(bb + 1) <= nbu + 1u;
                } else {
                    bb = -1;
                    near = false;
                    if (r2 >= lo2 && r2 < hi2) {
                        for (int e = 0; e <= a.nb; ++e) {
                            bb += r2 >= T.e2f[e];
                            near |= fabsf(r2 - T.e2f[e]) < T.guard[e];
                        }
                    }
                }
                const bool hit = valid && !near && (unsigned)bb < nbu;
                nearbits |= (valid && near) ? (NearMask)1 << (u * kGM + g) : (NearMask)0;
                put_hit<SWEEP, REC>(a, c, g, hit, bb, base[g], dx, dy, dz, q.w, entry);
            }
        }
        // the next tile's slot (written also after the last tile: the other
        // buffer is then unused)
        if (stager) {
#pragma unroll
            for (int s = 0; s < kStage; ++s)
                stage_store<SINGLE, REC>(st[s], c.tiles + (buf ^ 1) * kTile + threadIdx.x + 64 * kNW * s,
                                         c.tent + (buf ^ 1) * kTile + threadIdx.x + 64 * kNW * s, c.cst, c.cshift,
                                         a.g.hf, a.pw != nullptr);
        }
        // the marked near-edge pairs, binned exactly (rare)
        if (__ballot(nearbits != 0) != 0ull) {
#pragma unroll
            for (int g = 0; g < kGM; ++g) {
                // bits u kGM + g of this primary
                NearMask m = nearbits & (kNearPrimary << g);
                while (m != 0) {
                    const int bit = sizeof(NearMask) == 8 ? __builtin_ctzll(m) : __builtin_ctz((uint32_t)m);
                    m &= m - 1;
                    const int i = (bit / kGM) * 64 + c.lane;
                    const float4 q = cur[i];
                    const uint32_t entry = cure[i];
                    float dx, dy, dz;
                    separation<SINGLE>(a, q, px[g], py[g], pz[g], dx, dy, dz);
                    const int b = exact_pair<SINGLE>(a.pd, c.cs + c.wave + kNW * g, c.cstart, entry, c.mask,
                                                     c.cshift, c.cx, c.cy, c.cz, a.g.k, a.g.nc, a.g.box, a.nb, T.e2);
                    put_hit<SWEEP, REC>(a, c, g, b >= 0, b, base[g], dx, dy, dz, q.w, entry);
                }
            }
        }
        __syncthreads();
        buf ^= 1;
    }
}

// Exact layout: counts of sweep 0 -> one allocation per wavefront; cnt
// becomes the offset of each bin inside its primary's allocation, and
// (offset, count) of every (p, b) is published.
__device__ void exact_layout(const BinArgs& a, ItemCtx& c, uint32_t (&base)[kGM]) {
    const int lane = c.lane;
    // each bin's room is its count rounded up to a multiple of four: list
    // offsets are published in units of four slots
    uint32_t tot[kGM], cl[kGM], ex[kGM];
    uint32_t sum = 0;
#pragma unroll
    for (int g = 0; g < kGM; ++g) {
        tot[g] = cl[g] = ex[g] = 0;
        if (g >= c.ng) continue;
        const int cn = lane < a.nb ? (int)c.cnt[g * kMaxBins + lane] : 0;
        const int cv = (cn + 3) & ~3;
        int incl = cv;
        for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        tot[g] = (uint32_t)__shfl(incl, 63, 64);
        cl[g] = (uint32_t)cn;
        ex[g] = (uint32_t)(incl - cv);
        if (lane < a.nb) c.cnt[g * kMaxBins + lane] = ex[g];
        sum += tot[g];
    }
    if (c.ng == 0) return;
    const int slot = c.slot;
    // cursors, regions and the capacity count units of four slots
    const unsigned long long region = a.capacity / a.nslots;
    unsigned long long b0 = 0;
    if (lane == 0) b0 = atomicAdd(a.cursor + slot * 16, (unsigned long long)(sum / 4));
    b0 = __shfl(b0, 0, 64);
    const bool ok = b0 + sum / 4 <= region;
    if (!ok && lane == 0) atomicOr(a.overflow, 1);
    uint32_t run = (uint32_t)(b0 + (unsigned long long)slot * region);
#pragma unroll
    for (int g = 0; g < kGM; ++g) {
        if (g >= c.ng) continue;
        const int64_t pl = c.cs + c.wave + kNW * g - a.p_begin;
        if (lane < a.nb) {
            a.cnt[pl * a.nb + lane] = ok ? cl[g] : 0u;
            a.boff[pl * a.nb + lane] = ok ? run + ex[g] / 4 : 0u;
        }
        if (ok) base[g] = run;
        run += tot[g] / 4;
    }
}

// Binning of the pairs of a work item: up to kItemPrims primaries of one home
// cell (FIX = false), or one primary of the fix-up list (FIX = true).
// Candidates are staged in LDS once per tile for the whole workgroup, in the
// home cell's frame, and every wavefront tests them against its primaries
// (kGM at most), double-buffered so that the loads of the next tile overlap
// the tests.
//   FIX = false: one sweep. The primaries of an item share the stencil, whose
//     candidate count measures the local density; with the shell volumes it
//     predicts each bin's count, and a margin of 1.15x + 4 sigma + 8 gives its
//     region in the primary's allocation. Every hit is written in place; a
//     primary with more hits in some bin than its region holds is appended to
//     the fix-up list instead of being published.
//   FIX = true: two sweeps with exact counts (count, allocate, write).
// bin_item takes the primaries first .. last - 1 of home cell gc; every
// thread of the workgroup calls it with the same item.
template <bool SINGLE, bool UNIFORM, int REC, bool FIX>
__device__ __forceinline__ void bin_item(const BinArgs& a, ItemCtx& c, Pieces& S, BinTables& T, int gc,
                                         int64_t first, int64_t last, int slot) {
    c.slot = slot;
    c.cs = max(first, a.p_begin);
    const int64_t ce = min(last, a.p_end);
    if (c.cs >= ce) return;
    const int cat = gc / a.g.ncell;
    const int loc = gc - cat * a.g.ncell;
    c.cz = loc % a.g.nc;
    c.cy = (loc / a.g.nc) % a.g.nc;
    c.cx = loc / (a.g.nc * a.g.nc);
    c.cstart = a.pt_off[cat];
    c.cst = (uint32_t)c.cstart;
    c.cshift = 32 - a.g.code_bits;
    c.mask = a.g.idx_mask;
    if (c.wave == 0) {
        if constexpr (SINGLE) {
            build_pieces(S, a, cat, 0, 0, 0);
        } else {
            // The item's primaries bound the box the candidates are cut to:
            // all of them (at most kItemPrims), also where a chunk boundary
            // splits the item, so that the cut, and with it the tiles and the
            // order in which each list receives its hits, is the same in every
            // chunking and batch.
            const ItemBox box = item_box(a.pf, first, last, a.reach2);
            build_pieces<true>(S, a, cat, c.cx, c.cy, c.cz, box);
        }
    }
    __syncthreads();
    c.np = S.n[0];
    c.total = S.pref[c.np];
    c.total_full = S.n[1];
    const int lane = c.lane;

    // this wavefront's primaries: cs + wave + kNW g, g < ng
    const int rem = (int)(ce - c.cs);
    c.ng = rem > c.wave ? (rem - c.wave + kNW - 1) / kNW : 0;
    float px[kGM], py[kGM], pz[kGM];
    uint32_t base[kGM];
#pragma unroll
    for (int g = 0; g < kGM; ++g) {
        px[g] = py[g] = pz[g] = 0.f;
        base[g] = kNoBase;
        if (g < c.ng) {
            // uniform over the wavefront: scalar registers
            const float4 P = a.pf[c.cs + c.wave + kNW * g];
            px[g] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(P.x)));
            py[g] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(P.y)));
            pz[g] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(P.z)));
        }
    }

    if constexpr (FIX) {
        for (int i = lane; i < kGM * kMaxBins; i += 64) c.cnt[i] = 0u;
        wave_sync();
        bin_sweep<0, SINGLE, UNIFORM, REC>(a, c, px, py, pz, base);
        wave_sync();
        exact_layout(a, c, base);
        wave_sync();
        bin_sweep<1, SINGLE, UNIFORM, REC>(a, c, px, py, pz, base);
        return;
    } else {
        // Predicted regions, the same for every primary of the item, and one
        // allocation for the item's primaries of this chunk, laid out bin by
        // bin: bin b holds the lists of capacity cap_b of primaries 0 .. n-1
        // side by side. A harmonic wavefront reads one bin of consecutive
        // primaries, so its lists lie in a few items' blocks rather than in
        // as many places as it has lanes (the FP64 pass, whose gathers wait
        // on the list entries, was measured 1.6 times faster with this layout).
        const int nitem = (int)(ce - c.cs);
        if (c.wave == 0) {
            int cap = 0;
            if (lane < a.nb) {
                const float pred = (float)c.total_full * (float)a.vol[lane] * a.inv_vst;
                // a multiple of four: the offsets count blocks of four slots
                cap = ((int)ceilf(1.15f * pred + 4.0f * sqrtf(pred) + 8.0f) + 3) & ~3;
            }
            int incl = cap;
            for (int o = 1; o < 64; o <<= 1) {
                const int v = __shfl_up(incl, o, 64);
                if (lane >= o) incl += v;
            }
            if (lane <= a.nb) T.capoff[lane] = (uint32_t)(incl - cap);
            const uint32_t captot = (uint32_t)__shfl(incl, 63, 64);
            if (lane == 0) {
                // in units of four slots (every capacity is a multiple of four)
                const unsigned long long sum = (unsigned long long)(captot / 4) * (unsigned)nitem;
                const unsigned long long region = a.capacity / a.nslots;
                const int slot = c.slot;
                const unsigned long long b0 = atomicAdd(a.cursor + slot * 16, sum);
                const bool fits = b0 + sum <= region;
                if (!fits) atomicOr(a.overflow, 1);
                T.ibase = fits ? (uint32_t)(b0 + (unsigned long long)slot * region) : kNoBase;
            }
        }
        __syncthreads();
        const uint32_t ibase = T.ibase;
        const bool ok = ibase != kNoBase;
        // write cursor and region end of (primary wave + kNW g, bin b): the
        // region [nitem capoff[b] + i cap_b, + cap_b) of the item's allocation
        for (int i = lane; i < kGM * kMaxBins; i += 64) {
            const int g = i / kMaxBins, b = i % kMaxBins;
            uint32_t st = 0, cb = 0;
            if (b < a.nb) {
                const uint32_t co = T.capoff[b];
                cb = T.capoff[b + 1] - co;
                st = (uint32_t)nitem * co + (uint32_t)(c.wave + kNW * g) * cb;
            }
            c.cnt[i] = st;
            c.end[i] = st + cb;
        }
#pragma unroll
        for (int g = 0; g < kGM; ++g)
            if (g < c.ng) base[g] = ibase;
        wave_sync();
        bin_sweep<2, SINGLE, UNIFORM, REC>(a, c, px, py, pz, base);
        wave_sync();
#pragma unroll
        for (int g = 0; g < kGM; ++g) {
            if (g >= c.ng) continue;
            const int64_t pl = c.cs + c.wave + kNW * g - a.p_begin;
            uint32_t cv = 0, cap = 0, st = 0;
            if (lane < a.nb) {
                cap = T.capoff[lane + 1] - T.capoff[lane];
                st = c.end[g * kMaxBins + lane] - cap;
                cv = c.cnt[g * kMaxBins + lane] - st;
            }
            const bool over = __ballot(lane < a.nb && cv > cap) != 0;
            if (over && ok && lane == 0) {
                const int k = atomicAdd(a.nfix, 1);
                a.fix[k] = make_int2(gc, (int)pl);
            }
            if (lane < a.nb) {
                const bool pub = ok && !over;
                a.cnt[pl * a.nb + lane] = pub ? cv : 0u;
                a.boff[pl * a.nb + lane] = pub ? ibase + st / 4 : 0u;
            }
        }
    }
}

// The binning launch: one workgroup per work item, or (FIX) a fixed grid
// whose workgroups take the fix-up list's primaries in turn.
template <bool SINGLE, bool UNIFORM, int REC, bool FIX>
__global__ void __launch_bounds__(64 * kNW) k_pair_bin(BinArgs a) {
    extern __shared__ unsigned char smem[];
    BinTables& T = *reinterpret_cast<BinTables*>(smem);
    for (int i = threadIdx.x; i <= a.nb; i += blockDim.x) {
        T.e2[i] = a.e2[i];
        T.e2f[i] = a.e2f[i];
        T.guard[i] = a.guard[i];
    }
    size_t off = (sizeof(BinTables) + 15) / 16 * 16;
    float4* tiles = reinterpret_cast<float4*>(smem + off);
    off += sizeof(float4) * 2 * kTile;
    uint32_t* tent = reinterpret_cast<uint32_t*>(smem + off);
    off += sizeof(uint32_t) * 2 * kTile;
    Pieces S = pieces_view(smem + off, a.npmax);
    off += pieces_lds_bytes(a.npmax);
    ItemCtx c;
    c.wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    c.lane = lane_id();
    c.cnt = reinterpret_cast<uint32_t*>(smem + off) + c.wave * (kGM * kMaxBins);
    c.end = reinterpret_cast<uint32_t*>(smem + off) + (kNW + c.wave) * (kGM * kMaxBins);
    c.T = &T;
    c.S = &S;
    c.tiles = tiles;
    c.tent = tent;

    if constexpr (FIX) {
        // the fix-up list the binning launch left on the device, walked by a
        // fixed grid (no host round trip between the two launches)
        const int nfix = *a.nfix;
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(a.nfix_total, nfix);
        for (int64_t item = blockIdx.x; item < nfix; item += gridDim.x) {
            const int2 f = a.fix[item];
            __syncthreads();  // the previous item's pieces and tiles are no longer read
            // a fix-up item (one primary) allocates from the region of its primary
            bin_item<SINGLE, UNIFORM, REC, true>(a, c, S, T, f.x, a.p_begin + f.y, a.p_begin + f.y + 1,
                                                 f.y % a.nslots);
        }
    } else {
        const int64_t item = a.item_lo + xcd_block(blockIdx.x, (int64_t)gridDim.x);
        if (item >= a.item_hi) return;
        const int gc = a.item_cell[item];
        const int64_t first = (int64_t)a.cell_start[gc] + (item - a.item_start[gc]) * kItemPrims;
        const int64_t last = min(first + kItemPrims, (int64_t)a.cell_start[gc + 1]);
        // consecutive items take the regions in turn: the items that hold
        // the chunk's primaries are consecutive, so every region gets the
        // same share of them (to within one)
        bin_item<SINGLE, UNIFORM, REC, false>(a, c, S, T, gc, first, last, (int)((item - a.item_lo) % a.nslots));
    }
}

// ---------------------------------------------------------------- harmonics

// Chebyshev coefficients of the z-polynomial parts of the harmonics. The
// value of order (l, m) carries the monic polynomial q_l^m(z) of degree l - m
// (q_m = 1, q_{m+1} = z, q_l = z q_{l-1} - beta(l, m) q_{l-2}, the three-term
// recurrence of the associated Legendre functions divided by their leading
// coefficient and by (1 - z^2)^(m/2)). Written in Chebyshev polynomials,
// q_l^m = sum_k d[m][l][k] T_k(z), the coefficients follow from the same
// recurrence with z T_0 = T_1 and z T_k = (T_{k+1} + T_{k-1}) / 2. They are
// all non-negative (q_l^m is a Gegenbauer polynomial of index m + 1/2 > 0),
// so they sum to q_l^m(1) = max |q_l^m| and the change of basis amplifies no
// rounding error. The m = 0 chain runs to degree 2 lmax (self moments).
__host__ __device__ constexpr double beta_d(int l, int m) {
    return (double)((l + m - 1) * (l - m - 1)) / (double)((2 * l - 1) * (2 * l - 3));
}

template <int LMAX>
struct ChebTable {
    static constexpr int N = 2 * LMAX + 1;
    double d[LMAX + 1][N][N];
    constexpr ChebTable() : d{} {
        for (int m = 0; m <= LMAX; ++m) {
            const int ltop = m == 0 ? 2 * LMAX : LMAX;
            d[m][m][0] = 1.0;
            if (m + 1 <= ltop) d[m][m + 1][1] = 1.0;
            for (int l = m + 2; l <= ltop; ++l) {
                const double b = beta_d(l, m);
                for (int k = 0; k < N; ++k) {
                    double zk = 0.5 * (k + 1 < N ? d[m][l - 1][k + 1] : 0.0);
                    if (k == 1) zk += d[m][l - 1][0];
                    if (k >= 2) zk += 0.5 * d[m][l - 1][k - 1];
                    d[m][l][k] = zk - b * d[m][l - 2][k];
                }
            }
        }
    }
};

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

// Finer splits above lmax 12: the m range in np parts (3 or 4), the self
// moments with part 0, chosen to minimise the largest part's values. Returns
// the first m of part p (p = np gives lmax + 1).
__host__ __device__ constexpr int values_of_m(int lmax, int m) { return m == 0 ? lmax + 1 : 2 * (lmax - m + 1); }
__host__ __device__ constexpr int part_first_m(int lmax, int np, int p) {
    if (p <= 0) return 0;
    if (p >= np) return lmax + 1;
    // cumulative values before m = M (the self moments count with m = 0)
    int cum[64] = {};
    cum[0] = 2 * lmax + 1;
    for (int m = 0; m <= lmax; ++m) cum[m + 1] = cum[m] + values_of_m(lmax, m);
    int best = 1 << 30, b1 = 1, b2 = 2, b3 = 3;
    for (int x1 = 1; x1 <= lmax; ++x1)
        for (int x2 = x1 + 1; x2 <= (np >= 3 ? lmax : x1 + 1); ++x2)
            for (int x3 = x2 + 1; x3 <= (np >= 4 ? lmax : x2 + 1); ++x3) {
                const int e2 = np >= 3 ? x2 : lmax + 1, e3 = np >= 4 ? x3 : lmax + 1;
                int worst = cum[x1];
                if (np >= 3 && cum[e2] - cum[x1] > worst) worst = cum[e2] - cum[x1];
                if (np >= 4 && cum[e3] - cum[e2] > worst) worst = cum[e3] - cum[e2];
                const int last = np >= 4 ? e3 : (np >= 3 ? e2 : x1);
                if (cum[lmax + 1] - cum[last] > worst) worst = cum[lmax + 1] - cum[last];
                if (worst < best) {
                    best = worst;
                    b1 = x1;
                    b2 = x2;
                    b3 = x3;
                }
            }
    return p == 1 ? b1 : (p == 2 ? b2 : b3);
}

// Part G of the m range: G = 0 the whole range; G = 1, 2 the two halves of
// m_split; G = 3 .. 5 three parts; G = 6 .. 9 four parts.
__host__ __device__ constexpr int part_np(int G) { return G == 0 ? 1 : (G <= 2 ? 2 : (G <= 5 ? 3 : 4)); }
__host__ __device__ constexpr int part_ix(int G) { return G == 0 ? 0 : (G <= 2 ? G - 1 : (G <= 5 ? G - 3 : G - 6)); }
__host__ __device__ constexpr int part_mlo(int lmax, int G) {
    return G <= 2 ? (G == 2 ? m_split(lmax) + 1 : 0) : part_first_m(lmax, part_np(G), part_ix(G));
}
__host__ __device__ constexpr int part_mhi(int lmax, int G) {
    return G <= 2 ? (G == 1 ? m_split(lmax) : lmax) : part_first_m(lmax, part_np(G), part_ix(G) + 1) - 1;
}

template <typename T, int LMAX, int G>
struct Acc {
    static constexpr int MLO = part_mlo(LMAX, G);
    static constexpr int MHI = part_mhi(LMAX, G);
    static constexpr bool SELF = MLO == 0;
    static constexpr int V0 = value_offset(LMAX, MLO);
    static constexpr int V1 = value_offset(LMAX, MHI + 1);
    static constexpr int NA = V1 - V0;            // a_lm values held
    static constexpr int NS = SELF ? 2 * LMAX + 1 : 0;
    T a[NA > 0 ? NA : 1];
    T s[NS > 0 ? NS : 1];
};

// Highest order of the self moments a lane accumulates: 2 lmax, or lmax with
// SLO. The self moments enter the multipoles only through the removal of the
// degenerate triangles, and there the coefficient of the order-L' moment,
// summed over m, vanishes for every L' other than the multipole's own L (the
// orthogonality of the 3j symbols (l1 l2 L; m -m 0) over m). A run whose
// multipoles all have L <= lmax, and that exports no per-m sums, needs none
// of the orders above lmax.
__host__ __device__ constexpr int self_top(int lmax, bool slo) { return slo ? lmax : 2 * lmax; }

// Accumulates one neighbour (unit vector x,y,z; weight w) in the Chebyshev
// basis: the slot of order (l, m) sums c_m T_{l-m}(z) with c_m = w (x - i y)^m
// (and the self moments w^2 T_L(z)); cheb_to_monic turns the sums into the
// monic polynomial basis once the list is done. The Chebyshev values are
// shared by every m and cost one fused multiply-add per degree, where the
// monic recurrence runs once per m. With UNIT all weights are 1: the self
// moments of order L <= lmax then equal the m = 0 sums and are not
// accumulated twice (the caller copies them). With SLO the self moments stop
// at order lmax (those above are left 0; see self_top).
//
// Above lmax 12 the orders m >= 1 are accumulated in the monic basis itself,
// by the recurrence per pair (direct_m). The Chebyshev form bounds the error
// of a converted sum by q_l^m(1) times that of the Chebyshev sums, and for
// large m the Gegenbauer polynomial q_l^m peaks at z = +-1 far above its
// values elsewhere (by about 1800 at l = 16, m = 8), which at lmax 16 cost
// FP32 sums a few 1e-5 of the largest coefficient; the recurrence is stable.
__host__ __device__ constexpr bool direct_m(int lmax) { return lmax >= 13; }

template <typename T, int LMAX, int G, bool UNIT, bool SLO = false>
__device__ __forceinline__ void add_hit(Acc<T, LMAX, G>& A, T x, T y, T z, T w) {
    using AC = Acc<T, LMAX, G>;
    constexpr int MLO = AC::MLO, MHI = AC::MHI, V0 = AC::V0;
    constexpr bool SHARE = UNIT && MLO == 0 && AC::SELF;  // s[l] == a[l] for l <= lmax
    constexpr int STOP = self_top(LMAX, SLO);
    constexpr bool DIRECT = direct_m(LMAX);
    // highest Chebyshev degree used: the m = 0 sums, the self moments, and
    // the orders m >= MLO unless they are accumulated directly
    constexpr int KCH = DIRECT ? (MLO == 0 ? LMAX : 0) : LMAX - MLO;
    constexpr int KTOP = AC::SELF ? (STOP > KCH ? STOP : KCH) : KCH;
    T t[KTOP + 1];
    t[0] = (T)1;
    if constexpr (KTOP >= 1) t[1] = z;
    const T z2 = z + z;
#pragma unroll
    for (int k = 2; k <= KTOP; ++k) t[k] = fma(z2, t[k - 1], -t[k - 2]);
    if constexpr (MLO == 0) {
        // with UNIT the degree-0 sum is the number of neighbours, set by the caller
#pragma unroll
        for (int k = UNIT ? 1 : 0; k <= LMAX; ++k) A.a[k - V0] = UNIT ? A.a[k - V0] + t[k] : fma(w, t[k], A.a[k - V0]);
    }
    if constexpr (AC::SELF) {
        const T w2 = UNIT ? (T)1 : w * w;
#pragma unroll
        for (int k = 0; k <= STOP; ++k)
            if (!(SHARE && k <= LMAX)) A.s[k] = UNIT ? A.s[k] + t[k] : fma(w2, t[k], A.s[k]);
    }
    if constexpr (MHI >= 1) {
        // c_m = w (x - i y)^m
        T cr = UNIT ? x : w * x, ci = UNIT ? -y : -(w * y);
#pragma unroll
        for (int m = 1; m <= MHI; ++m) {
            if (m > 1) {
                const T u = fma(cr, x, ci * y);
                ci = fma(ci, x, -(cr * y));
                cr = u;
            }
            if (m >= MLO) {
                const int vo = value_offset(LMAX, m) - V0;
                const int nl = LMAX - m + 1;
                if constexpr (DIRECT) {
                    // q_m = 1, q_{m+1} = z, q_l = z q_{l-1} - beta(l, m) q_{l-2}
                    T q0 = (T)1, q1 = z;
                    A.a[vo] += cr;
                    A.a[vo + nl] += ci;
#pragma unroll
                    for (int k = 1; k < nl; ++k) {
                        if (k >= 2) {
                            const T q2 = fma(z, q1, -(T)beta_d(m + k, m) * q0);
                            q0 = q1;
                            q1 = q2;
                        }
                        A.a[vo + k] = fma(q1, cr, A.a[vo + k]);
                        A.a[vo + nl + k] = fma(q1, ci, A.a[vo + nl + k]);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < nl; ++k) {
                        A.a[vo + k] = fma(t[k], cr, A.a[vo + k]);
                        A.a[vo + nl + k] = fma(t[k], ci, A.a[vo + nl + k]);
                    }
                }
            }
        }
    }
}

// In-place change of basis of n consecutive sums of one m from Chebyshev
// T_0 .. T_{n-1} to q_m^m .. q_{m+n-1}^m: top down, so that every sum still
// read holds its Chebyshev value (q_{m+j} uses T_j, T_{j-2}, ...).
template <typename T, int LMAX>
__device__ __forceinline__ void cheb_run_to_monic(const ChebTable<LMAX>& D, T* v, int m, int n) {
#pragma unroll
    for (int j = n - 1; j >= 1; --j) {
        T s = (T)0;
#pragma unroll
        for (int k = j; k >= 0; k -= 2) s = fma((T)D.d[m][m + j][k], v[k], s);
        v[j] = s;
    }
}

template <typename T, int LMAX, int G, bool SLO = false>
__device__ __forceinline__ void cheb_to_monic(Acc<T, LMAX, G>& A) {
    using AC = Acc<T, LMAX, G>;
    constexpr ChebTable<LMAX> D{};
    // with direct_m only the m = 0 sums and the self moments are Chebyshev sums
    constexpr int MTOP = direct_m(LMAX) ? 0 : AC::MHI;
#pragma unroll
    for (int m = AC::MLO; m <= MTOP; ++m) {
        const int vo = value_offset(LMAX, m) - AC::V0;
        const int nl = LMAX - m + 1;
        cheb_run_to_monic<T, LMAX>(D, A.a + vo, m, nl);
        if (m >= 1) cheb_run_to_monic<T, LMAX>(D, A.a + vo + nl, m, nl);
    }
    if constexpr (AC::SELF) cheb_run_to_monic<T, LMAX>(D, A.s, 0, self_top(LMAX, SLO) + 1);
}

template <typename T, int LMAX, int G, bool UNIT, bool SLO>
__global__ void __launch_bounds__(64) k_pair_alm(AlmArgs a) {
    using AC = Acc<T, LMAX, G>;
    constexpr int NV = n_values(LMAX);
    // One wavefront per workgroup: 64 consecutive primaries of one bin. The
    // wavefronts of a block of 256 primaries are consecutive, bin by bin.
    const int lane = lane_id();
    const int64_t nprim = a.p_end - a.p_begin;
    const int64_t nwaves = ((nprim + 255) / 256) * a.nb * 4;
    const int64_t wv = xcd_block(blockIdx.x, (int64_t)gridDim.x);
    if (wv >= nwaves) return;
    const int64_t blk = wv / (4 * a.nb);
    const int rem = (int)(wv - blk * 4 * a.nb);
    const int b = rem >> 2;
    const int64_t pl = blk * 256 + (rem & 3) * 64 + lane;
    const int64_t p = a.p_begin + pl;
    const bool active = pl < nprim;

    AC acc;
#pragma unroll
    for (int i = 0; i < (AC::NA > 0 ? AC::NA : 1); ++i) acc.a[i] = (T)0;
#pragma unroll
    for (int i = 0; i < (AC::NS > 0 ? AC::NS : 1); ++i) acc.s[i] = (T)0;

    uint32_t n = 0, off = 0;
    if (active) {
        n = a.cnt[pl * a.nb + b];
        off = a.boff[pl * a.nb + b];
    }
    if constexpr (sizeof(T) == 4) {
        // FP32: the binning pass wrote each hit as (dx, dy, dz, w_j), or
        // with unit weights as the octahedral code of its direction. Two
        // sets of K records per lane in ping-pong: each half of an iteration
        // first refills the other set with the next K records, then
        // accumulates its own set, loaded one half earlier. The loads are
        // unconditional (at a clamped index past the end of the list), so the
        // loads in flight are the same on every path: the wait before a set
        // is used covers exactly that set, loaded a whole half (K hits of
        // arithmetic) before. (Conditional loads, or rotating registers,
        // would make every hit wait for the newest load.) Four records per
        // set, eight where the sums alone take more than 128 registers: such
        // a lane runs at two waves per SIMD, and a set of eight 16-byte
        // records is a whole 128-byte line of its list (with four, the two
        // halves of a line are fetched a set apart, and were measured slower
        // even at three waves). With 8-byte codes, sets of sixteen (whole
        // lines again) were measured slower than sets of eight.
        constexpr int K = AC::NA + AC::NS > 128 ? 8 : 4;
        // an empty list reads the first record of the buffer (not accumulated)
        const size_t roff = n > 0 ? 4 * (size_t)off : 0;  // offsets count blocks of four records
        const uint32_t last = n > 0 ? n - 1 : 0;
        // with UNIT the records are the 8-byte direction codes (p, q)
        const float4* rec = a.rec + roff;
        const float2* rec2 = reinterpret_cast<const float2*>(a.rec) + roff;
        using RecT = std::conditional_t<UNIT, float2, float4>;
        auto load_rec = [&](uint32_t i) -> RecT {
            if constexpr (UNIT) {
                return rec2[i];
            } else {
                return rec[i];
            }
        };
        RecT qa[K], qb[K];
#pragma unroll
        for (int i = 0; i < K; ++i) qa[i] = load_rec(min((uint32_t)i, last));
        auto hit = [&](const RecT q) {
            if constexpr (UNIT) {
                const float3 d = oct_decode(q.x, q.y);
                const float inv = __builtin_amdgcn_rsqf(d.x * d.x + d.y * d.y + d.z * d.z);
                add_hit<T, LMAX, G, UNIT, SLO>(acc, d.x * inv, d.y * inv, d.z * inv, 1.f);
            } else {
                const float d2 = q.x * q.x + q.y * q.y + q.z * q.z;
                const float inv = __builtin_amdgcn_rsqf(d2);
                add_hit<T, LMAX, G, UNIT, SLO>(acc, q.x * inv, q.y * inv, q.z * inv, q.w);
            }
        };
        for (uint32_t t = 0; t < n; t += 2 * K) {
#pragma unroll
            for (int i = 0; i < K; ++i) qb[i] = load_rec(min(t + K + i, last));
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (t + i < n) hit(qa[i]);
#pragma unroll
            for (int i = 0; i < K; ++i) qa[i] = load_rec(min(t + 2 * K + i, last));
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (t + K + i < n) hit(qb[i]);
        }
    } else {
        // FP64: the lane gathers its neighbours through the list entries,
        // with the same ping-pong of unconditional loads as the FP32 path in
        // two stages: a set's entries are loaded one half before its points
        // are gathered, and the points one half before they are accumulated.
        // A slot past the end of the list gathers the primary itself (not
        // accumulated), so every address is valid. The gathers are
        // latency-bound: the kernels that split the m range (lmax >= 7, two
        // waves per SIMD or one) keep six entries and points per set in
        // flight (lmax 10: 360 ms per step with two, 320 with three, 287 with
        // four, 274 with six or eight).
        constexpr int K = G == 0 ? 2 : 6;
        const int64_t pself = active ? p : a.p_begin;
        const int64_t cstart = a.pt_off[a.catid[pself]];
        const double4 P64 = a.pd[pself];
        const uint32_t mask = a.g.idx_mask;
        const uint32_t* lst = n > 0 ? a.list + 4 * (size_t)off : a.list;  // offsets count blocks of four entries
        const uint32_t last = n > 0 ? n - 1 : 0;
        auto entry = [&](uint32_t r) { return lst[min(r, last)]; };
        auto gather = [&](uint32_t r, uint32_t e) { return a.pd[r < n ? cstart + (int64_t)(e & mask) : pself]; };
        auto hit = [&](const double4 d) {
            double dx = d.x - P64.x, dy = d.y - P64.y, dz = d.z - P64.z;
            const double L = a.g.box, hL = 0.5 * a.g.box;
            dx = dx > hL ? dx - L : (dx < -hL ? dx + L : dx);
            dy = dy > hL ? dy - L : (dy < -hL ? dy + L : dy);
            dz = dz > hL ? dz - L : (dz < -hL ? dz + L : dz);
            const double r2 = dx * dx + dy * dy + dz * dz;
            double inv = __builtin_amdgcn_rsq(r2);
            inv = inv * fma(-0.5 * r2 * inv, inv, 1.5);
            inv = inv * fma(-0.5 * r2 * inv, inv, 1.5);
            add_hit<T, LMAX, G, UNIT, SLO>(acc, (T)(dx * inv), (T)(dy * inv), (T)(dz * inv), (T)d.w);
        };
        uint32_t ea[K], eb[K];
        double4 da[K], db[K];
#pragma unroll
        for (int i = 0; i < K; ++i) ea[i] = entry((uint32_t)i);
#pragma unroll
        for (int i = 0; i < K; ++i) da[i] = gather((uint32_t)i, ea[i]);
#pragma unroll
        for (int i = 0; i < K; ++i) eb[i] = entry((uint32_t)(K + i));
        for (uint32_t t = 0; t < n; t += 2 * K) {
#pragma unroll
            for (int i = 0; i < K; ++i) db[i] = gather(t + K + i, eb[i]);
#pragma unroll
            for (int i = 0; i < K; ++i) ea[i] = entry(t + 2 * K + i);
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (t + i < n) hit(da[i]);
#pragma unroll
            for (int i = 0; i < K; ++i) da[i] = gather(t + 2 * K + i, ea[i]);
#pragma unroll
            for (int i = 0; i < K; ++i) eb[i] = entry(t + 3 * K + i);
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (t + K + i < n) hit(db[i]);
        }
    }
    if (!active) return;
    // the degree-0 sum is the list length: exact below 2^24 hits in FP32, and
    // above that rounded to FP32 like any FP32 sum (lists hold at most 2^27)
    if constexpr (UNIT && AC::MLO == 0) acc.a[0 - AC::V0] = (T)n;
    if constexpr (UNIT && AC::MLO == 0 && AC::SELF) {
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) acc.s[l] = acc.a[l - AC::V0];
    }
    cheb_to_monic<T, LMAX, G, SLO>(acc);
    T* A = reinterpret_cast<T*>(a.A);
    const int64_t ld = a.ldA;
#pragma unroll
    for (int i = 0; i < AC::NA; ++i) A[((int64_t)b * NV + AC::V0 + i) * ld + pl] = acc.a[i];
    if constexpr (AC::SELF) {
        // with SLO the orders above lmax are zero and not stored (the
        // self-moment sums of such a run do not read them)
#pragma unroll
        for (int i = 0; i <= self_top(LMAX, SLO); ++i)
            A[((int64_t)b * NV + n_alm_values(LMAX) + i) * ld + pl] = acc.s[i];
    }
}

// Long lists (thousands of neighbours per (p, b), for example with many
// randoms): one wavefront per list, its 64 lanes taking consecutive records
// (each load is one contiguous 1 KiB block), every lane accumulating its own
// partial sums, which a butterfly of lane exchanges adds in a fixed order at
// the end. A lane per list would touch 64 cache lines per load there and
// thrash L1. FP32 and lmax <= 6 (higher orders have the arithmetic to hide
// the lane-per-list loads, and their partial sums would cost occupancy).
constexpr int kWaveListWaves = 4;

template <int LMAX, bool UNIT, bool SLO>
__global__ void __launch_bounds__(64 * kWaveListWaves) k_pair_alm_wave(AlmArgs a) {
    using AC = Acc<float, LMAX, 0>;
    constexpr int NV = n_values(LMAX);
    const int lane = lane_id();
    const int64_t nprim = a.p_end - a.p_begin;
    const int64_t wv = xcd_block(blockIdx.x, (int64_t)gridDim.x) * kWaveListWaves + (threadIdx.x >> 6);
    if (wv >= nprim * a.nb) return;
    const int64_t pl = wv / a.nb;
    const int b = (int)(wv - pl * a.nb);
    AC acc;
#pragma unroll
    for (int i = 0; i < AC::NA; ++i) acc.a[i] = 0.f;
#pragma unroll
    for (int i = 0; i < AC::NS; ++i) acc.s[i] = 0.f;
    const uint32_t n = a.cnt[pl * a.nb + b];
    // the same ping-pong of unconditional loads as the lane-per-list kernel,
    // over blocks of 64 consecutive records (n is uniform over the wavefront)
    constexpr int K = 2;
    const size_t roff = n > 0 ? 4 * (size_t)a.boff[pl * a.nb + b] : 0;  // offsets count blocks of four records
    const uint32_t last = n > 0 ? n - 1 : 0;
    // with UNIT the records are the 8-byte direction codes (p, q)
    const float4* rec = a.rec + roff;
    const float2* rec2 = reinterpret_cast<const float2*>(a.rec) + roff;
    using RecT = std::conditional_t<UNIT, float2, float4>;
    auto load_rec = [&](uint32_t i) -> RecT {
        if constexpr (UNIT) {
            return rec2[i];
        } else {
            return rec[i];
        }
    };
    RecT qa[K], qb[K];
#pragma unroll
    for (int i = 0; i < K; ++i) qa[i] = load_rec(min((uint32_t)(64 * i + lane), last));
    auto hit = [&](const RecT q) {
        if constexpr (UNIT) {
            const float3 d = oct_decode(q.x, q.y);
            const float inv = __builtin_amdgcn_rsqf(d.x * d.x + d.y * d.y + d.z * d.z);
            add_hit<float, LMAX, 0, UNIT, SLO>(acc, d.x * inv, d.y * inv, d.z * inv, 1.f);
        } else {
            const float d2 = q.x * q.x + q.y * q.y + q.z * q.z;
            const float inv = __builtin_amdgcn_rsqf(d2);
            add_hit<float, LMAX, 0, UNIT, SLO>(acc, q.x * inv, q.y * inv, q.z * inv, q.w);
        }
    };
    for (uint32_t t0 = 0; t0 < n; t0 += 128 * K) {
#pragma unroll
        for (int i = 0; i < K; ++i) qb[i] = load_rec(min(t0 + 64 * (K + i) + lane, last));
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (t0 + 64 * i + lane < n) hit(qa[i]);
#pragma unroll
        for (int i = 0; i < K; ++i) qa[i] = load_rec(min(t0 + 64 * (2 * K + i) + lane, last));
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (t0 + 64 * (K + i) + lane < n) hit(qb[i]);
    }
    // every lane ends with the total of every value
#pragma unroll
    for (int i = 0; i < AC::NA; ++i)
        for (int o = 32; o > 0; o >>= 1) acc.a[i] += __shfl_xor(acc.a[i], o, 64);
    if constexpr (UNIT) acc.a[0] = (float)n;  // the degree-0 sum: the list length
    if constexpr (UNIT) {
#pragma unroll
        for (int l = 0; l <= LMAX; ++l) acc.s[l] = acc.a[l];
#pragma unroll
        for (int i = LMAX + 1; i <= self_top(LMAX, SLO); ++i)
            for (int o = 32; o > 0; o >>= 1) acc.s[i] += __shfl_xor(acc.s[i], o, 64);
    } else {
#pragma unroll
        for (int i = 0; i <= self_top(LMAX, SLO); ++i)
            for (int o = 32; o > 0; o >>= 1) acc.s[i] += __shfl_xor(acc.s[i], o, 64);
    }
    cheb_to_monic<float, LMAX, 0, SLO>(acc);
    // lane i writes value i
    float* A = reinterpret_cast<float*>(a.A);
    const int64_t ld = a.ldA;
#pragma unroll
    for (int i = 0; i < AC::NA; ++i)
        if (lane == i % 64) A[((int64_t)b * NV + i) * ld + pl] = acc.a[i];
#pragma unroll
    for (int i = 0; i < AC::NS; ++i)
        if (lane == (AC::NA + i) % 64) A[((int64_t)b * NV + n_alm_values(LMAX) + i) * ld + pl] = acc.s[i];
}

template <typename T, int LMAX, int G>
hipError_t launch_alm_one(const AlmArgs& a, hipStream_t s) {
    const int64_t nprim = a.p_end - a.p_begin;
    if constexpr (sizeof(T) == 4 && G == 0 && LMAX <= 6) {
        if (a.wave_per_list) {
            const int64_t nw = (nprim * a.nb + kWaveListWaves - 1) / kWaveListWaves;
            const int64_t nwg = (nw + 7) / 8 * 8;
            const dim3 grid((unsigned)nwg), block(64 * kWaveListWaves);
            if (a.unit_w) {
                if (a.self_lo) hipLaunchKernelGGL((k_pair_alm_wave<LMAX, true, true>), grid, block, 0, s, a);
                else hipLaunchKernelGGL((k_pair_alm_wave<LMAX, true, false>), grid, block, 0, s, a);
            } else {
                if (a.self_lo) hipLaunchKernelGGL((k_pair_alm_wave<LMAX, false, true>), grid, block, 0, s, a);
                else hipLaunchKernelGGL((k_pair_alm_wave<LMAX, false, false>), grid, block, 0, s, a);
            }
            return hipGetLastError();
        }
    }
    const int64_t nwaves = ((nprim + 255) / 256) * a.nb * 4;
    const int64_t nwg = (nwaves + 7) / 8 * 8;
    const dim3 grid((unsigned)nwg), block(64);
    if constexpr (sizeof(T) == 4 && G == 0) {
        // unit weights: the FP32 single-launch kernel shares the m = 0 sums;
        // self_lo: the self moments stop at order lmax
        if (a.unit_w) {
            if (a.self_lo) hipLaunchKernelGGL((k_pair_alm<T, LMAX, G, true, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_pair_alm<T, LMAX, G, true, false>), grid, block, 0, s, a);
        } else {
            if (a.self_lo) hipLaunchKernelGGL((k_pair_alm<T, LMAX, G, false, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_pair_alm<T, LMAX, G, false, false>), grid, block, 0, s, a);
        }
    } else {
        hipLaunchKernelGGL((k_pair_alm<T, LMAX, G, false, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

// FP32 keeps every value of a bin in one lane up to lmax 10, and splits the
// m range over two launches at lmax 11 and 12 and three from 13; FP64 splits
// it over two launches from lmax 7 and four from 13 (register budget). Every
// launch rereads the lists.
template <typename T, int LMAX, int G0, int NP>
hipError_t launch_alm_parts(const AlmArgs& a, hipStream_t s) {
    hipError_t e = launch_alm_one<T, LMAX, G0>(a, s);
    if constexpr (NP > 1) {
        if (e != hipSuccess) return e;
        return launch_alm_parts<T, LMAX, G0 + 1, NP - 1>(a, s);
    }
    return e;
}

template <int LMAX>
hipError_t launch_alm_lmax(const AlmArgs& a, int fp64, hipStream_t s) {
    if (!fp64) {
        if constexpr (LMAX <= 10) return launch_alm_one<float, LMAX, 0>(a, s);
        else if constexpr (LMAX <= 12) return launch_alm_parts<float, LMAX, 1, 2>(a, s);
        else return launch_alm_parts<float, LMAX, 3, 3>(a, s);
    } else {
        if constexpr (LMAX <= 6) return launch_alm_one<double, LMAX, 0>(a, s);
        else if constexpr (LMAX <= 12) return launch_alm_parts<double, LMAX, 1, 2>(a, s);
        else return launch_alm_parts<double, LMAX, 6, 4>(a, s);
    }
}

}  // namespace

template <bool SINGLE, bool UNIFORM, int REC, bool FIX>
hipError_t launch_bin_variant(const BinArgs& a, hipStream_t s, int64_t nblk, size_t lds) {
    const hipError_t e = allow_full_lds((const void*)k_pair_bin<SINGLE, UNIFORM, REC, FIX>);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_pair_bin<SINGLE, UNIFORM, REC, FIX>), dim3((unsigned)nblk), dim3(64 * kNW), lds, s, a);
    return hipGetLastError();
}

template <int REC, bool FIX>
hipError_t launch_bin_rec(const BinArgs& a, hipStream_t s, int64_t nblk, size_t lds) {
    if (a.g.single) {
        return a.uniform ? launch_bin_variant<true, true, REC, FIX>(a, s, nblk, lds)
                         : launch_bin_variant<true, false, REC, FIX>(a, s, nblk, lds);
    }
    return a.uniform ? launch_bin_variant<false, true, REC, FIX>(a, s, nblk, lds)
                     : launch_bin_variant<false, false, REC, FIX>(a, s, nblk, lds);
}

hipError_t launch_pair_bin(const BinArgs& a, hipStream_t s) {
    const int64_t nitems = a.item_hi - a.item_lo;
    if (a.p_end <= a.p_begin || nitems <= 0) return hipSuccess;
    // a multiple of 8 blocks, so that the XCD remap is a permutation
    const int64_t nblk = (nitems + 7) / 8 * 8;
    const size_t lds = pair_bin_lds_bytes(a.npmax);
    if (!a.rec) return launch_bin_rec<0, false>(a, s, nblk, lds);
    return a.rec_oct ? launch_bin_rec<2, false>(a, s, nblk, lds) : launch_bin_rec<4, false>(a, s, nblk, lds);
}

hipError_t launch_pair_fix(const BinArgs& a, hipStream_t s) {
    if (a.p_end <= a.p_begin) return hipSuccess;
    // the list's length is read on the device: a fixed grid of 8 workgroups per CU
    const int64_t nblk = kFixGrid;
    const size_t lds = pair_bin_lds_bytes(a.npmax);
    if (!a.rec) return launch_bin_rec<0, true>(a, s, nblk, lds);
    return a.rec_oct ? launch_bin_rec<2, true>(a, s, nblk, lds) : launch_bin_rec<4, true>(a, s, nblk, lds);
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
        case 13: return launch_alm_lmax<13>(a, fp64, s);
        case 14: return launch_alm_lmax<14>(a, fp64, s);
        case 15: return launch_alm_lmax<15>(a, fp64, s);
        case 16: return launch_alm_lmax<16>(a, fp64, s);
        default: return hipErrorInvalidValue;
    }
}

size_t pair_bin_lds_bytes(int npmax) {
    return (sizeof(BinTables) + 15) / 16 * 16 + (sizeof(float4) + sizeof(uint32_t)) * 2 * kTile +
           pieces_lds_bytes(npmax) +
           sizeof(uint32_t) * 2 * kNW * kGM * kMaxBins;
}

}  // namespace tpcf
