// Device helpers of the cell-list pair kernels (the 3PCF binning pass and
// the 2PCF pair counts): wavefront utilities, the XCD-aware block map, and the
// flattening of a home cell's stencil into one candidate range.
// Internal to libtpcf; included by HIP sources only.
#pragma once
#include "tpcf_internal.h"

namespace tpcf {

namespace {

__device__ inline int lane_id() { return threadIdx.x & 63; }

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// XCD-aware block remap: the hardware hands consecutive workgroups to the 8
// XCDs in turn; this gives every XCD a contiguous range of logical blocks so
// that neighbouring primaries share that XCD's L2. The map is a permutation
// of [0, nblocks) when nblocks is a multiple of 8; launches round up to that.
__device__ inline int64_t xcd_block(int64_t bid, int64_t nblocks) {
    int64_t per = (nblocks + 7) / 8;
    return (bid % 8) * per + bid / 8;
}

// Bin tables shared by the workgroup.
struct BinTables {
    double e2[kMaxBins + 1];
    float e2f[kMaxBins + 1];
    float guard[kMaxBins + 1];
    uint32_t capoff[kMaxBins + 1];  // predicted regions of a primary: bin b has capoff[b+1] - capoff[b] slots
    uint32_t ibase;                 // the work item's list allocation (entry pairs), or kNoBase
};

// Candidate table of a home cell in LDS. Pieces are runs of consecutive cells
// of the cell's stencil, flattened into one candidate range [0, pref[n]).
//   rec[r]  = (j offset = start - pref, sx, sy, zo): candidate g of piece r is
//             point g + off, shifted into the home cell's frame by
//             (sx, sy, (izf + zo) h), izf = the candidate's cell z index;
//   code[r] = ((ox+k)(2k+1) + (oy+k))(2k+1) + k | wrap << 16, wrap = the
//             periodic shift signs (+1) of x, y, z in 2-bit fields.
struct Pieces {
    float4* rec;
    int* pref;
    int* code;
    int* n;
};

__host__ __device__ inline size_t pieces_lds_bytes(int npmax) {
    size_t b = sizeof(float4) * (size_t)npmax + sizeof(int) * (size_t)(2 * npmax + 1) + sizeof(int) * 4;
    return (b + 15) / 16 * 16;
}

__device__ inline Pieces pieces_view(unsigned char* base, int npmax) {
    Pieces w;
    w.rec = reinterpret_cast<float4*>(base);
    w.pref = reinterpret_cast<int*>(w.rec + npmax);
    w.code = w.pref + npmax + 1;
    w.n = w.code + npmax;
    return w;
}

__device__ inline double wrap_shift(int bits, int axis, double L) {
    return (double)(((bits >> (2 * axis)) & 3) - 1) * L;
}

// Bounding box of a work item's primaries in the home cell's frame, and the
// squared reach beyond which no candidate can pair with any of them.
struct ItemBox {
    float xlo, xhi, ylo, yhi, zlo, zhi;
    float r2;
};

// Box of the primaries [first, last) (at most 64 points of one cell, in the
// sorted order) in the home cell's frame, formed by one wavefront.
__device__ inline ItemBox item_box(const float4* pf, int64_t first, int64_t last, float r2) {
    const int lane = lane_id();
    const bool in = lane < last - first;
    const float4 P = pf[in ? first + lane : first];
    ItemBox b{P.x, P.x, P.y, P.y, P.z, P.z, r2};
    for (int o = 32; o > 0; o >>= 1) {
        b.xlo = fminf(b.xlo, __shfl_xor(b.xlo, o, 64));
        b.xhi = fmaxf(b.xhi, __shfl_xor(b.xhi, o, 64));
        b.ylo = fminf(b.ylo, __shfl_xor(b.ylo, o, 64));
        b.yhi = fmaxf(b.yhi, __shfl_xor(b.yhi, o, 64));
        b.zlo = fminf(b.zlo, __shfl_xor(b.zlo, o, 64));
        b.zhi = fmaxf(b.zhi, __shfl_xor(b.zhi, o, 64));
    }
    return b;
}

// Builds the flattened candidate ranges of the primary in cell (cx,cy,cz).
// Every stencil run (fixed ox, oy; oz in [oz_lo, oz_hi]) becomes at most two
// pieces of consecutive cells: the part that wraps through the z boundary and
// the part that does not.
// A is any argument block with the grid (g), the stencil runs (runs, nruns)
// and the per-cell point ranges (cell_start).
// CUT: the points of a cell are in increasing z (the grid's order), so along a
// piece the candidates' z in the home frame, computed as the staging does,
// never decreases. Each piece is cut to the candidates whose z lies within
// the reach of the item's box over the xy gap to the piece's column (two
// binary searches over the piece); a column beyond the reach is dropped. The
// cut keeps every candidate within sqrt(box.r2) of a point of the box. The
// uncut candidate count (the stencil's, for density estimates) goes to n[1].
template <bool CUT = false, class A>
__device__ void build_pieces(Pieces& W, const A& a, int cat, int cx, int cy, int cz,
                             const ItemBox& box = ItemBox{}) {
    const int lane = lane_id();
    const int nc = a.g.nc, k = a.g.k, K2 = 2 * k + 1;
    const int base = cat * a.g.ncell;
    int total_pieces = 0, full = 0;
    for (int r0 = 0; r0 < a.nruns; r0 += 64) {
        const int r = r0 + lane;
        int s0 = 0, e0 = 0, s1 = 0, e1 = 0, c0 = 0, c1 = 0;
        float zo0 = 0.f, zo1 = 0.f, sx = 0.f, sy = 0.f;
        bool has_wrap = false, has_in = false;
        if (r < a.nruns) {
            const StencilRun st = a.runs[r];
            int qx = cx + st.ox, qy = cy + st.oy;
            int wx = 0, wy = 0;
            if (qx < 0) { qx += nc; wx = -1; } else if (qx >= nc) { qx -= nc; wx = 1; }
            if (qy < 0) { qy += nc; wy = -1; } else if (qy >= nc) { qy -= nc; wy = 1; }
            const int col = base + (qx * nc + qy) * nc;
            const int zlo = cz + st.oz_lo, zhi = cz + st.oz_hi;
            const int cbk = ((st.ox + k) * K2 + (st.oy + k)) * K2 + k;
            const int wxy = (wx + 1) | ((wy + 1) << 2);
            sx = (float)(st.ox * a.g.h);
            sy = (float)(st.oy * a.g.h);
            if (zlo < 0) {
                // cells zlo..min(zhi,-1) are nc+zlo..nc+min(zhi,-1); z offset = izf - nc - cz
                const int za = zlo + nc, zb = min(zhi, -1) + nc;
                s0 = a.cell_start[col + za];
                e0 = a.cell_start[col + zb + 1];
                zo0 = (float)(-nc - cz);
                c0 = cbk | ((wxy | (0 << 4)) << 16);
                has_wrap = true;
            } else if (zhi > nc - 1) {
                // cells max(zlo,nc)..zhi are those minus nc; z offset = izf + nc - cz
                const int za = max(zlo, nc) - nc, zb = zhi - nc;
                s0 = a.cell_start[col + za];
                e0 = a.cell_start[col + zb + 1];
                zo0 = (float)(nc - cz);
                c0 = cbk | ((wxy | (2 << 4)) << 16);
                has_wrap = true;
            }
            const int lo_in = max(zlo, 0), hi_in = min(zhi, nc - 1);
            if (hi_in >= lo_in) {
                s1 = a.cell_start[col + lo_in];
                e1 = a.cell_start[col + hi_in + 1];
                zo1 = (float)(-cz);
                c1 = cbk | ((wxy | (1 << 4)) << 16);
                has_in = true;
            }
            full += (has_wrap ? e0 - s0 : 0) + (has_in ? e1 - s1 : 0);
            if constexpr (CUT) {
                const float hf = a.g.hf;
                const float gx = fmaxf(0.f, fmaxf(sx - box.xhi, box.xlo - (sx + hf)));
                const float gy = fmaxf(0.f, fmaxf(sy - box.yhi, box.ylo - (sy + hf)));
                const float d2 = gx * gx + gy * gy;
                if (d2 > box.r2) {
                    has_wrap = has_in = false;
                } else {
                    const float hz = sqrtf(box.r2 - d2);
                    const float zlo_c = box.zlo - hz, zhi_c = box.zhi + hz;
                    // candidate j's z in the home frame, as stage_store forms it
                    auto zh = [&](int j, float zo) {
                        const float4 q = a.pf[j];
                        return fmaf((float)(int)(q.w + zo), hf, q.z);
                    };
                    auto cut = [&](int& sb, int& se, float zo) {
                        int lo = sb, hi = se;  // first candidate with z >= zlo_c
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (zh(mid, zo) < zlo_c) lo = mid + 1; else hi = mid;
                        }
                        const int b = lo;
                        hi = se;  // first candidate past it with z > zhi_c
                        while (lo < hi) {
                            const int mid = (lo + hi) >> 1;
                            if (zh(mid, zo) <= zhi_c) lo = mid + 1; else hi = mid;
                        }
                        sb = b;
                        se = lo;
                    };
                    if (has_wrap) {
                        cut(s0, e0, zo0);
                        has_wrap = e0 > s0;
                    }
                    if (has_in) {
                        cut(s1, e1, zo1);
                        has_in = e1 > s1;
                    }
                }
            }
        }
        const int np = (int)has_wrap + (int)has_in;
        int incl = np;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off, 64);
            if (lane >= off) incl += t;
        }
        int q = total_pieces + incl - np;
        if (has_wrap) {
            W.rec[q] = make_float4(__int_as_float(s0), sx, sy, zo0);
            W.pref[q] = e0 - s0;
            W.code[q] = c0;
            ++q;
        }
        if (has_in) {
            W.rec[q] = make_float4(__int_as_float(s1), sx, sy, zo1);
            W.pref[q] = e1 - s1;
            W.code[q] = c1;
        }
        total_pieces += __shfl(incl, 63, 64);
    }
    wave_sync();
    // exclusive prefix of the piece lengths (held in pref) -> pref, and the
    // point offset off = start - pref into rec.x
    int carry = 0;
    for (int q0 = 0; q0 < total_pieces; q0 += 64) {
        const int q = q0 + lane;
        const int len = q < total_pieces ? W.pref[q] : 0;
        int incl = len;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off, 64);
            if (lane >= off) incl += t;
        }
        wave_sync();
        if (q < total_pieces) {
            const int pr = carry + incl - len;
            W.pref[q] = pr;
            W.rec[q].x = __int_as_float(__float_as_int(W.rec[q].x) - pr);
        }
        carry += __shfl(incl, 63, 64);
        wave_sync();
    }
    for (int off = 32; off > 0; off >>= 1) full += __shfl_xor(full, off, 64);
    if (lane == 0) {
        W.pref[total_pieces] = carry;
        W.n[0] = total_pieces;
        W.n[1] = full;
    }
    wave_sync();
}

// Wrap signs (+1, 2 bits per axis) of stencil offset `code` seen from cell
// (cx, cy, cz): -1 where the neighbour cell index wrapped below 0, +1 above nc-1.
__device__ inline int wrap_bits_of(int code, int cx, int cy, int cz, int k, int nc) {
    const int K2 = 2 * k + 1;
    const int ox = code / (K2 * K2) - k, oy = (code / K2) % K2 - k, oz = code % K2 - k;
    auto w = [&](int c, int o) { const int q = c + o; return q < 0 ? 0 : (q >= nc ? 2 : 1); };
    return w(cx, ox) | (w(cy, oy) << 2) | (w(cz, oz) << 4);
}

}  // namespace

}  // namespace tpcf
