// Edge correction of the anisotropic 3PCF by explicit randoms: the
// Szapudi-Szalay estimator of eq. (ssest), zeta = (D - R)^3 / R^3, read as a
// ratio of two functions of the triangle (arXiv:2408.03036, Sec. 4).
//
// With N and R the data-minus-randoms and random triplet counts of one
// (r1, r2) bin pair, each a real function of the two side directions and
// expanded in the orthonormal basis Y_l1m(r1) conj(Y_l2m(r2)) (the per-m
// coefficients NNN^m of the contraction, normalised by their analytic RRR),
// N = zeta R at every pair of directions gives
//   N^m_{l1 l2} = sum zeta^{m'}_{l1' l2'} R^{m-m'}_{l1'' l2''}
//                 g(l1 m; l1' m'; l1'') g(l2 m; l2' m'; l2''),
// g(l m; l' m'; l'') = integral of conj(Y_lm) Y_l'm' Y_l'',m-m' (real), all
// indices truncated at lmax. The real (reflection-symmetric) sector is solved:
// every coefficient is real and X^{-m} = X^m, so the unknowns are zeta^m for
// m >= 0 and the columns of m' > 0 collect the terms of +m' and -m'.
//
//  k_edge_assemble  one thread per (system, row, column) of the n x n systems
//                   (n = number of (l1, l2, m >= 0) with m <= l1, l2 <= lmax)
//  k_edge_solve     one workgroup per system: Gaussian elimination with
//                   partial pivoting in FP64 in the workspace, then back
//                   substitution; writes zeta^m in the export layout
//  k_edge_mult      TripoSH sums of zeta^m for the requested multipoles
#include "tpcf_internal.h"

namespace tpcf {

namespace {

__global__ void k_edge_assemble(EdgeArgs a) {
    const int n = a.n;
    const int64_t nn = (int64_t)n * n;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn * a.nsys) return;
    const int q = (int)(t / nn);              // system = b1 nb + b2
    const int row = (int)((t / n) % n), col = (int)(t % n);
    const int S = a.lmax + 1, S2 = 2 * a.lmax + 1;
    const int nbb = a.nsys;
    const int4 r = a.units[row], c = a.units[col];  // (l1, l2, m)
    const int l1 = r.x, l2 = r.y, m = r.z;
    double acc = 0.0;
    for (int s = 0; s < (c.z > 0 ? 2 : 1); ++s) {
        const int mq = s == 0 ? c.z : -c.z;   // m' of this term
        const int mpp = m - mq;
        const int am = mpp < 0 ? -mpp : mpp;
        if (am > a.lmax) continue;
        // g(l, m; l', m'; l'') at ((((l S + m) S + l') S2 + m' + lmax) S + l'')
        const double* g1 = a.gaunt + ((((int64_t)l1 * S + m) * S + c.x) * S2 + mq + a.lmax) * S;
        const double* g2 = a.gaunt + ((((int64_t)l2 * S + m) * S + c.y) * S2 + mq + a.lmax) * S;
        const double* Rm = a.R + (int64_t)am * S * S * nbb;
        for (int c1 = am; c1 <= a.lmax; ++c1) {
            const double v1 = g1[c1];
            if (v1 == 0.0) continue;
            for (int c2 = am; c2 <= a.lmax; ++c2) {
                const double v2 = g2[c2];
                if (v2 == 0.0) continue;
                acc += v1 * v2 * Rm[((int64_t)c1 * S + c2) * nbb + q] * a.inv_rrr_R[q];
            }
        }
    }
    a.M[t] = acc;
    if (col == 0)
        a.rhs[(int64_t)q * n + row] = a.N[(((int64_t)m * S + l1) * S + l2) * nbb + q] * a.inv_rrr_N[q];
}

constexpr int kSolveThreads = 256;

// Maximum |M[i][k]| over rows i >= k of the workgroup's system (first index on ties).
__device__ void pivot_search(const double* M, int n, int k, double* sv, int* si, int& piv) {
    double best = -1.0;
    int bi = k;
    for (int i = k + (int)threadIdx.x; i < n; i += kSolveThreads) {
        const double v = fabs(M[(int64_t)i * n + k]);
        if (v > best) {
            best = v;
            bi = i;
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int o = kSolveThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            const double v = sv[threadIdx.x + o];
            const int i = si[threadIdx.x + o];
            if (v > sv[threadIdx.x] || (v == sv[threadIdx.x] && i < si[threadIdx.x])) {
                sv[threadIdx.x] = v;
                si[threadIdx.x] = i;
            }
        }
        __syncthreads();
    }
    piv = si[0];
}

__global__ void __launch_bounds__(kSolveThreads) k_edge_solve(EdgeArgs a) {
    __shared__ double sv[kSolveThreads];
    __shared__ int si[kSolveThreads];
    __shared__ double fac[kMaxEdgeUnknowns];
    const int q = blockIdx.x;
    if (q >= a.nsys) return;
    const int n = a.n;
    double* M = a.M + (int64_t)q * n * n;
    double* x = a.rhs + (int64_t)q * n;
    for (int k = 0; k < n; ++k) {
        int piv;
        pivot_search(M, n, k, sv, si, piv);
        if (!(sv[0] > 0.0)) {
            if (threadIdx.x == 0) atomicOr(a.bad, 1);
            return;  // uniform: every thread read the same sv[0]
        }
        if (piv != k) {
            for (int j = k + (int)threadIdx.x; j < n; j += kSolveThreads) {
                const double t = M[(int64_t)k * n + j];
                M[(int64_t)k * n + j] = M[(int64_t)piv * n + j];
                M[(int64_t)piv * n + j] = t;
            }
            if (threadIdx.x == 0) {
                const double t = x[k];
                x[k] = x[piv];
                x[piv] = t;
            }
        }
        __syncthreads();
        const double ip = 1.0 / M[(int64_t)k * n + k];
        for (int i = k + 1 + (int)threadIdx.x; i < n; i += kSolveThreads) fac[i] = M[(int64_t)i * n + k] * ip;
        __syncthreads();
        // rows below the pivot: M[i][j] -= f_i M[k][j] (j > k), x[i] -= f_i x[k]
        const int w = n - k;  // columns k+1 .. n-1 and the right-hand side (as column n)
        const int64_t cnt = (int64_t)(n - k - 1) * w;
        for (int64_t e = threadIdx.x; e < cnt; e += kSolveThreads) {
            const int i = k + 1 + (int)(e / w);
            const int j = k + 1 + (int)(e % w);
            if (j < n) M[(int64_t)i * n + j] -= fac[i] * M[(int64_t)k * n + j];
            else x[i] -= fac[i] * x[k];
        }
        __syncthreads();
    }
    // back substitution, one unknown at a time: x[k] /= M[k][k], then the
    // rows above subtract its column
    for (int k = n - 1; k >= 0; --k) {
        if (threadIdx.x == 0) x[k] /= M[(int64_t)k * n + k];
        __syncthreads();
        const double xk = x[k];
        for (int i = (int)threadIdx.x; i < k; i += kSolveThreads) x[i] -= M[(int64_t)i * n + k] * xk;
        __syncthreads();
    }
    const int S = a.lmax + 1;
    for (int u = (int)threadIdx.x; u < n; u += kSolveThreads) {
        const int4 r = a.units[u];
        a.zeta[(((int64_t)r.z * S + r.x) * S + r.y) * a.nsys + q] = x[u];
    }
}

__global__ void k_edge_mult(EdgeArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)a.n_mult * a.nsys) return;
    const int tm = (int)(t / a.nsys), q = (int)(t % a.nsys);
    const int S = a.lmax + 1;
    const int l1 = a.mult[3 * tm], l2 = a.mult[3 * tm + 1];
    const int mm = l1 < l2 ? l1 : l2;
    double v = 0.0;
    for (int m = 0; m <= mm; ++m)
        v += a.coef[(int64_t)tm * S + m] * a.zeta[(((int64_t)m * S + l1) * S + l2) * a.nsys + q];
    a.out[t] = v;
}

}  // namespace

hipError_t launch_edge_aniso(const EdgeArgs& a, hipStream_t s) {
    if (a.n < 1 || a.n > kMaxEdgeUnknowns || a.nsys < 1) return hipErrorInvalidValue;
    const int64_t nt = (int64_t)a.n * a.n * a.nsys;
    hipLaunchKernelGGL(k_edge_assemble, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_edge_solve, dim3((unsigned)a.nsys), dim3(kSolveThreads), 0, s, a);
    const int64_t nm = (int64_t)a.n_mult * a.nsys;
    if (nm > 0) hipLaunchKernelGGL(k_edge_mult, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace tpcf
