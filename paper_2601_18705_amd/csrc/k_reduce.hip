// Cholesky QR of the swept columns (Algorithm 1 step 5): the Cholesky factor of
// the Gram matrix and the triangular right-multiply that forms the orthonormal
// factor; and the assembly of the L-step operators (Sec. 4.3) from the raw
// projection sums.  The Gram matrices and projection sums themselves are formed
// on the matrix cores (k_mfma.hip).
#include "dlr_internal.h"

namespace dlr {

namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------------------------- Cholesky
// G (r x r, symmetric); column scaling s_k = 1/sqrt(G_kk); upper Cholesky of s G s = R'^T R';
// R = R' diag(1/s); Rinv = diag(s) R'^{-1}.  A pivot below the breakdown threshold (relative
// residual 1e-6 of a column against the previous ones) flags status_code: the columns are too
// close to dependent for Cholesky QR and the CGS2 fallback recomputes the factor.
// One wavefront, no barriers: lane j holds column j of the (symmetric) matrix in registers,
// padded to RMAX x RMAX with the identity.  Per pivot k the lanes form their entry of row k of
// R' and publish it in an LDS row, from which every lane reads R'_ki for its trailing entries
// i > k (the wavefront's LDS accesses execute in order, so no barrier is needed).  The inverse
// is formed row by row from the bottom the same way, lane j holding column j of R'^{-1}.
__device__ __forceinline__ double lane_value(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int RMAX>
__global__ __launch_bounds__(64) void k_chol(int r, const double* __restrict__ G, double* __restrict__ R,
                                             double* __restrict__ Rinv, int* status, int status_code,
                                             int* near_identity, double identity_tol) {
    static_assert(RMAX <= 64, "one lane per column");
    __shared__ double row[64];
    __shared__ double scl[64];
    const int j = threadIdx.x;
    const bool col = j < r;
    const int jc = col ? j : r - 1;
    const double gjj = G[jc * r + jc];
    bool bad = col && !(gjj > 0.0 && isfinite(gjj));
    const double sj = col ? ((gjj > 0.0) ? 1.0 / sqrt(gjj) : 0.0) : 1.0;
    scl[j] = sj;
    double a[RMAX];
    double dev = 0.0;   // max |G_ij - delta_ij| of this column
#pragma unroll
    for (int i = 0; i < RMAX; ++i) {
        const double g = G[(i < r ? i : r - 1) * r + jc];
        a[i] = (i < r && col) ? scl[i] * g * sj : (i == j ? 1.0 : 0.0);
        if (i < r && col) dev = fmax(dev, fabs(g - (i == j ? 1.0 : 0.0)));
    }
    if (near_identity) {
        // the Gram matrix of an already orthonormal basis: the second Cholesky QR pass may be skipped
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off));
        if (j == 0) *near_identity = (dev < identity_tol) ? 1 : 0;
    }
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);   // one pivot's LDS reads at a time (register pressure)
        const double piv = lane_value(a[k], k);
        if (k < r && !(piv > 1e-12)) bad = true;
        const double rkk = sqrt(fmax(piv, 1e-300));
        const double rkj = (j > k) ? a[k] / rkk : (j == k ? rkk : 0.0);
        a[k] = rkj;   // row k of R' (not touched again)
        row[j] = rkj;
#pragma unroll
        for (int i = k + 1; i < RMAX; ++i) a[i] = fma(-row[i], rkj, a[i]);
    }
    // R'^{-1}: Ri_ij = (delta_ij - sum_{i < m} R'_im Ri_mj) / R'_ii  (Ri_mj = 0 for m > j)
    double ri[RMAX];
#pragma unroll
    for (int i = RMAX - 1; i >= 0; --i) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        row[j] = a[i];   // row i of R'
        double part = 0.0;
#pragma unroll
        for (int m = i + 1; m < RMAX; ++m) part = fma(row[m], ri[m], part);
        ri[i] = ((i == j ? 1.0 : 0.0) - part) / row[i];
    }
    if (col) {
#pragma unroll
        for (int i = 0; i < RMAX; ++i) {
            if (i < r) {
                R[i * r + j] = (i <= j && sj > 0.0) ? a[i] / sj : 0.0;
                Rinv[i * r + j] = (i <= j) ? scl[i] * ri[i] : 0.0;
            }
        }
    }
    const unsigned long long anybad = __ballot(bad);
    if (j == 0 && anybad) atomicOr(status, status_code);
}

// ---------------------------------------------------------------------------------------------- X = V Rinv
template <typename TV, int RMAX>
__global__ __launch_bounds__(kBlock) void k_trmm(int n, int r, const TV* __restrict__ V, size_t ldv,
                                                 const double* __restrict__ Rinv, double* __restrict__ X) {
    __shared__ double sR[RMAX * RMAX];
    for (int o = threadIdx.x; o < r * r; o += kBlock) sR[(o / r) * RMAX + o % r] = Rinv[o];
    __syncthreads();
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double v[RMAX];
    const size_t ve = (size_t)e;
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
        const double x = (double)V[(size_t)(j < r ? j : r - 1) * ldv + ve];
        v[j] = (j < r) ? x : 0.0;
    }
    // k fully unrolled: the triangle j <= k is resolved at compile time (r (r+1)/2 multiply-adds)
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        if (k < r) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j <= k; ++j) acc = fma(v[j], sR[j * RMAX + k], acc);
            X[(size_t)k * n + e] = acc;
        }
    }
}

// X = X Rinv in place (no aliasing qualifiers: every thread loads its cell's row before it stores),
// skipped when *skip is set
template <int RMAX>
__global__ __launch_bounds__(kBlock) void k_trmm_inplace(int n, int r, double* X, const double* __restrict__ Rinv,
                                                         const int* __restrict__ skip) {
    if (*skip) return;
    __shared__ double sR[RMAX * RMAX];
    for (int o = threadIdx.x; o < r * r; o += kBlock) sR[(o / r) * RMAX + o % r] = Rinv[o];
    __syncthreads();
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double v[RMAX];
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
        const double x = X[(size_t)(j < r ? j : r - 1) * n + e];
        v[j] = (j < r) ? x : 0.0;
    }
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        if (k < r) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j <= k; ++j) acc = fma(v[j], sR[j * RMAX + k], acc);
            X[(size_t)k * n + e] = acc;
        }
    }
}

// ops layout: Axp, Axm, Ayp, Aym, Mt, Ms, G (r x r each), qX[r], b[4][r]
//   A_x^+ = <X, D_x^+ X> = (I - M0)/hx   (X orthonormal), A_x^- = (I - M0^T)/hx, same for y;
//   M_t = <X, sigma X> + I/(c dt);  G = S0^T P with P_ik = <X0_i, X_k> (old solution onto new X)
__global__ __launch_bounds__(kBlock) void k_project_ops(int r, const double* __restrict__ raw, double hx, double hy,
                                                        double inv_cdt, const double* __restrict__ S0,
                                                        double* __restrict__ ops) {
    __shared__ double sM4[kMaxRank * kMaxRank];
    __shared__ double sS[kMaxRank * kMaxRank];
    const int rr = r * r;
    stage_lds(sM4, raw + 4 * rr, rr);
    stage_lds(sS, S0, rr);
    __syncthreads();
    const double* M0 = raw;
    const double* M1 = raw + rr;
    const double* M2 = raw + 2 * rr;
    const double* M3 = raw + 3 * rr;
    const double* vec = raw + 5 * rr;
    for (int o = threadIdx.x; o < rr; o += blockDim.x) {
        const int i = o / r, j = o % r;
        const double id = (i == j) ? 1.0 : 0.0;
        ops[0 * rr + o] = (id - M0[o]) / hx;
        ops[1 * rr + o] = (id - M0[j * r + i]) / hx;
        ops[2 * rr + o] = (id - M1[o]) / hy;
        ops[3 * rr + o] = (id - M1[j * r + i]) / hy;
        ops[4 * rr + o] = M2[o] + id * inv_cdt;
        ops[5 * rr + o] = M3[o];
        double g = 0.0;
        for (int m = 0; m < r; ++m) g += sS[m * r + i] * sM4[m * r + j];
        ops[6 * rr + o] = g;
    }
    for (int o = threadIdx.x; o < 5 * r; o += blockDim.x) {
        const int kind = o / r;
        const double h = (kind == 1 || kind == 2) ? hx : hy;
        ops[7 * rr + o] = (kind == 0) ? vec[o] : vec[o] / h;
    }
}

}  // namespace

void launch_chol(hipStream_t s, int r, const double* G, double* R, double* Rinv, int* status, int status_code,
                 int* near_identity, double identity_tol) {
    if (r <= 8)
        hipLaunchKernelGGL(k_chol<8>, dim3(1), dim3(64), 0, s, r, G, R, Rinv, status, status_code, near_identity,
                           identity_tol);
    else if (r <= 16)
        hipLaunchKernelGGL(k_chol<16>, dim3(1), dim3(64), 0, s, r, G, R, Rinv, status, status_code, near_identity,
                           identity_tol);
    else if (r <= 32)
        hipLaunchKernelGGL(k_chol<32>, dim3(1), dim3(64), 0, s, r, G, R, Rinv, status, status_code, near_identity,
                           identity_tol);
    else
        hipLaunchKernelGGL(k_chol<64>, dim3(1), dim3(64), 0, s, r, G, R, Rinv, status, status_code, near_identity,
                           identity_tol);
}

void launch_trmm_inplace(hipStream_t s, int n, int r, double* X, const double* Rinv, const int* skip) {
    dim3 g((n + kBlock - 1) / kBlock), b(kBlock);
    if (r <= 8)
        hipLaunchKernelGGL((k_trmm_inplace<8>), g, b, 0, s, n, r, X, Rinv, skip);
    else if (r <= 16)
        hipLaunchKernelGGL((k_trmm_inplace<16>), g, b, 0, s, n, r, X, Rinv, skip);
    else if (r <= 32)
        hipLaunchKernelGGL((k_trmm_inplace<32>), g, b, 0, s, n, r, X, Rinv, skip);
    else
        hipLaunchKernelGGL((k_trmm_inplace<64>), g, b, 0, s, n, r, X, Rinv, skip);
}

template <typename TV>
void launch_trmm(hipStream_t s, int n, int r, const TV* V, size_t ldv, const double* Rinv, double* X) {
    dim3 g((n + kBlock - 1) / kBlock), b(kBlock);
    if (r <= 8)
        hipLaunchKernelGGL((k_trmm<TV, 8>), g, b, 0, s, n, r, V, ldv, Rinv, X);
    else if (r <= 16)
        hipLaunchKernelGGL((k_trmm<TV, 16>), g, b, 0, s, n, r, V, ldv, Rinv, X);
    else if (r <= 32)
        hipLaunchKernelGGL((k_trmm<TV, 32>), g, b, 0, s, n, r, V, ldv, Rinv, X);
    else
        hipLaunchKernelGGL((k_trmm<TV, 64>), g, b, 0, s, n, r, V, ldv, Rinv, X);
}
template void launch_trmm<double>(hipStream_t, int, int, const double*, size_t, const double*, double*);
template void launch_trmm<float>(hipStream_t, int, int, const float*, size_t, const double*, double*);

__global__ __launch_bounds__(kBlock) void k_small_matmul(int r, const double* __restrict__ A,
                                                         const double* __restrict__ B, double* __restrict__ C) {
    __shared__ double sA[kMaxRank * kMaxRank], sB[kMaxRank * kMaxRank];
    stage_lds(sA, A, r * r);
    stage_lds(sB, B, r * r);
    __syncthreads();
    for (int o = threadIdx.x; o < r * r; o += blockDim.x) {
        const int i = o / r, j = o % r;
        double s = 0.0;
        for (int k = 0; k < r; ++k) s += sA[i * r + k] * sB[k * r + j];
        C[o] = s;
    }
}

void launch_small_matmul(hipStream_t s, int r, const double* A, const double* B, double* C) {
    hipLaunchKernelGGL(k_small_matmul, dim3(1), dim3(kBlock), 0, s, r, A, B, C);
}

void launch_project_finalize(hipStream_t s, int r, const double* partials, int nblocks, double hx, double hy,
                             double inv_cdt, const double* S0, double* ops) {
    // raw sums go into the tail of ops (beyond the operator block) as scratch
    const int rr = r * r;
    double* raw = ops + 7 * rr + 5 * r;
    const double area = hx * hy;
    launch_project_sum(s, r, partials, nblocks, area, raw);
    hipLaunchKernelGGL(k_project_ops, dim3(1), dim3(kBlock), 0, s, r, raw, hx, hy, inv_cdt, S0, ops);
}

}  // namespace dlr
