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
// G = sum of partials (block order); column scaling s_k = 1/sqrt(G_kk); upper Cholesky
// of s G s = R'^T R'; R = R' diag(1/s); Rinv = diag(s) R'^{-1}.  A pivot below the
// breakdown threshold (relative residual 1e-6 of a column against the previous
// ones) flags status_code: the columns are too close to dependent for Cholesky QR
// and the CGS2 fallback recomputes the factor.
// One workgroup of four wavefronts, the matrix in LDS.  Per pivot k the threads of row k
// form row k of R' and the trailing upper triangle gets the rank-one update, row i by
// wavefront i mod 4 with the columns on the lanes (contiguous, conflict-free LDS accesses,
// and only the live entries are touched), two barriers per pivot.  Wavefront 0 then forms
// R'^{-1} row by row from the bottom, the lanes holding its columns.
constexpr int kCholThreads = 256;
static_assert(kMaxRank <= 64, "one lane per column");

__global__ __launch_bounds__(kCholThreads) void k_chol(int r, const double* __restrict__ partials, int nblocks,
                                                       double* __restrict__ R, double* __restrict__ Rinv,
                                                       int* status, int status_code) {
    __shared__ double A[kMaxRank * kMaxRank];
    __shared__ double Ri[kMaxRank * kMaxRank];
    __shared__ double rowk[kMaxRank];
    __shared__ double sc[kMaxRank];
    __shared__ int bad;
    const int tid = threadIdx.x, rr = r * r;
    const int lane = tid & 63, wv = tid >> 6;
    if (tid == 0) bad = 0;
    stage_lds(A, partials, rr);
    __syncthreads();
    for (int b = 1; b < nblocks; ++b) {
        stage_lds(Ri, partials + (size_t)b * rr, rr);
        __syncthreads();
        for (int o = tid; o < rr; o += kCholThreads) A[o] += Ri[o];
        __syncthreads();
    }
    for (int k = tid; k < r; k += kCholThreads) {
        const double gkk = A[k * r + k];
        if (!(gkk > 0.0) || !isfinite(gkk)) bad = 1;
        sc[k] = (gkk > 0.0) ? 1.0 / sqrt(gkk) : 0.0;
    }
    __syncthreads();
    for (int i = wv; i < r; i += 4)
        if (lane < r) {
            A[i * r + lane] *= sc[i] * sc[lane];
            Ri[i * r + lane] = 0.0;
        }
    __syncthreads();
    for (int k = 0; k < r; ++k) {
        const double piv = A[k * r + k];
        const double rkk = sqrt(fmax(piv, 1e-300));
        if (tid == 0 && !(piv > 1e-12)) bad = 1;
        // row k of R' (A keeps it: row k is not touched again)
        if (tid >= k && tid < r) {
            const double v = (tid == k) ? rkk : A[k * r + tid] / rkk;
            rowk[tid] = v;
            A[k * r + tid] = v;
        }
        __syncthreads();
        // trailing update of the upper triangle: A_ij -= R'_ki R'_kj, k < i <= j
        if (lane < r) {
            const double rj = rowk[lane];
#pragma unroll 2
            for (int i = k + 1 + wv; i < r; i += 4)
                if (lane >= i) A[i * r + lane] -= rowk[i] * rj;
        }
        __syncthreads();
    }
    // R'^{-1}, row i from rows i+1.. : Ri_ij = (delta_ij - sum_{i < m < r} R'_im Ri_mj) / R'_ii
    // (Ri_mj = 0 for m > j, so the uniform bound adds exact zeros)
    if (wv == 0 && lane < r) {
        for (int i = r - 1; i >= 0; --i) {
            double part = 0.0;
#pragma unroll 8
            for (int m = i + 1; m < r; ++m) part += A[i * r + m] * Ri[m * r + lane];
            if (lane >= i) Ri[i * r + lane] = (((i == lane) ? 1.0 : 0.0) - part) / A[i * r + i];
        }
    }
    __syncthreads();
    for (int i = wv; i < r; i += 4)
        if (lane < r) {
            const int o = i * r + lane;
            R[o] = (i <= lane && sc[lane] > 0.0) ? A[o] / sc[lane] : 0.0;
            Rinv[o] = (i <= lane) ? sc[i] * Ri[o] : 0.0;
        }
    if (tid == 0 && bad) atomicOr(status, status_code);
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

void launch_chol(hipStream_t s, int r, const double* partials, int nblocks, double* R, double* Rinv, int* status,
                 int status_code) {
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(kCholThreads), 0, s, r, partials, nblocks, R, Rinv, status, status_code);
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
