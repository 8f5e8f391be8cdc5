// Tall-skinny reductions over cells (or ordinates): Gram matrices for the
// Cholesky-QR orthonormalisation of the swept columns and of L, the triangular
// right-multiply that forms the orthonormal factor, and the Galerkin
// projections of the L-step (A(Omega), M_t, M_s, <X0, X>, <X, q>, inflow faces).
// Every sum is split over blocks and the partials are added in a fixed order,
// so results are bitwise reproducible run to run.
#include "dlr_internal.h"

namespace dlr {

namespace {

constexpr int kBlock = 256;
constexpr int kGramChunk = 64;

// ---------------------------------------------------------------------------------------------- Gram
// partial_b[i*r + j] = scalar * sum_{e in block b} wgt_e V_i(e) V_j(e), V [r][n].
template <typename TV, int EPT>
__global__ __launch_bounds__(kBlock) void k_gram(int n, int r, const TV* __restrict__ V, size_t ldv, int pad_ny,
                                                 const double* __restrict__ weight, double scalar,
                                                 double* __restrict__ partials) {
    __shared__ double sV[kMaxRank * kGramChunk];
    __shared__ double sw[kGramChunk];
    const int rr = r * r;
    double acc[EPT];
    int oi[EPT], oj[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        acc[k] = 0.0;
        const int o = threadIdx.x + k * kBlock;
        oi[k] = (o < rr) ? o / r : 0;
        oj[k] = (o < rr) ? o % r : 0;
    }
    for (long c0 = (long)blockIdx.x * kGramChunk; c0 < n; c0 += (long)gridDim.x * kGramChunk) {
        const int cn = (int)min((long)kGramChunk, n - c0);
        __syncthreads();
        for (int idx = threadIdx.x; idx < r * kGramChunk; idx += kBlock) {
            const int k = idx / kGramChunk, c = idx % kGramChunk;
            const long e = c0 + c;
            sV[k * kGramChunk + c] =
                (c < cn) ? (double)V[(size_t)k * ldv + (pad_ny ? padded_cell(e, pad_ny) : (size_t)e)] : 0.0;
        }
        for (int c = threadIdx.x; c < kGramChunk; c += kBlock) sw[c] = (c < cn) ? (weight ? weight[c0 + c] : 1.0) : 0.0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const double* vi = sV + oi[k] * kGramChunk;
            const double* vj = sV + oj[k] * kGramChunk;
            double a = acc[k];
            for (int c = 0; c < kGramChunk; ++c) a += (vi[c] * sw[c]) * vj[c];
            acc[k] = a;
        }
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int o = threadIdx.x + k * kBlock;
        if (o < rr) partials[(size_t)blockIdx.x * rr + o] = acc[k] * scalar;
    }
}

// ---------------------------------------------------------------------------------------------- Cholesky
// G = sum of partials (block order); column scaling s_k = 1/sqrt(G_kk); upper Cholesky
// of s G s = R'^T R'; R = R' diag(1/s); Rinv = diag(s) R'^{-1}.  A pivot below the
// breakdown threshold (relative residual 1e-6 of a column against the previous
// ones) flags status_code: the columns are too close to dependent for Cholesky QR
// and the CGS2 fallback recomputes the factor.
__global__ __launch_bounds__(kBlock) void k_chol(int r, const double* __restrict__ partials, int nblocks,
                                                 double* __restrict__ R, double* __restrict__ Rinv, int* status,
                                                 int status_code) {
    __shared__ double A[kMaxRank * kMaxRank];
    __shared__ double Rp[kMaxRank * kMaxRank];
    __shared__ double sc[kMaxRank];
    __shared__ int bad;
    const int rr = r * r;
    if (threadIdx.x == 0) bad = 0;
    for (int o = threadIdx.x; o < rr; o += kBlock) {
        double g = 0.0;
        for (int b = 0; b < nblocks; ++b) g += partials[(size_t)b * rr + o];
        A[o] = g;
        Rp[o] = 0.0;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < r; k += kBlock) {
        const double gkk = A[k * r + k];
        if (!(gkk > 0.0) || !isfinite(gkk)) bad = 1;
        sc[k] = (gkk > 0.0) ? 1.0 / sqrt(gkk) : 0.0;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < rr; o += kBlock) A[o] *= sc[o / r] * sc[o % r];
    __syncthreads();
    for (int k = 0; k < r; ++k) {
        const double piv = A[k * r + k];
        if (threadIdx.x == 0 && !(piv > 1e-12)) bad = 1;
        const double rkk = sqrt(fmax(piv, 1e-300));
        for (int j = threadIdx.x; j < r; j += kBlock)
            if (j >= k) Rp[k * r + j] = (j == k) ? rkk : A[k * r + j] / rkk;
        __syncthreads();
        for (int o = threadIdx.x; o < rr; o += kBlock) {
            const int i = o / r, j = o % r;
            if (i > k && j > k) A[o] -= Rp[k * r + i] * Rp[k * r + j];
        }
        __syncthreads();
    }
    // inverse of the upper-triangular R' column by column (back substitution)
    for (int j = threadIdx.x; j < r; j += kBlock) {
        for (int i = r - 1; i >= 0; --i) {
            double v;
            if (i > j) {
                v = 0.0;
            } else {
                v = (i == j) ? 1.0 : 0.0;
                for (int m = i + 1; m <= j; ++m) v -= Rp[i * r + m] * A[m * r + j];
                v /= Rp[i * r + i];
            }
            A[i * r + j] = v;   // A now holds R'^{-1}; column j is written only by thread j
        }
    }
    __syncthreads();
    for (int o = threadIdx.x; o < rr; o += kBlock) {
        const int i = o / r, j = o % r;
        R[o] = (sc[j] > 0.0) ? Rp[o] / sc[j] : 0.0;
        Rinv[o] = sc[i] * A[o];
    }
    if (threadIdx.x == 0 && bad) atomicOr(status, status_code);
}

// ---------------------------------------------------------------------------------------------- X = V Rinv
template <typename TV, int RMAX>
__global__ __launch_bounds__(kBlock) void k_trmm(int n, int r, const TV* __restrict__ V, size_t ldv, int pad_ny,
                                                 const double* __restrict__ Rinv, double* __restrict__ X) {
    __shared__ double sR[RMAX * RMAX];
    for (int o = threadIdx.x; o < r * r; o += kBlock) sR[(o / r) * RMAX + o % r] = Rinv[o];
    __syncthreads();
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double v[RMAX];
    const size_t ve = pad_ny ? padded_cell(e, pad_ny) : (size_t)e;
#pragma unroll
    for (int j = 0; j < RMAX; ++j) v[j] = (j < r) ? (double)V[(size_t)j * ldv + ve] : 0.0;
#pragma unroll 4
    for (int k = 0; k < r; ++k) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < RMAX; ++j)
            if (j <= k) acc += v[j] * sR[j * RMAX + k];
        X[(size_t)k * n + e] = acc;
    }
}

// ---------------------------------------------------------------------------------------------- projections
// Raw split-K sums per block, layout [5 r^2 matrices][5 r vectors]:
//   M0 = sum X_i(i,j) X_j(i-1,j)      (x-upwind neighbour for mu > 0, 0 on column 0)
//   M1 = sum X_i(i,j) X_j(i,j-1)      (y-upwind neighbour for eta > 0, 0 on row 0)
// with column-major cells e = i*ny + j, so (i-1,j) = e - ny and (i,j-1) = e - 1.
//   M2 = sum sigma_e X_i X_j,  M3 = sum sigma_s,e X_i X_j,  M4 = sum X0_i X_j
//   v0 = sum q_e X_i,  v1..v4 = sum over the left/right/bottom/top cells of X_i
constexpr int kProjChunk = 32;

template <int EPT>
__global__ __launch_bounds__(kBlock) void k_project(int nx, int ny, int r, const double* __restrict__ X,
                                                    const double* __restrict__ X0, const double* __restrict__ sigma,
                                                    const double* __restrict__ sig_s, const double* __restrict__ q,
                                                    double* __restrict__ partials) {
    __shared__ double sX[kMaxRank * kProjChunk];
    __shared__ double sL[kMaxRank * kProjChunk];
    __shared__ double sD[kMaxRank * kProjChunk];
    __shared__ double s0[kMaxRank * kProjChunk];
    __shared__ double ss[kProjChunk], sss[kProjChunk], sq[kProjChunk];
    __shared__ int sside[kProjChunk];
    const long n = (long)nx * ny;
    const int rr = r * r;
    double a0[EPT], a1[EPT], a2[EPT], a3[EPT], a4[EPT];
    int oi[EPT], oj[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        a0[k] = a1[k] = a2[k] = a3[k] = a4[k] = 0.0;
        const int o = threadIdx.x + k * kBlock;
        oi[k] = (o < rr) ? o / r : 0;
        oj[k] = (o < rr) ? o % r : 0;
    }
    // vector entries: slot = threadIdx.x + m * kBlock < 5 r (two slots cover r <= 64)
    double vacc[2] = {0.0, 0.0};
    for (long c0 = (long)blockIdx.x * kProjChunk; c0 < n; c0 += (long)gridDim.x * kProjChunk) {
        const int cn = (int)min((long)kProjChunk, n - c0);
        __syncthreads();
        for (int idx = threadIdx.x; idx < r * kProjChunk; idx += kBlock) {
            const int k = idx / kProjChunk, c = idx % kProjChunk;
            double x = 0.0, xl = 0.0, xd = 0.0, x0 = 0.0;
            if (c < cn) {
                const long e = c0 + c;
                const int i = (int)(e / ny), j = (int)(e % ny);
                const double* col = X + (size_t)k * n;
                x = col[e];
                xl = (i > 0) ? col[e - ny] : 0.0;
                xd = (j > 0) ? col[e - 1] : 0.0;
                x0 = X0[(size_t)k * n + e];
            }
            sX[k * kProjChunk + c] = x;
            sL[k * kProjChunk + c] = xl;
            sD[k * kProjChunk + c] = xd;
            s0[k * kProjChunk + c] = x0;
        }
        for (int c = threadIdx.x; c < kProjChunk; c += kBlock) {
            const long e = c0 + c;
            const bool ok = c < cn;
            ss[c] = ok ? sigma[e] : 0.0;
            sss[c] = ok ? sig_s[e] : 0.0;
            sq[c] = ok ? q[e] : 0.0;
            int f = 0;
            if (ok) {
                const int i = (int)(e / ny), j = (int)(e % ny);
                f = (i == 0 ? 1 : 0) | (i == nx - 1 ? 2 : 0) | (j == 0 ? 4 : 0) | (j == ny - 1 ? 8 : 0);
            }
            sside[c] = f;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            const double* xi = sX + oi[k] * kProjChunk;
            const double* xj = sX + oj[k] * kProjChunk;
            const double* xlj = sL + oj[k] * kProjChunk;
            const double* xdj = sD + oj[k] * kProjChunk;
            const double* x0i = s0 + oi[k] * kProjChunk;
            double b0 = a0[k], b1 = a1[k], b2 = a2[k], b3 = a3[k], b4 = a4[k];
            for (int c = 0; c < kProjChunk; ++c) {
                const double u = xi[c];
                const double v = xj[c];
                b0 += u * xlj[c];
                b1 += u * xdj[c];
                b2 += (u * ss[c]) * v;
                b3 += (u * sss[c]) * v;
                b4 += x0i[c] * v;
            }
            a0[k] = b0; a1[k] = b1; a2[k] = b2; a3[k] = b3; a4[k] = b4;
        }
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int vslot = threadIdx.x + m * kBlock;
            if (vslot < 5 * r) {
                const int vkind = vslot / r, vi = vslot % r;
                const double* xi = sX + vi * kProjChunk;
                double acc = vacc[m];
                for (int c = 0; c < kProjChunk; ++c) {
                    if (vkind == 0) acc += sq[c] * xi[c];
                    else if (sside[c] & (1 << (vkind - 1))) acc += xi[c];
                }
                vacc[m] = acc;
            }
        }
    }
    double* out = partials + (size_t)blockIdx.x * (5 * rr + 5 * r);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int o = threadIdx.x + k * kBlock;
        if (o < rr) {
            out[o] = a0[k];
            out[rr + o] = a1[k];
            out[2 * rr + o] = a2[k];
            out[3 * rr + o] = a3[k];
            out[4 * rr + o] = a4[k];
        }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int vslot = threadIdx.x + m * kBlock;
        if (vslot < 5 * r) out[5 * rr + vslot] = vacc[m];
    }
}

__global__ __launch_bounds__(kBlock) void k_project_reduce(int total, const double* __restrict__ partials,
                                                           int nblocks, double area, double* __restrict__ raw) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= total) return;
    double acc = 0.0;
    for (int b = 0; b < nblocks; ++b) acc += partials[(size_t)b * total + o];
    raw[o] = acc * area;
}

// ops layout: Axp, Axm, Ayp, Aym, Mt, Ms, G (r x r each), qX[r], b[4][r]
//   A_x^+ = <X, D_x^+ X> = (I - M0)/hx   (X orthonormal), A_x^- = (I - M0^T)/hx, same for y;
//   M_t = <X, sigma X> + I/(c dt);  G = S0^T P with P_ik = <X0_i, X_k> (old solution onto new X)
__global__ __launch_bounds__(kBlock) void k_project_ops(int r, const double* __restrict__ raw, double hx, double hy,
                                                        double inv_cdt, const double* __restrict__ S0,
                                                        double* __restrict__ ops) {
    const int rr = r * r;
    const double* M0 = raw;
    const double* M1 = raw + rr;
    const double* M2 = raw + 2 * rr;
    const double* M3 = raw + 3 * rr;
    const double* M4 = raw + 4 * rr;
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
        for (int m = 0; m < r; ++m) g += S0[m * r + i] * M4[m * r + j];
        ops[6 * rr + o] = g;
    }
    for (int o = threadIdx.x; o < 5 * r; o += blockDim.x) {
        const int kind = o / r;
        const double h = (kind == 1 || kind == 2) ? hx : hy;
        ops[7 * rr + o] = (kind == 0) ? vec[o] : vec[o] / h;
    }
}

}  // namespace

template <typename TV>
void launch_gram(hipStream_t s, int n, int r, const TV* V, size_t ldv, int pad_ny, const double* weight,
                 double scalar_weight, double* partials, int nblocks) {
    const int ept = (r * r + kBlock - 1) / kBlock;
    if (ept <= 1)
        hipLaunchKernelGGL((k_gram<TV, 1>), dim3(nblocks), dim3(kBlock), 0, s, n, r, V, ldv, pad_ny, weight, scalar_weight,
                           partials);
    else if (ept <= 4)
        hipLaunchKernelGGL((k_gram<TV, 4>), dim3(nblocks), dim3(kBlock), 0, s, n, r, V, ldv, pad_ny, weight, scalar_weight,
                           partials);
    else
        hipLaunchKernelGGL((k_gram<TV, 16>), dim3(nblocks), dim3(kBlock), 0, s, n, r, V, ldv, pad_ny, weight, scalar_weight,
                           partials);
}
template void launch_gram<double>(hipStream_t, int, int, const double*, size_t, int, const double*, double, double*,
                                  int);
template void launch_gram<float>(hipStream_t, int, int, const float*, size_t, int, const double*, double, double*, int);

void launch_chol(hipStream_t s, int r, const double* partials, int nblocks, double* R, double* Rinv, int* status,
                 int status_code) {
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(kBlock), 0, s, r, partials, nblocks, R, Rinv, status, status_code);
}

template <typename TV>
void launch_trmm(hipStream_t s, int n, int r, const TV* V, size_t ldv, int pad_ny, const double* Rinv, double* X) {
    dim3 g((n + kBlock - 1) / kBlock), b(kBlock);
    if (r <= 8)
        hipLaunchKernelGGL((k_trmm<TV, 8>), g, b, 0, s, n, r, V, ldv, pad_ny, Rinv, X);
    else if (r <= 16)
        hipLaunchKernelGGL((k_trmm<TV, 16>), g, b, 0, s, n, r, V, ldv, pad_ny, Rinv, X);
    else if (r <= 32)
        hipLaunchKernelGGL((k_trmm<TV, 32>), g, b, 0, s, n, r, V, ldv, pad_ny, Rinv, X);
    else
        hipLaunchKernelGGL((k_trmm<TV, 64>), g, b, 0, s, n, r, V, ldv, pad_ny, Rinv, X);
}
template void launch_trmm<double>(hipStream_t, int, int, const double*, size_t, int, const double*, double*);
template void launch_trmm<float>(hipStream_t, int, int, const float*, size_t, int, const double*, double*);

void launch_project(hipStream_t s, int nx, int ny, int r, const double* X, const double* X0, const double* sigma,
                    const double* sig_s, const double* q, double area, double hx, double hy, double* partials,
                    int nblocks) {
    (void)area; (void)hx; (void)hy;
    const int ept = (r * r + kBlock - 1) / kBlock;
    if (ept <= 1)
        hipLaunchKernelGGL((k_project<1>), dim3(nblocks), dim3(kBlock), 0, s, nx, ny, r, X, X0, sigma, sig_s, q, partials);
    else if (ept <= 4)
        hipLaunchKernelGGL((k_project<4>), dim3(nblocks), dim3(kBlock), 0, s, nx, ny, r, X, X0, sigma, sig_s, q, partials);
    else
        hipLaunchKernelGGL((k_project<16>), dim3(nblocks), dim3(kBlock), 0, s, nx, ny, r, X, X0, sigma, sig_s, q,
                           partials);
}

void launch_project_finalize(hipStream_t s, int r, const double* partials, int nblocks, double hx, double hy,
                             double inv_cdt, const double* S0, double* ops) {
    // raw sums go into the tail of ops (beyond the operator block) as scratch
    const int rr = r * r;
    const int total = 5 * rr + 5 * r;
    double* raw = ops + 7 * rr + 5 * r;
    const double area = hx * hy;
    hipLaunchKernelGGL(k_project_reduce, dim3((total + kBlock - 1) / kBlock), dim3(kBlock), 0, s, total, partials,
                       nblocks, area, raw);
    hipLaunchKernelGGL(k_project_ops, dim3(1), dim3(kBlock), 0, s, r, raw, hx, hy, inv_cdt, S0, ops);
}

}  // namespace dlr
