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
// padded to RMAX x RMAX with the identity, and column j of an identity block B.  Pivot k divides
// row k by r_kk = sqrt(pivot) (one reciprocal, then products) and subtracts R'_ki times it from
// each row i > k, in both blocks.  After the last pivot the first block is R' and the second is
// E with E A = R', i.e. E = R'^{-T}: lane j holds row j of R'^{-1}, so no separate inversion is
// needed; row k of both is final after pivot k and stored then.  The row values R'_ki reach the
// lanes through an LDS row (the wavefront's LDS accesses execute in order, so no barrier is
// needed); the entries of row k + 1, which the next pivot needs at once, come through lane reads.
__device__ __forceinline__ double lane_value(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int RMAX>
__global__ __launch_bounds__(64) void k_chol(int r, const double* __restrict__ G, double* __restrict__ R,
                                             double* __restrict__ Rinv, int* status, int status_code,
                                             int* near_identity, double identity_tol, int identity_on_flag) {
    static_assert(RMAX <= 64, "one lane per column");
    if (identity_on_flag && (*status & status_code)) {
        for (int o = threadIdx.x; o < r * r; o += 64) {
            const double v = (o / r == o % r) ? 1.0 : 0.0;
            R[o] = v;
            Rinv[o] = v;
        }
        return;
    }
    __shared__ double row[64];
    __shared__ double scl[64];
    const int j = threadIdx.x;
    const bool col = j < r;
    const int jc = col ? j : r - 1;
    const double gjj = G[jc * r + jc];
    bool bad = col && !(gjj > 0.0 && isfinite(gjj));
    const double sj = col ? ((gjj > 0.0) ? 1.0 / sqrt(gjj) : 0.0) : 1.0;
    const double unscale = (col && gjj > 0.0) ? sqrt(gjj) : 0.0;   // 1 / s_j (R = R' diag(1/s))
    scl[j] = sj;
    double a[RMAX], bm[RMAX];
    double dev = 0.0;   // max |G_ij - delta_ij| of this column
    // The column's entries are loaded first, all at once, and cleared by a bit mask where unused:
    // a select between a loaded value and a constant is compiled into a branch around the load,
    // which then waits for each load in turn.
    double gv[RMAX];
#pragma unroll
    for (int i = 0; i < RMAX; ++i) {
        const unsigned long long keep = (i < r && col) ? ~0ull : 0ull;
        gv[i] = __longlong_as_double(__double_as_longlong(G[(i < r ? i : r - 1) * r + jc]) & keep);
    }
#pragma unroll
    for (int i = 0; i < RMAX; ++i) {
        const double g = gv[i];
        a[i] = (i < r && col) ? scl[i] * g * sj : (i == j ? 1.0 : 0.0);
        bm[i] = (i == j) ? 1.0 : 0.0;
        if (i < r && col) dev = fmax(dev, fabs(g - (i == j ? 1.0 : 0.0)));
    }
    if (near_identity) {
        // the Gram matrix of an already orthonormal basis: the second Cholesky QR pass may be skipped
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off));
        if (j == 0) *near_identity = (dev < identity_tol) ? 1 : 0;
    }
    double piv = lane_value(a[0], 0);
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        __atomic_signal_fence(__ATOMIC_SEQ_CST);   // one pivot's LDS reads at a time (register pressure)
        if (k < r && !(piv > 1e-12)) bad = true;
        const double rkk = sqrt(fmax(piv, 1e-300));
        const double inv = 1.0 / rkk;
        const double rkj = (j > k) ? a[k] * inv : (j == k ? rkk : 0.0);
        const double bk = bm[k] * inv;
        // row k of R' and entry k of row j of R'^{-1} are final: stored now, their registers freed
        if (col && k < r) {
            R[k * r + j] = (k <= j) ? rkj * unscale : 0.0;
            Rinv[j * r + k] = (k >= j) ? sj * bk : 0.0;
        }
        row[j] = rkj;
        if (k + 1 < RMAX) {
            const double x = lane_value(rkj, k + 1);   // R'_{k,k+1}
            a[k + 1] = fma(-x, rkj, a[k + 1]);
            bm[k + 1] = fma(-x, bk, bm[k + 1]);
            piv = lane_value(a[k + 1], k + 1);
        }
#pragma unroll
        for (int i = k + 2; i < RMAX; ++i) {
            const double x = row[i];   // R'_{k,i}
            a[i] = fma(-x, rkj, a[i]);
            bm[i] = fma(-x, bk, bm[i]);
        }
    }
    const unsigned long long anybad = __ballot(bad);
    if (j == 0 && anybad) atomicOr(status, status_code);
}

// ---------------------------------------------------------------------------------------------- X = V Rinv
// X = V Rinv with Rinv upper triangular, on the matrix cores.  Per 16-cell tile a wavefront forms
// D = Rinv^T V^T (blocks of 16 output planes x 16 cells) with v_mfma_f64_16x16x4: Rinv^T stays in
// registers for the launch, V is read straight from memory as the B operand (four planes of 16
// consecutive cells per instruction; planes past r are clamped to a valid one that meets a zero of Rinv),
// and output block mb only takes the k-steps j <= 16 mb + 15 of the triangle.  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; its accumulator element v is D[4 v + l/16][l%16], so a store writes
// 16 consecutive cells of four planes.  V may be X (in place): a wavefront loads all rows of its tiles
// before it stores any, and the tiles of different wavefronts are disjoint.  Nothing is done when skip
// is given and set.  With GEN the matrix is a general rin x rout one (row-major, leading dimension
// ldm) and every k-step of every output block is taken; otherwise rin = rout = ldm = r.
typedef double dv4 __attribute__((ext_vector_type(4)));

template <typename TV, int RMAX, int T, bool GEN = false>
__global__ __launch_bounds__(kBlock) void k_trmm_mfma(int n, int r, const TV* V, size_t ldv,
                                                      const double* __restrict__ Rinv, double* X,
                                                      const int* __restrict__ skip, int rout = 0, int ldm = 0) {
    static_assert(RMAX % 16 == 0, "16-plane blocks");
    if (skip && *skip) return;
    constexpr int NB = RMAX / 16, KS = RMAX / 4;
    if (!GEN) rout = r, ldm = r;
    const int lane = threadIdx.x & 63, c = lane & 15, kr = lane >> 4;
    double A[NB][KS];
#pragma unroll
    for (int mb = 0; mb < NB; ++mb)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int j = 4 * ks + kr, k = 16 * mb + c;
            const bool in = GEN ? (j < r && k < rout) : (ks <= 4 * mb + 3 && j <= k && k < r);
            A[mb][ks] = in ? Rinv[j * ldm + k] : 0.0;
        }
    const long tiles = ((long)n + 15) / 16;
    const long wave = ((long)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const long nwaves = (long)gridDim.x * (kBlock / 64);
    for (long t0 = wave * T; t0 < tiles; t0 += nwaves * T) {
        double xb[T][KS];
        long e[T];
#pragma unroll
        for (int u = 0; u < T; ++u) {
            e[u] = min((t0 + u) * 16 + c, (long)n - 1);
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) xb[u][ks] = (double)V[(size_t)min(4 * ks + kr, r - 1) * ldv + e[u]];
        }
#pragma unroll
        for (int u = 0; u < T; ++u) {
            dv4 acc[NB];
#pragma unroll
            for (int mb = 0; mb < NB; ++mb) {
                acc[mb] = dv4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ks = 0; ks < KS; ++ks)
                    if (GEN || ks <= 4 * mb + 3)
                        acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[mb][ks], xb[u][ks], acc[mb], 0, 0, 0);
            }
            if ((t0 + u) * 16 + c < n) {
#pragma unroll
                for (int mb = 0; mb < NB; ++mb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int k = 16 * mb + 4 * v + kr;
                        if (k < rout) X[(size_t)k * n + e[u]] = acc[mb][v];
                    }
            }
        }
    }
}

template <typename TV>
void launch_trmm_any(hipStream_t s, int n, int r, const TV* V, size_t ldv, const double* Rinv, double* X,
                     const int* skip) {
    const long tiles = ((long)n + 15) / 16;
    const dim3 b(kBlock);
    auto grid = [&](int t) { return dim3((unsigned)std::min<long>((tiles + 4 * t - 1) / (4 * t), 2048)); };
    if (r <= 16)
        hipLaunchKernelGGL((k_trmm_mfma<TV, 16, 2>), grid(2), b, 0, s, n, r, V, ldv, Rinv, X, skip);
    else if (r <= 32)
        hipLaunchKernelGGL((k_trmm_mfma<TV, 32, 2>), grid(2), b, 0, s, n, r, V, ldv, Rinv, X, skip);
    else
        hipLaunchKernelGGL((k_trmm_mfma<TV, 64, 1>), grid(1), b, 0, s, n, r, V, ldv, Rinv, X, skip);
}

// ops layout: Axp, Axm, Ayp, Aym, Mt, Ms, G (r x r each), qX[r], b[4][r]
//   A_x^+ = <X, D_x^+ X> = (I - M0)/hx   (X orthonormal), A_x^- = (I - M0^T)/hx, same for y;
//   M_t = <X, sigma X> + I/(c dt);  G = S0^T P with P_ik = <X0_i, X_k> (old solution onto new X)
__global__ __launch_bounds__(kBlock) void k_project_ops(int r, int r0, const double* __restrict__ raw, double hx,
                                                        double hy, double inv_cdt, const double* __restrict__ S0,
                                                        double* __restrict__ ops) {
    __shared__ double sM4[kMaxRank * kMaxRank];
    __shared__ double sS[kMaxRank * kMaxRank];
    const int rr = r * r;
    stage_lds(sM4, raw + 4 * rr, rr);
    stage_lds(sS, S0, r0 * r0);
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
        double g = 0.0;   // S0 is r0 x r0; rows of G past r0 stay zero
        if (i < r0)
            for (int m = 0; m < r0; ++m) g += sS[m * r0 + i] * sM4[m * r + j];
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
                 int* near_identity, double identity_tol, bool identity_on_flag) {
    const int f = identity_on_flag ? 1 : 0;
    if (r <= 8)
        hipLaunchKernelGGL(k_chol<8>, dim3(1), dim3(64), 0, s, r, G, R, Rinv, status, status_code, near_identity,
                           identity_tol, f);
    else if (r <= 16)
        hipLaunchKernelGGL(k_chol<16>, dim3(1), dim3(64), 0, s, r, G, R, Rinv, status, status_code, near_identity,
                           identity_tol, f);
    else if (r <= 32)
        hipLaunchKernelGGL(k_chol<32>, dim3(1), dim3(64), 0, s, r, G, R, Rinv, status, status_code, near_identity,
                           identity_tol, f);
    else
        hipLaunchKernelGGL(k_chol<64>, dim3(1), dim3(64), 0, s, r, G, R, Rinv, status, status_code, near_identity,
                           identity_tol, f);
}

void launch_trmm_inplace(hipStream_t s, int n, int r, double* X, const double* Rinv, const int* skip) {
    launch_trmm_any<double>(s, n, r, X, (size_t)n, Rinv, X, skip);
}

template <typename TV>
void launch_trmm(hipStream_t s, int n, int r, const TV* V, size_t ldv, const double* Rinv, double* X) {
    launch_trmm_any<TV>(s, n, r, V, ldv, Rinv, X, nullptr);
}

void launch_gemm_tall(hipStream_t s, int n, int rin, int rout, const double* V, const double* M, int ldm,
                      double* X) {
    const long tiles = ((long)n + 15) / 16;
    const dim3 b(kBlock), g((unsigned)std::min<long>((tiles + 3) / 4, 2048));
    if (rin <= 32)
        hipLaunchKernelGGL((k_trmm_mfma<double, 32, 1, true>), g, b, 0, s, n, rin, V, (size_t)n, M, X, nullptr,
                           rout, ldm);
    else
        hipLaunchKernelGGL((k_trmm_mfma<double, 64, 1, true>), g, b, 0, s, n, rin, V, (size_t)n, M, X, nullptr,
                           rout, ldm);
}
template void launch_trmm<double>(hipStream_t, int, int, const double*, size_t, const double*, double*);
template void launch_trmm<float>(hipStream_t, int, int, const float*, size_t, const double*, double*);

__global__ __launch_bounds__(kBlock) void k_small_matmul(int r, const double* __restrict__ A,
                                                         const double* __restrict__ B, double* __restrict__ C,
                                                         int b_transposed) {
    __shared__ double sA[kMaxRank * kMaxRank], sB[kMaxRank * kMaxRank];
    stage_lds(sA, A, r * r);
    stage_lds(sB, B, r * r);
    __syncthreads();
    // B[k][j] is sB[k * r + j], or sB[j * r + k] when B^T is wanted
    const int bk = b_transposed ? 1 : r, bj = b_transposed ? r : 1;
    for (int o = threadIdx.x; o < r * r; o += blockDim.x) {
        const int i = o / r, j = o % r;
        double s = 0.0;
        for (int k = 0; k < r; ++k) s += sA[i * r + k] * sB[k * bk + j * bj];
        C[o] = s;
    }
}

void launch_small_matmul(hipStream_t s, int r, const double* A, const double* B, double* C, bool b_transposed) {
    hipLaunchKernelGGL(k_small_matmul, dim3(1), dim3(kBlock), 0, s, r, A, B, C, b_transposed ? 1 : 0);
}


// Raw projection sums taken on a basis Xq whose orthonormal form is X = Xq T (T = R^{-1} of a Cholesky
// QR pass, r x r): the matrices with X on both sides become T^T M T, <X0, X> becomes M4 T and the
// vectors T^T v.  Block b < 5 transforms matrix b, block 5 the five vectors (in place).
__global__ __launch_bounds__(kBlock) void k_project_rotate(int r, const double* __restrict__ T,
                                                           double* __restrict__ raw) {
    __shared__ double sT[kMaxRank * kMaxRank], sM[kMaxRank * kMaxRank], sP[kMaxRank * kMaxRank];
    const int rr = r * r, b = blockIdx.x;
    stage_lds(sT, T, rr);
    if (b < 5)
        stage_lds(sM, raw + (size_t)b * rr, rr);
    else
        stage_lds(sM, raw + 5 * (size_t)rr, 5 * r);
    __syncthreads();
    if (b < 5) {
        for (int o = threadIdx.x; o < rr; o += kBlock) {   // sP = M T
            const int i = o / r, j = o % r;
            double acc = 0.0;
            for (int k = 0; k < r; ++k) acc = fma(sM[i * r + k], sT[k * r + j], acc);
            sP[o] = acc;
        }
        __syncthreads();
        for (int o = threadIdx.x; o < rr; o += kBlock) {
            double v = sP[o];
            if (b != 4) {   // T^T (M T)
                const int i = o / r, j = o % r;
                double acc = 0.0;
                for (int k = 0; k < r; ++k) acc = fma(sT[k * r + i], sP[k * r + j], acc);
                v = acc;
            }
            raw[(size_t)b * rr + o] = v;
        }
    } else {
        for (int o = threadIdx.x; o < 5 * r; o += kBlock) {
            const int kind = o / r, i = o % r;
            double acc = 0.0;
            for (int k = 0; k < r; ++k) acc = fma(sT[k * r + i], sM[kind * r + k], acc);
            raw[5 * (size_t)rr + o] = acc;
        }
    }
}

void launch_project_finalize(hipStream_t s, int r, const double* partials, int nblocks, double hx, double hy,
                             double inv_cdt, const double* S0, double* ops, int r0, const double* T) {
    if (r0 < 0) r0 = r;
    // raw sums go into the tail of ops (beyond the operator block) as scratch
    const int rr = r * r;
    double* raw = ops + 7 * rr + 5 * r;
    const double area = hx * hy;
    launch_project_sum(s, r, partials, nblocks, area, raw);
    if (T) hipLaunchKernelGGL(k_project_rotate, dim3(6), dim3(kBlock), 0, s, r, T, raw);
    hipLaunchKernelGGL(k_project_ops, dim3(1), dim3(kBlock), 0, s, r, r0, raw, hx, hy, inv_cdt, S0, ops);
}

}  // namespace dlr
