// Small dense FP64 stages of the DLR step:
//  * DEIM interpolation points on the angular basis (Sec. 4.2), computed as the
//    row pivots of Gaussian elimination with partial pivoting on W -- after j
//    elimination steps column j of the Schur complement is exactly the DEIM
//    residual of W_j against W_1..W_{j-1} at the chosen points -- with the
//    smallest-index rule for near ties;
//  * the DEIM quadrature weights c = What^{-T} beta (Sec. 4.1);
//  * the L-step (eq. "L step"): for every ordinate the r x r block
//    B_q = |mu| A_x + |eta| A_y + M_t is inverted by Gauss-Jordan, the isotropic
//    coupling is removed with the Schur complement (I - Cbar M_s / 4 pi) Lbar = zeta,
//    Cbar = sum w_q B_q^{-1}, zeta = sum w_q B_q^{-1} Q_q, and L_q = B_q^{-1} (M_s Lbar / 4 pi + Q_q);
//  * a one-sided (Hestenes) Jacobi SVD of the r x r coupling matrix.
#include "dlr_internal.h"

namespace dlr {

namespace {

// ---------------------------------------------------------------------------------------------- block reductions
template <int NT>
__device__ double block_max(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] = fmax(sh[t], sh[t + w]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

template <int NT>
__device__ int block_min_int(int v, int* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] = min(sh[t], sh[t + w]);
        __syncthreads();
    }
    const int r = sh[0];
    __syncthreads();
    return r;
}

constexpr int kDeimThreads = 1024;
constexpr int kMaxOrdinates = 16384;

// ---------------------------------------------------------------------------------------------- DEIM
__global__ __launch_bounds__(kDeimThreads) void k_deim(DeimArgs a) {
    __shared__ double shd[kDeimThreads];
    __shared__ int shi[kDeimThreads];
    __shared__ unsigned char piv[kMaxOrdinates];
    __shared__ double beta[kMaxRank];
    __shared__ double M[kMaxRank * (kMaxRank + 1)];
    __shared__ int sel[kMaxRank];
    __shared__ int bad;
    const int nq = a.nq, r = a.r, tid = threadIdx.x;
    const double* __restrict__ W = a.W;
    double* __restrict__ U = a.work;
    if (tid == 0) bad = 0;
    for (int q = tid; q < nq; q += kDeimThreads) piv[q] = 0;
    for (int i = tid; i < r * nq; i += kDeimThreads) U[i] = W[i];
    // beta_j = int W_j = sum_q w_q W_j(q)
    for (int j = 0; j < r; ++j) {
        double acc = 0.0;
        for (int q = tid; q < nq; q += kDeimThreads) acc += a.w[q] * W[(size_t)j * nq + q];
        shd[tid] = acc;
        __syncthreads();
        for (int w = kDeimThreads / 2; w > 0; w >>= 1) {
            if (tid < w) shd[tid] += shd[tid + w];
            __syncthreads();
        }
        if (tid == 0) beta[j] = shd[0];
        __syncthreads();
    }
    for (int j = 0; j < r; ++j) {
        const double* col = U + (size_t)j * nq;
        double m = 0.0;
        for (int q = tid; q < nq; q += kDeimThreads)
            if (!piv[q]) m = fmax(m, fabs(col[q]));
        m = block_max<kDeimThreads>(m, shd);
        const double thr = (1.0 - a.tie_tol) * m;
        int p = 0x7fffffff;
        double second = 0.0;
        for (int q = tid; q < nq; q += kDeimThreads) {
            if (piv[q]) continue;
            const double v = fabs(col[q]);
            if (v >= thr) p = min(p, q);
            else second = fmax(second, v);
        }
        p = block_min_int<kDeimThreads>(p, shi);
        second = block_max<kDeimThreads>(second, shd);
        if (a.forced) {
            const int f = a.forced[j];
            if (tid == 0 && (f < 0 || f >= nq || piv[f])) bad = 1;
            p = (f >= 0 && f < nq) ? f : 0;
        }
        if (tid == 0) {
            sel[j] = p;
            piv[p] = 1;
            a.margins[j] = (m > 0.0) ? (m - second) / m : 0.0;
            if (!(m > 0.0)) bad = 1;
        }
        __syncthreads();
        // eliminate column j from the remaining rows, columns k > j
        const double pv = col[p];
        for (int q = tid; q < nq; q += kDeimThreads) {
            if (piv[q]) continue;
            const double l = col[q] / pv;
            for (int k = j + 1; k < r; ++k) U[(size_t)k * nq + q] -= l * U[(size_t)k * nq + p];
        }
        __syncthreads();
    }
    // c = What^{-T} beta: solve M c = beta with M[i][j] = What[j][i] = W_i(Omega^(j))
    const int ld = r + 1;
    for (int o = tid; o < r * r; o += kDeimThreads) {
        const int i = o / r, j = o % r;
        M[i * ld + j] = W[(size_t)i * nq + sel[j]];
    }
    for (int i = tid; i < r; i += kDeimThreads) M[i * ld + r] = beta[i];
    __syncthreads();
    for (int k = 0; k < r; ++k) {
        if (tid == 0) {
            int pr = k;
            double best = fabs(M[k * ld + k]);
            for (int i = k + 1; i < r; ++i)
                if (fabs(M[i * ld + k]) > best) { best = fabs(M[i * ld + k]); pr = i; }
            shi[0] = pr;
            if (!(best > 0.0)) bad = 1;
        }
        __syncthreads();
        const int pr = shi[0];
        if (pr != k)
            for (int c = tid; c <= r; c += kDeimThreads) {
                const double t = M[k * ld + c];
                M[k * ld + c] = M[pr * ld + c];
                M[pr * ld + c] = t;
            }
        __syncthreads();
        const double inv = 1.0 / M[k * ld + k];
        for (int i = tid; i < r; i += kDeimThreads) shd[i] = (i == k) ? 0.0 : M[i * ld + k] * inv;
        __syncthreads();
        for (int o = tid; o < r * ld; o += kDeimThreads) {
            const int i = o / ld, c = o % ld;
            if (i != k) M[o] -= shd[i] * M[k * ld + c];
        }
        __syncthreads();
    }
    for (int i = tid; i < r; i += kDeimThreads) {
        const int d = i;
        a.cw[i] = M[i * ld + r] / M[i * ld + i];
        a.sel[d] = sel[d];
        const double mu = a.mu[sel[d]], eta = a.eta[sel[d]];
        a.sel_mu[d] = mu;
        a.sel_eta[d] = eta;
        a.inflow_x[d] = a.psib[mu > 0.0 ? 0 : 1];
        a.inflow_y[d] = a.psib[eta > 0.0 ? 2 : 3];
        double s = 0.0;
        for (int j = 0; j < r; ++j) s += a.S[i * r + j] * beta[j];
        a.a0[i] = s;
    }
    // C0[k][d] = sum_j S[k][j] W_j(Omega^(d))
    for (int o = tid; o < r * r; o += kDeimThreads) {
        const int k = o / r, d = o % r;
        double s = 0.0;
        for (int j = 0; j < r; ++j) s += a.S[k * r + j] * W[(size_t)j * nq + sel[d]];
        a.C0[o] = s;
    }
    if (tid == 0 && bad) atomicOr(a.status, a.forced ? (int)kStatusBadForcedSel : (int)kStatusSingularSolve);
}

// ---------------------------------------------------------------------------------------------- Gauss-Jordan
// In-place Gauss-Jordan with partial pivoting on an r x ld augmented matrix in LDS
// (first r columns = the matrix); afterwards columns r.. hold the solutions.
__device__ void gauss_jordan(double* Aug, int r, int ld, double* fac, int* pivrow, int* bad) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int k = 0; k < r; ++k) {
        if (tid == 0) {
            int pr = k;
            double best = fabs(Aug[k * ld + k]);
            for (int i = k + 1; i < r; ++i)
                if (fabs(Aug[i * ld + k]) > best) { best = fabs(Aug[i * ld + k]); pr = i; }
            *pivrow = pr;
            if (!(best > 0.0) || !isfinite(best)) *bad = 1;
        }
        __syncthreads();
        const int pr = *pivrow;
        if (pr != k)
            for (int c = tid; c < ld; c += nt) {
                const double t = Aug[k * ld + c];
                Aug[k * ld + c] = Aug[pr * ld + c];
                Aug[pr * ld + c] = t;
            }
        __syncthreads();
        const double inv = 1.0 / Aug[k * ld + k];
        __syncthreads();
        for (int c = tid; c < ld; c += nt) Aug[k * ld + c] *= inv;
        for (int i = tid; i < r; i += nt) fac[i] = (i == k) ? 0.0 : Aug[i * ld + k];
        __syncthreads();
        for (int o = tid; o < r * ld; o += nt) {
            const int i = o / ld, c = o % ld;
            if (i != k) Aug[o] -= fac[i] * Aug[k * ld + c];
        }
        __syncthreads();
    }
}

constexpr int kLsThreads = 256;

// per ordinate: B_q^{-1} and y_q = B_q^{-1} Q_q
__global__ __launch_bounds__(kLsThreads) void k_lstep_solve(LstepArgs a) {
    extern __shared__ double dyn[];
    __shared__ double fac[kMaxRank];
    __shared__ int pivrow, bad;
    const int r = a.r, rr = r * r, q = blockIdx.x, tid = threadIdx.x;
    const int ld = 2 * r + 1;
    double* Aug = dyn;
    const double mu = a.mu[q], eta = a.eta[q];
    const double* Ax = a.ops + (mu > 0.0 ? 0 : 1) * rr;
    const double* Ay = a.ops + (eta > 0.0 ? 2 : 3) * rr;
    const double* Mt = a.ops + 4 * rr;
    const double* G = a.ops + 6 * rr;
    const double* qX = a.ops + 7 * rr;
    const double* b = qX + r;
    const int sx = mu > 0.0 ? 0 : 1, sy = eta > 0.0 ? 2 : 3;
    const double amu = fabs(mu), aeta = fabs(eta);
    if (tid == 0) bad = 0;
    for (int o = tid; o < r * ld; o += kLsThreads) {
        const int i = o / ld, c = o % ld;
        double v;
        if (c < r) {
            v = amu * Ax[i * r + c] + aeta * Ay[i * r + c] + Mt[i * r + c];
        } else if (c < 2 * r) {
            v = (c - r == i) ? 1.0 : 0.0;
        } else {
            double lt = 0.0;   // old solution projected on the new basis: sum_j W0_j(q) G[j][i]
            for (int j = 0; j < r; ++j) lt += a.W0[(size_t)j * a.nq + q] * G[j * r + i];
            v = qX[i] + lt * a.inv_cdt + amu * a.psib[sx] * b[(sx - 0) * r + i] + aeta * a.psib[sy] * b[sy * r + i];
        }
        Aug[o] = v;
    }
    __syncthreads();
    gauss_jordan(Aug, r, ld, fac, &pivrow, &bad);
    double* Bi = a.Binv + (size_t)q * rr;
    for (int o = tid; o < rr; o += kLsThreads) Bi[o] = Aug[(o / r) * ld + r + (o % r)];
    for (int i = tid; i < r; i += kLsThreads) a.y[(size_t)q * r + i] = Aug[i * ld + 2 * r];
    if (tid == 0 && bad) atomicOr(a.status, (int)kStatusSingularSolve);
}

// partial sums over a contiguous range of ordinates of w_q B_q^{-1} and w_q y_q
__global__ __launch_bounds__(kLsThreads) void k_lstep_reduce(LstepArgs a) {
    const int r = a.r, rr = r * r, tot = rr + r;
    const int per = (a.nq + gridDim.x - 1) / gridDim.x;
    const int q0 = blockIdx.x * per, q1 = min(a.nq, q0 + per);
    for (int o = threadIdx.x; o < tot; o += kLsThreads) {
        double acc = 0.0;
        if (o < rr)
            for (int q = q0; q < q1; ++q) acc += a.w[q] * a.Binv[(size_t)q * rr + o];
        else
            for (int q = q0; q < q1; ++q) acc += a.w[q] * a.y[(size_t)q * r + (o - rr)];
        a.red_partials[(size_t)blockIdx.x * tot + o] = acc;
    }
}

// (I - Cbar M_s / 4 pi) Lbar = zeta ; v = M_s Lbar / (4 pi)
__global__ __launch_bounds__(kLsThreads) void k_lstep_schur(LstepArgs a) {
    extern __shared__ double dyn[];
    __shared__ double fac[kMaxRank];
    __shared__ double Cb[kMaxRank * kMaxRank];
    __shared__ int pivrow, bad;
    const int r = a.r, rr = r * r, tot = rr + r, ld = r + 1, tid = threadIdx.x;
    const double* Ms = a.ops + 5 * rr;
    double* Aug = dyn;
    if (tid == 0) bad = 0;
    for (int o = tid; o < tot; o += kLsThreads) {
        double acc = 0.0;
        for (int b = 0; b < a.red_blocks; ++b) acc += a.red_partials[(size_t)b * tot + o];
        if (o < rr) Cb[o] = acc;
        else Aug[(o - rr) * ld + r] = acc;
    }
    __syncthreads();
    for (int o = tid; o < rr; o += kLsThreads) {
        const int i = o / r, j = o % r;
        double s = 0.0;
        for (int k = 0; k < r; ++k) s += Cb[i * r + k] * Ms[k * r + j];
        Aug[i * ld + j] = ((i == j) ? 1.0 : 0.0) - s / kFourPi;
    }
    __syncthreads();
    gauss_jordan(Aug, r, ld, fac, &pivrow, &bad);
    for (int i = tid; i < r; i += kLsThreads) {
        double s = 0.0;
        for (int k = 0; k < r; ++k) s += Ms[i * r + k] * Aug[k * ld + r];
        a.v[i] = s / kFourPi;
    }
    if (tid == 0 && bad) atomicOr(a.status, (int)kStatusSingularSolve);
}

// L_q = B_q^{-1} v + y_q, stored column-major L[i][q]
__global__ __launch_bounds__(kLsThreads) void k_lstep_apply(LstepArgs a) {
    const int r = a.r, rr = r * r;
    const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (long)a.nq * r) return;
    const int q = (int)(o / r), i = (int)(o % r);
    const double* Bi = a.Binv + (size_t)q * rr + (size_t)i * r;
    double s = a.y[(size_t)q * r + i];
    for (int j = 0; j < r; ++j) s += Bi[j] * a.v[j];
    a.L[(size_t)i * a.nq + q] = s;
}

// ---------------------------------------------------------------------------------------------- SVD
// S = R^T.  One-sided Jacobi: rotate column pairs of S (and of V = I) until
// every pair is orthogonal to working precision; then sort by column norm
// (descending), sign each V column so its largest-magnitude entry is positive,
// and return V and S' = S V (column k = U_k sigma_k).
constexpr int kSvdThreads = 1024;

__global__ __launch_bounds__(kSvdThreads) void k_svd(int r, const double* __restrict__ Rin,
                                                     double* __restrict__ Vout, double* __restrict__ Sout,
                                                     int* status) {
    __shared__ double S[kMaxRank * kMaxRank];
    __shared__ double V[kMaxRank * kMaxRank];
    __shared__ double rc[kMaxRank / 2 + 1], rs[kMaxRank / 2 + 1];
    __shared__ int pos[kMaxRank + 1];
    __shared__ double nrm[kMaxRank];
    __shared__ int order[kMaxRank];
    __shared__ int rotated;
    const int tid = threadIdx.x;
    const int rr = r * r;
    for (int o = tid; o < rr; o += kSvdThreads) {
        const int i = o / r, j = o % r;
        S[j * r + i] = Rin[o];
        V[o] = (i == j) ? 1.0 : 0.0;
    }
    const double tol = fmax(1e-15, r * 2.3e-16);
    const int re = r + (r & 1);   // even number of positions; position r (if any) is a dummy
    const int np = re / 2;
    const int G = (r <= 32) ? 32 : 64;   // lanes per pair (rows handled per lane: ceil(r / G))
    __syncthreads();
    int sweep = 0;
    for (; sweep < 40; ++sweep) {
        if (tid == 0) rotated = 0;
        for (int i = tid; i < re; i += kSvdThreads) pos[i] = i;
        __syncthreads();
        for (int round = 0; round < re - 1; ++round) {
            // pairs (pos[k], pos[re-1-k]); pair k handled by lanes [k*G, k*G+G)
            for (int base = 0; base < np * G; base += kSvdThreads) {
                const int t = base + tid;
                const int k = t / G, lane = t % G;
                double al = 0.0, be = 0.0, ga = 0.0;
                int p = -1, qq = -1;
                if (k < np) {
                    p = pos[k];
                    qq = pos[re - 1 - k];
                    if (p < r && qq < r)
                        for (int i = lane; i < r; i += G) {
                            const double sp = S[i * r + p], sq = S[i * r + qq];
                            al += sp * sp;
                            be += sq * sq;
                            ga += sp * sq;
                        }
                }
                for (int off = G / 2; off > 0; off >>= 1) {
                    al += __shfl_xor(al, off, G);
                    be += __shfl_xor(be, off, G);
                    ga += __shfl_xor(ga, off, G);
                }
                if (k < np && lane == 0) {
                    double c = 1.0, s = 0.0;
                    if (p < r && qq < r && ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
                        const double zeta = (be - al) / (2.0 * ga);
                        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                        c = 1.0 / sqrt(1.0 + tt * tt);
                        s = c * tt;
                        rotated = 1;
                    }
                    rc[k] = c;
                    rs[k] = s;
                }
            }
            __syncthreads();
            for (int o = tid; o < np * r; o += kSvdThreads) {
                const int k = o / r, i = o % r;
                const int p = pos[k], qq = pos[re - 1 - k];
                if (p < r && qq < r && rs[k] != 0.0) {
                    const double c = rc[k], s = rs[k];
                    const double sp = S[i * r + p], sq = S[i * r + qq];
                    S[i * r + p] = c * sp - s * sq;
                    S[i * r + qq] = s * sp + c * sq;
                    const double vp = V[i * r + p], vq = V[i * r + qq];
                    V[i * r + p] = c * vp - s * vq;
                    V[i * r + qq] = s * vp + c * vq;
                }
            }
            __syncthreads();
            // round-robin rotation of positions 1..re-1
            if (tid == 0) {
                const int last = pos[re - 1];
                for (int i = re - 1; i > 1; --i) pos[i] = pos[i - 1];
                pos[1] = last;
            }
            __syncthreads();
        }
        const int rot = rotated;
        __syncthreads();
        if (!rot) break;
    }
    if (tid == 0 && sweep >= 40) atomicOr(status, (int)kStatusSvdNoConv);
    for (int k = tid; k < r; k += kSvdThreads) {
        double s = 0.0;
        for (int i = 0; i < r; ++i) s += S[i * r + k] * S[i * r + k];
        nrm[k] = sqrt(s);
    }
    __syncthreads();
    if (tid == 0) {   // stable selection sort, descending
        for (int k = 0; k < r; ++k) order[k] = k;
        for (int k = 0; k < r; ++k) {
            int best = k;
            for (int m = k + 1; m < r; ++m)
                if (nrm[order[m]] > nrm[order[best]]) best = m;
            const int t = order[best];
            for (int m = best; m > k; --m) order[m] = order[m - 1];
            order[k] = t;
        }
    }
    __syncthreads();
    for (int k = tid; k < r; k += kSvdThreads) {
        const int src = order[k];
        int m = 0;
        double best = -1.0;
        for (int i = 0; i < r; ++i)
            if (fabs(V[i * r + src]) > best) { best = fabs(V[i * r + src]); m = i; }
        const double sg = (V[m * r + src] < 0.0) ? -1.0 : 1.0;
        for (int i = 0; i < r; ++i) {
            Vout[i * r + k] = sg * V[i * r + src];
            Sout[i * r + k] = sg * S[i * r + src];
        }
    }
}

// X[k][c] = sum_j V[j][c] M[j][k]
__global__ __launch_bounds__(256) void k_rmul(int n, int r, const double* __restrict__ V, const double* __restrict__ M,
                                              double* __restrict__ X) {
    __shared__ double sM[kMaxRank * kMaxRank];
    for (int o = threadIdx.x; o < r * r; o += blockDim.x) sM[o] = M[o];
    __syncthreads();
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double v[kMaxRank];
    for (int j = 0; j < r; ++j) v[j] = V[(size_t)j * n + c];
    for (int k = 0; k < r; ++k) {
        double s = 0.0;
        for (int j = 0; j < r; ++j) s += v[j] * sM[j * r + k];
        X[(size_t)k * n + c] = s;
    }
}

// beta_k = sum_q w_q W_k(q), coef = S beta
__global__ __launch_bounds__(256) void k_wsum(int nq, int r, const double* __restrict__ W,
                                              const double* __restrict__ w, const double* __restrict__ S,
                                              double* __restrict__ beta, double* __restrict__ coef) {
    __shared__ double sh[256];
    __shared__ double sb[kMaxRank];
    for (int k = 0; k < r; ++k) {
        double acc = 0.0;
        for (int q = threadIdx.x; q < nq; q += 256) acc += w[q] * W[(size_t)k * nq + q];
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) sb[k] = sh[0];
        __syncthreads();
    }
    for (int i = threadIdx.x; i < r; i += 256) {
        beta[i] = sb[i];
        double s = 0.0;
        for (int j = 0; j < r; ++j) s += S[i * r + j] * sb[j];
        coef[i] = s;
    }
}

}  // namespace

void launch_deim(hipStream_t s, const DeimArgs& a) {
    hipLaunchKernelGGL(k_deim, dim3(1), dim3(kDeimThreads), 0, s, a);
}

void launch_lstep(hipStream_t s, const LstepArgs& a) {
    const int r = a.r;
    const size_t solve_lds = (size_t)r * (2 * r + 1) * sizeof(double);
    const size_t schur_lds = (size_t)r * (r + 1) * sizeof(double);
    if (solve_lds > 64 * 1024)
        (void)hipFuncSetAttribute((const void*)k_lstep_solve, hipFuncAttributeMaxDynamicSharedMemorySize, (int)solve_lds);
    hipLaunchKernelGGL(k_lstep_solve, dim3(a.nq), dim3(kLsThreads), solve_lds, s, a);
    hipLaunchKernelGGL(k_lstep_reduce, dim3(a.red_blocks), dim3(kLsThreads), 0, s, a);
    hipLaunchKernelGGL(k_lstep_schur, dim3(1), dim3(kLsThreads), schur_lds, s, a);
    const long tot = (long)a.nq * r;
    hipLaunchKernelGGL(k_lstep_apply, dim3((unsigned)((tot + kLsThreads - 1) / kLsThreads)), dim3(kLsThreads), 0, s, a);
}

void launch_svd(hipStream_t s, int r, const double* R, double* V, double* Snew, int* status) {
    hipLaunchKernelGGL(k_svd, dim3(1), dim3(kSvdThreads), 0, s, r, R, V, Snew, status);
}

void launch_rmul(hipStream_t s, int n, int r, const double* V, const double* M, double* X) {
    hipLaunchKernelGGL(k_rmul, dim3((n + 255) / 256), dim3(256), 0, s, n, r, V, M, X);
}

void launch_wsum(hipStream_t s, int nq, int r, const double* W, const double* w, const double* S, double* beta,
                 double* coef) {
    hipLaunchKernelGGL(k_wsum, dim3(1), dim3(256), 0, s, nq, r, W, w, S, beta, coef);
}

}  // namespace dlr
