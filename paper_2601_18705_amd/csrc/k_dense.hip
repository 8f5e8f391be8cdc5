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
constexpr int kDeimThreads = 1024;
constexpr int kDeimWaves = kDeimThreads / 64;
constexpr int kMaxOrdinates = 16384;

// Reductions over the workgroup: wavefront shuffles, one slot per wavefront in LDS, one barrier;
// every thread then combines the slots in wavefront order, so all threads hold the same result.
__device__ double block_max1(double v, double* slots) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    if ((threadIdx.x & 63) == 0) slots[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = slots[0];
    for (int w = 1; w < kDeimWaves; ++w) m = fmax(m, slots[w]);
    return m;
}
__device__ void block_minidx_max(int& p, double& v, int* islots, double* dslots) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        p = min(p, __shfl_xor(p, off));
        v = fmax(v, __shfl_xor(v, off));
    }
    if ((threadIdx.x & 63) == 0) {
        islots[threadIdx.x >> 6] = p;
        dslots[threadIdx.x >> 6] = v;
    }
    __syncthreads();
    p = islots[0];
    v = dslots[0];
    for (int w = 1; w < kDeimWaves; ++w) {
        p = min(p, islots[w]);
        v = fmax(v, dslots[w]);
    }
}

// ---------------------------------------------------------------------------------------------- DEIM
__global__ __launch_bounds__(kDeimThreads) void k_deim(DeimArgs a) {
    __shared__ double shd[kDeimThreads];
    __shared__ int shi[kDeimThreads];
    __shared__ double slotA[kDeimWaves], slotB[kDeimWaves];
    __shared__ int islot[kDeimWaves];
    __shared__ unsigned char piv[kMaxOrdinates];
    __shared__ double beta[kMaxRank];
    __shared__ double M[kMaxRank * (kMaxRank + 1)];
    __shared__ int sel[kMaxRank];
    __shared__ int bad;
    const int nq = a.nq, r = a.r, tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const double* __restrict__ W = a.W;
    double* __restrict__ U = a.work;
    if (tid == 0) bad = 0;
    for (int q = tid; q < nq; q += kDeimThreads) piv[q] = 0;
#pragma unroll 8
    for (int i = tid; i < r * nq; i += kDeimThreads) U[i] = W[i];
    // beta_j = int W_j = sum_q w_q W_j(q): wavefront j % 16 sums column j in lane order
    for (int j = wv; j < r; j += kDeimWaves) {
        double acc = 0.0;
#pragma unroll 8
        for (int q = lane; q < nq; q += 64) acc += a.w[q] * W[(size_t)j * nq + q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) beta[j] = acc;
    }
    __syncthreads();
    for (int j = 0; j < r; ++j) {
        const double* col = U + (size_t)j * nq;
        double m = 0.0;
        for (int q = tid; q < nq; q += kDeimThreads)
            if (!piv[q]) m = fmax(m, fabs(col[q]));
        m = block_max1(m, slotA);   // also orders the previous elimination before these reads
        const double thr = (1.0 - a.tie_tol) * m;
        int p = 0x7fffffff;
        double second = 0.0;
        for (int q = tid; q < nq; q += kDeimThreads) {
            if (piv[q]) continue;
            const double v = fabs(col[q]);
            if (v >= thr) p = min(p, q);
            else second = fmax(second, v);
        }
        block_minidx_max(p, second, islot, slotB);
        if (a.forced) {
            const int f = a.forced[j];
            if (tid == 0 && (f < 0 || f >= nq || piv[f])) bad = 1;
            p = (f >= 0 && f < nq) ? f : 0;
        }
        if (tid == 0) {
            sel[j] = p;
            a.margins[j] = (m > 0.0) ? (m - second) / m : 0.0;
            if (!(m > 0.0)) bad = 1;
        }
        // the owner of row p marks it; every thread only tests the rows it owns
        if (p % kDeimThreads == tid) piv[p] = 1;
        // eliminate column j from the remaining rows, columns k > j, eight columns at a time so the
        // loads of a batch are in flight together
        const double pv = col[p];
        for (int k0 = j + 1; k0 < r; k0 += 8) {
            double up[8];
#pragma unroll
            for (int b = 0; b < 8; ++b) up[b] = (k0 + b < r) ? U[(size_t)(k0 + b) * nq + p] : 0.0;
            for (int q = tid; q < nq; q += kDeimThreads) {
                if (piv[q]) continue;
                const double l = col[q] / pv;
                double x[8];
#pragma unroll
                for (int b = 0; b < 8; ++b) x[b] = (k0 + b < r) ? U[(size_t)(k0 + b) * nq + q] : 0.0;
#pragma unroll
                for (int b = 0; b < 8; ++b)
                    if (k0 + b < r) U[(size_t)(k0 + b) * nq + q] = x[b] - l * up[b];
            }
        }
    }
    __syncthreads();
    // c = What^{-T} beta: solve M c = beta with M[i][j] = What[j][i] = W_i(Omega^(j))
    const int ld = r + 1;
    __shared__ double sS[kMaxRank * kMaxRank];
    __shared__ double Wh[kMaxRank * kMaxRank];   // Wh[i][j] = W_i(Omega^(sel j))
    stage_lds(sS, a.S, r * r);
    for (int o = tid; o < r * r; o += kDeimThreads) {
        const int i = o / r, j = o % r;
        const double v = W[(size_t)i * nq + sel[j]];
        M[i * ld + j] = v;
        Wh[o] = v;
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
        for (int j = 0; j < r; ++j) s += sS[i * r + j] * beta[j];
        a.a0[i] = s;
    }
    // C0[k][d] = sum_j S[k][j] W_j(Omega^(d))
    for (int o = tid; o < r * r; o += kDeimThreads) {
        const int k = o / r, d = o % r;
        double s = 0.0;
        for (int j = 0; j < r; ++j) s += sS[k * r + j] * Wh[j * r + d];
        a.C0[o] = s;
    }
    if (tid == 0 && bad) atomicOr(a.status, a.forced ? (int)kStatusBadForcedSel : (int)kStatusSingularSolve);
}

// ---------------------------------------------------------------------------------------------- Gauss-Jordan
// In-place Gauss-Jordan with partial pivoting on an r x ld augmented matrix in LDS
// (first r columns = the matrix); afterwards columns r.. hold the solutions.  Per pivot k:
// wavefront 0 finds the pivot row (largest |A_ik|, i >= k, lowest index on ties); then the
// new row k (the pivot row scaled by 1/pivot) goes to prow while the old row k moves to the
// pivot row's place, and the factors of the other rows are read; then every other row is
// updated and row k written.  Three barriers per pivot; r <= 64.
__device__ void gauss_jordan(double* Aug, int r, int ld, double* fac, double* prow, int* pivrow, double* pivval,
                             int* bad) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int k = 0; k < r; ++k) {
        if (tid < 64) {
            const int i = k + tid;
            double v = (i < r) ? fabs(Aug[i * ld + k]) : -1.0;
            int idx = (i < r) ? i : 0x7fffffff;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(v, off);
                const int oi = __shfl_xor(idx, off);
                if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
            }
            if (tid == 0) {
                const int p = (idx < r) ? idx : k;
                *pivrow = p;
                *pivval = Aug[p * ld + k];
                if (!(v > 0.0) || !isfinite(v)) *bad = 1;
            }
        }
        __syncthreads();
        const int pr = *pivrow;
        const double inv = 1.0 / *pivval;   // read before this phase moves the old row k
        for (int c = tid; c < ld; c += nt) {
            const double ak = Aug[k * ld + c], ap = Aug[pr * ld + c];
            prow[c] = ap * inv;
            if (pr != k) Aug[pr * ld + c] = ak;
        }
        for (int i = tid; i < r; i += nt)
            fac[i] = (i == k) ? 0.0 : ((i == pr) ? Aug[k * ld + k] : Aug[i * ld + k]);
        __syncthreads();
        // rows by wavefront (i = wave + 4 a), columns by lane (c = lane + 64 b): no integer division
        {
            const int lane = tid & 63, wv = tid >> 6;
            const int nw = nt >> 6;
            double pv[3];   // ld <= 2 * 64 + 1 columns
#pragma unroll
            for (int b = 0; b < 3; ++b) pv[b] = prow[lane + 64 * b < ld ? lane + 64 * b : ld - 1];
            for (int i0 = wv; i0 < r; i0 += 4 * nw) {
                double x[12], f[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int i = i0 + a * nw;
                    f[a] = fac[i < r ? i : r - 1];
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const int c = lane + 64 * b;
                        x[a * 3 + b] = Aug[(i < r ? i : r - 1) * ld + (c < ld ? c : ld - 1)];
                    }
                }
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int i = i0 + a * nw;
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        const int c = lane + 64 * b;
                        if (i < r && c < ld) Aug[i * ld + c] = (i == k) ? pv[b] : x[a * 3 + b] - f[a] * pv[b];
                    }
                }
            }
        }
        __syncthreads();
    }
}

constexpr int kLsThreads = 256;

// per ordinate: B_q^{-1} and y_q = B_q^{-1} Q_q
__global__ __launch_bounds__(kLsThreads) void k_lstep_solve(LstepArgs a) {
    extern __shared__ double dyn[];
    __shared__ double fac[kMaxRank];
    __shared__ double prow[2 * kMaxRank + 1];
    __shared__ double pivval;
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
    double* sG = dyn + (size_t)r * ld;   // r x r after the augmented matrix
    __shared__ double sW0[kMaxRank];
    stage_lds(sG, G, rr);
    for (int j = tid; j < r; j += kLsThreads) sW0[j] = a.W0[(size_t)j * a.nq + q];
    __syncthreads();
    // rows by wavefront, columns by lane (ld <= 129)
    const int lane = tid & 63, wv = tid >> 6;
    constexpr int kLsWaves = kLsThreads / 64;
#pragma unroll 2
    for (int i = wv; i < r; i += kLsWaves) {
#pragma unroll
        for (int bc = 0; bc < 3; ++bc) {
            const int c = lane + 64 * bc;
            if (c >= ld) continue;
            double v;
            if (c < r) {
                v = amu * Ax[i * r + c] + aeta * Ay[i * r + c] + Mt[i * r + c];
            } else if (c < 2 * r) {
                v = (c - r == i) ? 1.0 : 0.0;
            } else {
                double lt = 0.0;   // old solution projected on the new basis: sum_j W0_j(q) G[j][i]
                for (int j = 0; j < r; ++j) lt += sW0[j] * sG[j * r + i];
                v = qX[i] + lt * a.inv_cdt + amu * a.psib[sx] * b[(sx - 0) * r + i] +
                    aeta * a.psib[sy] * b[sy * r + i];
            }
            Aug[i * ld + c] = v;
        }
    }
    __syncthreads();
    gauss_jordan(Aug, r, ld, fac, prow, &pivrow, &pivval, &bad);
    double* Bi = a.Binv + (size_t)q * rr;
    for (int i = wv; i < r; i += kLsWaves)
        if (lane < r) Bi[i * r + lane] = Aug[i * ld + r + lane];
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
        if (o < rr) {
#pragma unroll 8
            for (int q = q0; q < q1; ++q) acc += a.w[q] * a.Binv[(size_t)q * rr + o];
        } else {
#pragma unroll 8
            for (int q = q0; q < q1; ++q) acc += a.w[q] * a.y[(size_t)q * r + (o - rr)];
        }
        a.red_partials[(size_t)blockIdx.x * tot + o] = acc;
    }
}

// (I - Cbar M_s / 4 pi) Lbar = zeta ; v = M_s Lbar / (4 pi)
__global__ __launch_bounds__(kLsThreads) void k_lstep_schur(LstepArgs a) {
    extern __shared__ double dyn[];
    __shared__ double fac[kMaxRank];
    __shared__ double prow[kMaxRank + 1];
    __shared__ double pivval;
    __shared__ double Cb[kMaxRank * kMaxRank];
    __shared__ int pivrow, bad;
    const int r = a.r, rr = r * r, tot = rr + r, ld = r + 1, tid = threadIdx.x;
    const double* Ms = a.ops + 5 * rr;
    double* Aug = dyn;
    if (tid == 0) bad = 0;
    __shared__ double sMs[kMaxRank * kMaxRank];
    stage_lds(sMs, Ms, rr);
    for (int o = tid; o < tot; o += kLsThreads) {
        double acc = 0.0;
#pragma unroll 8
        for (int b = 0; b < a.red_blocks; ++b) acc += a.red_partials[(size_t)b * tot + o];
        if (o < rr) Cb[o] = acc;
        else Aug[(o - rr) * ld + r] = acc;
    }
    __syncthreads();
    for (int o = tid; o < rr; o += kLsThreads) {
        const int i = o / r, j = o % r;
        double s = 0.0;
        for (int k = 0; k < r; ++k) s += Cb[i * r + k] * sMs[k * r + j];
        Aug[i * ld + j] = ((i == j) ? 1.0 : 0.0) - s / kFourPi;
    }
    __syncthreads();
    gauss_jordan(Aug, r, ld, fac, prow, &pivrow, &pivval, &bad);
    for (int i = tid; i < r; i += kLsThreads) {
        double s = 0.0;
        for (int k = 0; k < r; ++k) s += sMs[i * r + k] * Aug[k * ld + r];
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
#pragma unroll 8
    for (int j = 0; j < r; ++j) s += Bi[j] * a.v[j];
    a.L[(size_t)i * a.nq + q] = s;
}

// ---------------------------------------------------------------------------------------------- SVD
// S = R^T.  One-sided Jacobi: rotate column pairs of S (and of V = I) until
// every pair is orthogonal to working precision; then sort by column norm
// (descending), sign each V column so its largest-magnitude entry is positive,
// and return V and S' = S V (column k = U_k sigma_k).
//
// Round-robin (circle) schedule: in round t slot 0 holds column 0 and slot i >= 1
// holds column 1 + (i - 1 + t) mod (re - 1); slots k and re-1-k form pair k.  The
// pairs of a round are disjoint, so the sixteen lanes of pair k compute its rotation
// from their own rows and apply it at once: one barrier per round.
constexpr int kSvdLanes = 16;   // lanes per column pair: one DPP row
constexpr int kSvdThreads = kSvdLanes * kMaxRank / 2;

// v moved across the lanes of a DPP row (ctrl: quad_perm, row_half_mirror, row_mirror)
template <int CTRL>
__device__ inline double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// sum over the 16 lanes of a DPP row, in every lane: swap neighbours, swap pairs, then add the
// mirrored half-row and the mirrored row
__device__ inline double row16_sum(double v) {
    v += dpp_move<0xB1>(v);    // quad_perm(1,0,3,2)
    v += dpp_move<0x4E>(v);    // quad_perm(2,3,0,1)
    v += dpp_move<0x141>(v);   // row_half_mirror
    v += dpp_move<0x140>(v);   // row_mirror
    return v;
}

__global__ __launch_bounds__(kSvdThreads) void k_svd(int r, const double* __restrict__ Rin,
                                                     double* __restrict__ Vout, double* __restrict__ Sout,
                                                     int* status) {
    __shared__ double S[kMaxRank * kMaxRank];
    __shared__ double V[kMaxRank * kMaxRank];
    __shared__ double nrm[kMaxRank];
    __shared__ int order[kMaxRank];
    const int tid = threadIdx.x;
    const int rr = r * r;
    // column-major: column c of S = R^T is row c of R, S[c * r + i] = R[c][i]; the lanes of a pair
    // read consecutive rows of a column (no bank conflicts)
    for (int o = tid; o < rr; o += kSvdThreads) {
        const int c = o / r, i = o % r;
        S[o] = Rin[o];
        V[o] = (i == c) ? 1.0 : 0.0;
    }
    const double tol = fmax(1e-15, r * 2.3e-16);
    const int re = r + (r & 1);   // even number of slots; column r (if any) is a dummy
    const int np = re / 2;
    const int k = tid / kSvdLanes, lane = tid % kSvdLanes;
    __syncthreads();
    int sweep = 0;
    bool converged = false;
    for (; sweep < 40 && !converged; ++sweep) {
        int rotated = 0;
        for (int round = 0; round < re - 1; ++round) {
            if (k < np) {
                const int sa = k, sb = re - 1 - k;
                // (x + round) mod (re - 1) for 0 <= x, round < re - 1, without an integer division
                int tp = sa - 1 + round, tq = sb - 1 + round;
                if (tp >= re - 1) tp -= re - 1;
                if (tq >= re - 1) tq -= re - 1;
                const int p = (sa == 0) ? 0 : 1 + tp;
                const int q = 1 + tq;
                if (p < r && q < r) {
                    // the pair's rows of this lane (i = lane + 16 t), loaded once, clamped and masked
                    double sp[4], sq[4], vp[4], vq[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int i = lane + kSvdLanes * t;
                        const int ic = i < r ? i : r - 1;
                        sp[t] = S[p * r + ic];
                        sq[t] = S[q * r + ic];
                        vp[t] = V[p * r + ic];
                        vq[t] = V[q * r + ic];
                    }
                    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const bool on = lane + kSvdLanes * t < r;
                        const double x = on ? sp[t] : 0.0, y = on ? sq[t] : 0.0;
                        al += x * x;
                        be += y * y;
                        ga += x * y;
                    }
                    al = row16_sum(al);
                    be = row16_sum(be);
                    ga = row16_sum(ga);
                    if (ga != 0.0 && ga * ga > tol * tol * (al * be)) {
                        // tan of the rotation angle, t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)) with
                        // zeta = (be - al) / (2 ga), written without forming zeta
                        const double d = be - al;
                        const double sgn = (d * ga >= 0.0) ? 1.0 : -1.0;
                        const double tt = sgn * (2.0 * fabs(ga)) / (fabs(d) + sqrt(d * d + 4.0 * ga * ga));
                        const double c = 1.0 / sqrt(1.0 + tt * tt);
                        const double sn = c * tt;
                        rotated = 1;
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int i = lane + kSvdLanes * t;
                            if (i < r) {
                                S[p * r + i] = c * sp[t] - sn * sq[t];
                                S[q * r + i] = sn * sp[t] + c * sq[t];
                                V[p * r + i] = c * vp[t] - sn * vq[t];
                                V[q * r + i] = sn * vp[t] + c * vq[t];
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
        converged = !__syncthreads_or(rotated);
    }
    if (tid == 0 && !converged) atomicOr(status, (int)kStatusSvdNoConv);
    if (tid == 0) status[2] = sweep;   // diagnostic: sweeps taken
    for (int c = tid; c < r; c += kSvdThreads) {
        double sum = 0.0;
        for (int i = 0; i < r; ++i) sum += S[c * r + i] * S[c * r + i];
        nrm[c] = sqrt(sum);
    }
    __syncthreads();
    // stable descending order: rank of column c = columns with a larger norm, or an equal norm
    // and a smaller index
    for (int c = tid; c < r; c += kSvdThreads) {
        int rank = 0;
        for (int m = 0; m < r; ++m) rank += (nrm[m] > nrm[c] || (nrm[m] == nrm[c] && m < c)) ? 1 : 0;
        order[rank] = c;
    }
    __syncthreads();
    for (int c = tid; c < r; c += kSvdThreads) {
        const int src = order[c];
        int m = 0;
        double best = -1.0;
        for (int i = 0; i < r; ++i)
            if (fabs(V[src * r + i]) > best) { best = fabs(V[src * r + i]); m = i; }
        const double sg = (V[src * r + m] < 0.0) ? -1.0 : 1.0;
        for (int i = 0; i < r; ++i) {
            Vout[i * r + c] = sg * V[src * r + i];
            Sout[i * r + c] = sg * S[src * r + i];
        }
    }
}

// X[k][c] = sum_j V[j][c] M[j][k]; one thread per output, consecutive threads along c
__global__ __launch_bounds__(256) void k_rmul(int n, int r, const double* __restrict__ V, const double* __restrict__ M,
                                              double* __restrict__ X) {
    __shared__ double sM[kMaxRank * kMaxRank];
    stage_lds(sM, M, r * r);
    __syncthreads();
    const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (long)n * r) return;
    const int k = (int)(o / n), c = (int)(o % n);
    double s = 0.0;
#pragma unroll 8
    for (int j = 0; j < r; ++j) s += V[(size_t)j * n + c] * sM[j * r + k];
    X[(size_t)k * n + c] = s;
}

// beta_k = sum_q w_q W_k(q), coef = S beta; wavefront k sums column k (fixed lane order)
__global__ __launch_bounds__(1024) void k_wsum(int nq, int r, const double* __restrict__ W,
                                               const double* __restrict__ w, const double* __restrict__ S,
                                               double* __restrict__ beta, double* __restrict__ coef) {
    __shared__ double sb[kMaxRank];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = wv; k < r; k += 16) {
        double acc = 0.0;
#pragma unroll 8
        for (int q = lane; q < nq; q += 64) acc += w[q] * W[(size_t)k * nq + q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) sb[k] = acc;
    }
    __syncthreads();
    __shared__ double sS[kMaxRank * kMaxRank];
    stage_lds(sS, S, r * r);
    __syncthreads();
    for (int i = threadIdx.x; i < r; i += blockDim.x) {
        beta[i] = sb[i];
        double s = 0.0;
        for (int j = 0; j < r; ++j) s += sS[i * r + j] * sb[j];
        coef[i] = s;
    }
}

}  // namespace

void launch_deim(hipStream_t s, const DeimArgs& a) {
    hipLaunchKernelGGL(k_deim, dim3(1), dim3(kDeimThreads), 0, s, a);
}

void launch_lstep(hipStream_t s, const LstepArgs& a) {
    const int r = a.r;
    const size_t solve_lds = ((size_t)r * (2 * r + 1) + (size_t)r * r) * sizeof(double);
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
    hipLaunchKernelGGL(k_rmul, dim3((unsigned)(((long)n * r + 255) / 256)), dim3(256), 0, s, n, r, V, M, X);
}

void launch_wsum(hipStream_t s, int nq, int r, const double* W, const double* w, const double* S, double* beta,
                 double* coef) {
    hipLaunchKernelGGL(k_wsum, dim3(1), dim3(1024), 0, s, nq, r, W, w, S, beta, coef);
}

}  // namespace dlr
