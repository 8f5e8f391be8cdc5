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
#include "wave_ops.h"

namespace dlr {

namespace {

// ---------------------------------------------------------------------------------------------- block reductions
constexpr int kMaxOrdinates = 16384;

// ---------------------------------------------------------------------------------------------- Gauss-Jordan
// The same solve on one wavefront without barriers, for systems of a single workgroup's
// critical path: lane i holds row i of the augmented system in registers, the pivot of
// column k is the largest remaining |A_ik| (ties to the lowest row) found by a DPP wavefront
// maximum and a ballot, the pivot row is broadcast through prow (the wavefront's LDS accesses execute in
// order), and column k is eliminated from every other row.  The solution overwrites the
// right-hand-side column (x_k in row k).  Called by the whole workgroup; wavefront 0 works.
template <int RMAX>
__device__ __forceinline__ void gauss_jordan_wave_impl(double* Aug, int r, int ld, double* prow, int* bad) {
    const int i = threadIdx.x;
    const bool live = i < r;
    const int ic = live ? i : r - 1;
    double a[RMAX];
#pragma unroll
    for (int c = 0; c < RMAX; ++c) {
        const double v = Aug[ic * ld + (c < r ? c : r - 1)];
        a[c] = (live && c < r) ? v : 0.0;
    }
    double b = live ? Aug[ic * ld + r] : 0.0;
    bool used = !live, isbad = false;
    int mypiv = -1;
    double mydiag = 1.0;
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        if (k < r) {
            __atomic_signal_fence(__ATOMIC_SEQ_CST);   // one pivot's LDS traffic at a time
            const double mine = used ? -1.0 : fabs(a[k]);
            const double v = wave_max(mine);
            // the lowest row holding the maximum (the lowest free row when no value compares equal)
            const unsigned long long hit = __ballot(mine == v);
            const int p = hit ? __builtin_ctzll(hit) : __builtin_ctzll(__ballot(!used));
            if (!(v > 0.0) || !isfinite(v)) isbad = true;
            if (i == p) {
#pragma unroll
                for (int c = k; c < RMAX; ++c) prow[c] = a[c];
                prow[RMAX] = b;
                used = true;
                mypiv = k;
                mydiag = a[k];
            }
            const double f = (i == p) ? 0.0 : a[k] / prow[k];
#pragma unroll
            for (int c = k + 1; c < RMAX; ++c) a[c] = fma(-f, prow[c], a[c]);
            b = fma(-f, prow[RMAX], b);
        }
    }
    if (mypiv >= 0) Aug[mypiv * ld + r] = b / mydiag;
    if (__ballot(isbad) != 0ull && i == 0) *bad = 1;
}

__device__ __forceinline__ void gauss_jordan_wave(double* Aug, int r, int ld, double* prow, int* bad) {
    __syncthreads();
    if (threadIdx.x < 64) {
        if (r <= 8)
            gauss_jordan_wave_impl<8>(Aug, r, ld, prow, bad);
        else if (r <= 16)
            gauss_jordan_wave_impl<16>(Aug, r, ld, prow, bad);
        else if (r <= 32)
            gauss_jordan_wave_impl<32>(Aug, r, ld, prow, bad);
        else
            gauss_jordan_wave_impl<64>(Aug, r, ld, prow, bad);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------------------------- DEIM
// Algorithm 1 step 2 (Sec. 4.2): the DEIM points of W are the pivots of Gaussian elimination
// with partial pivoting on the rows of W (ordinates): for column j, the pivot is the
// lowest-index row whose |value| is within the tie tolerance of the column maximum over the
// rows not yet chosen (margin = relative gap to the largest value below that threshold), and
// the column is eliminated from the remaining rows.  Then c solves What^T c = beta with
// beta = W^T w, and C0 = S W[sel]^T, a0 = S beta.
//
// The rows are spread over ceil(nq / 256) workgroups, one row per thread, kept in registers.
// Per column one exchange among the workgroups: each group publishes its maximum m_g, its
// lowest-index row at or above its own threshold (1 - tol) m_g with that row's values, and its
// largest value below that threshold.  The group(s) holding the global maximum M have the
// global threshold, so the pivot is the lowest of their candidates, and every other group lies
// entirely below the threshold -- unless some m_g lies in [(1 - tol) M, M), a near-tie across
// groups.  All groups see the same published values and detect that case alike; it falls back
// to a second exchange of each group's lowest-index row at or above the global threshold.  A
// forced selection (the parity replay) always takes the two-exchange path: (1) each group's
// maximum, (2) the rows at or above the global threshold.  Exchanged values are agent-scope atomics in a double-buffered area; a group
// counts itself after its stores have completed and polls the count, bounded by a spin limit
// (kStatusDeimStall) so that a stall cannot hang the device.  All groups reach the same
// decisions from the same data; group 0 then solves for c and writes the outputs.
constexpr int kDeimThreads = 256;
constexpr int kDeimWaves = kDeimThreads / 64;
constexpr int kDeimMaxGroups = kMaxOrdinates / kDeimThreads;
constexpr size_t kXEx1 = 0;                                                        // [2][groups]
constexpr size_t kXEx2 = kXEx1 + 2 * kDeimMaxGroups;                              // [2][groups][2 + kMaxRank]
constexpr size_t kXBeta = kXEx2 + 2 * (size_t)kDeimMaxGroups * (2 + kMaxRank);    // [groups][kMaxRank]
constexpr size_t kXExM = kXBeta + (size_t)kDeimMaxGroups * kMaxRank;              // [2][groups][3 + kMaxRank]
static_assert(kXExM + 2 * (size_t)kDeimMaxGroups * (3 + kMaxRank) <= kDeimXchgDoubles, "DEIM exchange area");
constexpr unsigned kDeimSpinLimit = 1u << 20;

__device__ __forceinline__ void xstore(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double xload(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_vm_stores() {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt and lgkmcnt unconstrained
}
// Every group arrives at exchange number `target / groups`: the stores of each wavefront have
// completed, then thread 0 counts the group and polls until all groups have counted.  After one
// wait has timed out the group stops polling (its results are flagged invalid anyway).
__device__ void group_sync(unsigned* arrive, unsigned target, int* stall) {
    wait_vm_stores();
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned polls = 0;
        while (!*stall && __hip_atomic_load(arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++polls > kDeimSpinLimit) {
                *stall = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
}

// RT: rank bound; GM: bound on the number of workgroups.  With GM <= 8 the polling wavefront loads
// every group's candidate row together with the maxima (one round trip fewer per column).
template <int RT, int GM>
__global__ __launch_bounds__(kDeimThreads) void k_deim(DeimArgs a) {
    __shared__ double sv[kDeimWaves], sv2[kDeimWaves];
    __shared__ int si[kDeimWaves];
    __shared__ double sM, sSecond;
    __shared__ int sP, sFallback, sHaveRow;
    __shared__ size_t sSrc;   // offset of the pivot row's values in the exchange area
    __shared__ double up[2][RT];   // pivot rows of the current and the previous column
    __shared__ double bw[kDeimWaves][RT];
    __shared__ int bad, stall;
    const int G = gridDim.x, g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nq = a.nq, r = a.r;
    const int q = g * kDeimThreads + tid;
    const bool in = q < nq;
    double* X = a.xchg;
    // the launch's tag: from the host, or read from the counter before the last group advances it
    const unsigned long long seq =
        a.seq_ctr ? (unsigned long long)__hip_atomic_load(a.seq_ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                  : a.launch_seq;
    if (tid == 0) {
        bad = 0;
        stall = 0;
    }
    for (int i = tid; i < 2 * RT; i += kDeimThreads) up[i / RT][i % RT] = 0.0;
    // row q of W, and this group's part of beta = W^T w (wavefront sums, then wavefront order).
    // Every load is issued unconditionally (clamped index) and the unused values cleared by a bit
    // mask: a select on `in` lets the compiler put each load under its own branch and wait there.
    double u[RT];
    const double wq = in ? a.w[q] : 0.0;
    const int qc = in ? q : nq - 1;
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        const double v = a.W[(size_t)(i < r ? i : r - 1) * nq + qc];
        const unsigned long long keep = (in && i < r) ? ~0ull : 0ull;
        u[i] = __longlong_as_double(__double_as_longlong(v) & keep);
    }
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        double b = wq * u[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) b += __shfl_xor(b, off);
        if (lane == 0) bw[wv][i] = b;
    }
    __syncthreads();
    for (int i = tid; i < r; i += kDeimThreads) {
        double b = 0.0;
        for (int w = 0; w < kDeimWaves; ++w) b += bw[w][i];
        xstore(&X[kXBeta + (size_t)g * kMaxRank + i], b);
    }
    // Look-ahead elimination: when pivot j is known, a row forms its updated column j + 1 at once
    // (the next column's search needs only that one) and applies the pivot to its whole row
    // while the exchange of column j + 1 is in flight.  Each entry still receives the pivots'
    // updates in column order, so the arithmetic is that of plain column-by-column elimination.
    // The whole-row update has no per-column condition: columns up to j are no longer read (their
    // values go stale), and the pivot rows are zero from column r on.
    bool pivoted = false;
    bool defer = false;    // pivot j - 1 still to be applied to this row
    double lprev = 0.0;    // this row's multiplier of pivot j - 1
    double unext = 0.0;    // column j of this row with pivot j - 1 applied (when defer)
    unsigned nsync = 0;
    for (int j = 0; j < r; ++j) {
        double* urow = up[j & 1];
        const double* prow = up[(j + 1) & 1];
        // The row update reads the pivot row whole, then updates every entry without a branch (a
        // per-column condition had been compiled into a chain of uniform branches, each with its
        // own LDS wait).
        auto finish_prev = [&]() {
            if (defer) {
                double pr[RT];
#pragma unroll
                for (int i = 0; i < RT; ++i) pr[i] = prow[i];
#pragma unroll
                for (int i = 0; i < RT; ++i) u[i] = fma(-lprev, pr[i], u[i]);
                defer = false;
            }
        };
        double uj = 0.0;
#pragma unroll
        for (int i = 0; i < RT; ++i) uj = (i == j) ? u[i] : uj;
        if (defer) uj = unext;
        const bool elig = in && !pivoted;
        const double v = elig ? fabs(uj) : -1.0;
        // the two-exchange step (2): lowest-index row at or above thr (or the forced row) with its
        // values, largest value below thr; sets sP, sSecond, and sSrc to the pivot row's values
        auto exchange_above = [&](double thr) {
            int pi = (elig && v >= thr) ? q : 0x7fffffff;
            double sec = (elig && v < thr) ? v : 0.0;
            if (a.forced) {
                const int f = a.forced[j];
                pi = (q == f) ? q : 0x7fffffff;
                if (q == f && !elig) bad = 1;
            }
            pi = wave_min(pi);
            sec = wave_max(sec);
            if (lane == 0) {
                si[wv] = pi;
                sv2[wv] = sec;
            }
            __syncthreads();
            int pw = si[0];
            double sw = sv2[0];
            for (int w = 1; w < kDeimWaves; ++w) {
                pw = min(pw, si[w]);
                sw = fmax(sw, sv2[w]);
            }
            double* slot = &X[kXEx2 + ((size_t)(j & 1) * kDeimMaxGroups + g) * (2 + kMaxRank)];
            if (q == pw) {
#pragma unroll
                for (int i = 0; i < RT; ++i)
                    if (i < r) xstore(&slot[2 + i], u[i]);
            }
            if (tid == 0) {
                xstore(&slot[0], (double)pw);
                xstore(&slot[1], sw);
            }
            group_sync(a.xcount, (++nsync) * (unsigned)G, &stall);
            if (wv == 0) {
                const double* sl = &X[kXEx2 + ((size_t)(j & 1) * kDeimMaxGroups + lane) * (2 + kMaxRank)];
                double pg = (lane < G) ? xload(&sl[0]) : 2147483647.0;
                double sg = (lane < G) ? xload(&sl[1]) : 0.0;
                pg = wave_min(pg);
                sg = wave_max(sg);
                if (lane == 0) {
                    sP = (pg < 2147483647.0) ? (int)pg : -1;
                    sSecond = sg;
                    sSrc = (pg < 2147483647.0)
                               ? kXEx2 + ((size_t)(j & 1) * kDeimMaxGroups + (int)pg / kDeimThreads) * (2 + kMaxRank) + 2
                               : 0;
                }
            }
            __syncthreads();
        };
        // this group's maximum over the rows not yet chosen
        const double m = wave_max(v);
        if (lane == 0) sv[wv] = m;
        __syncthreads();
        double mw = sv[0];
        for (int w = 1; w < kDeimWaves; ++w) mw = fmax(mw, sv[w]);
        if (!a.forced) {
            // one exchange: m_g, the lowest-index row at or above (1 - tol) m_g with its values,
            // and the largest value below that threshold
            const double thl = (1.0 - a.tie_tol) * mw;
            int pi = (elig && v >= thl) ? q : 0x7fffffff;
            double sec = (elig && v < thl) ? v : 0.0;
            pi = wave_min(pi);
            sec = wave_max(sec);
            if (lane == 0) {
                si[wv] = pi;
                sv2[wv] = sec;
            }
            __syncthreads();
            int pw = si[0];
            double sw = sv2[0];
            for (int w = 1; w < kDeimWaves; ++w) {
                pw = min(pw, si[w]);
                sw = fmax(sw, sv2[w]);
            }
            // The candidate word, stored last (after the group's other stores have completed),
            // carries the launch and the column: tag * 2^15 + index (index 2^14 = none).  Readers
            // poll it instead of a shared arrival counter.  A group cannot reach column j + 2 (and
            // overwrite this slot) before every group has published column j + 1, i.e. finished
            // reading column j.
            const double tag = (double)(((seq & 0xffffffffull) << 6) | (unsigned long long)j);
            double* slot = &X[kXExM + ((size_t)(j & 1) * kDeimMaxGroups + g) * (3 + kMaxRank)];
            if (q == pw) {
                finish_prev();   // the published row carries every earlier pivot's update
#pragma unroll
                for (int i = 0; i < RT; ++i)
                    if (i < r) xstore(&slot[3 + i], u[i]);
            }
            if (tid == 0) {
                xstore(&slot[0], mw);
                xstore(&slot[1], sw);
            }
            wait_vm_stores();
            __syncthreads();
            if (tid == 0) xstore(&slot[2], tag * 32768.0 + (double)(pw < nq ? pw : 16384));
            finish_prev();   // the rest of pivot j - 1's update, while the exchange is in flight
            if (wv == 0) {
                const double* sl = &X[kXExM + ((size_t)(j & 1) * kDeimMaxGroups + lane) * (3 + kMaxRank)];
                double word = 0.0;
                bool seen = lane >= G;
                unsigned polls = 0;
                for (;;) {
                    if (!seen) {
                        word = xload(&sl[2]);
                        seen = floor(word / 32768.0) == tag;
                    }
                    if (__all(seen)) break;
                    if (stall || ++polls > kDeimSpinLimit) {
                        stall = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                // every group's maxima and (GM <= 8) candidate row, complete once the words are seen
                const double* base = &X[kXExM + (size_t)(j & 1) * kDeimMaxGroups * (3 + kMaxRank)];
                const double mg = (lane < G) ? xload(&sl[0]) : -1.0;
                const double sg = (lane < G) ? xload(&sl[1]) : 0.0;
                constexpr int KS = GM <= 8 ? (8 * RT + 63) / 64 : 1;
                double rv[KS];
                if (GM <= 8) {
#pragma unroll
                    for (int k = 0; k < KS; ++k) {
                        const int idx = lane + 64 * k, gg = idx / r, i = idx - gg * r;
                        rv[k] = xload(&base[(size_t)(gg < G ? gg : 0) * (3 + kMaxRank) + 3 + (gg < G ? i : 0)]);
                    }
                }
                const double ci = word - tag * 32768.0;
                const double cg = (lane < G && ci < 16384.0) ? ci : 2147483647.0;
                const double Mx = wave_max(mg);
                const double Mpos = fmax(Mx, 0.0);
                const double thr = (1.0 - a.tie_tol) * Mpos;
                const bool band = lane < G && mg >= thr && mg < Mx;
                double cand = (lane < G && mg == Mx) ? cg : 2147483647.0;
                double scnd = (lane < G) ? ((mg < thr) ? fmax(mg, 0.0) : ((mg == Mx) ? sg : 0.0)) : 0.0;
                cand = wave_min(cand);
                scnd = wave_max(scnd);
                const bool fallback = __ballot(band) != 0ull;
                const bool found = cand < 2147483647.0;
                const int pg = found ? (int)cand / kDeimThreads : 0;
                bool have = false;
                if (!fallback && found) {
                    // the pivot row into LDS: from the loaded rows, or one more load
                    if (GM <= 8) {
#pragma unroll
                        for (int k = 0; k < KS; ++k) {
                            const int idx = lane + 64 * k, gg = idx / r, i = idx - gg * r;
                            if (gg == pg) urow[i] = rv[k];
                        }
                    } else {
                        for (int i = lane; i < r; i += 64) urow[i] = xload(&base[(size_t)pg * (3 + kMaxRank) + 3 + i]);
                    }
                    have = true;
                }
                if (lane == 0) {
                    sM = Mpos;
                    sFallback = fallback ? 1 : 0;
                    sHaveRow = have ? 1 : 0;
                    sP = found ? (int)cand : -1;
                    sSecond = scnd;
                    sSrc = found ? kXExM + ((size_t)(j & 1) * kDeimMaxGroups + pg) * (3 + kMaxRank) + 3 : 0;
                }
            }
            __syncthreads();
            if (sFallback) exchange_above((1.0 - a.tie_tol) * sM);
        } else {
            finish_prev();
            // (1) the maximum over the rows not yet chosen, (2) the rows at or above the threshold
            if (tid == 0) xstore(&X[kXEx1 + (size_t)(j & 1) * kDeimMaxGroups + g], mw);
            group_sync(a.xcount, (++nsync) * (unsigned)G, &stall);
            if (wv == 0) {
                const double mg =
                    wave_max((lane < G) ? xload(&X[kXEx1 + (size_t)(j & 1) * kDeimMaxGroups + lane]) : -1.0);
                if (lane == 0) {
                    sM = fmax(mg, 0.0);
                    sHaveRow = 0;
                }
            }
            __syncthreads();
            exchange_above((1.0 - a.tie_tol) * sM);
        }
        const double M = sM;
        const int p = sP;
        if (p < 0) {   // no row qualifies (an invalid forced index): flag and stop, consistently in all groups
            if (tid == 0) bad = 1;
            break;
        }
        const bool reload = sFallback || !sHaveRow;
        if (reload) {
            for (int i = tid; i < r; i += kDeimThreads) urow[i] = xload(&X[sSrc + i]);
            __syncthreads();
        }
        if (tid == 0 && g == 0) {
            a.sel[j] = p;
            a.margins[j] = (M > 0.0) ? (M - sSecond) / M : 0.0;
        }
        if (tid == 0 && !(M > 0.0)) bad = 1;
        // pivot j: this row's multiplier, applied to column j + 1 now and to the rest later
        if (q == p) pivoted = true;
        if (in && !pivoted && j + 1 < r) {
            lprev = uj / urow[j];
            double un = 0.0;
#pragma unroll
            for (int i = 0; i < RT; ++i) un = (i == j + 1) ? u[i] : un;
            unext = fma(-lprev, urow[j + 1], un);
            defer = true;
        }
    }
    // the last group to leave resets the counters for the next launch
    __syncthreads();
    if (tid == 0) {
        const unsigned prev = __hip_atomic_fetch_add(&a.xcount[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == (unsigned)G - 1u) {
            __hip_atomic_store(&a.xcount[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.xcount[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a.seq_ctr) {   // stays at 2^31 or above (the host's tags are below)
                const unsigned nx = (unsigned)seq + 1u;
                __hip_atomic_store(a.seq_ctr, nx < (1u << 31) ? nx + (1u << 31) : nx, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (stall) atomicOr(a.status, (int)kStatusDeimStall);
        if (bad) atomicOr(a.status, a.forced ? (int)kStatusBadForcedSel : (int)kStatusSingularSolve);
    }
}

// After the selection: beta (sum of the groups' parts in group order), What^T c = beta by
// Gauss-Jordan with partial pivoting, and the per-direction outputs.  One workgroup.
__global__ __launch_bounds__(kDeimThreads) void k_deim_tail(DeimArgs a, int groups) {
    __shared__ double beta[kMaxRank];
    __shared__ int sel[kMaxRank];
    __shared__ double Aug[kMaxRank * (kMaxRank + 1)];
    __shared__ double sS[kMaxRank * kMaxRank];
    __shared__ double Wh[kMaxRank * kMaxRank];   // Wh[i][d] = W_i(Omega^(sel d))
    __shared__ double fac[kMaxRank];
    __shared__ double prow[kMaxRank + 1];
    __shared__ double pivval;
    __shared__ int pivrow, bad;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nq = a.nq, r = a.r;
    const double* X = a.xchg;
    if (tid == 0) bad = 0;
    __shared__ double bparts[kDeimMaxGroups * kMaxRank];
    __shared__ double smu[kMaxRank], seta[kMaxRank];
    stage_lds(bparts, X + kXBeta, groups * kMaxRank);
    stage_lds(sS, a.S, r * r);
    for (int i = tid; i < r; i += kDeimThreads) {
        const int sv = a.sel[i];
        sel[i] = (sv >= 0 && sv < nq) ? sv : 0;
    }
    __syncthreads();
    for (int i = tid; i < r; i += kDeimThreads) {
        double b = 0.0;
        for (int w = 0; w < groups; ++w) b += bparts[w * kMaxRank + i];
        beta[i] = b;
        smu[i] = a.mu[sel[i]];
        seta[i] = a.eta[sel[i]];
    }
    // What: the r x r gather, all loads of a thread issued before its stores
    const int ld = r + 1;
    for (int base = tid; base < r * r; base += 8 * kDeimThreads) {
        double v[8];
        int o8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int o = base + u * kDeimThreads;
            const int oc = o < r * r ? o : r * r - 1;
            const int i = oc / r, jj = oc - (oc / r) * r;
            o8[u] = o;
            v[u] = a.W[(size_t)i * nq + sel[jj]];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (o8[u] < r * r) {
                const int i = o8[u] / r, jj = o8[u] - (o8[u] / r) * r;
                Aug[i * ld + jj] = v[u];
                Wh[o8[u]] = v[u];
            }
    }
    __syncthreads();
    for (int i = tid; i < r; i += kDeimThreads) Aug[i * ld + r] = beta[i];
    gauss_jordan_wave(Aug, r, ld, prow, &bad);
    for (int i = tid; i < r; i += kDeimThreads) {
        a.cw[i] = Aug[i * ld + r];
        const double mu = smu[i], eta = seta[i];
        a.sel_mu[i] = mu;
        a.sel_eta[i] = eta;
        a.inflow_x[i] = a.psib[mu > 0.0 ? 0 : 1];
        a.inflow_y[i] = a.psib[eta > 0.0 ? 2 : 3];
        double s = 0.0;
        for (int jj = 0; jj < r; ++jj) s += sS[i * r + jj] * beta[jj];
        a.a0[i] = s;
    }
    // C0[k][d] = sum_j S[k][j] W_j(Omega^(d))
    for (int k = wv; k < r; k += kDeimWaves)
        for (int d = lane; d < r; d += 64) {
            double s = 0.0;
            for (int jj = 0; jj < r; ++jj) s += sS[k * r + jj] * Wh[jj * r + d];
            a.C0[k * r + d] = s;
        }
    if (tid == 0 && bad) atomicOr(a.status, (int)kStatusSingularSolve);
}

constexpr int kLsThreads = 256;

// Right-hand sides of the L-step for ranks 33 to 64, one thread per (ordinate, basis index):
// Q_q = qX + (old solution on the new basis) / (c dt) + inflow, with G = S0^T P staged in LDS; written
// to y, which the solve below reads and overwrites with B_q^{-1} Q_q.
__global__ __launch_bounds__(256) void k_lstep_rhs(LstepArgs a) {
    __shared__ double sG[kMaxRank * kMaxRank];
    const int r = a.r, rr = r * r;
    stage_lds(sG, a.ops + 6 * rr, rr);
    __syncthreads();
    const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (long)a.nq * r) return;
    const int q = (int)(o / r), i = (int)(o % r);
    const double* qX = a.ops + 7 * rr;
    const double* bv = qX + r;
    const double mu = a.mu[q], eta = a.eta[q];
    const int sx = mu > 0.0 ? 0 : 1, sy = eta > 0.0 ? 2 : 3;
    double lt = 0.0;   // sum_j W0_j(q) G[j][i]
#pragma unroll 8
    for (int j = 0; j < r; ++j) lt = fma(a.W0[(size_t)j * a.nq + q], sG[j * r + i], lt);
    a.y[o] = qX[i] + lt * a.inv_cdt + fabs(mu) * a.psib[sx] * bv[sx * r + i] + fabs(eta) * a.psib[sy] * bv[sy * r + i];
}

// Ranks 33 to 64: one workgroup of 128 threads per ordinate, Gauss-Jordan on [B_q | I] (64 x 128, the
// identity past r).  Thread t holds the 8 x 8 block of rows 8 (t / 16) .. + 7 and columns 8 (t % 16) .. + 7
// in registers.  Per pivot k the threads of block column k / 8 copy their entries of column k, and those
// of block row k / 8 their entries of row k, to LDS (two buffers each, one barrier per pivot); every
// thread then reads 8 column and 8 row values and updates its block.  As in the one-wavefront form no
// rows are exchanged (B_q's symmetric part is positive definite; a zero or non-finite pivot flags a
// singular solve).  Afterwards the threads of block columns 8..15 hold B_q^{-1}; it goes to memory and
// to LDS, where 64 threads form y_q = B_q^{-1} Q_q (Q_q from k_lstep_rhs).
__global__ __launch_bounds__(128) void k_lstep_solve_w2(LstepArgs a) {
    constexpr int RT = 64, NB = 8;
    __shared__ double colk[2][RT];
    __shared__ double rowk[2][2 * RT];
    __shared__ double Bs[RT * (RT + 1)];
    __shared__ double Qs[RT];
    __shared__ int bad;
    const int t = threadIdx.x, pb = t >> 4, sb = t & 15;   // block row, block column
    const int r = a.r, rr = r * r, q = blockIdx.x;
    const double mu = a.mu[q], eta = a.eta[q];
    const double* Ax = a.ops + (mu > 0.0 ? 0 : 1) * rr;
    const double* Ay = a.ops + (eta > 0.0 ? 2 : 3) * rr;
    const double* Mt = a.ops + 4 * rr;
    const double amu = fabs(mu), aeta = fabs(eta);
    if (t == 0) bad = 0;
    if (t < RT) {
        const double Q = a.y[(size_t)q * r + (t < r ? t : r - 1)];
        Qs[t] = t < r ? Q : 0.0;
    }
    double blk[NB][NB];
    if (sb < NB) {
        // columns 8 sb .. of B (the identity past r); clamped loads, 0/1 masks instead of selects of loads
#pragma unroll
        for (int ii = 0; ii < NB; ++ii) {
            const int i = NB * pb + ii, ic = i < r ? i : r - 1;
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) {
                const int c = NB * sb + jj, cc = c < r ? c : r - 1;
                const double v = amu * Ax[ic * r + cc] + aeta * Ay[ic * r + cc] + Mt[ic * r + cc];
                const double keep = (i < r && c < r) ? 1.0 : 0.0;
                blk[ii][jj] = keep * v + (i == c ? 1.0 - keep : 0.0);
            }
        }
    } else {
#pragma unroll
        for (int ii = 0; ii < NB; ++ii)
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) blk[ii][jj] = (NB * pb + ii == NB * (sb - NB) + jj) ? 1.0 : 0.0;
    }
    // The eight pivots of a block are unrolled, so the block-local index k % 8 is a constant: the owners
    // copy fixed registers, every entry takes the same update, and the pivot row is then overwritten
    // by the threads that hold it (no selects on the pivot index)
    bool sing = false;
#pragma unroll 1
    for (int kb = 0; kb < NB; ++kb) {
#pragma unroll
        for (int kk = 0; kk < NB; ++kk) {
            const int k = NB * kb + kk, buf = kk & 1;
            if (sb == kb) {   // column k of this thread's rows
#pragma unroll
                for (int ii = 0; ii < NB; ++ii) colk[buf][NB * pb + ii] = blk[ii][kk];
            }
            if (pb == kb) {   // row k of this thread's columns
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) rowk[buf][NB * sb + jj] = blk[kk][jj];
            }
            __syncthreads();
            const double piv = colk[buf][k];
            if (!(fabs(piv) > 0.0) || !isfinite(piv)) sing = true;
            const double inv = 1.0 / piv;
            double f[NB], cv[NB];
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) f[jj] = rowk[buf][NB * sb + jj] * inv;
#pragma unroll
            for (int ii = 0; ii < NB; ++ii) cv[ii] = colk[buf][NB * pb + ii];
#pragma unroll
            for (int ii = 0; ii < NB; ++ii)
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) blk[ii][jj] = fma(-cv[ii], f[jj], blk[ii][jj]);
            if (pb == kb) {   // the pivot row becomes row k / pivot
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) blk[kk][jj] = f[jj];
            }
        }
    }
    if (sing) bad = 1;
    if (sb >= NB) {
        double* Bi = a.Binv + (size_t)q * rr;
#pragma unroll
        for (int ii = 0; ii < NB; ++ii) {
            const int i = NB * pb + ii;
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) {
                const int c = NB * (sb - NB) + jj;
                Bs[i * (RT + 1) + c] = blk[ii][jj];
                if (i < r && c < r) Bi[i * r + c] = blk[ii][jj];
            }
        }
    }
    __syncthreads();
    if (t < r) {
        double y = 0.0;
        for (int j = 0; j < r; ++j) y = fma(Bs[t * (RT + 1) + j], Qs[j], y);
        a.y[(size_t)q * r + t] = y;
    }
    if (t == 0 && bad) atomicOr(a.status, (int)kStatusSingularSolve);
}

// Ranks up to 32: one wavefront per ordinate, lane c holding column c of [B_q | I] (2 RT <= 64
// columns, rows in registers, padded to RT with the identity).  B_q = |mu| A_x + |eta| A_y + M_t is
// the Galerkin projection, on the orthonormal basis X, of the upwind transport operator plus
// sigma_t + 1/(c dt); its symmetric part is positive definite, so Gauss-Jordan elimination needs
// no row exchanges (a zero or non-finite pivot still flags a singular solve).  Per pivot
// k, lane k's column goes through a per-wavefront LDS buffer to all lanes.  Afterwards the lanes
// of the identity part hold B_q^{-1} column by column; y_q = B_q^{-1} Q_q from an LDS copy.
template <int RT>
__global__ __launch_bounds__(256) void k_lstep_solve_wave(LstepArgs a) {
    constexpr int kW = 4;   // wavefronts (ordinates) per block
    __shared__ double colk[kW][RT];
    __shared__ double Bs[kW][RT * (RT + 1)];
    __shared__ double Qs[kW][RT];
    __shared__ int bad;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = a.r, rr = r * r;
    const int q = blockIdx.x * kW + wv;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    if (q < a.nq) {
        const double mu = a.mu[q], eta = a.eta[q];
        const double* Ax = a.ops + (mu > 0.0 ? 0 : 1) * rr;
        const double* Ay = a.ops + (eta > 0.0 ? 2 : 3) * rr;
        const double* Mt = a.ops + 4 * rr;
        const double* G = a.ops + 6 * rr;
        const double* qX = a.ops + 7 * rr;
        const double* bv = qX + r;
        const int sx = mu > 0.0 ? 0 : 1, sy = eta > 0.0 ? 2 : 3;
        const double amu = fabs(mu), aeta = fabs(eta);
        // column c of [B | I]: c < RT the matrix (identity outside r x r), c >= RT the identity
        const bool matcol = lane < RT;
        const int c = matcol ? lane : lane - RT;
        const int cc = c < r ? c : r - 1;
        double acol[RT];
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            const int ic = i < r ? i : r - 1;
            const double v = amu * Ax[ic * r + cc] + aeta * Ay[ic * r + cc] + Mt[ic * r + cc];
            acol[i] = (matcol && i < r && c < r) ? v : ((i == c) ? 1.0 : 0.0);
        }
        // right-hand side Q_q (lane i < r): qX + (old solution on the new basis) / (c dt) + inflow
        if (lane < r) {
            double lt = 0.0;   // sum_j W0_j(q) G[j][i]
#pragma unroll 8
            for (int j = 0; j < r; ++j) lt += a.W0[(size_t)j * a.nq + q] * G[j * r + lane];
            Qs[wv][lane] = qX[lane] + lt * a.inv_cdt + amu * a.psib[sx] * bv[sx * r + lane] +
                           aeta * a.psib[sy] * bv[sy * r + lane];
        }
        bool sing = false;
#pragma unroll
        for (int k = 0; k < RT; ++k) {
            if (lane == k) {
#pragma unroll
                for (int i = 0; i < RT; ++i) colk[wv][i] = acol[i];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const double piv = colk[wv][k];
            if (!(fabs(piv) > 0.0) || !isfinite(piv)) sing = true;
            const double akk = acol[k] / piv;   // row k of the normalised pivot row
            acol[k] = akk;
#pragma unroll
            for (int i = 0; i < RT; ++i)
                if (i != k) acol[i] -= colk[wv][i] * akk;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (sing && lane == 0) bad = 1;
        // B_q^{-1}: lane RT + j holds column j
        if (!matcol && c < r) {
            double* Bi = a.Binv + (size_t)q * rr;
#pragma unroll
            for (int i = 0; i < RT; ++i)
                if (i < r) {
                    Bi[i * r + c] = acol[i];
                    Bs[wv][i * (RT + 1) + c] = acol[i];
                }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < r) {
            double y = 0.0;
            for (int j = 0; j < r; ++j) y += Bs[wv][lane * (RT + 1) + j] * Qs[wv][j];
            a.y[(size_t)q * r + lane] = y;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && bad) atomicOr(a.status, (int)kStatusSingularSolve);
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
    gauss_jordan_wave(Aug, r, ld, prow, &bad);
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

// RMAX: rank bound (32 or 64); RMAX / 2 column pairs of 16 lanes, each lane RMAX / 16 rows.
template <int RMAX>
__global__ __launch_bounds__(kSvdLanes * RMAX / 2) void k_svd(int r, const double* __restrict__ Rin,
                                                               double* __restrict__ Vout, double* __restrict__ Sout,
                                                               int* status, const double* __restrict__ Tl) {
    constexpr int NT = kSvdLanes * RMAX / 2, RT = RMAX / kSvdLanes;
    __shared__ double S[RMAX * RMAX];
    __shared__ double V[RMAX * RMAX];
    __shared__ double nrm[RMAX];
    __shared__ int order[RMAX];
    __shared__ double sTl[RMAX * RMAX];   // with Tl: Tl; sP: the sorted S V
    __shared__ double sP[RMAX * RMAX];
    const int tid = threadIdx.x;
    const int rr = r * r;
    if (Tl) stage_lds(sTl, Tl, rr);   // read at the end; the barriers of the sweeps order it
    // column-major: column c of S = R^T is row c of R, S[c * r + i] = R[c][i]; the lanes of a pair
    // read consecutive rows of a column (no bank conflicts)
    for (int o = tid; o < rr; o += NT) {
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
                    double sp[RT], sq[RT], vp[RT], vq[RT];
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
                        const int i = lane + kSvdLanes * t;
                        const int ic = i < r ? i : r - 1;
                        sp[t] = S[p * r + ic];
                        sq[t] = S[q * r + ic];
                        vp[t] = V[p * r + ic];
                        vq[t] = V[q * r + ic];
                    }
                    double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                    for (int t = 0; t < RT; ++t) {
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
                        // zeta = (be - al) / (2 ga), written without forming zeta.  The angle need not be
                        // exact (a slightly different rotation is still a rotation; the sweeps go on until
                        // every pair is orthogonal), so the quotient takes the hardware reciprocal and two
                        // Newton steps; cos and sin come from an exact reciprocal square root, which keeps
                        // the rotation orthogonal to working precision.
                        const double d = be - al;
                        const double sgn = (d * ga >= 0.0) ? 1.0 : -1.0;
                        const double den = fabs(d) + sqrt(d * d + 4.0 * ga * ga);   // >= 2 |ga| > 0
                        double rc = __builtin_amdgcn_rcp(den);
                        rc = fma(rc, fma(-den, rc, 1.0), rc);
                        rc = fma(rc, fma(-den, rc, 1.0), rc);
                        const double tt = sgn * (2.0 * fabs(ga)) * rc;
                        const double c = rsqrt(1.0 + tt * tt);
                        const double sn = c * tt;
                        rotated = 1;
#pragma unroll
                        for (int t = 0; t < RT; ++t) {
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
    for (int c = tid; c < r; c += NT) {
        double sum = 0.0;
        for (int i = 0; i < r; ++i) sum += S[c * r + i] * S[c * r + i];
        nrm[c] = sqrt(sum);
    }
    __syncthreads();
    // stable descending order: rank of column c = columns with a larger norm, or an equal norm
    // and a smaller index
    for (int c = tid; c < r; c += NT) {
        int rank = 0;
        for (int m = 0; m < r; ++m) rank += (nrm[m] > nrm[c] || (nrm[m] == nrm[c] && m < c)) ? 1 : 0;
        order[rank] = c;
    }
    __syncthreads();
    for (int c = tid; c < r; c += NT) {
        const int src = order[c];
        int m = 0;
        double best = -1.0;
        for (int i = 0; i < r; ++i)
            if (fabs(V[src * r + i]) > best) { best = fabs(V[src * r + i]); m = i; }
        const double sg = (V[src * r + m] < 0.0) ? -1.0 : 1.0;
        for (int i = 0; i < r; ++i) {
            Vout[i * r + c] = sg * V[src * r + i];
            if (Tl)
                sP[i * r + c] = sg * S[src * r + i];
            else
                Sout[i * r + c] = sg * S[src * r + i];
        }
    }
    if (Tl) {   // Sout = Tl (S V), one output per thread and pass (consecutive threads: consecutive columns)
        __syncthreads();
        for (int o = tid; o < rr; o += NT) {
            const int i = o / r, c = o % r;
            double acc = 0.0;
            for (int k = 0; k < r; ++k) acc = fma(sTl[i * r + k], sP[k * r + c], acc);
            Sout[o] = acc;
        }
    }
}

// X[k][c] = sum_j V[j][c] M[j][k]; one thread per output, consecutive threads along c
__global__ __launch_bounds__(256) void k_rmul(int n, int rin, int rout, int ldm, const double* __restrict__ V,
                                              const double* __restrict__ M, double* __restrict__ X) {
    __shared__ double sM[kMaxRank * kMaxRank];
    stage_lds(sM, M, rin * ldm);
    __syncthreads();
    const long o = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (long)n * rout) return;
    const int k = (int)(o / n), c = (int)(o % n);
    double s = 0.0;
#pragma unroll 8
    for (int j = 0; j < rin; ++j) s += V[(size_t)j * n + c] * sM[j * ldm + k];
    X[(size_t)k * n + c] = s;
}

// Rank-r truncation of an SVD result held as U Sigma (columns U_k sigma_k of the ra x ra row-major Sv):
// Q R of its first r columns by classical Gram-Schmidt with two passes.  Sv is staged in LDS once; the
// working column sits in LDS, thread j forms its product with accepted column j serially over the rows
// (rows padded to 65 doubles, so the threads' reads fall in different banks), then 64 threads subtract
// them.  Norms are serial sums in one thread, so nothing depends on timing.  A column with nothing left
// after the passes (a zero singular value) takes the unit vector with the largest remainder, which
// keeps Q orthonormal; R_kk is then 0.
__global__ __launch_bounds__(256) void k_trunc(int ra, int r, const double* __restrict__ Sv, double* __restrict__ Q,
                                               double* __restrict__ R) {
    constexpr int kC = kMaxRank / 2, kP = 65;
    __shared__ double sQ[kC * kP];
    __shared__ double sv[64];
    __shared__ double sh[kC];
    __shared__ double sR[kC * kC];
    __shared__ double sS[kMaxRank * kMaxRank];
    __shared__ double snrm[2];
    const int t = threadIdx.x;
    for (int o = t; o < r * r; o += 256) sR[o] = 0.0;
    stage_lds(sS, Sv, ra * ra);
    __syncthreads();
    // two passes of v -= Q_{<k} (Q_{<k}^T v) on the vector in sv; with rcol >= 0 the coefficients are
    // added to column rcol of R.  Called by every thread (it holds barriers).
    auto orth = [&](int k, int rcol) {
        for (int pass = 0; pass < 2; ++pass) {
            if (t < k) {
                double d = 0.0;
                for (int i = 0; i < 64; ++i) d = fma(sQ[t * kP + i], sv[i], d);
                sh[t] = d;
                if (rcol >= 0) sR[t * r + rcol] += d;
            }
            __syncthreads();
            if (t < 64) {
                double v = sv[t];
                for (int j = 0; j < k; ++j) v = fma(-sh[j], sQ[j * kP + t], v);
                sv[t] = v;
            }
            __syncthreads();
        }
    };
    auto norm = [&](int slot) {
        if (t == 0) {
            double s2 = 0.0;
            for (int i = 0; i < 64; ++i) s2 = fma(sv[i], sv[i], s2);
            snrm[slot] = sqrt(s2);
        }
        __syncthreads();
    };
    for (int k = 0; k < r; ++k) {
        if (t < 64) sv[t] = t < ra ? sS[t * ra + k] : 0.0;
        __syncthreads();
        norm(0);
        orth(k, k);
        norm(1);
        const double own = snrm[0], nrm = snrm[1];
        double rkk = nrm;
        if (!(own > 0.0 && nrm > 1e-12 * own)) {   // the same decision in every thread
            double bn = -1.0;
            int best = 0;
            for (int m = 0; m < ra; ++m) {
                if (t < 64) sv[t] = (t == m) ? 1.0 : 0.0;
                __syncthreads();
                orth(k, -1);
                norm(1);
                if (snrm[1] > bn) bn = snrm[1], best = m;
                __syncthreads();
            }
            if (t < 64) sv[t] = (t == best) ? 1.0 : 0.0;
            __syncthreads();
            orth(k, -1);
            norm(1);
            rkk = 0.0;
        }
        const double scale = 1.0 / snrm[1];
        if (t < 64) {
            const double qv = t < ra ? sv[t] * scale : 0.0;
            sQ[k * kP + t] = qv;
            if (t < ra) Q[t * r + k] = qv;
        }
        if (t == 0) sR[k * r + k] = rkk;
        __syncthreads();
    }
    for (int o = t; o < r * r; o += 256) R[o] = sR[o];
}

// beta_k = sum_q w_q W_k(q), coef = S beta; wavefront k sums column k (fixed lane order)
__global__ __launch_bounds__(1024) void k_wsum(int nq, int r, const double* __restrict__ W,
                                               const double* __restrict__ w, const double* __restrict__ S,
                                               double* __restrict__ beta, double* __restrict__ coef,
                                               const double* __restrict__ mu, const double* __restrict__ eta,
                                               double* __restrict__ gside, int transpose_s,
                                               const double* __restrict__ Tl) {
    __shared__ double sb[kMaxRank];
    __shared__ double sgs[4][kMaxRank];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool sides = gside != nullptr;
    // columns k and k + 16 of a wavefront are summed together (twice the loads in flight); each keeps
    // its own lane order and butterfly.  With the side vectors, the ordinate's weight times its
    // exit cosine goes to the side it leaves through (left mu < 0, right mu > 0, bottom eta < 0,
    // top eta > 0).
    for (int k = wv; k < r; k += 32) {
        const int k2 = k + 16;
        const bool two = k2 < r;
        double acc = 0.0, acc2 = 0.0;
        double g[4] = {0.0, 0.0, 0.0, 0.0}, g2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
        for (int q = lane; q < nq; q += 64) {
            const double wq = w[q];
            const double x = W[(size_t)k * nq + q];
            const double x2 = two ? W[(size_t)k2 * nq + q] : 0.0;
            acc += wq * x;
            if (two) acc2 += wq * x2;
            if (sides) {
                const double m = mu[q], e = eta[q];
                const double fx = wq * fabs(m), fy = wq * fabs(e);
                const int sx = m > 0.0 ? 1 : 0, sy = e > 0.0 ? 3 : 2;
#pragma unroll
                for (int sd = 0; sd < 4; ++sd) {
                    const double f = sd == sx ? fx : (sd == sy ? fy : 0.0);
                    g[sd] += f * x;
                    g2[sd] += f * x2;
                }
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            acc += __shfl_xor(acc, off);
            acc2 += __shfl_xor(acc2, off);
        }
        if (sides) {
#pragma unroll
            for (int sd = 0; sd < 4; ++sd)
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    g[sd] += __shfl_xor(g[sd], off);
                    g2[sd] += __shfl_xor(g2[sd], off);
                }
        }
        if (lane == 0) {
            sb[k] = acc;
            if (two) sb[k2] = acc2;
            if (sides)
                for (int sd = 0; sd < 4; ++sd) {
                    sgs[sd][k] = g[sd];
                    if (two) sgs[sd][k2] = g2[sd];
                }
        }
    }
    __syncthreads();
    __shared__ double sS[kMaxRank * kMaxRank];
    __shared__ double sT[kMaxRank * kMaxRank];
    __shared__ double sE[kMaxRank * (kMaxRank + 1)];
    // without S (the identity) the matrix used is Tl itself
    stage_lds(sS, S ? S : Tl, r * r);
    if (S && Tl) stage_lds(sT, Tl, r * r);
    __syncthreads();
    // S[i][j] is sS[i * r + j], or sS[j * r + i] when the matrix given is S^T; with Tl the matrix used
    // is Tl S (formed in LDS first)
    int si = (S && transpose_s) ? 1 : r, sj = (S && transpose_s) ? r : 1;
    if (S && Tl) {
        // sE = Tl S.  S[k][j] is read as a row of the (transposed) matrix given when transpose_s, so
        // it is first copied with an odd stride (r + 1): consecutive threads (consecutive j) then read
        // different LDS banks instead of one bank r doubles apart
        const int ld = r + 1;
        for (int o = threadIdx.x; o < r * r; o += blockDim.x) {
            const int k = o / r, j = o % r;
            sE[j * ld + k] = sS[k * si + j * sj];   // sE holds S^T with stride ld
        }
        __syncthreads();
        for (int o = threadIdx.x; o < r * r; o += blockDim.x) {
            const int i = o / r, j = o % r;
            double acc = 0.0;
            for (int k = 0; k < r; ++k) acc = fma(sT[i * r + k], sE[j * ld + k], acc);
            sS[o] = acc;   // every read of the old sS was before the barrier above
        }
        __syncthreads();
        si = r;
        sj = 1;
    }
    for (int i = threadIdx.x; i < r; i += blockDim.x) {
        beta[i] = sb[i];
        double s = 0.0;
        for (int j = 0; j < r; ++j) s += sS[i * si + j * sj] * sb[j];
        coef[i] = s;
    }
    if (sides)
        for (int t = threadIdx.x; t < 4 * r; t += blockDim.x) {
            const int sd = t / r, i = t - sd * r;
            double s = 0.0;
            for (int j = 0; j < r; ++j) s += sS[i * si + j * sj] * sgs[sd][j];
            gside[t] = s;
        }
}

// One thread per instance.
__global__ __launch_bounds__(256) void k_gather_si(int n, const int* const* flags, const int* const* status,
                                                   const double* const* rel, int* dst_i, double* dst_d) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int* f = flags[k];
    __hip_atomic_store(dst_i + 4 * k, f[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(dst_i + 4 * k + 1, f[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(dst_i + 4 * k + 2, f[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(dst_i + 4 * k + 3, status[k][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(reinterpret_cast<unsigned long long*>(dst_d) + k,
                       (unsigned long long)__double_as_longlong(rel[k][0]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence_system();
}

// One workgroup: the runs and the status words, each value by its own thread.
__global__ __launch_bounds__(256) void k_publish(PublishArgs a) {
    int off = 0;
    for (int k = 0; k < 3; ++k) {
        for (int i = threadIdx.x; i < a.n[k]; i += blockDim.x)
            __hip_atomic_store(reinterpret_cast<unsigned long long*>(a.dst) + off + i,
                               (unsigned long long)__double_as_longlong(a.src[k][i]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        off += a.n[k];
    }
    for (int i = threadIdx.x; i < a.nstatus; i += blockDim.x)
        __hip_atomic_store(a.dst_status + i, a.status[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    for (int i = threadIdx.x; i < a.ni; i += blockDim.x)
        __hip_atomic_store(a.idst + i, a.isrc[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence_system();
    if (a.seq_dst) {   // every thread's values are fenced before the barrier; the word the host polls comes last
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(a.seq_dst, a.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

}  // namespace

void launch_deim(hipStream_t s, const DeimArgs& a) {
    const unsigned groups = (unsigned)((a.nq + kDeimThreads - 1) / kDeimThreads);
    if (groups <= 8) {
        if (a.r <= 8)
            hipLaunchKernelGGL((k_deim<8, 8>), dim3(groups), dim3(kDeimThreads), 0, s, a);
        else if (a.r <= 16)
            hipLaunchKernelGGL((k_deim<16, 8>), dim3(groups), dim3(kDeimThreads), 0, s, a);
        else if (a.r <= 32)
            hipLaunchKernelGGL((k_deim<32, 8>), dim3(groups), dim3(kDeimThreads), 0, s, a);
        else
            hipLaunchKernelGGL((k_deim<64, 8>), dim3(groups), dim3(kDeimThreads), 0, s, a);
    } else {
        if (a.r <= 8)
            hipLaunchKernelGGL((k_deim<8, kDeimMaxGroups>), dim3(groups), dim3(kDeimThreads), 0, s, a);
        else if (a.r <= 16)
            hipLaunchKernelGGL((k_deim<16, kDeimMaxGroups>), dim3(groups), dim3(kDeimThreads), 0, s, a);
        else if (a.r <= 32)
            hipLaunchKernelGGL((k_deim<32, kDeimMaxGroups>), dim3(groups), dim3(kDeimThreads), 0, s, a);
        else
            hipLaunchKernelGGL((k_deim<64, kDeimMaxGroups>), dim3(groups), dim3(kDeimThreads), 0, s, a);
    }
    hipLaunchKernelGGL(k_deim_tail, dim3(1), dim3(kDeimThreads), 0, s, a, (int)groups);
}

void launch_lstep(hipStream_t s, const LstepArgs& a) {
    const int r = a.r;
    const size_t schur_lds = (size_t)r * (r + 1) * sizeof(double);
    const unsigned wave_blocks = (unsigned)((a.nq + 3) / 4);
    if (r <= 8) {
        hipLaunchKernelGGL((k_lstep_solve_wave<8>), dim3(wave_blocks), dim3(256), 0, s, a);
    } else if (r <= 16) {
        hipLaunchKernelGGL((k_lstep_solve_wave<16>), dim3(wave_blocks), dim3(256), 0, s, a);
    } else if (r <= 32) {
        hipLaunchKernelGGL((k_lstep_solve_wave<32>), dim3(wave_blocks), dim3(256), 0, s, a);
    } else {
        const long tot = (long)a.nq * r;
        hipLaunchKernelGGL(k_lstep_rhs, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_lstep_solve_w2, dim3(a.nq), dim3(128), 0, s, a);
    }
    hipLaunchKernelGGL(k_lstep_reduce, dim3(a.red_blocks), dim3(kLsThreads), 0, s, a);
    hipLaunchKernelGGL(k_lstep_schur, dim3(1), dim3(kLsThreads), schur_lds, s, a);
    const long tot = (long)a.nq * r;
    hipLaunchKernelGGL(k_lstep_apply, dim3((unsigned)((tot + kLsThreads - 1) / kLsThreads)), dim3(kLsThreads), 0, s, a);
}

void launch_svd(hipStream_t s, int r, const double* R, double* V, double* Snew, int* status, const double* Tl) {
    if (r <= 32)
        hipLaunchKernelGGL(k_svd<32>, dim3(1), dim3(kSvdLanes * 16), 0, s, r, R, V, Snew, status, Tl);
    else
        hipLaunchKernelGGL(k_svd<64>, dim3(1), dim3(kSvdLanes * 32), 0, s, r, R, V, Snew, status, Tl);
}

void launch_rmul(hipStream_t s, int n, int r, const double* V, const double* M, double* X) {
    hipLaunchKernelGGL(k_rmul, dim3((unsigned)(((long)n * r + 255) / 256)), dim3(256), 0, s, n, r, r, r, V, M, X);
}

void launch_rmul_rect(hipStream_t s, int n, int rin, int rout, const double* V, const double* M, int ldm,
                      double* X) {
    hipLaunchKernelGGL(k_rmul, dim3((unsigned)(((long)n * rout + 255) / 256)), dim3(256), 0, s, n, rin, rout, ldm,
                       V, M, X);
}

void launch_trunc(hipStream_t s, int ra, int r, const double* Sv, double* Q, double* R) {
    hipLaunchKernelGGL(k_trunc, dim3(1), dim3(256), 0, s, ra, r, Sv, Q, R);
}

void launch_gather_si(hipStream_t s, int n, const int* const* flags, const int* const* status,
                      const double* const* rel, int* dst_i, double* dst_d) {
    if (n > 0) hipLaunchKernelGGL(k_gather_si, dim3((n + 255) / 256), dim3(256), 0, s, n, flags, status, rel, dst_i, dst_d);
}

void launch_publish(hipStream_t s, const PublishArgs& a) {
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(256), 0, s, a);
}

void launch_wsum(hipStream_t s, int nq, int r, const double* W, const double* w, const double* S, double* beta,
                 double* coef, const double* mu, const double* eta, double* gside, bool s_transposed,
                 const double* Tl) {
    hipLaunchKernelGGL(k_wsum, dim3(1), dim3(1024), 0, s, nq, r, W, w, S, beta, coef, mu, eta, gside,
                       s_transposed ? 1 : 0, Tl);
}

}  // namespace dlr
