// Tall-skinny contractions over the cells on the FP64 matrix cores:
//   * Gram matrices V^T V of the swept columns (Cholesky QR of Algorithm 1 step 5);
//   * the Galerkin projections of the L-step (Sec. 4.3): <X_i, X_j(left neighbour)>,
//     <X_i, X_j(lower neighbour)>, <X_i, sigma X_j>, <X_i, sigma_s X_j>, <X0_i, X_j>,
//     and the vectors <q, X_i> and the sums of X_i over the four boundary sides.
//
// Each block walks chunks of 64 consecutive (column-major) cells, stages the r
// basis columns of a chunk in LDS as FP64, and its four wavefronts each own a
// fixed set of 16 x 16 output tiles, accumulated with v_mfma_f64_16x16x4 over
// the 16 four-cell k-steps of the chunk.  Partial sums are written per block and
// added by k_sum_partials in a fixed order, so every result is bitwise
// reproducible.
#include "dlr_internal.h"

namespace dlr {

namespace {

typedef double dv4 __attribute__((ext_vector_type(4)));
typedef double dv2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;   // four wavefronts
constexpr int kPC = 64;         // cells per chunk = 16 k-steps of 4 cells
constexpr int kPS = kPC + 4;    // LDS row stride (doubles): one leading neighbour slot, spreads the banks

__device__ __forceinline__ dv4 mfma4(double a, double b, dv4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Operands of v_mfma_f64_16x16x4: lane l supplies A[l%16][l/16] and B[l/16][l%16]; its accumulator
// element v holds D[4*v + l/16][l%16] (measured on gfx950; the FP32 16x16x4 form differs).
__device__ __forceinline__ void store_tile(double* out, int r, int ti, int tj, dv4 acc, double scale) {
    const int lane = threadIdx.x & 63;
    const int j = tj * 16 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = ti * 16 + 4 * v + (lane >> 4);
        if (i < r && j < r) out[i * r + j] = acc[v] * scale;
    }
}

typedef float fv4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ fv4 mfma4(float a, float b, fv4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Accumulator layout of v_mfma_f32_16x16x4: lane l, element v holds D[4*(l/16) + v][l%16].
__device__ __forceinline__ void store_tile(double* out, int r, int ti, int tj, fv4 acc, double scale) {
    const int lane = threadIdx.x & 63;
    const int j = tj * 16 + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = ti * 16 + 4 * (lane >> 4) + v;
        if (i < r && j < r) out[i * r + j] = (double)acc[v] * scale;
    }
}

typedef short bf4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ short to_bf16(float x) {
    unsigned u = __builtin_bit_cast(unsigned, x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(short h) {
    return __builtin_bit_cast(float, (unsigned)(unsigned short)h << 16);
}
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi): the pair carries about 16 mantissa bits
struct bf4x2 {
    bf4 hi, lo;
};
__device__ __forceinline__ bf4x2 split_bf16(float a, float b, float c, float d) {
    const float v[4] = {a, b, c, d};
    bf4x2 o;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const short h = to_bf16(v[j]);
        o.hi[j] = h;
        o.lo[j] = to_bf16(v[j] - from_bf16(h));
    }
    return o;
}
// v_mfma_f32_16x16x16_bf16: lane l supplies A[l%16][4*(l/16) + j] and B[4*(l/16) + j][l%16], j = 0..3;
// the accumulator layout is that of the FP32 16x16x4 form (measured on gfx950).
__device__ __forceinline__ fv4 mfma16(bf4 a, bf4 b, fv4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// A B with split operands: hi*hi + hi*lo + lo*hi (the lo*lo term is below FP32 rounding of the sum)
__device__ __forceinline__ fv4 mfma16x3(const bf4x2& a, const bf4x2& b, fv4 c) {
    c = mfma16(a.lo, b.hi, c);
    c = mfma16(a.hi, b.lo, c);
    return mfma16(a.hi, b.hi, c);
}

template <typename TO> struct AccOf;
template <> struct AccOf<double> { typedef dv4 type; };
template <> struct AccOf<float> { typedef fv4 type; };

// ------------------------------------------------------------------------------------------------ Gram
// partial_b[i*r + j] = scale * sum over the cells of block b of V_i(e) wt(e) V_j(e), wt = weight or 1.
// Operands come straight from memory, no LDS: a wavefront takes passes of 32 cells, and in a pass lane l
// holds cells 8 (l/16) .. 8 (l/16) + 7 of plane 16 tb + l%16 for each 16-plane block tb (one 32- or
// 64-byte load per block).  k-step s (0..7) of v_mfma_f64_16x16x4 pairs cell 8 (l/16) + s of the A and B
// operands, so the eight k-steps cover the pass's 32 cells (the sum over cells is order-free).  Only the
// tiles ti <= tj are formed (the matrix is symmetric; the mirror is written at the end).  Planes past r are
// clamped to a valid one (their rows and columns are not stored), cells past n are zero.  The four
// wavefronts' sums are added through LDS in wavefront order, so every result is bitwise reproducible.
template <typename TV, int RT>
__global__ __launch_bounds__(kThreads) void k_gram_mfma(long n, int r, const TV* __restrict__ V, size_t ldv,
                                                        const double* __restrict__ weight, double scale,
                                                        double* __restrict__ partials) {
    constexpr int NT = RT * (RT + 1) / 2;
    __shared__ double sacc[NT * 4 * 64];
    const int lane = threadIdx.x & 63, w = (threadIdx.x >> 6) & 3, p = lane & 15, g = lane >> 4;
    dv4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = dv4{0.0, 0.0, 0.0, 0.0};
    size_t base[RT];
#pragma unroll
    for (int tb = 0; tb < RT; ++tb) base[tb] = (size_t)min(16 * tb + p, r - 1) * ldv;
    // 8 consecutive cells as two or four 16-byte loads: planes and their leading dimension are aligned
    const bool vec = (ldv % 8 == 0) && ((reinterpret_cast<uintptr_t>(V) & 63) == 0);
    const long passes = (n + 31) / 32;
    const long stride = (long)gridDim.x * 4;
    double cur[RT][8], wt[8];
    auto load = [&](long ps) {
        const long c0 = ps * 32 + 8 * g;
        if (vec && c0 + 8 <= n) {
#pragma unroll
            for (int tb = 0; tb < RT; ++tb) {
                const TV* q = V + base[tb] + c0;
                if constexpr (sizeof(TV) == 4) {
                    const fv4 x = *reinterpret_cast<const fv4*>(q), y = *reinterpret_cast<const fv4*>(q + 4);
#pragma unroll
                    for (int k = 0; k < 4; ++k) cur[tb][k] = x[k], cur[tb][4 + k] = y[k];
                } else {
#pragma unroll
                    for (int k = 0; k < 8; k += 2) {
                        const dv2 x = *reinterpret_cast<const dv2*>(q + k);
                        cur[tb][k] = x[0], cur[tb][k + 1] = x[1];
                    }
                }
            }
        } else {
#pragma unroll
            for (int tb = 0; tb < RT; ++tb)
#pragma unroll
                for (int k = 0; k < 8; ++k) cur[tb][k] = c0 + k < n ? (double)V[base[tb] + c0 + k] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) wt[k] = (weight && c0 + k < n) ? weight[c0 + k] : 1.0;
    };
    long ps = blockIdx.x * 4 + w;
    if (ps < passes) load(ps);
    for (; ps < passes; ps += stride) {
        double v[RT][8], vw[RT][8];
#pragma unroll
        for (int tb = 0; tb < RT; ++tb)
#pragma unroll
            for (int k = 0; k < 8; ++k) v[tb][k] = cur[tb][k], vw[tb][k] = cur[tb][k] * wt[k];
        if (ps + stride < passes) load(ps + stride);   // in flight during the products below
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            int t = 0;
#pragma unroll
            for (int ti = 0; ti < RT; ++ti)
#pragma unroll
                for (int tj = ti; tj < RT; ++tj, ++t) acc[t] = mfma4(v[ti][k], vw[tj][k], acc[t]);
        }
    }
    // wavefront 0 writes its sums, wavefronts 1..3 add theirs in order, then the block's partial is stored
#pragma unroll 1
    for (int ww = 0; ww < 4; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    double& dst = sacc[(t * 4 + e) * 64 + lane];
                    dst = (ww == 0 ? 0.0 : dst) + acc[t][e];
                }
        }
        __syncthreads();
    }
    double* out = partials + (size_t)blockIdx.x * r * r;
    for (int o = threadIdx.x; o < NT * 4 * 64; o += kThreads) {
        const int t = o / 256, e = (o / 64) % 4, l = o % 64;
        int ti = 0, tj = 0, tt = t;
        while (tt >= RT - ti) tt -= RT - ti, ++ti;
        tj = ti + tt;
        const int i = ti * 16 + 4 * e + (l >> 4), j = tj * 16 + (l & 15);   // D[4 e + l/16][l%16]
        if (i < r && j < r) {
            const double val = sacc[o] * scale;
            out[i * r + j] = val;
            if (ti != tj) out[j * r + i] = val;
        }
    }
}

// ------------------------------------------------------------------------------------------ projections
// Partial layout per block: [5 r^2 matrices][5 r vectors]
//   M0 = sum X_i(i,j) X_j(i-1,j)   (x-upwind neighbour, 0 on column 0)
//   M1 = sum X_i(i,j) X_j(i,j-1)   (y-upwind neighbour, 0 on row 0)
//   M2 = sum sigma X_i X_j,  M3 = sum sigma_s X_i X_j,  M4 = sum X0_i X_j (rows i >= r0 zero: X0
//   has r0 <= r columns, fewer than X when the basis was augmented)
//   v0 = sum q X_i,  v1..v4 = sums of X_i over the left / right / bottom / top cells
// Column-major cells e = i*ny + j: (i-1,j) = e - ny and (i,j-1) = e - 1.
//
// A wavefront owns whole 16 x 16 tile pairs (ti, tj) and accumulates all five matrices of each,
// so per four-cell k-step it reads two A operands (X, X0 at ti) and three B operands (X at the
// left neighbour, the lower neighbour and the cell, at tj) once for five MFMAs.  With one tile
// pair (r <= 16) the four wavefronts split the k-steps instead and are added at the end.  The
// next chunk's global loads are issued before the current chunk's MFMAs (register staging).
template <int RT>
struct ProjShape {
    static constexpr int RP = 16 * RT;
    static constexpr int NPAIR = RT * RT;
    static constexpr int KS = NPAIR >= 4 ? 1 : 4;                       // k-step split across wavefronts
    static constexpr int PPW = NPAIR >= 4 ? (NPAIR + 3) / 4 : 1;         // tile pairs per wavefront
};

template <int RT, typename TO, bool BF16 = false>
__global__ __launch_bounds__(kThreads) void k_project_mfma(int nx, int ny, int r, int r0, const double* __restrict__ X,
                                                           const double* __restrict__ X0,
                                                           const double* __restrict__ sigma,
                                                           const double* __restrict__ sig_s,
                                                           const double* __restrict__ q,
                                                           double* __restrict__ partials) {
    using Sh = ProjShape<RT>;
    constexpr int RP = Sh::RP, PPW = Sh::PPW, KS = Sh::KS;
    constexpr int TPP = kThreads / RP;   // threads per basis column for the vectors
    typedef typename AccOf<TO>::type Acc;
    __shared__ TO sX[RP * kPS];          // slot c+1 holds cell c0+c, slot 0 the cell before the chunk
    __shared__ TO sXl[RP * kPS];         // X at the left neighbour (e - ny)
    __shared__ TO sX0[RP * kPS];
    constexpr bool kLowOp = sizeof(TO) < sizeof(double);
    __shared__ double sXv[kLowOp ? RP * (kPC + 1) : 1];   // X in FP64 for the vector sums (low-precision operands)
    __shared__ double sSig[kPC], sSs[kPC];
    __shared__ int sFlag[kPC];           // bit0 left side, bit1 right, bit2 bottom, bit3 top
    __shared__ double red[4][kThreads];
    const long n = (long)nx * ny;
    // the & 3 tells the compiler the range of the wavefront index, so that the tile-pair guards
    // below fold away and the MFMA accumulators stay put (no copies around each MFMA)
    const int lane = threadIdx.x & 63, w = (threadIdx.x >> 6) & 3;
    Acc acc[PPW][5];
#pragma unroll
    for (int pp = 0; pp < PPW; ++pp)
#pragma unroll
        for (int m = 0; m < 5; ++m) acc[pp][m] = Acc{0, 0, 0, 0};
    const int pv = threadIdx.x % RP, cv = threadIdx.x / RP;
    double vl = 0.0, vr = 0.0, vb = 0.0, vt = 0.0;
    const long nch = (n + kPC - 1) / kPC;

    // register staging of one chunk: thread t holds cell c0 + (t & 63) of planes (t >> 6) + 4u,
    // and threads t < RP the cell before the chunk (the lower neighbour of its first cell) of plane t
    constexpr int NP = RP / 4;
    const int sc = threadIdx.x & (kPC - 1), sp = threadIdx.x / kPC;
    double gX[NP], gL[NP], g0[NP], gH = 0.0;
    double gs = 0.0, gss = 0.0, gq = 0.0;   // gq: q at this thread's staged cell (every thread)
    // sum_e q(e) X_p(e) for this thread's staged planes p = sp + 4u, accumulated in registers as the
    // chunks are committed (summed over the wavefront's cells at the end)
    double vqr[NP];
#pragma unroll
    for (int u = 0; u < NP; ++u) vqr[u] = 0.0;
    bool edge = false, edge_cur = false;   // the staged / committed chunk holds cells on the grid boundary
    int gf = 0;
    auto stage = [&](long ch) {
        const long c0 = ch * kPC;
        const long e = c0 + sc;
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            const int p = sp + 4 * u;
            const bool ok = p < r && e < n;
            gX[u] = ok ? X[(size_t)p * n + e] : 0.0;
            gL[u] = (ok && e >= ny) ? X[(size_t)p * n + e - ny] : 0.0;
            g0[u] = (ok && p < r0) ? X0[(size_t)p * n + e] : 0.0;
        }
        if (threadIdx.x < RP) gH = (threadIdx.x < r && c0 > 0) ? X[(size_t)threadIdx.x * n + c0 - 1] : 0.0;
        gq = e < n ? q[e] : 0.0;
        const long jlo = c0 % ny;   // first column position of the chunk (it may run into the next column)
        edge = c0 < ny || c0 + kPC > n - ny || jlo == 0 || jlo + kPC >= ny;
        if (threadIdx.x < kPC) {
            gs = gss = 0.0;
            gf = 0;
            if (e < n) {
                gs = sigma[e];
                gss = sig_s[e];
                const int ei = (int)e, i = ei / ny, j = ei - i * ny;   // cell counts stay below 2^31
                gf = (i == 0 ? 1 : 0) | (i == nx - 1 ? 2 : 0) | (j == 0 ? 4 : 0) | (j == ny - 1 ? 8 : 0);
            }
        }
    };
    auto commit = [&]() {
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            const int p = sp + 4 * u;
            sX[p * kPS + sc + 1] = (TO)gX[u];
            if (kLowOp && edge) sXv[p * (kPC + 1) + sc + 1] = gX[u];
            vqr[u] = fma(gq, gX[u], vqr[u]);
            sXl[p * kPS + sc] = (TO)gL[u];
            sX0[p * kPS + sc] = (TO)g0[u];
        }
        if (threadIdx.x < RP) {
            sX[threadIdx.x * kPS] = (TO)gH;
            if (kLowOp && edge) sXv[threadIdx.x * (kPC + 1)] = gH;
        }
        edge_cur = edge;
        if (threadIdx.x < kPC) {
            sSig[threadIdx.x] = gs;
            sSs[threadIdx.x] = gss;
            sFlag[threadIdx.x] = gf;
        }
    };

    long ch = blockIdx.x;
    if (ch < nch) stage(ch);
    for (; ch < nch; ch += gridDim.x) {
        __syncthreads();   // the previous chunk's LDS reads are done
        commit();
        __syncthreads();
        if (ch + gridDim.x < nch) stage(ch + gridDim.x);   // in flight during the MFMAs below
        if constexpr (BF16) {
            // sixteen cells per k-step; this lane's four consecutive cells c4 .. c4+3
            for (int ks = (KS == 1 ? 0 : w); ks < kPC / 16; ks += KS) {
                const int c4 = 16 * ks + 4 * (lane >> 4);
                float sg[4], ss[4];
                bool bottom[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    sg[j] = (float)sSig[c4 + j];
                    ss[j] = (float)sSs[c4 + j];
                    bottom[j] = (sFlag[c4 + j] & 4) != 0;
                }
#pragma unroll
                for (int pp = 0; pp < PPW; ++pp) {
                    const int pr = (KS == 1) ? w + 4 * pp : 0;
                    if (pr < Sh::NPAIR) {
                        const int pa = (pr / RT) * 16 + (lane & 15), pb = (pr % RT) * 16 + (lane & 15);
                        float ax[4], a0[4], bx[4], bl[4], bd[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            ax[j] = (float)sX[pa * kPS + c4 + j + 1];
                            a0[j] = (float)sX0[pa * kPS + c4 + j];
                            bx[j] = (float)sX[pb * kPS + c4 + j + 1];
                            bl[j] = (float)sXl[pb * kPS + c4 + j];
                            bd[j] = bottom[j] ? 0.0f : (float)sX[pb * kPS + c4 + j];
                        }
                        const bf4x2 Ax = split_bf16(ax[0], ax[1], ax[2], ax[3]);
                        const bf4x2 A0 = split_bf16(a0[0], a0[1], a0[2], a0[3]);
                        acc[pp][0] = mfma16x3(Ax, split_bf16(bl[0], bl[1], bl[2], bl[3]), acc[pp][0]);
                        acc[pp][1] = mfma16x3(Ax, split_bf16(bd[0], bd[1], bd[2], bd[3]), acc[pp][1]);
                        acc[pp][2] = mfma16x3(
                            Ax, split_bf16(sg[0] * bx[0], sg[1] * bx[1], sg[2] * bx[2], sg[3] * bx[3]), acc[pp][2]);
                        acc[pp][3] = mfma16x3(
                            Ax, split_bf16(ss[0] * bx[0], ss[1] * bx[1], ss[2] * bx[2], ss[3] * bx[3]), acc[pp][3]);
                        acc[pp][4] = mfma16x3(A0, split_bf16(bx[0], bx[1], bx[2], bx[3]), acc[pp][4]);
                    }
                }
            }
        } else
        for (int ks = (KS == 1 ? 0 : w); ks < kPC / 4; ks += KS) {
            const int c = 4 * ks + (lane >> 4);
            const TO keep = (sFlag[c] & 4) ? (TO)0 : (TO)1;   // 0 without a lower neighbour
            const TO sg = (TO)sSig[c], ss = (TO)sSs[c];
#pragma unroll
            for (int pp = 0; pp < PPW; ++pp) {
                const int pr = (KS == 1) ? w + 4 * pp : 0;
                if (pr < Sh::NPAIR) {
                    const int pa = (pr / RT) * 16 + (lane & 15), pb = (pr % RT) * 16 + (lane & 15);
                    const TO ax = sX[pa * kPS + c + 1], a0 = sX0[pa * kPS + c];
                    const TO bx = sX[pb * kPS + c + 1];
                    const TO bl = sXl[pb * kPS + c];
                    const TO bd = keep * sX[pb * kPS + c];   // read unconditionally: no branch in the k-step
                    acc[pp][0] = mfma4(ax, bl, acc[pp][0]);
                    acc[pp][1] = mfma4(ax, bd, acc[pp][1]);
                    acc[pp][2] = mfma4(ax, sg * bx, acc[pp][2]);
                    acc[pp][3] = mfma4(ax, ss * bx, acc[pp][3]);
                    acc[pp][4] = mfma4(a0, bx, acc[pp][4]);
                }
            }
        }
        if (edge_cur && pv < r) {   // sums over the boundary sides: only chunks that hold such cells
            for (int c = cv; c < kPC; c += TPP) {
                const int f = sFlag[c];
                if (f == 0) continue;
                const double x = kLowOp ? sXv[pv * (kPC + 1) + c + 1] : (double)sX[pv * kPS + c + 1];
                if (f & 1) vl += x;
                if (f & 2) vr += x;
                if (f & 4) vb += x;
                if (f & 8) vt += x;
            }
        }
    }
    const int rr = r * r;
    double* out = partials + (size_t)blockIdx.x * (5 * rr + 5 * r);
    if (KS == 1) {
#pragma unroll
        for (int pp = 0; pp < PPW; ++pp) {
            const int pr = w + 4 * pp;
            if (pr < Sh::NPAIR)
#pragma unroll
                for (int m = 0; m < 5; ++m) store_tile(out + m * rr, r, pr / RT, pr % RT, acc[pp][m], 1.0);
        }
    } else {
        // four wavefronts hold k-step partials of the same tiles: add them in wavefront order via LDS
        __syncthreads();
        __shared__ double sacc[KS > 1 ? 4 * 5 * 256 : 1];
#pragma unroll
        for (int m = 0; m < 5; ++m)
#pragma unroll
            for (int v = 0; v < 4; ++v) sacc[((w * 5 + m) * 4 + v) * 64 + lane] = acc[0][m][v];
        __syncthreads();
        if (w == 0) {
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                Acc t = acc[0][m];
#pragma unroll
                for (int ww = 1; ww < 4; ++ww)
#pragma unroll
                    for (int v = 0; v < 4; ++v) t[v] += sacc[((ww * 5 + m) * 4 + v) * 64 + lane];
                store_tile(out + m * rr, r, 0, 0, t, 1.0);
            }
        }
    }
    // v0: each wavefront's staged planes p = sp + 4u, summed over its 64 cells in butterfly order
#pragma unroll
    for (int u = 0; u < NP; ++u) {
        double t = vqr[u];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
        const int p = sp + 4 * u;
        if (lane == 0 && p < r) out[5 * rr + p] = t;
    }
    // v1..v4: the boundary sides
    __syncthreads();
    red[0][threadIdx.x] = vl;
    red[1][threadIdx.x] = vr;
    red[2][threadIdx.x] = vb;
    red[3][threadIdx.x] = vt;
    __syncthreads();
    for (int o = threadIdx.x; o < 4 * r; o += kThreads) {
        const int kind = o / r, p = o % r;
        double acc_v = 0.0;
        for (int k = 0; k < TPP; ++k) acc_v += red[kind][p + k * RP];
        out[5 * rr + r + o] = acc_v;
    }
}

// ------------------------------------------------------------------------------------------ partial sums
// out[o] = scale * sum_b partials[b*total + o]: 16 slices of blocks (fixed stride order) per output, the
// slices added in order; 64 outputs per workgroup.
__global__ __launch_bounds__(1024) void k_sum_partials(int total, const double* __restrict__ partials, int nblocks,
                                                       double scale, double* __restrict__ out) {
    __shared__ double red[16][64];
    const int ol = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int o = blockIdx.x * 64 + ol;
    double a0 = 0.0, a1 = 0.0;
    if (o < total) {
        int b = sl;
#pragma unroll 8   // same order of additions; the loads of eight iterations in flight together
        for (; b + 16 < nblocks; b += 32) {
            a0 += partials[(size_t)b * total + o];
            a1 += partials[(size_t)(b + 16) * total + o];
        }
        if (b < nblocks) a0 += partials[(size_t)b * total + o];
    }
    red[sl][ol] = a0 + a1;
    __syncthreads();
    if (sl == 0 && o < total) {
        double s = 0.0;
        for (int k = 0; k < 16; ++k) s += red[k][ol];
        out[o] = s * scale;
    }
}

void sum_partials(hipStream_t s, int total, const double* partials, int nblocks, double scale, double* out) {
    hipLaunchKernelGGL(k_sum_partials, dim3((total + 63) / 64), dim3(1024), 0, s, total, partials, nblocks, scale,
                       out);
}

}  // namespace

template <typename TV>
void launch_gram(hipStream_t s, long n, int r, const TV* V, size_t ldv, const double* weight, double scale,
                 double* work, int nblocks, double* G) {
    const dim3 g(nblocks), b(kThreads);
    if (r <= 16)
        hipLaunchKernelGGL((k_gram_mfma<TV, 1>), g, b, 0, s, n, r, V, ldv, weight, scale, work);
    else if (r <= 32)
        hipLaunchKernelGGL((k_gram_mfma<TV, 2>), g, b, 0, s, n, r, V, ldv, weight, scale, work);
    else if (r <= 48)
        hipLaunchKernelGGL((k_gram_mfma<TV, 3>), g, b, 0, s, n, r, V, ldv, weight, scale, work);
    else
        hipLaunchKernelGGL((k_gram_mfma<TV, 4>), g, b, 0, s, n, r, V, ldv, weight, scale, work);
    sum_partials(s, r * r, work, nblocks, 1.0, G);
}
template void launch_gram<double>(hipStream_t, long, int, const double*, size_t, const double*, double, double*,
                                  int, double*);
template void launch_gram<float>(hipStream_t, long, int, const float*, size_t, const double*, double, double*, int,
                                 double*);

template <typename TO, bool BF16>
void launch_project_t(hipStream_t s, int nx, int ny, int r, int r0, const double* X, const double* X0,
                      const double* sigma, const double* sig_s, const double* q, double* partials, int nblocks) {
    const dim3 g(nblocks), b(kThreads);
    if (r <= 16)
        hipLaunchKernelGGL((k_project_mfma<1, TO, BF16>), g, b, 0, s, nx, ny, r, r0, X, X0, sigma, sig_s, q,
                           partials);
    else if (r <= 32)
        hipLaunchKernelGGL((k_project_mfma<2, TO, BF16>), g, b, 0, s, nx, ny, r, r0, X, X0, sigma, sig_s, q,
                           partials);
    else if (r <= 48)
        hipLaunchKernelGGL((k_project_mfma<3, TO, BF16>), g, b, 0, s, nx, ny, r, r0, X, X0, sigma, sig_s, q,
                           partials);
    else
        hipLaunchKernelGGL((k_project_mfma<4, TO, BF16>), g, b, 0, s, nx, ny, r, r0, X, X0, sigma, sig_s, q,
                           partials);
}

void launch_project(hipStream_t s, int nx, int ny, int r, const double* X, const double* X0, const double* sigma,
                    const double* sig_s, const double* q, double* partials, int nblocks, int operand_bits, int r0) {
    if (r0 < 0) r0 = r;
    if (operand_bits == 16)
        launch_project_t<float, true>(s, nx, ny, r, r0, X, X0, sigma, sig_s, q, partials, nblocks);
    else if (operand_bits == 32)
        launch_project_t<float, false>(s, nx, ny, r, r0, X, X0, sigma, sig_s, q, partials, nblocks);
    else
        launch_project_t<double, false>(s, nx, ny, r, r0, X, X0, sigma, sig_s, q, partials, nblocks);
}

void launch_project_sum(hipStream_t s, int r, const double* partials, int nblocks, double area, double* raw) {
    sum_partials(s, 5 * r * r + 5 * r, partials, nblocks, area, raw);
}

}  // namespace dlr
