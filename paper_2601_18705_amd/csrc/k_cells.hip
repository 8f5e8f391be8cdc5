// Per-cell kernels of the DLR step: linearisation, reconstruction of the old
// solution at the selected ordinates, the scalar-flux update inside source
// iteration, and the temperature update.  All are bandwidth-bound streams over
// the N cells.  Column-major fields ([r][N] for X) are read with unit stride
// across a wavefront.  The kernels that read or write the diagonal sweep layout
// walk tiles of 8 columns x 128 rows (32 threads per column, consecutive rows):
// a 128-byte line of that layout holds 8 lanes x 4 diagonals, so a workgroup
// writes and reads whole lines.
#include "dlr_internal.h"

#include <algorithm>

namespace dlr {

namespace {

constexpr int kBlock = 256;

// Deterministic block sum of one double (fixed tree order).
__device__ double block_sum(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Last-block-done reduction: each block stores its partial(s) with store_partial; the
// block that retires last sums all partials in index order and resets the counter.
// The partials and the counter are agent-scope atomics: they are performed at the
// device-coherent level, so no cache-wide fence is needed between the per-XCD L2s;
// thread 0 waits until its partial stores have completed before it counts the block.
__device__ __forceinline__ void store_partial(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_vm_stores() {
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt and lgkmcnt unconstrained
}
__device__ bool retire_block(unsigned* counter) {
    __shared__ bool last;
    __syncthreads();
    if (threadIdx.x == 0) {
        wait_vm_stores();
        const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    return last;
}
__device__ void reset_counter(unsigned* counter) {
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ double ordered_sum(const double* p, int count, int stride, double* sh) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x)
        acc += __hip_atomic_load(p + (size_t)i * stride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return block_sum(acc, sh);
}

// ---------------------------------------------------------------------------------------------- tiles
constexpr int kTileCols = 8, kTileRows = 128;

struct TileGrid {
    int nx, ny, ntx, nty;
    __device__ int count() const { return ntx * nty; }
    // cell k (0..3) of thread threadIdx.x in tile b; false outside the grid
    __device__ bool cell(int b, int k, int& i, int& j) const {
        const int tx = b / nty, ty = b % nty;
        i = tx * kTileCols + (threadIdx.x >> 5);
        j = ty * kTileRows + (threadIdx.x & 31) + 32 * k;
        return i < nx && j < ny;
    }
};
inline TileGrid tile_grid(int nx, int ny) {
    return TileGrid{nx, ny, (nx + kTileCols - 1) / kTileCols, (ny + kTileRows - 1) / kTileRows};
}
static_assert(kBlock * 4 == kTileCols * kTileRows, "four cells per thread");

// ---------------------------------------------------------------------------------------------- linearise
// Newton linearisation of backward Euler for the material energy (Sec. 2.2):
//   D = rho c_v + 4 pi dt sigma dB/dT, sigma_s = (4 pi dt sigma dB/dT / D) sigma,
//   q = sigma B(T0) rho c_v / D + q_ext / (4 pi), sigma_t = sigma + 1/(c dt).
// sigma_t goes to the four orientation copies of the diagonal layout.
__global__ __launch_bounds__(kBlock) void k_linearize(TileGrid g, const double* __restrict__ sigma,
                                                      const double* __restrict__ rho_cv,
                                                      const double* __restrict__ q_ext, const double* __restrict__ T,
                                                      double dt, double a, double c, double* __restrict__ D,
                                                      double* __restrict__ sig_s, double* __restrict__ q,
                                                      double* __restrict__ sig_t64, float* __restrict__ sig_t32,
                                                      size_t ldg, double* __restrict__ q_diag) {
    for (int b = blockIdx.x; b < g.count(); b += gridDim.x) {
        // the loads of the thread's four cells first (cells outside the grid read cell (0, 0)), then
        // the arithmetic and stores of the cells inside
        bool ok[4];
        int ci[4], cj[4];
        double tv[4], sv[4], cv[4], qx[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            ok[k] = g.cell(b, k, ci[k], cj[k]);
            if (!ok[k]) ci[k] = cj[k] = 0;
            const long e = (long)ci[k] * g.ny + cj[k];
            tv[k] = T[e];
            sv[k] = sigma[e];
            cv[k] = rho_cv[e];
            qx[k] = q_ext ? q_ext[e] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!ok[k]) continue;
            const int i = ci[k], j = cj[k];
            const long e = (long)i * g.ny + j;
            const double t = tv[k], s = sv[k], C = cv[k];
            const double t3 = t * t * t;
            const double B0 = a * c * t3 * t / kFourPi;
            const double dB = a * c * t3 / kPi;
            const double d = C + kFourPi * dt * s * dB;
            D[e] = d;
            sig_s[e] = (kFourPi * dt * s * dB / d) * s;
            const double qe = s * B0 * C / d + (q_ext ? qx[k] / kFourPi : 0.0);
            q[e] = qe;
            const double st = s + 1.0 / (c * dt);
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                const size_t pe = (size_t)o * ldg + diag_pos(g.nx, g.ny, o, i, j);
                if (sig_t64) sig_t64[pe] = st;
                if (sig_t32) sig_t32[pe] = (float)st;
                if (q_diag) q_diag[pe] = qe;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------- psi0
// Algorithm 1 step 3: psi_d^(0) = sum_k X0_k L0_k(Omega^(d)) = (X0 C0)[:, d] with
// C0 = S0 W0[sel]^T, folded into the fixed sweep source src0 = q + psi^(0)/(c dt),
// written in direction d's diagonal layout.  Also the source-iteration start
// phi = X0 S0 beta and s_e = sigma_s phi / (4 pi) (four orientation copies).
template <typename TS, int RMAX>
__global__ __launch_bounds__(kBlock) void k_psi0_wide(TileGrid g, int r, const double* __restrict__ X,
                                                 const double* __restrict__ C0, const double* __restrict__ a0,
                                                 const double* __restrict__ q, const double* __restrict__ sig_s,
                                                 double inv_cdt, const double* __restrict__ mu,
                                                 const double* __restrict__ eta, TS* __restrict__ src0, size_t ldg,
                                                 double* __restrict__ phi, TS* __restrict__ s_e, int* zero4) {
    if (zero4 && blockIdx.x == 0 && threadIdx.x < 4) zero4[threadIdx.x] = 0;
    // C0, a0 and the orientations are uniform across the workgroup: they are read with scalar
    // loads (through the scalar cache), which keeps the inner product off the LDS pipe
    const long n = (long)g.nx * g.ny;
    for (int b = blockIdx.x; b < g.count(); b += gridDim.x) {
        for (int kc = 0; kc < 4; ++kc) {
            int i, j;
            if (!g.cell(b, kc, i, j)) continue;
            const long e = (long)i * g.ny + j;
            // acc[d] = sum_k X_k(e) C0[k][d] in passes of 16 directions: a row of C0 is 16
            // contiguous doubles (wide scalar loads into 32 SGPRs); X_k(e) is re-read from cache
            constexpr int kPass = RMAX < 16 ? RMAX : 16;
            double ph = 0.0;
#pragma unroll 1
            for (int k = 0; k < r; ++k) ph += X[(size_t)k * n + e] * a0[k];
            phi[e] = ph;
            size_t pos[4];
#pragma unroll
            for (int o = 0; o < 4; ++o) pos[o] = diag_pos(g.nx, g.ny, o, i, j);
            const TS se = (TS)(sig_s[e] * ph / kFourPi);
#pragma unroll
            for (int o = 0; o < 4; ++o) s_e[(size_t)o * ldg + pos[o]] = se;
            const double qe = q[e];
#pragma unroll 1
            for (int d0 = 0; d0 < r; d0 += kPass) {
                double acc[kPass];
#pragma unroll
                for (int d = 0; d < kPass; ++d) acc[d] = 0.0;
#pragma unroll 1
                for (int k = 0; k < r; ++k) {
                    const double xk = X[(size_t)k * n + e];
#pragma unroll
                    for (int d = 0; d < kPass; ++d) acc[d] += xk * C0[k * r + (d0 + d < r ? d0 + d : r - 1)];
                }
#pragma unroll
                for (int d = 0; d < kPass; ++d) {
                    if (d0 + d >= r) break;
                    const int o = orient_of(mu[d0 + d], eta[d0 + d]);
                    const size_t pd = o == 0 ? pos[0] : o == 1 ? pos[1] : o == 2 ? pos[2] : pos[3];
                    src0[(size_t)(d0 + d) * ldg + pd] = (TS)(qe + acc[d] * inv_cdt);
                }
            }
        }
    }
}

// Four consecutive values as vector accesses (16-byte aligned), on the compiler's native vector types
// (the field-wise HIP vector structs can be split into narrower memory instructions).
typedef float fv4 __attribute__((ext_vector_type(4)));
typedef double dv2 __attribute__((ext_vector_type(2)));
__device__ inline void load_quad(const float* p, float (&v)[4]) {
    const fv4 x = *reinterpret_cast<const fv4*>(p);
    v[0] = x[0], v[1] = x[1], v[2] = x[2], v[3] = x[3];
}
__device__ inline void load_quad(const double* p, double (&v)[4]) {
    const dv2 x = *reinterpret_cast<const dv2*>(p), y = *reinterpret_cast<const dv2*>(p + 2);
    v[0] = x[0], v[1] = x[1], v[2] = y[0], v[3] = y[1];
}
__device__ inline void store_quad(float* p, const float (&v)[4]) {
    *reinterpret_cast<fv4*>(p) = fv4{v[0], v[1], v[2], v[3]};
}
__device__ inline void store_quad(double* p, const double (&v)[4]) {
    *reinterpret_cast<dv2*>(p) = dv2{v[0], v[1]};
    *reinterpret_cast<dv2*>(p + 2) = dv2{v[2], v[3]};
}

typedef double dv4 __attribute__((ext_vector_type(4)));

// Ranks up to 32 on the matrix cores, in workgroup tiles of 8 columns x RT rows.
// MFMA phase: per 16-cell piece of one column the wavefront forms D = C0^T X^T (blocks of 16 directions
// x 16 cells) with v_mfma_f64_16x16x4.  C0^T (zero-padded to RMAX x RMAX) stays in registers for the
// launch; X is read straight from memory as the B operand (four k rows of 16 consecutive cells per
// instruction, rows past r clamped to a valid row that meets a zero of C0).  Lane l supplies A[l%16][l/16]
// and B[l/16][l%16], and its accumulator element v is D[4 v + l/16][l%16].  The src0 values and
// sigma_s phi / (4 pi) go to LDS (one row per direction plus one); phi = X a0 is summed over the lane's k
// rows and across the four lane rows and written directly.
// Store phase: in a direction's diagonal layout the tile's column holds RT consecutive positions t, which
// touch RT/4 + 1 aligned groups of four; a thread writes one group of one column (a 16-byte store, or
// single values in the groups cut by the tile's top and bottom rows), so eight consecutive threads cover
// whole 128-byte lines (one in FP32, two in FP64).  The s_e row is written the same way into each of the
// four orientation copies.
template <typename TS, int RMAX, int RT>
__global__ __launch_bounds__(kBlock) void k_psi0_mfma(int nx, int ny, int r, const double* __restrict__ X,
                                                      const double* __restrict__ C0, const double* __restrict__ a0,
                                                      const double* __restrict__ q, const double* __restrict__ sig_s,
                                                      double inv_cdt, const double* __restrict__ mu,
                                                      const double* __restrict__ eta, TS* __restrict__ src0,
                                                      size_t ldg, double* __restrict__ phi, TS* __restrict__ s_e,
                                                      int* zero4) {
    static_assert(RMAX % 16 == 0 && RMAX <= 32 && RT % 16 == 0, "16-direction blocks, 16-cell pieces");
    if (zero4 && blockIdx.x == 0 && threadIdx.x < 4) zero4[threadIdx.x] = 0;
    constexpr int NB = RMAX / 16, KS = RMAX / 4;
    constexpr int NP = 8 * RT / 16;                     // 16-cell pieces per tile
    constexpr int SD = 8 * RT + 32 / (int)sizeof(TS);   // LDS row stride: two-way bank access in both phases
    constexpr int NG = RT / 4 + 1;                      // aligned groups one column's RT positions touch
    static_assert(NP % 8 == 0, "pieces in pairs per wavefront");
    __shared__ TS sD[(RMAX + 1) * SD];
    __shared__ int so[RMAX];
    const int lane = threadIdx.x & 63, c = lane & 15, kr = lane >> 4, w = threadIdx.x >> 6;
    double A[NB][KS], al[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const int k = 4 * ks + kr;
        al[ks] = k < r ? a0[k] : 0.0;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int d = 16 * nb + c;
            A[nb][ks] = (k < r && d < r) ? C0[k * r + d] : 0.0;
        }
    }
    for (int k = threadIdx.x; k < RMAX; k += kBlock) so[k] = k < r ? orient_of(mu[k], eta[k]) : 0;
    const int nty = (ny + RT - 1) / RT, ntiles = ((nx + 7) / 8) * nty;
    const long n = (long)nx * ny;
    const int G = diag_groups(ny);
    for (int b = blockIdx.x; b < ntiles; b += gridDim.x) {
        const int i0 = (b / nty) * 8, j0 = (b % nty) * RT;
        __syncthreads();   // the previous tile's rows are stored (and so[] is set)
        // pairs of pieces (m0, m0 + 4), m0 = w, w + 8, ...: the next pair's X is loaded before the
        // current pair's products
        double xb[2][KS];
        auto load_pair = [&](int m0) {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int m = m0 + 4 * u, col = m / (RT / 16), row = (m % (RT / 16)) * 16 + c;
                const long e = (long)min(i0 + col, nx - 1) * ny + min(j0 + row, ny - 1);
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) xb[u][ks] = X[(size_t)min(4 * ks + kr, r - 1) * n + e];
            }
        };
        load_pair(w);
#pragma unroll 1
        for (int m0 = w; m0 < NP; m0 += 8) {
            double xc[2][KS];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) xc[u][ks] = xb[u][ks];
            if (m0 + 8 < NP) load_pair(m0 + 8);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int m = m0 + 4 * u, col = m / (RT / 16), row = (m % (RT / 16)) * 16 + c;
                const bool live = i0 + col < nx && j0 + row < ny;
                const long e = (long)min(i0 + col, nx - 1) * ny + min(j0 + row, ny - 1);
                const int loc = col * RT + row;
                dv4 acc[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[nb] = dv4{0.0, 0.0, 0.0, 0.0};
                double ph = 0.0;
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb)
                        acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[nb][ks], xc[u][ks], acc[nb], 0, 0, 0);
                    ph = fma(xc[u][ks], al[ks], ph);
                }
                ph += __shfl_xor(ph, 16);
                ph += __shfl_xor(ph, 32);
                if (live && kr == 0) phi[e] = ph;
                const double qe = q[e];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        sD[(16 * nb + 4 * v + kr) * SD + loc] = (TS)(qe + acc[nb][v] * inv_cdt);
                if (kr == 0) sD[RMAX * SD + loc] = (TS)(sig_s[e] * ph / kFourPi);
            }
        }
        __syncthreads();
        const int jmax = min(j0 + RT, ny) - 1;   // last row of the tile inside the grid
#pragma unroll 2
        for (int task = threadIdx.x; task < (r + 4) * NG * 8; task += kBlock) {
            const int cc = task & 7, gi = (task >> 3) % NG, dd = (task >> 3) / NG;
            const int i = i0 + cc;
            if (i >= nx) continue;
            const int o = dd < r ? so[dd] : dd - r;
            const TS* sv = sD + (dd < r ? dd : RMAX) * SD + cc * RT;
            TS* plane = dd < r ? src0 + (size_t)dd * ldg : s_e + (size_t)(dd - r) * ldg;
            const int ip = (o & 1) ? nx - 1 - i : i, l = ip & 63;
            const int tlo = ((o & 2) ? ny - 1 - jmax : j0) + l;   // first position of the column's rows
            const int gg = (tlo >> 2) + gi;
            TS v[4];
            int nok = 0, okm = 0;
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int jp = 4 * gg + s4 - l, j = (o & 2) ? ny - 1 - jp : jp;
                const bool ok = j >= j0 && j <= jmax;
                v[s4] = sv[ok ? j - j0 : 0];
                nok += ok;
                okm |= (int)ok << s4;
            }
            if (nok == 0) continue;
            TS* p = plane + (((size_t)(ip >> 6) * G + gg) * 64 + l) * 4;
            if (nok == 4) {
                store_quad(p, v);
            } else {
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4)
                    if (okm >> s4 & 1) p[s4] = v[s4];
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------- phi
// Scalar flux of the collocation system (Sec. 4.1): phi = beta^T What^{-1} Psi =
// sum_d cw_d psi_d, its pseudo-scattering source, and the relative change
// ||phi_new - phi_old||_2 / ||phi_new||_2 written to out[2] by the last block:
// k_phi_partial + k_phi_combine (with the plain SN kernels below).

// ---------------------------------------------------------------------------------------------- Psi relayout
// Psi (four diagonal layouts) -> compact cell planes.  A thread owns column i and the four rows j0..j0+3.
// In a direction's layout those rows are the consecutive diagonal positions t = a..a+3 (in reverse order
// when the orientation flips j), which lie in the aligned groups floor(a/4) and floor(a/4) + 1 of the
// column's lane: both are loaded as vectors and the four values picked by a & 3.  DU directions are
// loaded before any is stored; positions of rows beyond ny are clamped into the layout and not stored.
template <typename TS, int DU>
__global__ __launch_bounds__(kBlock) void k_psi_to_cm(TileGrid g, int r, const TS* __restrict__ psi, size_t ldg,
                                                      const double* __restrict__ mu, const double* __restrict__ eta,
                                                      TS* __restrict__ psi_cm, size_t ld) {
    __shared__ int so[kMaxRank];
    for (int i = threadIdx.x; i < r; i += blockDim.x) so[i] = orient_of(mu[i], eta[i]);
    __syncthreads();
    const int G = diag_groups(g.ny);
    const bool vec = (g.ny & 3) == 0;   // 16-byte aligned row quads in the compact planes
    for (int b = blockIdx.x; b < g.count(); b += gridDim.x) {
        const int tx = b / g.nty, ty = b % g.nty;
        // a wavefront covers the tile's 8 columns x 32 rows: its loads touch few, mostly whole,
        // lines of the diagonal layouts and its stores write whole 128-byte column segments
        const int i = tx * kTileCols + (threadIdx.x & 7);
        const int j0 = ty * kTileRows + (threadIdx.x >> 3) * 4;
        if (i >= g.nx || j0 >= g.ny) continue;
        TS* out = psi_cm + (size_t)i * g.ny + j0;
        for (int d0 = 0; d0 < r; d0 += DU) {
            TS lo[DU][4], hi[DU][4];
#pragma unroll
            for (int u = 0; u < DU; ++u) {
                const int d = min(d0 + u, r - 1);
                const int o = so[d];
                // the column's lane l in direction d's layout, and the first position a of the rows
                // (arithmetic on the orientation bits: indexed per-thread tables end up in LDS)
                const int ip = (o & 1) ? g.nx - 1 - i : i, l = ip & 63;
                const int a = ((o & 2) ? g.ny - 4 - j0 : j0) + l;
                const TS* p = psi + (size_t)d * ldg + ((size_t)(ip >> 6) * G * 64 + l) * 4;
                load_quad(p + (size_t)max(a >> 2, 0) * 256, lo[u]);
                load_quad(p + (size_t)min((a >> 2) + 1, G - 1) * 256, hi[u]);
            }
#pragma unroll
            for (int u = 0; u < DU; ++u) {
                const int d = d0 + u;
                if (d < r) {   // a guard, not a break: the loop must unroll (lo, hi stay in registers)
                    const int o = so[d];
                    const int l = ((o & 1) ? g.nx - 1 - i : i) & 63;
                    const int s = (((o & 2) ? g.ny - 4 - j0 : j0) + l) & 3;
                    // positions a & 3 .. (a & 3) + 3 of the two groups, selected on named values (an
                    // indexed array here is turned into address selects and placed in LDS)
                    const bool s1 = s & 1, s2 = s & 2;
                    TS a0 = s1 ? lo[u][1] : lo[u][0], a1 = s1 ? lo[u][2] : lo[u][1];
                    TS a2 = s1 ? lo[u][3] : lo[u][2], a3 = s1 ? hi[u][0] : lo[u][3];
                    const TS a4 = s1 ? hi[u][1] : hi[u][0], a5 = s1 ? hi[u][2] : hi[u][1];
                    a0 = s2 ? a2 : a0;
                    a1 = s2 ? a3 : a1;
                    a2 = s2 ? a4 : a2;
                    a3 = s2 ? a5 : a3;
                    const bool rev = o & 2;
                    TS v[4] = {rev ? a3 : a0, rev ? a2 : a1, rev ? a1 : a2, rev ? a0 : a3};
                    TS* q = out + (size_t)d * ld;
                    if (vec) {
                        store_quad(q, v);
                    } else {
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            if (j0 + k < g.ny) q[k] = v[k];
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------- T update
// Algorithm 1 step 9 with the mean intensity of the new factors phi = X (S beta):
//   T = T0 + dt sigma (phi - a c T0^4) / D,  and energy sum area * (rho c_v T + phi / c).
// With the side vectors gside[s] = S (sum over the ordinates leaving through side s of
// w_q |Omega_q . n| W_q), the intensity leaving a wall cell e through side s, summed over
// ordinates, is X(e) . gside[s]; times the face length this is the cell's share of the
// outflow tally of the time-discrete energy balance.
// RMAX >= r: the r values X_k(e) of a cell are loaded together (clamped rows, all in flight)
template <int RMAX>
__global__ __launch_bounds__(kBlock) void k_tupdate(TupdateArgs A) {
    __shared__ double sh[kBlock];
    __shared__ double sc[kMaxRank];
    __shared__ double sg[4][kMaxRank];
    const int n = A.nx * A.ny, r = A.r;
    for (int i = threadIdx.x; i < r; i += blockDim.x) sc[i] = A.coef[i];
    if (A.gside)
        for (int i = threadIdx.x; i < 4 * r; i += blockDim.x) sg[i / r][i % r] = A.gside[i];
    __syncthreads();
    double en = 0.0, ob = 0.0;
    bool bad = false;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        // The coefficients and side vectors are read from LDS in every pass: held in registers across
        // the loop (5 r doubles, the compiler's choice without this barrier) they left room for one
        // wavefront per SIMD, and a CU that holds another kernel's workgroup (the SVD beside this
        // kernel) took none of these blocks.
        asm volatile("" ::: "memory");
        double ph = 0.0;
        double v[RMAX];
        if (A.X) {
#pragma unroll
            for (int k = 0; k < RMAX; ++k) v[k] = A.X[(size_t)(k < r ? k : r - 1) * n + e];
#pragma unroll
            for (int k = 0; k < RMAX; ++k)
                if (k < r) ph = fma(v[k], sc[k], ph);
        } else {
            ph = A.phi[e];   // plain SN: the converged scalar flux
        }
        const double t0 = A.T[e];
        const double emis = A.a * A.c * t0 * t0 * t0 * t0;
        const double t = t0 + A.dt * A.sigma[e] * (ph - emis) / A.D[e];
        A.T[e] = t;
        A.phi[e] = ph;
        en += A.rho_cv[e] * t + ph / A.c;
        bad |= !(isfinite(ph) && isfinite(t));
        if (A.X && A.gside) {
            // column-major cells: e = i * ny + j
            const unsigned ci = (unsigned)e / (unsigned)A.ny, cj = (unsigned)e - ci * (unsigned)A.ny;
            const bool on[4] = {ci == 0u, ci == (unsigned)A.nx - 1u, cj == 0u, cj == (unsigned)A.ny - 1u};
            if (on[0] || on[1] || on[2] || on[3]) {
#pragma unroll
                for (int sd = 0; sd < 4; ++sd) {
                    if (!on[sd]) continue;
                    double o = 0.0;
#pragma unroll
                    for (int k = 0; k < RMAX; ++k)
                        if (k < r) o = fma(v[k], sg[sd][k], o);
                    ob = fma(sd < 2 ? A.hy : A.hx, o, ob);
                }
            }
        }
    }
    if (bad) atomicOr(A.status, (int)kStatusNonfinite);
    en = block_sum(en, sh);
    ob = block_sum(ob, sh);
    if (threadIdx.x == 0) {
        store_partial(&A.partials[2 * blockIdx.x], en);
        store_partial(&A.partials[2 * blockIdx.x + 1], ob);
    }
    if (retire_block(A.counter)) {
        const double E = ordered_sum(A.partials, gridDim.x, 2, sh);
        const double O = ordered_sum(A.partials + 1, gridDim.x, 2, sh);
        if (threadIdx.x == 0) {
            A.out[0] = E * A.area;
            if (A.gside) A.out[1] = O;
            reset_counter(A.counter);
        }
    }
}

// Outflow tally of plain SN from every ordinate's intensity: in its sweep coordinates an
// ordinate leaves through the last column i' = nx - 1 (x faces, length hy) and the last row
// j' = ny - 1 (y faces, length hx).  Each block takes ordinates d = block, block + grid, ...;
// out[1] = sum over d of w_d (|mu_d| hy sum_j' psi(nx-1, j') + |eta_d| hx sum_i' psi(i', ny-1)).
template <typename TS>
__global__ __launch_bounds__(kBlock) void k_sn_outflow(int nx, int ny, int nq, size_t ldg,
                                                       const double* __restrict__ mu, const double* __restrict__ eta,
                                                       const double* __restrict__ w, const TS* __restrict__ psi,
                                                       double hx, double hy, double* __restrict__ partials,
                                                       unsigned* counter, double* out) {
    __shared__ double sh[kBlock];
    const int ndg = diag_groups(ny);
    auto at = [&](const TS* p, int ip, int jp) {
        const int l = ip & 63, t = jp + l;
        return (double)p[((size_t)((ip >> 6) * ndg + (t >> 2)) * 64 + l) * 4 + (t & 3)];
    };
    double acc = 0.0;
    for (int d = blockIdx.x; d < nq; d += gridDim.x) {
        const TS* p = psi + (size_t)d * ldg;
        double sx = 0.0, sy = 0.0;
        for (int jp = threadIdx.x; jp < ny; jp += blockDim.x) sx += at(p, nx - 1, jp);
        for (int ip = threadIdx.x; ip < nx; ip += blockDim.x) sy += at(p, ip, ny - 1);
        acc += w[d] * (fabs(mu[d]) * hy * sx + fabs(eta[d]) * hx * sy);
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) store_partial(&partials[blockIdx.x], acc);
    if (retire_block(counter)) {
        const double O = ordered_sum(partials, gridDim.x, 1, sh);
        if (threadIdx.x == 0) {
            out[1] = O;
            reset_counter(counter);
        }
    }
}

// ---------------------------------------------------------------------------------------------- plain SN
// Discrete ordinates without the low-rank factorisation (the comparator of the DLR step):
// every ordinate is swept, phi = sum_q w_q psi_q, and psi of the previous step is the time
// source.  Ordinates are listed grouped by orientation (dirs[off[o] .. off[o+1])), so the
// directions of one orientation share a diagonal layout.

// src0_d = q + psi_old_d / (c dt) over whole planes (padding positions compute padding)
template <typename TS>
__global__ __launch_bounds__(kBlock) void k_sn_source(int nq, size_t ldg, const int* __restrict__ orient,
                                                      const double* __restrict__ q_diag,
                                                      const TS* __restrict__ psi_old, double inv_cdt,
                                                      TS* __restrict__ src0) {
    const size_t total = (size_t)nq * ldg;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (size_t)gridDim.x * blockDim.x) {
        const size_t d = k / ldg, pos = k - d * ldg;
        src0[k] = (TS)(q_diag[(size_t)orient[d] * ldg + pos] + (double)psi_old[k] * inv_cdt);
    }
}

// psi_d = B(T) for every ordinate, phi = 4 pi B(T), s_e = sigma_s phi / (4 pi) (isotropic start)
template <typename TS>
__global__ __launch_bounds__(kBlock) void k_sn_init(TileGrid g, int nq, size_t ldg, const int* __restrict__ orient,
                                                    const double* __restrict__ T, double a, double c,
                                                    TS* __restrict__ psi, double* __restrict__ phi) {
    const long n = (long)g.nx * g.ny;
    (void)n;
    for (int b = blockIdx.x; b < g.count(); b += gridDim.x) {
        for (int kc = 0; kc < 4; ++kc) {
            int i, j;
            if (!g.cell(b, kc, i, j)) continue;
            const long e = (long)i * g.ny + j;
            const double t = T[e];
            const double B = a * c * t * t * t * t / kFourPi;
            phi[e] = kFourPi * B;
            size_t pos[4];
#pragma unroll
            for (int o = 0; o < 4; ++o) pos[o] = diag_pos(g.nx, g.ny, o, i, j);
            for (int d = 0; d < nq; ++d) {
                const int o = orient[d];
                const size_t pd = o == 0 ? pos[0] : o == 1 ? pos[1] : o == 2 ? pos[2] : pos[3];
                psi[(size_t)d * ldg + pd] = (TS)B;
            }
        }
    }
}

// Scalar flux in two passes.  The directions of one orientation share a diagonal layout, so
// the first pass sums their weighted intensities position by position with contiguous
// four-element loads: phio[o][pos] = sum over the directions d of orientation o of
// w_d psi_d[pos].  Directions come as a list grouped by orientation (dirs, off) or, with
// dirs = nullptr, as nd directions filtered by the orientation of (mu_d, eta_d).
template <typename TS>
__global__ __launch_bounds__(kBlock) void k_phi_partial(size_t ldg, int nd, const int* __restrict__ dirs,
                                                        const int* __restrict__ off, const double* __restrict__ mu,
                                                        const double* __restrict__ eta,
                                                        const double* __restrict__ w, const TS* __restrict__ psi,
                                                        double* __restrict__ phio, const int* ctl) {
    typedef TS tv4 __attribute__((ext_vector_type(4)));
    if (ctl && *ctl) return;   // the source iteration has stopped
    const int o = blockIdx.y;
    // without a list, the block first lists the directions of orientation o in order (nd <= 64: the
    // selected directions of a rank-r factorisation), so the loop below has no per-direction branch
    // and unrolls with several loads in flight
    __shared__ int sdir[64];
    __shared__ int sndir;
    if (!dirs) {
        if (threadIdx.x < 64) {
            const int d = threadIdx.x;
            const bool m = d < nd && orient_of(mu[d], eta[d]) == o;
            const unsigned long long mask = __ballot(m);
            if (m) sdir[__popcll(mask & ((1ull << d) - 1ull))] = d;
            if (d == 0) sndir = __popcll(mask);
        }
        __syncthreads();
    }
    const int k0 = dirs ? off[o] : 0, cnt = dirs ? off[o + 1] - off[o] : sndir;
    const size_t nquad = ldg / 4;
    for (size_t qd = (size_t)blockIdx.x * blockDim.x + threadIdx.x; qd < nquad; qd += (size_t)gridDim.x * blockDim.x) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 8
        for (int k = 0; k < cnt; ++k) {
            const int d = dirs ? dirs[k0 + k] : sdir[k];
            const double wd = w[d];
            const tv4 v = *reinterpret_cast<const tv4*>(psi + (size_t)d * ldg + 4 * qd);
            a0 += wd * (double)v.x;
            a1 += wd * (double)v.y;
            a2 += wd * (double)v.z;
            a3 += wd * (double)v.w;
        }
        double* dst = phio + (size_t)o * ldg + 4 * qd;
        *reinterpret_cast<double2*>(dst) = make_double2(a0, a1);
        *reinterpret_cast<double2*>(dst + 2) = make_double2(a2, a3);
    }
}

// Second pass: phi = sum_o phio[o] at the cell's position in each orientation, the four
// copies of s_e = sigma_s phi / (4 pi), and the source-iteration change norm
// (||phi_new - phi_old||^2, ||phi_new||^2 and their ratio, summed in block order).
template <typename TS>
__global__ __launch_bounds__(kBlock) void k_phi_combine(TileGrid g, size_t ldg, const double* __restrict__ phio,
                                                           const double* __restrict__ sig_s,
                                                           const double* __restrict__ phi_old,
                                                           double* __restrict__ phi_new, TS* __restrict__ s_e,
                                                           double* __restrict__ partials, unsigned* counter,
                                                           double* out, SiControl ctl) {
    __shared__ double sh[kBlock];
    // every block reads the flag before the last one of this launch can set it
    if (ctl.flag && *ctl.flag) return;
    double d2 = 0.0, p2 = 0.0;
    for (int b = blockIdx.x; b < g.count(); b += gridDim.x) {
        // the loads of the thread's four cells first (cells outside the grid read cell (0, 0)), so
        // they are in flight together; then the sums and stores of the cells inside
        bool ok[4];
        long e[4];
        size_t pos[4][4];
        double po[4][4], pold[4], ss[4];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            int i, j;
            ok[kc] = g.cell(b, kc, i, j);
            if (!ok[kc]) i = j = 0;
            e[kc] = (long)i * g.ny + j;
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                pos[kc][o] = diag_pos(g.nx, g.ny, o, i, j);
                po[kc][o] = phio[(size_t)o * ldg + pos[kc][o]];
            }
            pold[kc] = phi_old[e[kc]];
            ss[kc] = sig_s[e[kc]];
        }
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            if (!ok[kc]) continue;
            double ph = 0.0;
#pragma unroll
            for (int o = 0; o < 4; ++o) ph += po[kc][o];
            const double diff = ph - pold[kc];
            d2 += diff * diff;
            p2 += ph * ph;
            phi_new[e[kc]] = ph;
            const TS se = (TS)(ss[kc] * ph / kFourPi);
#pragma unroll
            for (int o = 0; o < 4; ++o) s_e[(size_t)o * ldg + pos[kc][o]] = se;
        }
    }
    d2 = block_sum(d2, sh);
    p2 = block_sum(p2, sh);
    if (threadIdx.x == 0) {
        store_partial(&partials[2 * blockIdx.x], d2);
        store_partial(&partials[2 * blockIdx.x + 1], p2);
    }
    if (retire_block(counter)) {
        const double D2 = ordered_sum(partials, gridDim.x, 2, sh);
        const double P2 = ordered_sum(partials + 1, gridDim.x, 2, sh);
        if (threadIdx.x == 0) {
            const double rel = (P2 > 0.0) ? sqrt(D2) / sqrt(P2) : (D2 > 0.0 ? 1.0 : 0.0);
            out[0] = D2;
            out[1] = P2;
            out[2] = rel;
            if (ctl.flag) {
                const int it = ctl.flag[1] + 1;
                ctl.flag[1] = it;
                const int why = !isfinite(rel) ? 2 : (rel <= ctl.tol ? 1 : (it >= ctl.max_iter ? 3 : 0));
                if (why) {
                    ctl.flag[2] = why;
                    ctl.flag[0] = 1;
                }
            }
            reset_counter(counter);
        }
    }
}

// phi = X coef (the mean intensity of given factors: coef = S beta)
__global__ __launch_bounds__(kBlock) void k_phi_of_factors(int n, int r, const double* __restrict__ X,
                                                           const double* __restrict__ coef, double* __restrict__ phi) {
    __shared__ double sc[kMaxRank];
    for (int i = threadIdx.x; i < r; i += blockDim.x) sc[i] = coef[i];
    __syncthreads();
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        double ph = 0.0;
        for (int k = 0; k < r; ++k) ph += X[(size_t)k * n + e] * sc[k];
        phi[e] = ph;
    }
}

}  // namespace

constexpr int kMaxTileBlocks = 1024;

template <typename TS>
void launch_sn_source(hipStream_t s, int nq, size_t ldg, const int* orient, const double* q_diag, const TS* psi_old,
                      double inv_cdt, TS* src0) {
    const size_t total = (size_t)nq * ldg;
    const unsigned blocks = (unsigned)std::min<size_t>((total + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL((k_sn_source<TS>), dim3(blocks), dim3(kBlock), 0, s, nq, ldg, orient, q_diag, psi_old, inv_cdt,
                       src0);
}
template <typename TS>
void launch_sn_init(hipStream_t s, int nx, int ny, int nq, size_t ldg, const int* orient, const double* T, double a,
                    double c, TS* psi, double* phi) {
    const TileGrid g = tile_grid(nx, ny);
    hipLaunchKernelGGL((k_sn_init<TS>), dim3(std::min(g.ntx * g.nty, kMaxTileBlocks)), dim3(kBlock), 0, s, g, nq, ldg,
                       orient, T, a, c, psi, phi);
}
template <typename TS>
void launch_phi_two_pass(hipStream_t s, int nx, int ny, size_t ldg, int nd, const int* dirs, const int* off,
                         const double* mu, const double* eta, const double* w, const TS* psi, double* phio,
                         const double* sig_s, const double* phi_old, double* phi_new, TS* s_e, double* partials,
                         int nblocks, unsigned* counter, double* out, const SiControl* ctl = nullptr) {
    const unsigned bx = (unsigned)std::min<size_t>((ldg / 4 + kBlock - 1) / kBlock, 2048);
    const SiControl c = ctl ? *ctl : SiControl{nullptr, 0.0, 0};
    hipLaunchKernelGGL((k_phi_partial<TS>), dim3(bx, 4), dim3(kBlock), 0, s, ldg, nd, dirs, off, mu, eta, w, psi,
                       phio, c.flag);
    const TileGrid g = tile_grid(nx, ny);
    hipLaunchKernelGGL((k_phi_combine<TS>), dim3(nblocks), dim3(kBlock), 0, s, g, ldg, phio, sig_s, phi_old, phi_new,
                       s_e, partials, counter, out, c);
}
template <typename TS>
void launch_sn_phi(hipStream_t s, int nx, int ny, size_t ldg, const int* dirs, const int* off, const double* w,
                   const TS* psi, double* phio, const double* sig_s, const double* phi_old, double* phi_new, TS* s_e,
                   double* partials, int nblocks, unsigned* counter, double* out) {
    launch_phi_two_pass<TS>(s, nx, ny, ldg, 0, dirs, off, nullptr, nullptr, w, psi, phio, sig_s, phi_old, phi_new, s_e,
                            partials, nblocks, counter, out);
}
#define DLR_SN_INST(TS)                                                                                              \
    template void launch_sn_source<TS>(hipStream_t, int, size_t, const int*, const double*, const TS*, double, TS*); \
    template void launch_sn_init<TS>(hipStream_t, int, int, int, size_t, const int*, const double*, double, double,  \
                                     TS*, double*);                                                                  \
    template void launch_sn_phi<TS>(hipStream_t, int, int, size_t, const int*, const int*, const double*, const TS*, \
                                    double*, const double*, const double*, double*, TS*, double*, int, unsigned*,     \
                                    double*);
DLR_SN_INST(float)
DLR_SN_INST(double)
#undef DLR_SN_INST

void launch_phi_of_factors(hipStream_t s, int n, int r, const double* X, const double* coef, double* phi) {
    hipLaunchKernelGGL(k_phi_of_factors, dim3(std::min((n + kBlock - 1) / kBlock, 4096)), dim3(kBlock), 0, s, n, r, X,
                       coef, phi);
}

// ---------------------------------------------------------------------------------------------- launchers

void launch_linearize(hipStream_t s, int nx, int ny, const double* sigma, const double* rho_cv, const double* q_ext,
                      const double* T, double dt, double a, double c, double* D, double* sig_s, double* q,
                      double* sig_t64, float* sig_t32, size_t ldg, double* q_diag) {
    const TileGrid g = tile_grid(nx, ny);
    hipLaunchKernelGGL(k_linearize, dim3(std::min(g.ntx * g.nty, kMaxTileBlocks)), dim3(kBlock), 0, s, g, sigma,
                       rho_cv, q_ext, T, dt, a, c, D, sig_s, q, sig_t64, sig_t32, ldg, q_diag);
}

template <typename TS>
void launch_psi0(hipStream_t s, int nx, int ny, int r, const double* X, const double* C0, const double* a0,
                 const double* q, const double* sig_s, double inv_cdt, const double* mu, const double* eta,
                 TS* src0, size_t ldg, double* phi, TS* s_e, int* zero4) {
    constexpr int RT = sizeof(TS) == 4 ? 64 : 32;
    const int tiles = ((nx + 7) / 8) * ((ny + RT - 1) / RT);
    const dim3 b(kBlock), gm(std::min(tiles, 4096));
    if (r <= 16) {
        hipLaunchKernelGGL((k_psi0_mfma<TS, 16, RT>), gm, b, 0, s, nx, ny, r, X, C0, a0, q, sig_s, inv_cdt, mu, eta,
                           src0, ldg, phi, s_e, zero4);
    } else if (r <= 32) {
        hipLaunchKernelGGL((k_psi0_mfma<TS, 32, RT>), gm, b, 0, s, nx, ny, r, X, C0, a0, q, sig_s, inv_cdt, mu, eta,
                           src0, ldg, phi, s_e, zero4);
    } else {
        const TileGrid g = tile_grid(nx, ny);
        hipLaunchKernelGGL((k_psi0_wide<TS, 64>), dim3(std::min(g.ntx * g.nty, kMaxTileBlocks)), b, 0, s, g, r, X, C0,
                           a0, q, sig_s, inv_cdt, mu, eta, src0, ldg, phi, s_e, zero4);
    }
}
template void launch_psi0<double>(hipStream_t, int, int, int, const double*, const double*, const double*,
                                  const double*, const double*, double, const double*, const double*, double*, size_t,
                                  double*, double*, int*);
template void launch_psi0<float>(hipStream_t, int, int, int, const double*, const double*, const double*,
                                 const double*, const double*, double, const double*, const double*, float*, size_t,
                                 double*, float*, int*);

template <typename TS>
void launch_phi(hipStream_t s, int nx, int ny, int r, const TS* psi, size_t ldg, const double* mu, const double* eta,
                const double* cw, double* phio, const double* sig_s, const double* phi_old, double* phi_new, TS* s_e,
                double* partials, int nblocks, unsigned* counter, double* out, const SiControl* ctl) {
    launch_phi_two_pass<TS>(s, nx, ny, ldg, r, nullptr, nullptr, mu, eta, cw, psi, phio, sig_s, phi_old, phi_new, s_e,
                            partials, nblocks, counter, out, ctl);
}
template void launch_phi<double>(hipStream_t, int, int, int, const double*, size_t, const double*, const double*,
                                 const double*, double*, const double*, const double*, double*, double*, double*, int,
                                 unsigned*, double*, const SiControl*);
template void launch_phi<float>(hipStream_t, int, int, int, const float*, size_t, const double*, const double*,
                                const double*, double*, const double*, const double*, double*, float*, double*, int,
                                unsigned*, double*, const SiControl*);

template <typename TS>
void launch_psi_to_cm(hipStream_t s, int nx, int ny, int r, const TS* psi, size_t ldg, const double* mu,
                      const double* eta, TS* psi_cm, size_t ld) {
    const TileGrid g = tile_grid(nx, ny);
    hipLaunchKernelGGL((k_psi_to_cm<TS, sizeof(TS) == 4 ? 8 : 4>), dim3(std::min(g.ntx * g.nty, kMaxTileBlocks)), dim3(kBlock), 0, s, g, r, psi,
                       ldg, mu, eta, psi_cm, ld);
}
template void launch_psi_to_cm<double>(hipStream_t, int, int, int, const double*, size_t, const double*,
                                       const double*, double*, size_t);
template void launch_psi_to_cm<float>(hipStream_t, int, int, int, const float*, size_t, const double*, const double*,
                                      float*, size_t);

void launch_tupdate(hipStream_t s, const TupdateArgs& A, int nblocks) {
    const dim3 g(nblocks), b(kBlock);
    if (A.r <= 8)
        hipLaunchKernelGGL(k_tupdate<8>, g, b, 0, s, A);
    else if (A.r <= 16)
        hipLaunchKernelGGL(k_tupdate<16>, g, b, 0, s, A);
    else if (A.r <= 32)
        hipLaunchKernelGGL(k_tupdate<32>, g, b, 0, s, A);
    else
        hipLaunchKernelGGL(k_tupdate<64>, g, b, 0, s, A);
}

template <typename TS>
void launch_sn_outflow(hipStream_t s, int nx, int ny, int nq, size_t ldg, const double* mu, const double* eta,
                       const double* w, const TS* psi, double hx, double hy, double* partials, int nblocks,
                       unsigned* counter, double* out) {
    hipLaunchKernelGGL(k_sn_outflow<TS>, dim3(std::max(1, std::min(nblocks, nq))), dim3(kBlock), 0, s, nx, ny, nq,
                       ldg, mu, eta, w, psi, hx, hy, partials, counter, out);
}
template void launch_sn_outflow<double>(hipStream_t, int, int, int, size_t, const double*, const double*,
                                        const double*, const double*, double, double, double*, int, unsigned*,
                                        double*);
template void launch_sn_outflow<float>(hipStream_t, int, int, int, size_t, const double*, const double*,
                                       const double*, const float*, double, double, double*, int, unsigned*,
                                       double*);

}  // namespace dlr
