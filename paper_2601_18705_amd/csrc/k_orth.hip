// Weighted classical Gram-Schmidt with one reorthogonalisation (CGS2) and
// deterministic completion of rank-deficient columns -- the "stabilised
// Gram-Schmidt" of Algorithm 1 steps 5 and 8.  One workgroup does the whole
// factorisation V = Q R, so it is used where V is small (the angular factor L,
// n_ordinates x r) and as the fallback for the spatial factor when Cholesky QR
// reports a numerically dependent set of swept columns.
//
// A column whose residual after both passes is at most 1e-12 of its own norm is
// replaced by the next graded monomial (spatial: x^a y^b at cell centres mapped
// to [-1,1]^2; angular: mu^a eta^b), orthogonalised twice and skipped when its
// residual is below 1e-10 of its own norm; R_kk is then 0.
#include "dlr_internal.h"

#include <algorithm>

namespace dlr {

namespace {

constexpr int kOrthThreads = 1024;
constexpr int kOrthWaves = kOrthThreads / 64;
constexpr int kGrp = 16;                                   // dot products reduced together
constexpr int kMaxGroups = (kMaxRank + 1 + kGrp - 1) / kGrp;

struct OrthCtx {
    long n;
    const double* weight;   // per element or nullptr
    double wscalar;
    double* Q;              // [r][n]; column k doubles as the working vector v
};

__device__ __forceinline__ double wt(const OrthCtx& c, long e) { return c.weight ? c.weight[e] : c.wscalar; }

// Sum of a[0..16) over the 64 lanes of a wavefront, scattered: four exchange stages
// halve the live values (17 shuffles instead of 96); the lanes with (lane & 3) == 0
// return the total of value 8*b5 + 4*b4 + 2*b3 + b2 (b = bits of the lane id).
__device__ __forceinline__ double wave_reduce_scatter16(double (&a)[kGrp], int lane) {
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const int o = 32 >> st, c = 8 >> st;
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < c; ++i) {
            const double send = up ? a[i] : a[i + c];
            const double keep = up ? a[i + c] : a[i];
            a[i] = keep + __shfl_xor(send, o);
        }
    }
    double x = a[0];
    x += __shfl_xor(x, 2);
    x += __shfl_xor(x, 1);
    return x;
}

// hs[j] = sum_e Q_j(e) w(e) v(e) for j < k, and hs[k] = sum_e w(e) v(e)^2 when with_norm,
// where v = column kv of Q (kv >= k).  Each thread owns the elements e = t (mod kOrthThreads); the per-wave
// partials are added over the wavefronts in a fixed order.
__device__ void block_dots(const OrthCtx& c, int k, int kv, bool with_norm, double* hs, double* wsum) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int cnt = k + (with_norm ? 1 : 0);
    const double* v = c.Q + (size_t)kv * c.n;
    for (int g0 = 0; g0 < cnt; g0 += kGrp) {
        double a[kGrp];
#pragma unroll
        for (int i = 0; i < kGrp; ++i) a[i] = 0.0;
        const unsigned n32 = (unsigned)c.n;
        const int jend = min(k, g0 + kGrp) - g0;   // number of projections in this group
        const bool norm_here = with_norm && k >= g0 && k < g0 + kGrp;
#pragma unroll 1
        for (unsigned e = t; e < n32; e += kOrthThreads) {
            const double ve = v[e];
            const double wve = wt(c, e) * ve;
            unsigned off = (unsigned)g0 * n32 + e;
            const int inorm = norm_here ? k - g0 : -1;
#pragma unroll
            for (int i = 0; i < kGrp; ++i, off += n32) {
                if (i < jend) a[i] += c.Q[off] * wve;
                if (i == inorm) a[i] += wve * ve;
            }
        }
        const double tot = wave_reduce_scatter16(a, lane);
        if ((lane & 3) == 0) {
            const int idx = 8 * ((lane >> 5) & 1) + 4 * ((lane >> 4) & 1) + 2 * ((lane >> 3) & 1) + ((lane >> 2) & 1);
            wsum[((g0 / kGrp) * kOrthWaves + wv) * kGrp + idx] = tot;
        }
    }
    __syncthreads();
    if (t < cnt) {
        double s = 0.0;
        for (int w = 0; w < kOrthWaves; ++w) s += wsum[((t / kGrp) * kOrthWaves + w) * kGrp + t % kGrp];
        hs[t] = s;
    }
    __syncthreads();
}

// v <- v - Q_{<k} h on the thread's own elements
__device__ void block_update(const OrthCtx& c, int k, const double* h) {
    double* v = c.Q + (size_t)k * c.n;
    const unsigned n32 = (unsigned)c.n;
    for (unsigned e = threadIdx.x; e < n32; e += kOrthThreads) {
        double x = v[e];
        unsigned off = e;
        for (int j = 0; j < k; ++j, off += n32) x -= h[j] * c.Q[off];
        v[e] = x;
    }
}

__device__ void block_scale(const OrthCtx& c, int k, double inv) {
    double* v = c.Q + (size_t)k * c.n;
    for (long e = threadIdx.x; e < c.n; e += kOrthThreads) v[e] *= inv;
}

// Column k of Q holds the candidate v.  Three reductions: (dots with Q_{<k}, |v|^2), update,
// (dots), update, |v|^2 -- the two projection passes of CGS2; a single code path so the
// reduction is instantiated once.
__device__ void project_twice(const OrthCtx& c, int k, double* hs, double* hsum, double* wsum, double& own,
                              double& nrm) {
    for (int pass = 0; pass < 3; ++pass) {
        const int kk = (pass < 2) ? k : 0;
        block_dots(c, kk, k, pass != 1, hs, wsum);
        if (pass == 0) own = sqrt(fmax(hs[k], 0.0));
        if (pass == 2) {
            nrm = sqrt(fmax(hs[0], 0.0));
            break;
        }
        for (int j = threadIdx.x; j < k; j += kOrthThreads) hsum[j] = (pass == 0 ? 0.0 : hsum[j]) + hs[j];
        block_update(c, k, hs);
        __syncthreads();   // hs is read by every thread before the next pass overwrites it
    }
}

template <typename TV>
__global__ __launch_bounds__(kOrthThreads) void k_cgs2(long n, int r, const TV* __restrict__ V, size_t ldv,
                                                       const double* __restrict__ weight, double wscalar,
                                                       int comp_kind, int nx, int ny, const double* __restrict__ mu,
                                                       const double* __restrict__ eta, double* __restrict__ Q,
                                                       double* __restrict__ R, int* flag, int flag_mask,
                                                       int* status, int status_code) {
    __shared__ double hs[kMaxRank + 1], hsum[kMaxRank];
    __shared__ double wsum[kMaxGroups * kOrthWaves * kGrp];
    __shared__ int deg, ax;
    if (flag) {   // fallback mode: run only when the fast path flagged a breakdown
        const int f = *flag;
        if (!(f & flag_mask)) return;
    }
    const int t = threadIdx.x;
    OrthCtx c{n, weight, wscalar, Q};
    if (t == 0) { deg = 0; ax = 0; }
    for (int o = t; o < r * r; o += kOrthThreads) R[o] = 0.0;
    __syncthreads();
    bool out_of_completions = false;
    for (int k = 0; k < r; ++k) {
        double* v = Q + (size_t)k * n;
        for (long e = t; e < n; e += kOrthThreads)
            v[e] = (double)V[(size_t)k * ldv + (size_t)e];
        // attempt 0 is the column itself; later attempts are completion vectors
        for (int attempt = 0; attempt <= 100000; ++attempt) {
            double own, nrm;
            project_twice(c, k, hs, hsum, wsum, own, nrm);
            if (attempt == 0) {
                for (int j = t; j < k; j += kOrthThreads) R[j * r + k] = hsum[j];
                if (own > 0.0 && nrm > 1e-12 * own) {   // accepted: R_kk = nrm
                    block_scale(c, k, 1.0 / nrm);
                    if (t == 0) R[k * r + k] = nrm;
                    break;
                }
            } else if (nrm > 1e-10 * own) {             // completion accepted: R_kk stays 0
                block_scale(c, k, 1.0 / nrm);
                break;
            }
            if (attempt == 100000) {
                out_of_completions = true;
                break;
            }
            // next graded monomial: (deg, ax) -> (deg, ax-1) or (deg+1, deg+1)
            const int d = deg, a = ax;
            __syncthreads();
            if (t == 0) {
                if (ax > 0) ax = ax - 1; else { deg = deg + 1; ax = deg; }
            }
            for (long e = t; e < n; e += kOrthThreads) {
                double bx, by;
                if (comp_kind == 0) {   // column-major cells e = i*ny + j
                    const long i = e / ny, j = e % ny;
                    bx = -1.0 + (i + 0.5) * 2.0 / nx;
                    by = -1.0 + (j + 0.5) * 2.0 / ny;
                } else {
                    bx = mu[e];
                    by = eta[e];
                }
                double m = 1.0;
                for (int p = 0; p < a; ++p) m *= bx;
                for (int p = 0; p < d - a; ++p) m *= by;
                v[e] = m;
            }
        }
    }
    if (t == 0) {
        if (out_of_completions) atomicOr(status, status_code);
        if (flag) atomicAnd(flag, ~flag_mask);   // the fallback repaired the factor
    }
}

// Planes k = 0 .. count-1 of V (leading dimension ldv): the graded spatial monomial number first + k, in the
// completion's order (1, x, y, x^2, x y, y^2, ...: degree d, then the power of x from d down to 0) at the
// cell centres mapped to [-1, 1]^2, column-major cells e = i*ny + j.
__global__ __launch_bounds__(256) void k_monomials(int nx, int ny, int first, int count, double* __restrict__ V,
                                                  size_t ldv) {
    const long n = (long)nx * ny;
    const long total = n * count;
    for (long o = (long)blockIdx.x * blockDim.x + threadIdx.x; o < total; o += (long)gridDim.x * blockDim.x) {
        const int k = (int)(o / n);
        const long e = o - (long)k * n;
        const int idx = first + k;
        int d = 0;
        while ((d + 1) * (d + 2) / 2 <= idx) ++d;
        const int a = d - (idx - d * (d + 1) / 2);   // power of x
        const long i = e / ny, j = e % ny;
        const double bx = -1.0 + (i + 0.5) * 2.0 / nx, by = -1.0 + (j + 0.5) * 2.0 / ny;
        double m = 1.0;
        for (int p = 0; p < a; ++p) m *= bx;
        for (int p = 0; p < d - a; ++p) m *= by;
        V[(size_t)k * ldv + e] = m;
    }
}

}  // namespace

void launch_monomials(hipStream_t s, int nx, int ny, int first, int count, double* V, size_t ldv) {
    const long total = (long)nx * ny * count;
    if (total <= 0) return;
    hipLaunchKernelGGL(k_monomials, dim3((unsigned)std::min<long>((total + 255) / 256, 65536)), dim3(256), 0, s, nx, ny,
                       first, count, V, ldv);
}

template <typename TV>
void launch_cgs2(hipStream_t s, long n, int r, const TV* V, size_t ldv, const double* weight,
                 double wscalar, int comp_kind, int nx, int ny, const double* mu, const double* eta, double* Q,
                 double* R, int* flag, int flag_mask, int* status, int status_code) {
    hipLaunchKernelGGL((k_cgs2<TV>), dim3(1), dim3(kOrthThreads), 0, s, n, r, V, ldv, weight, wscalar,
                       comp_kind, nx, ny, mu, eta, Q, R, flag, flag_mask, status, status_code);
}
template void launch_cgs2<double>(hipStream_t, long, int, const double*, size_t, const double*, double, int, int,
                                  int, const double*, const double*, double*, double*, int*, int, int*, int);
template void launch_cgs2<float>(hipStream_t, long, int, const float*, size_t, const double*, double, int, int,
                                 int, const double*, const double*, double*, double*, int*, int, int*, int);

}  // namespace dlr
