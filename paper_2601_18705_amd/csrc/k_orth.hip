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

namespace dlr {

namespace {

constexpr int kOrthThreads = 1024;
constexpr int kSlices = kOrthThreads / kMaxRank;   // 16 slices x 64 columns for the dot products

__device__ double orth_block_sum(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = kOrthThreads / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

struct OrthCtx {
    long n;
    const double* weight;   // per element or nullptr
    double wscalar;
    double* Q;              // [r][n]
};

__device__ inline double wt(const OrthCtx& c, long e) { return c.weight ? c.weight[e] : c.wscalar; }

// Two passes of v <- v - Q_{<k} (Q_{<k}^T W v); accumulates the coefficients in hsum.
__device__ void project_twice(const OrthCtx& c, int k, double* hsum, double* red, double* h) {
    const int t = threadIdx.x;
    double* v = c.Q + (size_t)k * c.n;
    for (int j = t; j < k; j += kOrthThreads) hsum[j] = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        __syncthreads();
        const int j = t % kMaxRank, slice = t / kMaxRank;
        double acc = 0.0;
        if (j < k) {
            const double* qj = c.Q + (size_t)j * c.n;
            for (long e = slice; e < c.n; e += kSlices) acc += qj[e] * (wt(c, e) * v[e]);
        }
        red[slice * kMaxRank + j] = acc;
        __syncthreads();
        for (int jj = t; jj < k; jj += kOrthThreads) {
            double s = 0.0;
            for (int sl = 0; sl < kSlices; ++sl) s += red[sl * kMaxRank + jj];
            h[jj] = s;
            hsum[jj] += s;
        }
        __syncthreads();
        for (long e = t; e < c.n; e += kOrthThreads) {
            double x = v[e];
            for (int jj = 0; jj < k; ++jj) x -= h[jj] * c.Q[(size_t)jj * c.n + e];
            v[e] = x;
        }
    }
    __syncthreads();
}

__device__ double wnorm(const OrthCtx& c, int k, double* sh) {
    const double* v = c.Q + (size_t)k * c.n;
    double acc = 0.0;
    for (long e = threadIdx.x; e < c.n; e += kOrthThreads) acc += wt(c, e) * v[e] * v[e];
    return sqrt(orth_block_sum(acc, sh));
}

template <typename TV>
__global__ __launch_bounds__(kOrthThreads) void k_cgs2(long n, int r, const TV* __restrict__ V, size_t ldv, int pad_ny,
                                                       const double* __restrict__ weight, double wscalar,
                                                       int comp_kind, int nx, int ny, const double* __restrict__ mu,
                                                       const double* __restrict__ eta, double* __restrict__ Q,
                                                       double* __restrict__ R, int* flag, int flag_mask,
                                                       int* status, int status_code) {
    __shared__ double sh[kOrthThreads];
    __shared__ double red[kSlices * kMaxRank];
    __shared__ double h[kMaxRank], hsum[kMaxRank];
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
            v[e] = (double)V[(size_t)k * ldv + (pad_ny ? padded_cell(e, pad_ny) : (size_t)e)];
        __syncthreads();
        const double own = wnorm(c, k, sh);
        project_twice(c, k, hsum, red, h);
        const double nrm = wnorm(c, k, sh);
        for (int j = t; j < k; j += kOrthThreads) R[j * r + k] = hsum[j];
        if (own > 0.0 && nrm > 1e-12 * own) {
            for (long e = t; e < n; e += kOrthThreads) v[e] /= nrm;
            if (t == 0) R[k * r + k] = nrm;
            __syncthreads();
            continue;
        }
        // completion: next graded monomial that is independent of the accepted columns
        for (int guard = 0; guard < 100000; ++guard) {
            const int d = deg, a = ax;
            __syncthreads();
            if (t == 0) {   // advance the iterator: (deg, ax) -> (deg, ax-1) or (deg+1, deg+1)
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
            __syncthreads();
            const double un = wnorm(c, k, sh);
            project_twice(c, k, hsum, red, h);
            const double n2 = wnorm(c, k, sh);
            if (n2 > 1e-10 * un) {
                for (long e = t; e < n; e += kOrthThreads) v[e] /= n2;
                __syncthreads();
                break;
            }
            if (guard == 99999) out_of_completions = true;
        }
    }
    if (t == 0) {
        if (out_of_completions) atomicOr(status, status_code);
        if (flag) atomicAnd(flag, ~flag_mask);   // the fallback repaired the factor
    }
}

}  // namespace

template <typename TV>
void launch_cgs2(hipStream_t s, long n, int r, const TV* V, size_t ldv, int pad_ny, const double* weight,
                 double wscalar, int comp_kind, int nx, int ny, const double* mu, const double* eta, double* Q,
                 double* R, int* flag, int flag_mask, int* status, int status_code) {
    hipLaunchKernelGGL((k_cgs2<TV>), dim3(1), dim3(kOrthThreads), 0, s, n, r, V, ldv, pad_ny, weight, wscalar,
                       comp_kind, nx, ny, mu, eta, Q, R, flag, flag_mask, status, status_code);
}
template void launch_cgs2<double>(hipStream_t, long, int, const double*, size_t, int, const double*, double, int, int,
                                  int, const double*, const double*, double*, double*, int*, int, int*, int);
template void launch_cgs2<float>(hipStream_t, long, int, const float*, size_t, int, const double*, double, int, int,
                                 int, const double*, const double*, double*, double*, int*, int, int*, int);

}  // namespace dlr
