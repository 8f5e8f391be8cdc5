// Diffusion synthetic acceleration of the source iteration (Sec. 4 "Diffusion Synthetic
// Acceleration (DSA) for SN-like DLR method" and its appendix derivation), degree-0 cells.
//
// After a sweep took phi_old to phi_half, the diffusion approximation of the remaining error,
//   D delta = M_s (phi_half - phi_old),
//   D = (1/3) sum_j F_j^T M_t^{-1} F_j + F_0 + M_a,
// is solved and phi = phi_half + delta.  F_j are the central face operators of the degree-0
// elements ((F_x u)_i = (h_y / 2)(u_{i-1} - u_{i+1}), zero outside the grid; there is no
// volume gradient term), M_t = area sigma_t, M_a = area (sigma_t - sigma_s), and F_0 the jump
// penalty of eq. "penalty term": (1/4pi) sum_faces (1/2) kappa_f h_f [[u]][[v]] with
// kappa_f = sum_d c_d |Omega_d . n_f| (c: the collocation weights).  So, at cell (i, j),
//   (D u) = h_y^2 / (12 A) [ (u_i - u_{i+2}) / s_{i+1} - (u_{i-2} - u_i) / s_{i-1} ]   (x part)
//         + h_x^2 / (12 A) [ same along j ]
//         + c_x (2 u - u_{i-1} - u_{i+1}) + c_y (2 u - u_{j-1} - u_{j+1}) + A (sigma_t - sigma_s) u,
// with s = sigma_t, c_x = kappa_x h_y / (8 pi), c_y = kappa_y h_x / (8 pi), a term with s_k present
// only when cell k exists, and u = 0 outside the grid.  D is symmetric positive definite.
//
// Solver: conjugate gradients with the diagonal of D as preconditioner, FP64.  Each iteration
// is two kernels (stencil product with the new search direction formed on the fly, then the
// vector updates); their dot products are summed per block and then over blocks in block
// order by the last block to finish, so results are bitwise reproducible.  The iteration count
// is fixed by the host; once the relative residual is below the tolerance a device flag makes
// the remaining launches return at once.
#include "dlr_internal.h"

#include <algorithm>

namespace dlr {

namespace {

constexpr int kDsaBlock = 256;

__device__ double dsa_block_sum(double v, double* sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ void dsa_store(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double dsa_load(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// true in the block that retires last (partials stored before counting, agent-scope atomics)
__device__ bool dsa_retire(unsigned* counter) {
    __shared__ bool last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this block's partial stores are performed
        const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    return last;
}

__device__ double dsa_ordered_sum(const double* p, int count, int stride, double* sh) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += blockDim.x) acc += dsa_load(p + (size_t)i * stride);
    return dsa_block_sum(acc, sh);
}

// scalar slots
enum { kRZ = 0, kPQ, kAlpha, kBeta, kRR0, kRR, kIter, kDone, kScalars };

struct Stencil {
    int nx, ny;
    double wx, wy;      // h_y^2 / (12 A), h_x^2 / (12 A)
    double cx, cy;      // penalty coefficients
    double area, inv_cdt;
    const double* sig;     // sigma (sigma_t = sigma + 1 / (c dt))
    const double* sig_s;
    __device__ __forceinline__ double st(size_t k) const { return sig[k] + inv_cdt; }
    // value of u at (i, j), zero outside
    __device__ __forceinline__ bool in(int i, int j) const { return i >= 0 && i < nx && j >= 0 && j < ny; }
};

__device__ __forceinline__ double dsa_diag(const Stencil& S, int i, int j) {
    const size_t e = (size_t)i * S.ny + j;
    double dx = 0.0, dy = 0.0;
    if (i + 1 < S.nx) dx += 1.0 / S.st(e + S.ny);
    if (i >= 1) dx += 1.0 / S.st(e - S.ny);
    if (j + 1 < S.ny) dy += 1.0 / S.st(e + 1);
    if (j >= 1) dy += 1.0 / S.st(e - 1);
    return S.wx * dx + S.wy * dy + 2.0 * S.cx + 2.0 * S.cy + S.area * (S.st(e) - S.sig_s[e]);
}

// (D u)(i, j) for u given by a functor val(i, j) (zero outside)
template <typename F>
__device__ __forceinline__ double dsa_apply_at(const Stencil& S, int i, int j, F val) {
    const size_t e = (size_t)i * S.ny + j;
    const double u = val(i, j);
    double tx = 0.0, ty = 0.0;
    if (i + 1 < S.nx) tx += (u - val(i + 2, j)) / S.st(e + S.ny);
    if (i >= 1) tx -= (val(i - 2, j) - u) / S.st(e - S.ny);
    if (j + 1 < S.ny) ty += (u - val(i, j + 2)) / S.st(e + 1);
    if (j >= 1) ty -= (val(i, j - 2) - u) / S.st(e - 1);
    const double pen = S.cx * (2.0 * u - val(i - 1, j) - val(i + 1, j)) + S.cy * (2.0 * u - val(i, j - 1) - val(i, j + 1));
    return S.wx * tx + S.wy * ty + pen + S.area * (S.st(e) - S.sig_s[e]) * u;
}

// kappa_x = sum_d c_d |mu_d|, kappa_y = sum_d c_d |eta_d| (one wavefront, fixed order)
__global__ void k_dsa_kappa(int nd, const double* __restrict__ c, const double* __restrict__ mu,
                            const double* __restrict__ eta, double* __restrict__ kappa) {
    __shared__ double sh[64];
    double ax = 0.0, ay = 0.0;
    for (int d = threadIdx.x; d < nd; d += blockDim.x) {
        ax += c[d] * fabs(mu[d]);
        ay += c[d] * fabs(eta[d]);
    }
    ax = dsa_block_sum(ax, sh);
    ay = dsa_block_sum(ay, sh);
    if (threadIdx.x == 0) {
        kappa[0] = ax;
        kappa[1] = ay;
    }
}

__device__ __forceinline__ Stencil make_stencil(const DsaArgs& a) {
    Stencil S;
    S.nx = a.nx;
    S.ny = a.ny;
    S.area = a.hx * a.hy;
    S.wx = a.hy * a.hy / (12.0 * S.area);
    S.wy = a.hx * a.hx / (12.0 * S.area);
    S.cx = a.kappa[0] * a.hy / (8.0 * kPi);
    S.cy = a.kappa[1] * a.hx / (8.0 * kPi);
    S.inv_cdt = a.inv_cdt;
    S.sig = a.sigma;
    S.sig_s = a.sig_s;
    return S;
}

// r = A sigma_s (phi_half - phi_old), x = 0, z = r / diag, p = 0; rz, rr
__global__ __launch_bounds__(kDsaBlock) void k_dsa_init(DsaArgs a) {
    __shared__ double sh[kDsaBlock];
    if (a.skip && *a.skip) return;
    const Stencil S = make_stencil(a);
    const size_t n = (size_t)a.nx * a.ny;
    double rz = 0.0, rr = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / a.ny), j = (int)(e % a.ny);
        const double d = dsa_diag(S, i, j);
        const double r = S.area * a.sig_s[e] * (a.phi[e] - a.phi_old[e]);
        a.dg[e] = d;
        a.r[e] = r;
        a.x[e] = 0.0;
        a.z[e] = r / d;
        a.p[0][e] = 0.0;
        rz += r * (r / d);
        rr += r * r;
    }
    rz = dsa_block_sum(rz, sh);
    rr = dsa_block_sum(rr, sh);
    if (threadIdx.x == 0) {
        dsa_store(&a.partials[2 * blockIdx.x], rz);
        dsa_store(&a.partials[2 * blockIdx.x + 1], rr);
    }
    if (dsa_retire(a.counter)) {
        const double RZ = dsa_ordered_sum(a.partials, gridDim.x, 2, sh);
        const double RR = dsa_ordered_sum(a.partials + 1, gridDim.x, 2, sh);
        if (threadIdx.x == 0) {
            a.scal[kRZ] = RZ;
            a.scal[kRR0] = RR;
            a.scal[kRR] = RR;
            a.scal[kBeta] = 0.0;
            a.scal[kIter] = 0.0;
            a.scal[kDone] = (RR > 0.0 && RZ > 0.0 && isfinite(RR)) ? 0.0 : 1.0;
            __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// p_new = z + beta p_old (formed at the stencil points), q = D p_new; alpha = rz / (p_new . q)
__global__ __launch_bounds__(kDsaBlock) void k_dsa_apply(DsaArgs a, int par) {
    __shared__ double sh[kDsaBlock];
    if ((a.skip && *a.skip) || a.scal[kDone] != 0.0) return;
    const Stencil S = make_stencil(a);
    const double beta = a.scal[kBeta];
    const double* __restrict__ z = a.z;
    const double* __restrict__ po = a.p[par];
    double* __restrict__ pn = a.p[par ^ 1];
    const size_t n = (size_t)a.nx * a.ny;
    auto pval = [&](int i, int j) -> double {
        if (!S.in(i, j)) return 0.0;
        const size_t k = (size_t)i * S.ny + j;
        return z[k] + beta * po[k];
    };
    double pq = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / a.ny), j = (int)(e % a.ny);
        const double pe = z[e] + beta * po[e];
        const double q = dsa_apply_at(S, i, j, pval);
        pn[e] = pe;
        a.q[e] = q;
        pq += pe * q;
    }
    pq = dsa_block_sum(pq, sh);
    if (threadIdx.x == 0) dsa_store(&a.partials[2 * blockIdx.x], pq);
    if (dsa_retire(a.counter)) {
        const double PQ = dsa_ordered_sum(a.partials, gridDim.x, 2, sh);
        if (threadIdx.x == 0) {
            if (PQ > 0.0 && isfinite(PQ)) {
                a.scal[kPQ] = PQ;
                a.scal[kAlpha] = a.scal[kRZ] / PQ;
            } else {
                a.scal[kDone] = 1.0;   // breakdown: keep the current correction
            }
            __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// x += alpha p, r -= alpha q, z = r / diag; beta = rz_new / rz; done when |r| <= tol |r0|
__global__ __launch_bounds__(kDsaBlock) void k_dsa_update(DsaArgs a, int par) {
    __shared__ double sh[kDsaBlock];
    if ((a.skip && *a.skip) || a.scal[kDone] != 0.0) return;
    const double alpha = a.scal[kAlpha];
    const double* __restrict__ p = a.p[par ^ 1];
    const size_t n = (size_t)a.nx * a.ny;
    double rz = 0.0, rr = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const double r = a.r[e] - alpha * a.q[e];
        const double z = r / a.dg[e];
        a.x[e] += alpha * p[e];
        a.r[e] = r;
        a.z[e] = z;
        rz += r * z;
        rr += r * r;
    }
    rz = dsa_block_sum(rz, sh);
    rr = dsa_block_sum(rr, sh);
    if (threadIdx.x == 0) {
        dsa_store(&a.partials[2 * blockIdx.x], rz);
        dsa_store(&a.partials[2 * blockIdx.x + 1], rr);
    }
    if (dsa_retire(a.counter)) {
        const double RZ = dsa_ordered_sum(a.partials, gridDim.x, 2, sh);
        const double RR = dsa_ordered_sum(a.partials + 1, gridDim.x, 2, sh);
        if (threadIdx.x == 0) {
            const double it = a.scal[kIter] + 1.0;
            a.scal[kIter] = it;
            a.scal[kBeta] = RZ / a.scal[kRZ];
            a.scal[kRZ] = RZ;
            a.scal[kRR] = RR;
            if (!(RR > a.tol * a.tol * a.scal[kRR0]) || !(RZ > 0.0)) a.scal[kDone] = 1.0;
            __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// phi += delta and the four orientation copies of s_e = sigma_s phi / (4 pi) in the sweep layout
template <typename TS>
__global__ __launch_bounds__(kDsaBlock) void k_dsa_finish(DsaArgs a) {
    if (a.skip && *a.skip) return;
    TS* s_e = static_cast<TS*>(a.s_e);
    const size_t n = (size_t)a.nx * a.ny;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / a.ny), j = (int)(e % a.ny);
        const double ph = a.phi[e] + a.x[e];
        a.phi[e] = ph;
        if (s_e) {
            const TS se = (TS)(a.sig_s[e] * ph / kFourPi);
#pragma unroll
            for (int o = 0; o < 4; ++o) s_e[(size_t)o * a.ldg + diag_pos(a.nx, a.ny, o, i, j)] = se;
        }
    }
}

}  // namespace

void launch_dsa_kappa(hipStream_t s, int nd, const double* c, const double* mu, const double* eta, double* kappa) {
    hipLaunchKernelGGL(k_dsa_kappa, dim3(1), dim3(64), 0, s, nd, c, mu, eta, kappa);
}

int dsa_blocks(int nx, int ny) {
    const long n = (long)nx * ny;
    return (int)std::max<long>(1, std::min<long>((n + kDsaBlock - 1) / kDsaBlock, 2048));
}

void launch_dsa(hipStream_t s, const DsaArgs& a, bool fp32_layout) {
    const int nb = dsa_blocks(a.nx, a.ny);
    hipLaunchKernelGGL(k_dsa_init, dim3(nb), dim3(kDsaBlock), 0, s, a);
    for (int it = 0; it < a.max_iter; ++it) {
        hipLaunchKernelGGL(k_dsa_apply, dim3(nb), dim3(kDsaBlock), 0, s, a, it & 1);
        hipLaunchKernelGGL(k_dsa_update, dim3(nb), dim3(kDsaBlock), 0, s, a, it & 1);
    }
    if (fp32_layout)
        hipLaunchKernelGGL(k_dsa_finish<float>, dim3(nb), dim3(kDsaBlock), 0, s, a);
    else
        hipLaunchKernelGGL(k_dsa_finish<double>, dim3(nb), dim3(kDsaBlock), 0, s, a);
}

}  // namespace dlr
