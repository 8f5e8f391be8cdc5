// Internal declarations of the dlrtrt HIP library (gfx950).
//
// Storage layout on the device (one instance).  Cells are numbered column-major,
// e = i*ny + j (a grid column is contiguous); the C interface uses e = j*nx + i
// and the library transposes at creation and read-back only.
//   per-cell fields          [N] float64, N = nx*ny
//   spatial basis X          [r][N] float64 (column k of X contiguous)
//   sweep planes             in the sweep precision (double or float), diagonal layout (below):
//                            Psi, src0 [r][ldg] each in its own direction's orientation; sigma_t,
//                            s_e [4][ldg], one copy per orientation
//   Psi for the QR           [r][ld] compact cell planes (cell e = i*ny + j), ld = N rounded up to 64
//   angular basis W, L       [r][nq] float64 (column k contiguous over ordinates)
//   coupling S               [r][r] float64, row-major S[i*r + j]
// The state is psi = X S W^T with X, W orthonormal; S is kept as a general
// r x r matrix (the SVD rotation of the angular modes is applied to W and S
// only, which leaves psi and X unchanged).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dlr {

constexpr double kPi = 3.14159265358979323846;
constexpr double kFourPi = 4.0 * kPi;
constexpr int kMaxRank = 64;
constexpr int kSweepChunk = 32;   // rows published per edge-flag update in the sweep

// Copy count doubles from global memory to LDS with eight independent loads in flight per
// thread: the small dense kernels read data that the previous kernel has just written, often
// from another XCD's L2, and a loop that waits for each load in turn pays that latency
// count / blockDim times over.  Callers synchronise the block before reading dst.
//
// The loads are issued by every lane from a clamped (valid) address and masked afterwards:
// "x = ok ? p[i] : 0" compiles to an exec-masked load whose result register the other lanes
// then overwrite, which makes the wavefront wait for that load before issuing the next.  The
// small dense kernels and the triangular multiply use the same form; in the streaming MFMA
// staging loops the masked form measured faster and is kept there.
__device__ inline void stage_lds(double* dst, const double* __restrict__ src, int count) {
    for (int base = threadIdx.x; base < count; base += 8 * blockDim.x) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int o = base + u * blockDim.x;
            v[u] = src[o < count ? o : count - 1];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int o = base + u * blockDim.x;
            if (o < count) dst[o] = v[u];
        }
    }
}

// ----------------------------------------------------------------------------- diagonal sweep layout
// A direction's orientation o has bit 0 set when mu <= 0 and bit 1 when eta <= 0.  In its swept
// coordinates i' = i or nx-1-i, j' = j or ny-1-j the grid is cut into strips of 64 columns; the
// cell (i', j') of strip s = i'/64 is on lane l = i' % 64 and diagonal t = j' + l.  Element (s, t, l)
// is stored at ((s*ndg + t/4)*64 + l)*4 + t%4, ndg = diagonal groups of four per strip, so the 64
// lanes of a wavefront at four consecutive diagonals touch one contiguous block.
__host__ __device__ inline int orient_of(double mu, double eta) { return (mu > 0.0 ? 0 : 1) | (eta > 0.0 ? 0 : 2); }
__host__ __device__ inline int diag_groups(int ny) { return (ny + 63 + 15) / 16 * 4; }
__host__ __device__ inline size_t diag_plane(int nx, int ny) { return (size_t)((nx + 63) / 64) * diag_groups(ny) * 256; }
__host__ __device__ inline size_t diag_pos(int nx, int ny, int o, int i, int j) {
    const int ip = (o & 1) ? nx - 1 - i : i, jp = (o & 2) ? ny - 1 - j : j;
    const int l = ip & 63, t = jp + l;
    return ((size_t)((ip >> 6) * diag_groups(ny) + (t >> 2)) * 64 + l) * 4 + (t & 3);
}

// ----------------------------------------------------------------------------- per-cell kernels
// The kernels that touch the diagonal layout walk tiles of 8 columns x 128 rows.
void launch_linearize(hipStream_t s, int nx, int ny, const double* sigma, const double* rho_cv, const double* q_ext,
                      const double* T, double dt, double a, double c, double* D, double* sig_s, double* q,
                      double* sig_t64, float* sig_t32, size_t ldg, double* q_diag /* nullable: q, 4 copies */);

// zero4: nullptr, or four words set to 0 (the source-iteration control of the step)
template <typename TS>
void launch_psi0(hipStream_t s, int nx, int ny, int r, const double* X, const double* C0, const double* a0,
                 const double* q, const double* sig_s, double inv_cdt, const double* mu, const double* eta,
                 TS* src0, size_t ldg, double* phi, TS* s_e, int* zero4 = nullptr);

// Source iteration decided on the device: the scalar-flux kernels return at once while flag[0] is
// set; otherwise the last block of the second pass counts the iteration in flag[1] and sets
// flag[0] (with the reason in flag[2]: 1 converged, 2 non-finite change norm, 3 iteration limit)
// when the relative change is at most tol, is not finite, or the count reaches max_iter.
struct SiControl {
    int* flag;     // [4], zero at the start of each step
    double tol;
    int max_iter;
};
template <typename TS>
void launch_phi(hipStream_t s, int nx, int ny, int r, const TS* psi, size_t ldg, const double* mu, const double* eta,
                const double* cw, double* phio /* [4][ldg] work */, const double* sig_s, const double* phi_old,
                double* phi_new, TS* s_e, double* partials, int nblocks, unsigned* counter, double* out,
                const SiControl* ctl = nullptr);

// Psi (diagonal layouts) -> compact column-major cell planes [r][ld] (cell e = i * ny + j)
template <typename TS>
void launch_psi_to_cm(hipStream_t s, int nx, int ny, int r, const TS* psi, size_t ldg, const double* mu,
                      const double* eta, TS* psi_cm, size_t ld);

// Plain discrete ordinates (the comparator): orient[d] = orientation of ordinate d; dirs/off list the
// ordinates grouped by orientation; phio is [4][ldg] FP64 work space.
template <typename TS>
void launch_sn_source(hipStream_t s, int nq, size_t ldg, const int* orient, const double* q_diag, const TS* psi_old,
                      double inv_cdt, TS* src0);
template <typename TS>
void launch_sn_init(hipStream_t s, int nx, int ny, int nq, size_t ldg, const int* orient, const double* T, double a,
                    double c, TS* psi, double* phi);
template <typename TS>
void launch_sn_phi(hipStream_t s, int nx, int ny, size_t ldg, const int* dirs, const int* off, const double* w,
                   const TS* psi, double* phio, const double* sig_s, const double* phi_old, double* phi_new, TS* s_e,
                   double* partials, int nblocks, unsigned* counter, double* out);

// phi = X coef, coef = S beta (launch_wsum)
void launch_phi_of_factors(hipStream_t s, int n, int r, const double* X, const double* coef, double* phi);

// Temperature update (Algorithm 1 step 9) with the energy sum and, for DLR, the outflow tally.
struct TupdateArgs {
    int nx, ny, r;                  // r = 0 and X = nullptr: plain SN (phi holds the converged flux)
    const double* X;                // [r][N] column-major cells e = i * ny + j
    const double* coef;             // [r] S beta
    const double* gside;            // [4][r] side vectors of the outflow tally (launch_wsum), or nullptr
    const double *sigma, *rho_cv, *D;
    double dt, a, c, area, hx, hy;
    double *T, *phi;
    double* partials;               // [2 * nblocks]
    unsigned* counter;              // zero between launches
    double* out;                    // out[0] = energy, out[1] = outflow (when gside is set)
    int* status;
};
void launch_tupdate(hipStream_t s, const TupdateArgs& A, int nblocks);
// plain SN: out[1] = outflow tally from every ordinate's psi (diagonal planes of their orientations)
template <typename TS>
void launch_sn_outflow(hipStream_t s, int nx, int ny, int nq, size_t ldg, const double* mu, const double* eta,
                       const double* w, const TS* psi, double hx, double hy, double* partials, int nblocks,
                       unsigned* counter, double* out);

// ----------------------------------------------------------------------------- sweep
// compute wavefronts (64-column strips) per sweep workgroup: two with FP32 planes, one with FP64
// (measured at 1024^2 x 32 directions: FP32 158 us with two against 168 with one; FP64 sweeps the
// other way round)
constexpr int sweep_waves(bool fp64) { return fp64 ? 1 : 2; }
// One instance's sweep: everything but the launch-level fields below is fixed for the life of
// the instance, so the record is uploaded once and reused by every launch.
template <typename TS>
struct SweepArgs {
    int nx, ny, nd, nsuper, total_units;   // nsuper = superstrips of sweep_waves x 64 columns; units = nsuper * nd
    size_t ldg;                            // diagonal plane stride (elements), diag_plane
    const TS* src0;      // [nd][ldg] fixed source q + psi0 / (c dt), each in its direction's orientation
    const TS* sig_t;     // [4][ldg] one copy per orientation
    const TS* s_e;       // [4][ldg] sigma_s phi / (4 pi), one copy per orientation
    TS* psi;             // [nd][ldg]
    const double* mu;    // [nd] direction cosines of the swept directions
    const double* eta;   // [nd]
    const double* inflow_x;  // [nd] isotropic inflow on the x-inflow face (0 = vacuum)
    const double* inflow_y;  // [nd]
    double inv_hx, inv_hy;
    TS* edge;                        // [nd][nsuper][ny] outgoing x-face values of each superstrip
    unsigned long long* progress;    // [nd][nsuper] (launch << 32) | rows published
    int* status;                     // kStatusSweepStall is raised if a wait exceeds spin_limit polls
    unsigned spin_limit;
    const int* skip;                 // nullptr, or the instance's units are skipped while *skip is set
};

// One persistent launch sweeps the units of several instances: table[k] describes instance k,
// unit_end[k] = sum of total_units of instances 0..k.  Workgroups take units from one ticket in
// order, so a unit only waits on lower tickets of its own instance (already running).
struct SweepLaunch {
    int ninst;
    unsigned total_units;
    const unsigned* unit_end;        // [ninst], device
    unsigned* ticket;                // [2] work ticket, retired workgroups; zero before the launch, reset after
    unsigned long long launch_id;    // unique per launch in the process (tags progress words)
    int grid_blocks;
    // nullptr, or the launch id is read here at the start (values from 2^31 on, disjoint from the
    // host's ids) and advanced by the last workgroup to retire, so a launch recorded once in a
    // graph still tags every replay apart
    unsigned long long* id_ctr;
};
// prefetch: chunks of loads each compute wavefront keeps in flight (2, 4 or 8)
template <typename TS>
void launch_sweep(hipStream_t s, const SweepArgs<TS>* table, const SweepLaunch& L, int prefetch = 4);
// next process-wide sweep launch id
unsigned long long next_sweep_launch_id();

// ----------------------------------------------------------------------------- bilinear DG sweep
// Upwind sweep of the bilinear (Q1) DG discretisation (Sec. 4.4) for nd directions, natural
// layouts: cell e = j*nx + i, local node a = ix + 2*iy (ix, iy = 0 on the left / bottom side).
constexpr int kQ1Waves = 2;        // compute wavefronts (64-column strips) per Q1 workgroup
template <typename TS>
struct Q1Args {
    int nx, ny, nd, nsuper;        // nsuper = superstrips of kQ1Waves x 64 columns
    unsigned total_units;          // nsuper * nd
    int grid_blocks;
    double hx, hy;
    const double* mu;              // [nd] direction cosines
    const double* eta;             // [nd]
    const TS* sig;                 // [ny*nx] sigma_t
    const TS* src;                 // [nd][ny*nx][4] nodal source
    const TS* inx;                 // [nd][ny][2] inflow on each row's x-inflow face, nodes iy = 0, 1
    const TS* iny;                 // [nd][nx][2] inflow on each column's y-inflow face, nodes ix = 0, 1
    TS* psi;                       // [nd][ny*nx][4]
    TS* edge;                      // [nd][nsuper][ny][2] outgoing x-face values, sweep row order
    unsigned long long* progress;  // [nd][nsuper] (launch << 32) | rows published
    unsigned* ticket;              // [2] unit ticket, retired workgroups (zero between launches)
    int* status;                   // kStatusSweepStall if a wait exceeds spin_limit polls
    unsigned spin_limit;
    unsigned long long launch_id;
};
template <typename TS>
void launch_q1_sweep(hipStream_t s, const Q1Args<TS>& a);

// ----------------------------------------------------------------------------- reductions
// V planes are compact [r][ldv] (cell e at V[k * ldv + e]).
// G = scale * V^T diag(weight) V (r x r, row-major; weight nullable = 1), via per-block partials in
// work [nblocks][r^2].
template <typename TV>
void launch_gram(hipStream_t s, long n, int r, const TV* V, size_t ldv, const double* weight, double scale,
                 double* work, int nblocks, double* G);
// C = A B (or A B^T) for r x r row-major matrices
void launch_small_matmul(hipStream_t s, int r, const double* A, const double* B, double* C,
                         bool b_transposed = false);
// Cholesky QR step: the Gram matrix G -> R, Rinv; a pivot too small for Cholesky QR sets
// status_code in *status.  With near_identity, also writes 1 there when max |G - I| < identity_tol
// (the basis is already orthonormal to that tolerance), else 0.
// With identity_on_flag, a status_code bit already set in *status (an earlier pass flagged the columns
// for the CGS2 fallback) makes R = Rinv = I.
void launch_chol(hipStream_t s, int r, const double* G, double* R, double* Rinv, int* status, int status_code,
                 int* near_identity = nullptr, double identity_tol = 0.0, bool identity_on_flag = false);
// X = X Rinv in place for n x r column-major X; nothing when *skip is set
void launch_trmm_inplace(hipStream_t s, int n, int r, double* X, const double* Rinv, const int* skip);
template <typename TV>
void launch_trmm(hipStream_t s, int n, int r, const TV* V, size_t ldv, const double* Rinv, double* X);
// X = V M for a general rin x rout matrix M (row-major, leading dimension ldm): n x rin column-major V
// (planes of n cells) -> n x rout X, rin <= 64, rout <= 32; X must not overlap V
void launch_gemm_tall(hipStream_t s, int n, int rin, int rout, const double* V, const double* M, int ldm,
                      double* X);
// Raw projection sums per block, [nblocks][5 r^2 + 5 r] (layout in k_mfma.hip); the matrix sums use
// FP64 MFMA operands (operand_bits 64), FP32 operands (32) or BF16 operands (16), the last two with
// FP32 accumulation per block; the vector sums and the sum over blocks are FP64.  X0 has r0 columns
// (r0 < 0: r); the rows of <X0_i, X_j> past r0 are zero.
void launch_project(hipStream_t s, int nx, int ny, int r, const double* X, const double* X0, const double* sigma,
                    const double* sig_s, const double* q, double* partials, int nblocks, int operand_bits,
                    int r0 = -1);
// raw[o] = area * sum over blocks of partials[b][o]
void launch_project_sum(hipStream_t s, int r, const double* partials, int nblocks, double area, double* raw);
// Produces Axp, Axm, Ayp, Aym, Mt, Ms (r x r each, row-major), qX[r], b[4][r], G = S0^T P [r][r];
// S0 is r0 x r0 (r0 < 0: r) and the rows of G past r0 are zero.  With T given, the sums were taken on
// a basis Xq whose orthonormal form is X = Xq T, and the operators are those of X.
void launch_project_finalize(hipStream_t s, int r, const double* partials, int nblocks, double hx, double hy,
                             double inv_cdt, const double* S0, double* ops, int r0 = -1,
                             const double* T = nullptr);

// ----------------------------------------------------------------------------- small dense FP64 work
// DEIM exchange area: per column two exchanges among up to 64 workgroups (double-buffered),
// and the workgroups' parts of beta
constexpr size_t kDeimXchgDoubles =
    2 * 64 + 2 * 64 * (2 + (size_t)kMaxRank) + 64 * (size_t)kMaxRank + 2 * 64 * (3 + (size_t)kMaxRank);
struct DeimArgs {
    int nq, r;
    const double* W;       // [r][nq]
    const double* S;       // [r][r]
    const double* w;       // [nq]
    double tie_tol;
    const int* forced;     // [r] or nullptr
    double* xchg;          // [kDeimXchgDoubles] exchange area among the workgroups
    unsigned* xcount;      // [2] arrival / departure counters, zero between launches
    unsigned long long launch_seq;   // unique per launch (>= 1): tags the exchanged words
    unsigned* seq_ctr;     // nullptr, or the tag is read here (values from 2^31 on) and advanced by the last group
    int* sel;              // [r]
    double* cw;            // [r]
    double* C0;            // [r][r]  C0[k*r + d] = sum_j S[k][j] W[j][sel_d]
    double* a0;            // [r]     S beta
    double* margins;       // [r]
    double* sel_mu;        // [r]
    double* sel_eta;       // [r]
    double* inflow_x;      // [r]
    double* inflow_y;      // [r]
    const double* mu;      // [nq]
    const double* eta;     // [nq]
    double psib[4];        // inflow intensity per side (0 for vacuum)
    int* status;
};
void launch_deim(hipStream_t s, const DeimArgs& a);

struct LstepArgs {
    int nq, r;
    const double* mu;
    const double* eta;
    const double* w;
    const double* ops;     // layout of launch_project_finalize
    const double* W0;      // [r][nq] old angular basis
    double inv_cdt;
    double psib[4];        // inflow intensity per side (0 when not an inflow side)
    double* Binv;          // [nq][r][r]
    double* y;             // [nq][r]
    double* red_partials;  // [nblocks][r*r + r]
    int red_blocks;
    double* v;             // [r] M_s Lbar / (4 pi)
    double* L;             // [r][nq]
    int* status;
};
void launch_lstep(hipStream_t s, const LstepArgs& a);

// one-sided Jacobi SVD of S = R^T; writes V [r][r] and S' = S V (columns U_k sigma_k), or Tl S V
// with Tl given
void launch_svd(hipStream_t s, int r, const double* R, double* V, double* Snew, int* status,
                const double* Tl = nullptr);
// weighted CGS2 with monomial completion, one workgroup: V [r][n] -> Q [r][n], R [r][r] upper.
// comp_kind 0: spatial monomials on the nx x ny cell centres, 1: angular monomials in (mu, eta).
// With flag != nullptr the kernel runs only if (*flag & flag_mask) and then clears those bits.
template <typename TV>
void launch_cgs2(hipStream_t s, long n, int r, const TV* V, size_t ldv, const double* weight, double wscalar,
                 int comp_kind,
                 int nx, int ny, const double* mu, const double* eta, double* Q, double* R, int* flag,
                 int flag_mask, int* status, int status_code);
// planes k = 0 .. count-1 of V: graded spatial monomial number first + k (the CGS2 completion's order) at the
// cell centres of the nx x ny grid, column-major cells
void launch_monomials(hipStream_t s, int nx, int ny, int first, int count, double* V, size_t ldv);
// X[k][c] = sum_j V[j][c] M[j][k] for a [r][n] column-major V (general r x r right multiply)
void launch_rmul(hipStream_t s, int n, int r, const double* V, const double* M, double* X);
// the same with rin input planes, rout output planes and M of leading dimension ldm
void launch_rmul_rect(hipStream_t s, int n, int rin, int rout, const double* V, const double* M, int ldm,
                      double* X);
// Truncation of an SVD result to rank r (Sec. 3, the rank-2r representation rounded back to rank r):
// Sv (ra x ra, row-major) holds U_k sigma_k in column k, singular values descending.  Its first r
// columns are factored as Q R with Q^T Q = I (two Gram-Schmidt passes; a column whose remainder is at
// most 1e-12 of its own norm, or zero, is replaced by the unit vector that keeps the largest remainder,
// with R_kk = 0).  Q -> [ra][r] row-major, R -> [r][r] row-major.  One workgroup.
void launch_trunc(hipStream_t s, int ra, int r, const double* Sv, double* Q, double* R);
// beta[k] = sum_q w_q W[k][q];  coef = S beta.  With mu, eta and gside set, also the side vectors
// of the outflow tally: gside[s][i] = sum_j S[i][j] sum_{q leaving through side s} w_q |Omega_q . n_s| W[j][q]
// (sides 0 left, 1 right, 2 bottom, 3 top).
// s_transposed: the matrix given is S^T (as the angular QR's R factor, S = R^T).  Tl: the matrix
// used is Tl S (Tl r x r, row-major), for a spatial basis stored as X Tl^{-1}.  S = nullptr stands for
// the identity (then Tl is required): W is then L = W S^T itself.
void launch_wsum(hipStream_t s, int nq, int r, const double* W, const double* w, const double* S, double* beta,
                 double* coef, const double* mu = nullptr, const double* eta = nullptr, double* gside = nullptr,
                 bool s_transposed = false, const double* Tl = nullptr);

// The few values the host reads after a source iteration or a step, written by one small kernel
// straight into host-mapped pinned memory (system-scope stores): up to three runs of doubles,
// placed one after the other from dst, and nstatus status words into dst_status.
struct PublishArgs {
    const double* src[3];
    int n[3];
    double* dst;
    const int* status;
    int nstatus;
    int* dst_status;
    const int* isrc;   // optional: ni more ints to idst
    int ni;
    int* idst;
    unsigned* seq_dst;   // optional: seq written last, after every other value is visible to the host
    unsigned seq;
};
void launch_publish(hipStream_t s, const PublishArgs& a);
// For n instances: their source-iteration control words flag[0..2], status word and last relative
// change norm into host-mapped pinned memory: dst_i[4 k + 0..3], dst_d[k] (system-scope stores).
void launch_gather_si(hipStream_t s, int n, const int* const* flags, const int* const* status,
                      const double* const* rel, int* dst_i, double* dst_d);

// ----------------------------------------------------------------------------- diffusion synthetic acceleration
// One DSA correction of the source iteration: phi <- phi + delta with D delta = M_s (phi - phi_old),
// D the diffusion matrix of the degree-0 cells (k_dsa.hip), by Jacobi-preconditioned CG in FP64; then
// the four orientation copies of s_e = sigma_s phi / (4 pi) in the sweep layout.  Cells column-major.
struct DsaArgs {
    int nx, ny;
    double hx, hy, inv_cdt;
    const double* sigma;       // [N] sigma (sigma_t = sigma + inv_cdt)
    const double* sig_s;       // [N] pseudo-scattering opacity
    const double* kappa;       // [2] sum_d c_d |mu_d|, sum_d c_d |eta_d| (launch_dsa_kappa)
    const double* phi_old;     // [N] the iterate the sweep started from
    double* phi;               // [N] in: the swept phi, out: corrected
    double *x, *r, *z, *q, *dg;  // [N] each
    double* p[2];              // [N] each, search direction (double-buffered)
    double* partials;          // [2 * dsa_blocks]
    unsigned* counter;         // zero between launches
    double* scal;              // [8] CG scalars
    double tol;                // relative residual of the CG solve
    int max_iter;              // CG iterations launched (the rest return at once after convergence)
    void* s_e;                 // [4][ldg] in the sweep precision, or nullptr
    size_t ldg;
    const int* skip;           // nullptr, or every kernel returns at once while *skip is set
};
int dsa_blocks(int nx, int ny);
void launch_dsa_kappa(hipStream_t s, int nd, const double* c, const double* mu, const double* eta, double* kappa);
void launch_dsa(hipStream_t s, const DsaArgs& a, bool fp32_layout);

// status words written by kernels
enum DeviceStatus : int {
    kStatusOk = 0,
    kStatusQrBreakdownX = 1,
    kStatusQrBreakdownW = 2,
    kStatusNonfinite = 4,
    kStatusSingularSolve = 8,
    kStatusBadForcedSel = 16,
    kStatusSvdNoConv = 32,
    kStatusSweepStall = 64,
    kStatusNoCompletion = 128,
    kStatusDeimStall = 256,
};

}  // namespace dlr
