// C-ABI of the dlrtrt library (include/dlrtrt.h) and the host orchestration of
// one SN-like DLR time step (Algorithm 1 of the paper) as a sequence of HIP
// kernel launches on the instance's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <deque>
#include <map>
#include <tuple>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dlrtrt.h"
#include "dlr_internal.h"
#include "host_setup.h"

namespace {

thread_local std::string g_last_error;

dlr_status fail(dlr_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

struct HipError : std::runtime_error {
    using std::runtime_error::runtime_error;
};

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) throw HipError(std::string(what) + ": " + hipGetErrorString(e));
}

// Device memory: hipMalloc / hipFree, or the caller's pair from dlr_set_allocator.  Every
// allocation keeps the pair (and the stream) it was made with, so it goes back the same way.
struct AllocHook {
    void* (*alloc)(size_t, void*, void*) = nullptr;
    void (*release)(void*, void*, void*) = nullptr;
    void* user = nullptr;
};
std::mutex g_alloc_mu;
AllocHook g_hook;

struct DevMem {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    AllocHook hook;
    bool user_owned() const { return hook.alloc != nullptr; }
};

// false: out of memory (nothing allocated)
bool dev_alloc(DevMem& m, size_t bytes, hipStream_t stream) {
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        m.hook = g_hook;
    }
    m.bytes = bytes;
    m.stream = stream;
    if (m.hook.alloc) {
        m.ptr = m.hook.alloc(bytes, stream, m.hook.user);
        if (m.ptr && (reinterpret_cast<uintptr_t>(m.ptr) & 255) != 0)
            throw std::runtime_error("allocator hook returned memory not aligned to 256 bytes");
        return m.ptr != nullptr;
    }
    const hipError_t e = hipMalloc(&m.ptr, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        m.ptr = nullptr;
        return false;
    }
    return true;
}

// The caller has made sure that no queued work still uses the memory.
void dev_free(DevMem& m) {
    if (!m.ptr) return;
    if (m.hook.release)
        m.hook.release(m.ptr, m.stream, m.hook.user);
    else
        (void)hipFree(m.ptr);
    m.ptr = nullptr;
}

bool hook_installed() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_hook.alloc != nullptr;
}

// One device allocation carved into 256-byte aligned pieces.
struct Arena {
    char* base = nullptr;
    size_t used = 0, cap = 0;
    DevMem mem;
    // false: out of memory
    bool allocate(size_t bytes, hipStream_t stream) {
        if (!dev_alloc(mem, bytes, stream)) return false;
        base = static_cast<char*>(mem.ptr);
        cap = bytes;
        used = 0;
        return true;
    }
    void release() {
        dev_free(mem);
        base = nullptr;
    }
    template <typename T>
    T* take(size_t count) {
        const size_t bytes = ((count * sizeof(T)) + 255) & ~size_t(255);
        if (base == nullptr) {   // sizing pass
            used += bytes;
            return nullptr;
        }
        if (used + bytes > cap) throw HipError("arena overflow");
        T* p = reinterpret_cast<T*>(base + used);
        used += bytes;
        return p;
    }
};

}  // namespace

constexpr int kPinnedNorm = 4;                                     // SI norm words
constexpr int kPinnedDoubles = kPinnedNorm + 2 + 2 * dlr::kMaxRank;   // + energy, outflow, margins, weights
constexpr int kPinnedInts = 8;   // status words [0, 4), source-iteration control words [4, 7), publish number [7]
constexpr int kSiSpec = 6;       // source iterations queued at once before the host looks (at most)

struct dlr_instance {
    // ---- problem (host copies)
    bool sn = false;   // plain discrete ordinates (every ordinate swept, no factors)
    // augmented basis: the step's Galerkin space is spanned by the swept columns and the old basis
    // (ra = 2r columns) and the SVD truncates the result back to rank r; otherwise ra = r
    bool augment = false;
    int nx = 0, ny = 0, N = 0, npol = 0, naz = 0, nq = 0, r = 0, ra = 0, prec = 0;
    double x0 = 0, x1 = 0, y0 = 0, y1 = 0, hx = 0, hy = 0, area = 0, dt = 0, c = 0, a = 0;
    double si_tol = 0, tie = 0;
    int si_max_iter = 0;
    int bc[4] = {0, 0, 0, 0};
    double Tb[4] = {0, 0, 0, 0}, psib[4] = {0, 0, 0, 0};
    double inflow_power = 0, source_power = 0;   // constant terms of the energy balance
    bool has_qext = false;
    hipStream_t stream = nullptr;
    std::vector<double> h_mu, h_eta, h_w;
    // ---- status
    bool poisoned = false;
    dlr_status poison_code = DLR_OK;
    bool s_is_usigma = false;   // S columns are U_k sigma_k (true after a step)
    bool have_sel = false;
    bool force_pending = false;
    int64_t steps_done = 0;
    dlr_step_stats stats{};
    // ---- source-iteration state of the step in progress
    double* phi_cur = nullptr;
    double* phi_nxt = nullptr;
    int si_it = 0;
    bool si_conv = false;
    float sweep_ms_acc = 0.f;
    float si_ms_acc = 0.f;   // sweeps and scalar-flux passes of the step's source iterations
    // ---- device memory
    Arena arena;
    double *mu = nullptr, *eta = nullptr, *w = nullptr;
    double *sigma = nullptr, *rho_cv = nullptr, *q_ext = nullptr, *T = nullptr;
    double *D = nullptr, *sig_s = nullptr, *q = nullptr, *sig_t = nullptr;
    float* sig_t32 = nullptr;
    double *X = nullptr, *Xn = nullptr;
    double* Va = nullptr;   // augmented: [swept basis | X] (2r planes; X is its second half)
    // The plain step stores its spatial basis after one Cholesky QR pass: the orthonormal basis is
    // X Rxi (Rxi = Rx^{-1}, r x r, from the second pass), and the stored S carries Rxi, so that
    // psi = X S W^T holds for the stored pair.  Identity after creation and load, and for the
    // augmented basis (its X is orthonormal).
    double *Rx = nullptr, *Rxi = nullptr;
    double *S = nullptr, *Sn = nullptr;
    double *W = nullptr, *Wt = nullptr, *Wq = nullptr, *L = nullptr;
    void *psi = nullptr, *src0 = nullptr, *s_e = nullptr, *psi_cm = nullptr;
    double *phi = nullptr, *phi2 = nullptr;
    int *sel = nullptr, *forced = nullptr;
    int* sel_alt = nullptr;     // picks of a selection queued for the next step (swapped with sel when it starts)
    double *cw = nullptr, *C0 = nullptr, *a0 = nullptr, *margins = nullptr, *sel_mu = nullptr, *sel_eta = nullptr;
    double *inflow_x = nullptr, *inflow_y = nullptr, *deim_work = nullptr;
    unsigned* deim_count = nullptr;
    int* si_flag = nullptr;         // [4] source-iteration control of the step (dlr::SiControl)
    unsigned* deim_ctr = nullptr;   // DEIM tag counter of graph-recorded launches (from 2^31 on)
    bool device_si = false;         // source iteration decided on the device (graph-recorded steps)
    bool capturing = false;         // launches are being recorded into a graph: no timing events
    bool untimed = false;           // this step's beginning ran from a recorded graph (no step timing)
    bool lin_ready = false;         // the last step queued the next step's linearisation behind its statistics
    bool deim_ready = false;        // ... and its start event and angle selection (DEIM)
    int si_last = 0;                // source iterations of the last step: how many the next step queues at once
    int sw_prefetch = 0, sw_grid = 0;   // sweep launch shape (0: chosen by the tuner at the first sweep)
    void* edge = nullptr;
    unsigned long long* progress = nullptr;
    unsigned* ticket = nullptr;
    char* sweep_rec = nullptr;       // device SweepArgs record of this instance
    unsigned* unit_end = nullptr;    // [1] sweep units of this instance
    std::vector<char> h_sweep_rec;   // host copy of the sweep record (SweepArgs of the instance's precision)
    int nsuper = 0;
    size_t ld = 0;    // elements of one compact cell plane of Psi handed to the QR (N rounded up to 64)
    size_t ldg = 0;   // elements of one diagonal sweep plane (psi, src0, and the 4 copies of sigma_t, s_e)
    double* partials = nullptr;
    size_t partials_count = 0;
    double* tpart = nullptr;   // the temperature update's block sums (it runs beside kernels that use partials)
    double* norm_out = nullptr;
    double* energy_out = nullptr;
    unsigned* counters = nullptr;
    double *Gm = nullptr, *Ra = nullptr, *R1 = nullptr, *R1i = nullptr, *R2 = nullptr, *R2i = nullptr;
    double *ops = nullptr, *Binv = nullptr, *yv = nullptr, *red = nullptr, *vv = nullptr;
    double *Vsvd = nullptr, *beta = nullptr, *coef = nullptr, *gside = nullptr;
    int* status = nullptr;
    // diffusion synthetic acceleration (dlr_set_dsa): workspace in its own allocation
    bool dsa = false;
    double dsa_tol = 1e-8;
    int dsa_max_iter = 100;
    DevMem dsa_mem;
    double* dsa_ws = nullptr;     // [7 N] x, r, z, q, diag, p0, p1
    double* dsa_part = nullptr;   // [2 * dsa_blocks]
    double* dsa_scal = nullptr;   // [8]
    double* dsa_kappa = nullptr;  // [2]
    unsigned* dsa_count = nullptr;
    // plain SN only
    double *q_diag = nullptr, *phio = nullptr;
    int *orient = nullptr, *dirs = nullptr, *dir_off = nullptr;
    // pinned host mirrors
    double* h_norm = nullptr;   // pinned: SI norms [0, kPinnedNorm), then energy, margins[r], cw[r]
    int* h_status = nullptr;
    double* d_h_norm = nullptr;   // the device's addresses of the two pinned areas
    int* d_h_status = nullptr;
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    // second stream for work that does not depend on the main stream's latency-bound kernels
    // (the linearisation beside DEIM, the temperature update beside the SVD); nullptr: in order
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_si[3 * kSiSpec] = {};   // queued source iterations: sweep starts, sweep ends, flux ends
    unsigned pub_seq = 0;                 // number of the last publish the host waits for by polling
    // launch shapes
    int nb_cells = 256, nb_phi = 1024, nb_gram = 512, nb_gram_ang = 32, nb_proj = 512, red_blocks = 64;

    bool fp32() const { return prec != DLR_FP64; }
    size_t sweep_bytes() const { return fp32() ? sizeof(float) : sizeof(double); }
    int nsweep() const { return sn ? nq : r; }   // directions of one sweep launch

    // plain SN: all ordinates' psi and fixed source in the diagonal layout, q in 4 orientation copies
    void carve_sn(Arena& A) {
        const size_t n = (size_t)N, Q = (size_t)nq;
        mu = A.take<double>(Q);
        eta = A.take<double>(Q);
        w = A.take<double>(Q);
        orient = A.take<int>(Q);
        dirs = A.take<int>(Q);
        dir_off = A.take<int>(8);
        inflow_x = A.take<double>(Q);
        inflow_y = A.take<double>(Q);
        sigma = A.take<double>(n);
        rho_cv = A.take<double>(n);
        q_ext = has_qext ? A.take<double>(n) : nullptr;
        T = A.take<double>(n);
        D = A.take<double>(n);
        sig_s = A.take<double>(n);
        q = A.take<double>(n);
        q_diag = A.take<double>(4 * ldg);
        sig_t = fp32() ? nullptr : A.take<double>(4 * ldg);
        sig_t32 = fp32() ? A.take<float>(4 * ldg) : nullptr;
        psi = A.take<char>(Q * ldg * sweep_bytes());
        src0 = A.take<char>(Q * ldg * sweep_bytes());
        s_e = A.take<char>(4 * ldg * sweep_bytes());
        phio = A.take<double>(4 * ldg);
        phi = A.take<double>(n);
        phi2 = A.take<double>(n);
        edge = A.take<char>(Q * (size_t)nsuper * ny * sweep_bytes());
        progress = A.take<unsigned long long>(Q * (size_t)nsuper);
        ticket = A.take<unsigned>(4);
        sweep_rec = A.take<char>(sizeof(dlr::SweepArgs<double>));
        unit_end = A.take<unsigned>(4);
        partials = A.take<double>(partials_count);
        norm_out = A.take<double>(4);
        energy_out = A.take<double>(2);
        counters = A.take<unsigned>(8);
        status = A.take<int>(4);
    }

    void carve(Arena& A) {
        if (sn) return carve_sn(A);
        const size_t n = (size_t)N, R = (size_t)r, Q = (size_t)nq;
        const size_t RA = (size_t)ra;   // Galerkin rank of the step's dense work
        mu = A.take<double>(Q);
        eta = A.take<double>(Q);
        w = A.take<double>(Q);
        sigma = A.take<double>(n);
        rho_cv = A.take<double>(n);
        q_ext = has_qext ? A.take<double>(n) : nullptr;
        T = A.take<double>(n);
        D = A.take<double>(n);
        sig_s = A.take<double>(n);
        q = A.take<double>(n);
        sig_t = fp32() ? nullptr : A.take<double>(4 * ldg);
        sig_t32 = fp32() ? A.take<float>(4 * ldg) : nullptr;
        if (augment) {
            Va = A.take<double>(2 * R * n);
            X = Va ? Va + R * n : nullptr;
        } else {
            X = A.take<double>(R * n);
        }
        Xn = A.take<double>(RA * n);
        Rx = A.take<double>(R * R);
        Rxi = A.take<double>(R * R);
        S = A.take<double>(R * R);
        Sn = A.take<double>(RA * RA);
        W = A.take<double>(RA * Q);   // planes past r stay zero (the L-step reads ra planes of W0)
        Wt = A.take<double>(RA * Q);
        Wq = A.take<double>(RA * Q);
        L = A.take<double>(RA * Q);
        psi = A.take<char>(R * ldg * sweep_bytes());
        src0 = A.take<char>(R * ldg * sweep_bytes());
        s_e = A.take<char>(4 * ldg * sweep_bytes());
        phio = A.take<double>(4 * ldg);
        psi_cm = A.take<char>(R * ld * sweep_bytes());
        phi = A.take<double>(n);
        phi2 = A.take<double>(n);
        sel = A.take<int>(R);
        forced = A.take<int>(R);
        sel_alt = A.take<int>(R);
        cw = A.take<double>(R);
        C0 = A.take<double>(R * R);
        a0 = A.take<double>(R);
        margins = A.take<double>(R);
        sel_mu = A.take<double>(R);
        sel_eta = A.take<double>(R);
        inflow_x = A.take<double>(R);
        inflow_y = A.take<double>(R);
        deim_work = A.take<double>(dlr::kDeimXchgDoubles);
        deim_count = A.take<unsigned>(4);
        si_flag = A.take<int>(4);
        deim_ctr = A.take<unsigned>(4);
        edge = A.take<char>(R * (size_t)nsuper * ny * sweep_bytes());
        progress = A.take<unsigned long long>(R * (size_t)nsuper);
        ticket = A.take<unsigned>(4);
        sweep_rec = A.take<char>(sizeof(dlr::SweepArgs<double>));
        unit_end = A.take<unsigned>(4);
        partials = A.take<double>(partials_count);
        tpart = A.take<double>(2 * (size_t)nb_cells);
        norm_out = A.take<double>(4);
        energy_out = A.take<double>(2);
        counters = A.take<unsigned>(8);
        Gm = A.take<double>(RA * RA);
        Ra = A.take<double>(RA * RA);
        R1 = A.take<double>(RA * RA);
        R1i = A.take<double>(RA * RA);
        R2 = A.take<double>(RA * RA);
        R2i = A.take<double>(RA * RA);
        ops = A.take<double>(12 * RA * RA + 10 * RA);
        Binv = A.take<double>(Q * RA * RA);
        yv = A.take<double>(Q * RA);
        red = A.take<double>((size_t)red_blocks * (RA * RA + RA));
        vv = A.take<double>(RA);
        Vsvd = A.take<double>(RA * RA);
        beta = A.take<double>(RA);
        coef = A.take<double>(RA);
        gside = A.take<double>(4 * RA);
        status = A.take<int>(4);
    }
};

namespace {

dlr_status validate(const dlr_problem* p, bool sn = false) {
    if (!p) return fail(DLR_ERR_ARG, "problem is NULL");
    if (p->abi_version != DLR_ABI_VERSION) return fail(DLR_ERR_ARG, "abi_version mismatch");
    if (p->nx < 1 || p->ny < 1) return fail(DLR_ERR_ARG, "nx, ny must be >= 1");
    if ((long long)p->nx * p->ny > (1LL << 30)) return fail(DLR_ERR_ARG, "grid too large");
    if (!(p->x1 > p->x0) || !(p->y1 > p->y0)) return fail(DLR_ERR_ARG, "empty domain");
    if (p->n_polar < 1 || p->n_azim < 4 || p->n_azim % 4 != 0)
        return fail(DLR_ERR_ARG, "n_polar >= 1 and n_azim a positive multiple of 4 required");
    const long long nq = (long long)p->n_polar * p->n_azim;
    if (nq > 16384) return fail(DLR_ERR_ARG, "at most 16384 ordinates");
    const long long ncell = (long long)p->nx * p->ny;
    if (!sn && (p->rank < 1 || p->rank > dlr::kMaxRank || p->rank > nq || p->rank > ncell))
        return fail(DLR_ERR_ARG, "rank must satisfy 1 <= rank <= min(64, ordinates, cells)");
    if (!(p->dt > 0) || !(p->c > 0) || !(p->a >= 0) || !std::isfinite(p->dt) || !std::isfinite(p->c) ||
        !std::isfinite(p->a))
        return fail(DLR_ERR_ARG, "dt, c > 0 and a >= 0 required");
    if (!p->sigma_a || !p->rho_cv || !p->T_init) return fail(DLR_ERR_ARG, "sigma_a, rho_cv, T_init required");
    for (long long e = 0; e < ncell; ++e) {
        if (!(p->sigma_a[e] > 0) || !std::isfinite(p->sigma_a[e])) return fail(DLR_ERR_ARG, "sigma_a must be > 0");
        if (!(p->rho_cv[e] > 0) || !std::isfinite(p->rho_cv[e])) return fail(DLR_ERR_ARG, "rho_cv must be > 0");
        if (!(p->T_init[e] >= 0) || !std::isfinite(p->T_init[e])) return fail(DLR_ERR_ARG, "T_init must be >= 0");
        if (p->q_ext && (!(p->q_ext[e] >= 0) || !std::isfinite(p->q_ext[e])))
            return fail(DLR_ERR_ARG, "q_ext must be >= 0");
    }
    for (int s = 0; s < 4; ++s) {
        if (p->bc[s] == DLR_BC_REFLECT)
            return fail(DLR_ERR_UNSUPPORTED, "reflecting walls are not available on the GPU path");
        if (p->bc[s] != DLR_BC_VACUUM && p->bc[s] != DLR_BC_INFLOW) return fail(DLR_ERR_ARG, "unknown bc");
        if (!(p->T_b[s] >= 0) || !std::isfinite(p->T_b[s])) return fail(DLR_ERR_ARG, "T_b must be >= 0");
    }
    if (p->precision != DLR_FP64 && p->precision != DLR_FP32_SWEEP && p->precision != DLR_FP32_SWEEP_BF16_PROJ)
        return fail(DLR_ERR_ARG, "unknown precision");
    if (!(p->si_tol > 0) || p->si_max_iter < 1) return fail(DLR_ERR_ARG, "si_tol > 0 and si_max_iter >= 1");
    if (!sn && (!(p->deim_tie_tol >= 0) || !(p->deim_tie_tol < 1)))
        return fail(DLR_ERR_ARG, "0 <= deim_tie_tol < 1");
    return DLR_OK;
}

template <typename TS>
dlr_status step_once(dlr_instance* I);

// The host waits for a publish by polling the number it writes last (after every value it publishes
// is visible): no event on the stream, whose marker would leave the GPU idle for a few microseconds
// between the kernels around it.  After 50 ms of polling the wait becomes a stream synchronisation,
// which also reports a device error that kept the publish from running.
unsigned next_publish(dlr_instance* I) {
    if (++I->pub_seq == 0) I->pub_seq = 1;
    return I->pub_seq;
}
void wait_published(dlr_instance* I, unsigned seq) {
    const volatile unsigned* word = reinterpret_cast<const volatile unsigned*>(I->h_status + 7);
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned n = 1; *word != seq; ++n) {
        __builtin_ia32_pause();
        if ((n & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50)) {
            hip_check(hipStreamSynchronize(I->stream), "stream sync");
            if (*word != seq) throw std::runtime_error("a publish did not arrive although its stream has drained");
            break;
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
}

// published: a launch_publish of the four status words is already queued on the stream (then `seq`, if
// not 0, is its number, and the host waits for that instead of the whole stream)
dlr_status check_device_status(dlr_instance* I, bool published = false, unsigned seq = 0) {
    if (!published)
        hip_check(hipMemcpyAsync(I->h_status, I->status, 4 * sizeof(int), hipMemcpyDeviceToHost, I->stream),
                  "status copy");
    if (published && seq)
        wait_published(I, seq);
    else
        hip_check(hipStreamSynchronize(I->stream), "stream sync");
    const int st = *I->h_status;
    if (st == 0) return DLR_OK;
    std::string m = "device status";
    dlr_status code = DLR_ERR_NUMERIC;
    if (st & dlr::kStatusNonfinite) { m += " non-finite"; code = DLR_ERR_NONFINITE; }
    if (st & dlr::kStatusQrBreakdownX) m += " spatial-QR-breakdown";
    if (st & dlr::kStatusQrBreakdownW) m += " angular-QR-breakdown";
    if (st & dlr::kStatusSingularSolve) m += " singular-solve";
    if (st & dlr::kStatusSvdNoConv) m += " svd-not-converged";
    if (st & dlr::kStatusSweepStall) { m += " sweep-wait-stalled"; code = DLR_ERR_TIMEOUT; }
    if (st & dlr::kStatusDeimStall) { m += " deim-exchange-stalled"; code = DLR_ERR_TIMEOUT; }
    if (st & dlr::kStatusNoCompletion) m += " no-completion-vector";
    if (st & dlr::kStatusBadForcedSel) { m += " bad-forced-selection"; code = DLR_ERR_ARG; }
    I->poisoned = true;
    I->poison_code = code;
    return fail(code, m);
}

// Queue the copies of (up to three) runs of doubles into the pinned area from word `at`, and of the
// first `nstatus` status words, as one kernel.
void publish(dlr_instance* I, hipStream_t s, int at, const double* a, int na, const double* b, int nb, const double* c,
             int nc, int nstatus, unsigned seq = 0) {
    dlr::PublishArgs p{};
    p.src[0] = a; p.n[0] = a ? na : 0;
    p.src[1] = b; p.n[1] = b ? nb : 0;
    p.src[2] = c; p.n[2] = c ? nc : 0;
    p.dst = I->d_h_norm + at;
    p.status = I->status; p.nstatus = nstatus; p.dst_status = I->d_h_status;
    if (seq) {
        p.seq_dst = reinterpret_cast<unsigned*>(I->d_h_status + 7);
        p.seq = seq;
    }
    dlr::launch_publish(s, p);
}


// The sweep record of an instance (fixed for its life; DEIM rewrites the pointed-to direction data).
template <typename TS>
dlr::SweepArgs<TS> make_sweep_record(const dlr_instance* I) {
    dlr::SweepArgs<TS> sa{};
    sa.nx = I->nx; sa.ny = I->ny; sa.nd = I->nsweep(); sa.nsuper = I->nsuper; sa.total_units = I->nsuper * sa.nd;
    sa.ldg = I->ldg;
    sa.src0 = static_cast<const TS*>(I->src0);
    sa.sig_t = I->fp32() ? reinterpret_cast<const TS*>(I->sig_t32) : reinterpret_cast<const TS*>(I->sig_t);
    sa.s_e = static_cast<const TS*>(I->s_e);
    sa.psi = static_cast<TS*>(I->psi);
    sa.mu = I->sn ? I->mu : I->sel_mu;
    sa.eta = I->sn ? I->eta : I->sel_eta;
    sa.inflow_x = I->inflow_x; sa.inflow_y = I->inflow_y;
    sa.inv_hx = 1.0 / I->hx; sa.inv_hy = 1.0 / I->hy;
    sa.edge = static_cast<TS*>(I->edge); sa.progress = I->progress;
    sa.status = I->status;
    sa.spin_limit = 1u << 20;
    sa.skip = I->si_flag;   // zero except in graph-recorded steps once the source iteration has stopped
    return sa;
}

void upload_sweep_record(dlr_instance* I) {
    I->h_sweep_rec.resize(sizeof(dlr::SweepArgs<double>));
    if (I->fp32()) {
        const dlr::SweepArgs<float> a = make_sweep_record<float>(I);
        std::memcpy(I->h_sweep_rec.data(), &a, sizeof(a));
    } else {
        const dlr::SweepArgs<double> a = make_sweep_record<double>(I);
        std::memcpy(I->h_sweep_rec.data(), &a, sizeof(a));
    }
    const unsigned units = (unsigned)(I->nsuper * I->nsweep());
    hip_check(hipMemcpy(I->sweep_rec, I->h_sweep_rec.data(), I->h_sweep_rec.size(), hipMemcpyHostToDevice), "record");
    hip_check(hipMemcpy(I->unit_end, &units, sizeof(units), hipMemcpyHostToDevice), "record");
}

dlr::TupdateArgs tupdate_args(dlr_instance* I, const double* X, const double* gside) {
    dlr::TupdateArgs A{};
    A.nx = I->nx; A.ny = I->ny; A.r = X ? I->r : 0;
    A.X = X; A.coef = I->coef; A.gside = gside;
    A.sigma = I->sigma; A.rho_cv = I->rho_cv; A.D = I->D;
    A.dt = I->dt; A.a = I->a; A.c = I->c; A.area = I->area; A.hx = I->hx; A.hy = I->hy;
    A.T = I->T; A.phi = I->phi;
    A.partials = I->tpart ? I->tpart : I->partials;
    A.counter = I->counters + 1; A.out = I->energy_out; A.status = I->status;
    return A;
}

// DSA correction of the source iteration just checked (phi_cur = swept phi, phi_nxt = the iterate it
// started from), queued on the instance's stream before its next sweep.
void dsa_correct(dlr_instance* I) {
    dlr::DsaArgs a{};
    a.nx = I->nx; a.ny = I->ny; a.hx = I->hx; a.hy = I->hy; a.inv_cdt = 1.0 / (I->c * I->dt);
    a.sigma = I->sigma; a.sig_s = I->sig_s; a.kappa = I->dsa_kappa;
    a.phi_old = I->phi_nxt; a.phi = I->phi_cur;
    const size_t n = (size_t)I->N;
    double* w = I->dsa_ws;
    a.x = w; a.r = w + n; a.z = w + 2 * n; a.q = w + 3 * n; a.dg = w + 4 * n; a.p[0] = w + 5 * n; a.p[1] = w + 6 * n;
    a.partials = I->dsa_part; a.counter = I->dsa_count; a.scal = I->dsa_scal;
    a.tol = I->dsa_tol; a.max_iter = I->dsa_max_iter;
    a.s_e = I->s_e; a.ldg = I->ldg;
    a.skip = I->device_si ? I->si_flag : nullptr;   // no correction once the iteration has stopped
    dlr::launch_dsa(I->stream, a, I->fp32());
}

// Algorithm 1 step 1 on the instance's current temperature.
void launch_linearize(dlr_instance* I, hipStream_t s) {
    dlr::launch_linearize(s, I->nx, I->ny, I->sigma, I->rho_cv, I->q_ext, I->T, I->dt, I->a, I->c, I->D, I->sig_s,
                          I->q, I->sig_t, I->sig_t32, I->ldg, nullptr);
}

// Algorithm 1 step 2 on the instance's current W and S: DEIM (forced picks if pending), the weights,
// C0 = S W[sel]^T, a0 = S beta, and the DSA coefficients of the picks.
void launch_selection(dlr_instance* I, hipStream_t s, int* sel_out) {
    const int r = I->r;
    dlr::DeimArgs da{};
    da.nq = I->nq; da.r = r; da.W = I->W; da.S = I->S; da.w = I->w; da.tie_tol = I->tie;
    da.forced = I->force_pending ? I->forced : nullptr;
    da.xchg = I->deim_work; da.xcount = I->deim_count; da.launch_seq = dlr::next_sweep_launch_id();
    da.seq_ctr = I->device_si ? I->deim_ctr : nullptr; da.sel = sel_out; da.cw = I->cw; da.C0 = I->C0; da.a0 = I->a0; da.margins = I->margins;
    da.sel_mu = I->sel_mu; da.sel_eta = I->sel_eta; da.inflow_x = I->inflow_x; da.inflow_y = I->inflow_y;
    da.mu = I->mu; da.eta = I->eta;
    for (int k = 0; k < 4; ++k) da.psib[k] = I->psib[k];
    da.status = I->status;
    dlr::launch_deim(s, da);
    I->force_pending = false;
    if (I->dsa) dlr::launch_dsa_kappa(s, r, I->cw, I->sel_mu, I->sel_eta, I->dsa_kappa);
}

// ---------------------------------------------------------------------------------------------------------
// One DLR step in phases, so that a batch can interleave the phases of many instances:
//   phase_begin  linearise, DEIM, old solution at the new ordinates (Algorithm 1 steps 1-3)
//   [sweep]      one persistent launch per source iteration, alone or shared by a batch (step 4)
//   si_phi       scalar flux, convergence norm and status -> pinned host memory (step 4)
//   si_check     after the stream has reached si_phi: converged / failed / go on
//   phase_end    X, projections, L-step, W and S, temperature (steps 5-9)
//   step_publish, step_read  status check and statistics
// A step alone (step_once) queues its source iterations several at a time, decided on the device
// (si_queue), and the next step's linearisation behind its statistics.
template <typename TS>
void phase_begin(dlr_instance* I) {
    hipStream_t s = I->stream;
    const int r = I->r;
    const double cdt = I->c * I->dt;
    // A step alone queues the next step's start behind its statistics (start event, linearisation,
    // selection): they run while the host reads those.  A selection forced since is made again here.
    const bool queued = I->deim_ready;
    I->deim_ready = false;
    if (queued) {
        std::swap(I->ev[0], I->ev[1]);    // the last step's end event starts this step
        std::swap(I->sel, I->sel_alt);    // the queued selection's picks
    } else if (!I->capturing) {
        hip_check(hipEventRecord(I->ev[0], s), "event");
    }
    // 1. effective scattering and source (beside DEIM, which does not read them), unless the last step
    // queued them behind its statistics
    const bool lin = !I->lin_ready;
    I->lin_ready = false;
    const bool fork = lin && I->side;
    hipStream_t ls = s;
    if (fork) {
        hip_check(hipEventRecord(I->ev_fork, s), "event");
        hip_check(hipStreamWaitEvent(I->side, I->ev_fork, 0), "wait");
        ls = I->side;
    }
    if (lin) launch_linearize(I, ls);
    if (fork) hip_check(hipEventRecord(I->ev_join, I->side), "event");
    // 2. DEIM angle selection on W (and the weights, C0 = S W[sel]^T, a0 = S beta)
    if (!queued || I->force_pending) launch_selection(I, s, I->sel);
    if (fork) hip_check(hipStreamWaitEvent(s, I->ev_join, 0), "wait");
    // 3. old solution at the selected ordinates -> fixed source; SI start phi = X S beta
    dlr::launch_psi0<TS>(s, I->nx, I->ny, r, I->X, I->C0, I->a0, I->q, I->sig_s, 1.0 / cdt, I->sel_mu, I->sel_eta,
                         static_cast<TS*>(I->src0), I->ldg, I->phi, static_cast<TS*>(I->s_e), I->si_flag);
    I->phi_cur = I->phi;
    I->phi_nxt = I->phi2;
    I->si_it = 0;
    I->si_conv = false;
    I->sweep_ms_acc = 0.f;
    I->si_ms_acc = 0.f;
}

// ---------------------------------------------------------------------------------------------- sweep shape tuner
// The launch shape of an instance's sweep -- the chunks of loads each compute wavefront keeps in
// flight (the register prefetch depth) and the number of persistent workgroups -- is chosen by
// timing the candidates on the instance's own data at its first sweep, and kept per grid, count
// of swept directions and precision for the life of the process.  A sweep reads only its inputs,
// so the timing launches leave the results as they are, and the shape changes no arithmetic.
struct TuneKey {
    int nx, ny, nd, bytes;
    bool operator<(const TuneKey& o) const {
        return std::tie(nx, ny, nd, bytes) < std::tie(o.nx, o.ny, o.nd, o.bytes);
    }
};
struct SweepShape {
    int prefetch, grid;
};
std::mutex g_tune_mu;
std::map<TuneKey, SweepShape> g_tuned;

template <typename TS>
void sweep_launch(dlr_instance* I, int prefetch, int grid) {
    dlr::SweepLaunch L{};
    L.ninst = 1;
    L.total_units = (unsigned)(I->nsuper * I->nsweep());
    L.unit_end = I->unit_end;
    L.ticket = I->ticket;
    L.launch_id = dlr::next_sweep_launch_id();
    L.grid_blocks = (int)std::min<unsigned>(L.total_units, (unsigned)grid);
    dlr::launch_sweep<TS>(I->stream, reinterpret_cast<const dlr::SweepArgs<TS>*>(I->sweep_rec), L, prefetch);
}

template <typename TS>
void sweep_tune(dlr_instance* I) {
    const TuneKey key{I->nx, I->ny, I->nsweep(), (int)sizeof(TS)};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            I->sw_prefetch = it->second.prefetch;
            I->sw_grid = it->second.grid;
            return;
        }
    }
    // FP64 with 8 chunks in flight does not fit the register file (it spills)
    const int pre[3] = {2, 4, 8};
    const int npre = sizeof(TS) == 4 ? 3 : 2;
    const int grids[3] = {256, 512, 1024};
    SweepShape best{4, I->sn ? 1024 : 512};
    float best_ms = 0.f;
    bool have = false;
    for (int a = 0; a < npre; ++a)
        for (int b = 0; b < 3; ++b) {
            sweep_launch<TS>(I, pre[a], grids[b]);   // warm-up
            hip_check(hipEventRecord(I->ev[2], I->stream), "event");
            sweep_launch<TS>(I, pre[a], grids[b]);
            sweep_launch<TS>(I, pre[a], grids[b]);
            hip_check(hipEventRecord(I->ev[3], I->stream), "event");
            hip_check(hipEventSynchronize(I->ev[3]), "sync");
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, I->ev[2], I->ev[3]), "elapsed");
            if (!have || ms < best_ms) {
                best = SweepShape{pre[a], grids[b]};
                best_ms = ms;
                have = true;
            }
        }
    I->sw_prefetch = best.prefetch;
    I->sw_grid = best.grid;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.emplace(key, best);
}

// this instance alone: one sweep launch on its own stream, timed with events
template <typename TS>
void sweep_alone(dlr_instance* I) {
    if (I->sw_prefetch == 0) sweep_tune<TS>(I);
    hip_check(hipEventRecord(I->ev[2], I->stream), "event");
    sweep_launch<TS>(I, I->sw_prefetch, I->sw_grid);
    hip_check(hipEventRecord(I->ev[3], I->stream), "event");
}

template <typename TS>
void si_phi(dlr_instance* I) {
    hipStream_t s = I->stream;
    const dlr::SiControl ctl{I->si_flag, I->si_tol, I->si_max_iter};
    dlr::launch_phi<TS>(s, I->nx, I->ny, I->r, static_cast<const TS*>(I->psi), I->ldg, I->sel_mu, I->sel_eta, I->cw,
                        I->phio, I->sig_s, I->phi_cur, I->phi_nxt, static_cast<TS*>(I->s_e), I->partials, I->nb_phi,
                        I->counters + 0, I->norm_out, I->device_si ? &ctl : nullptr);
    std::swap(I->phi_cur, I->phi_nxt);
    // with the iteration decided on the device the host reads the control words once, at the end
    if (!I->device_si) publish(I, s, 0, I->norm_out, 3, nullptr, 0, nullptr, 0, 1);
}

// After the stream has passed si_phi.  Returns DLR_OK with I->si_conv set, or an error (handle poisoned).
dlr_status si_check(dlr_instance* I) {
    ++I->si_it;
    if (*I->h_status != 0) return check_device_status(I);
    const double rel = I->h_norm[2];
    if (!std::isfinite(rel)) {
        I->poisoned = true;
        I->poison_code = DLR_ERR_NONFINITE;
        return fail(DLR_ERR_NONFINITE, "non-finite scalar flux in source iteration");
    }
    I->stats.si_residual = rel;
    // I->phi names the converged flux after the step's iteration -- except in a step begun from a
    // recorded graph, whose launches hold the buffers as recorded (a DLR step does not read the
    // converged flux after the iteration: the temperature update forms phi from the new factors)
    const bool rename = I->phi_cur != I->phi && !I->untimed;
    if (rel <= I->si_tol) {
        I->si_conv = true;
        if (rename) std::swap(I->phi, I->phi2);
        return DLR_OK;
    }
    if (I->si_it >= I->si_max_iter) {
        if (rename) std::swap(I->phi, I->phi2);
        I->poisoned = true;
        I->poison_code = DLR_ERR_NOT_CONVERGED;
        return fail(DLR_ERR_NOT_CONVERGED, "source iteration reached si_max_iter");
    }
    return DLR_OK;
}

// Steps 5 to 8 up to the angular QR.  Everything this part writes is scratch (the new basis, the
// projections, the L-step, the angular factors); the state (X, S, W, T) is written only by
// phase_end_b, so a step alone can queue this part before the host knows that the source iteration
// has converged, and queue it again after further iterations if it had not.
template <typename TS>
void phase_end_a(dlr_instance* I) {
    hipStream_t s = I->stream;
    const int N = I->N, r = I->r, nq = I->nq, rg = I->ra;
    const double cdt = I->c * I->dt;
    TS* psi = static_cast<TS*>(I->psi);
    TS* psi_cm = static_cast<TS*>(I->psi_cm);
    // the orthonormal swept basis: the new X, or with the augmented basis the first half of Va
    double* Xq = I->augment ? I->Va : I->Xn;
    // 5. X from the swept columns: Cholesky QR (column-scaled) in the cell-area inner product; the
    // second pass re-orthonormalises in place unless the first already left the Gram matrix within
    // tol of the identity (1e-11 with FP64 sweeps, 1e-8 with FP32 sweeps: X then differs from the
    // exact orthonormal factor by less than that)
    dlr::launch_psi_to_cm<TS>(s, I->nx, I->ny, r, psi, I->ldg, I->sel_mu, I->sel_eta, psi_cm, I->ld);
    dlr::launch_gram<TS>(s, N, r, psi_cm, I->ld, nullptr, I->area, I->partials, I->nb_gram, I->Gm);
    dlr::launch_chol(s, r, I->Gm, I->R1, I->R1i, I->status, dlr::kStatusQrBreakdownX);
    dlr::launch_trmm<TS>(s, N, r, psi_cm, I->ld, I->R1i, Xq);
    dlr::launch_gram<double>(s, N, r, Xq, (size_t)N, nullptr, I->area, I->partials, I->nb_gram, I->Gm);
    if (I->augment) {
        dlr::launch_chol(s, r, I->Gm, I->R2, I->R2i, I->status, dlr::kStatusQrBreakdownX, I->status + 3,
                         I->fp32() ? 1e-8 : 1e-11);
        dlr::launch_trmm_inplace(s, N, r, Xq, I->R2i, I->status + 3);
    } else {
        // The second pass's factor is not multiplied into the cell planes: the orthonormal basis is
        // Xq Rxi, and the projections, the temperature update's coefficients and the new S take Rxi
        // instead (r x r work in place of a pass over the r planes).  When the first pass flagged the
        // columns, the fallback below rebuilds an orthonormal basis and Rxi is the identity.
        dlr::launch_chol(s, r, I->Gm, I->Rx, I->Rxi, I->status, dlr::kStatusQrBreakdownX, nullptr, 0.0, true);
    }
    // fallback (runs on the device only if a Cholesky pivot flagged near-dependent columns)
    dlr::launch_cgs2<TS>(s, N, r, psi_cm, I->ld, nullptr, I->area, 0, I->nx, I->ny, nullptr, nullptr, Xq,
                         I->R1, I->status, dlr::kStatusQrBreakdownX, I->status, dlr::kStatusNoCompletion);
    if (I->augment) {
        // 5 (augmented basis). Va = [swept basis | X0] (contiguous planes) -> Xn, 2r orthonormal
        // columns whose span holds the old solution: the same Cholesky QR twice, and the CGS2 with
        // spatial completion when X0 has columns (nearly) inside the swept span
        dlr::launch_gram<double>(s, N, rg, I->Va, (size_t)N, nullptr, I->area, I->partials, I->nb_gram, I->Gm);
        dlr::launch_chol(s, rg, I->Gm, I->R1, I->R1i, I->status, dlr::kStatusQrBreakdownX);
        dlr::launch_trmm<double>(s, N, rg, I->Va, (size_t)N, I->R1i, I->Xn);
        dlr::launch_gram<double>(s, N, rg, I->Xn, (size_t)N, nullptr, I->area, I->partials, I->nb_gram, I->Gm);
        dlr::launch_chol(s, rg, I->Gm, I->R2, I->R2i, I->status, dlr::kStatusQrBreakdownX, I->status + 3, 1e-11);
        dlr::launch_trmm_inplace(s, N, rg, I->Xn, I->R2i, I->status + 3);
        dlr::launch_cgs2<double>(s, N, rg, I->Va, (size_t)N, nullptr, I->area, 0, I->nx, I->ny, nullptr, nullptr,
                                 I->Xn, I->R1, I->status, dlr::kStatusQrBreakdownX, I->status,
                                 dlr::kStatusNoCompletion);
    }
    // 6-7. projections on the new basis (rg columns; the old basis X has r) and the L-step for every
    // ordinate
    dlr::launch_project(s, I->nx, I->ny, rg, I->Xn, I->X, I->sigma, I->sig_s, I->q, I->partials, I->nb_proj,
                        I->prec == DLR_FP32_SWEEP_BF16_PROJ ? 16 : (I->fp32() ? 32 : 64), r);
    dlr::launch_project_finalize(s, rg, I->partials, I->nb_proj, I->hx, I->hy, 1.0 / cdt, I->S, I->ops, r,
                                 I->augment ? nullptr : I->Rxi);
    dlr::LstepArgs la{};
    la.nq = nq; la.r = rg; la.mu = I->mu; la.eta = I->eta; la.w = I->w; la.ops = I->ops; la.W0 = I->W;
    la.inv_cdt = 1.0 / cdt;
    for (int k = 0; k < 4; ++k) la.psib[k] = I->psib[k];
    la.Binv = I->Binv; la.y = I->yv; la.red_partials = I->red; la.red_blocks = I->red_blocks; la.v = I->vv;
    la.L = I->L; la.status = I->status;
    dlr::launch_lstep(s, la);
    // 8. L = W S^T in the quadrature inner product: Cholesky QR twice, R = R2 R1; the CGS2 with
    // angular completion recomputes W and R on the device when a pivot flagged near-dependent columns
    dlr::launch_gram<double>(s, nq, rg, I->L, (size_t)nq, I->w, 1.0, I->partials, I->nb_gram_ang, I->Gm);
    dlr::launch_chol(s, rg, I->Gm, I->R1, I->R1i, I->status, dlr::kStatusQrBreakdownW);
    dlr::launch_trmm<double>(s, nq, rg, I->L, (size_t)nq, I->R1i, I->Wt);
    dlr::launch_gram<double>(s, nq, rg, I->Wt, (size_t)nq, I->w, 1.0, I->partials, I->nb_gram_ang, I->Gm);
    dlr::launch_chol(s, rg, I->Gm, I->R2, I->R2i, I->status, dlr::kStatusQrBreakdownW);
    dlr::launch_trmm<double>(s, nq, rg, I->Wt, (size_t)nq, I->R2i, I->Wq);
    dlr::launch_small_matmul(s, rg, I->R2, I->R1, I->Ra);
    dlr::launch_cgs2<double>(s, nq, rg, I->L, (size_t)nq, I->w, 0.0, 1, I->nx, I->ny, I->mu, I->eta, I->Wq, I->Ra,
                             I->status, dlr::kStatusQrBreakdownW, I->status, dlr::kStatusNoCompletion);
}

// The rest of steps 8 and 9: SVD (and the truncation of the augmented basis), new W and S, the
// temperature update; the new state.
template <typename TS>
void phase_end_b(dlr_instance* I) {
    hipStream_t s = I->stream;
    const int N = I->N, r = I->r, nq = I->nq, rg = I->ra;
    if (I->augment) {
        // 8 (end, augmented basis). SVD of the 2r x 2r S = Ra^T and truncation to its r largest singular
        // values: with (U Sigma)_r = Q R, the new state is X = Xn Q, S = R, W = Wq V_r.  The temperature
        // update then takes the mean intensity and outflow of the truncated state.
        dlr::launch_svd(s, rg, I->Ra, I->Vsvd, I->Sn, I->status);
        dlr::launch_trunc(s, rg, r, I->Sn, I->R1, I->S);
        dlr::launch_gemm_tall(s, N, rg, r, I->Xn, I->R1, r, I->X);
        dlr::launch_rmul_rect(s, nq, rg, r, I->Wq, I->Vsvd, rg, I->W);
        dlr::launch_wsum(s, nq, r, I->W, I->w, I->S, I->beta, I->coef, I->mu, I->eta, I->gside, false);
        dlr::launch_tupdate(s, tupdate_args(I, I->X, I->gside), I->nb_cells);
        if (!I->capturing) hip_check(hipEventRecord(I->ev[1], s), "event");
        return;
    }
    // 9. temperature update with the mean intensity of the new factors, energy sum and outflow.  The
    // mean intensity of the new state is X S W^T w with X = Xn Rxi and S W^T = L^T (the L-step's
    // result; the angular QR and the SVD only factor it), so the coefficients are Rxi L^T w and the
    // outflow side vectors Rxi L^T f_side: the temperature update needs nothing the SVD writes and
    // runs beside it on the second stream.  (Started right after the L-step instead, it took the CUs
    // that the angular QR's small kernels wait for.)
    hipStream_t ts = s;
    if (I->side) {
        hip_check(hipEventRecord(I->ev_fork, s), "event");
        hip_check(hipStreamWaitEvent(I->side, I->ev_fork, 0), "wait");
        ts = I->side;
    }
    dlr::launch_wsum(ts, nq, r, I->L, I->w, nullptr, I->beta, I->coef, I->mu, I->eta, I->gside, false, I->Rxi);
    dlr::launch_tupdate(ts, tupdate_args(I, I->Xn, I->gside), I->nb_cells);
    if (I->side) hip_check(hipEventRecord(I->ev_join, I->side), "event");
    // 8 (end). SVD of S: W <- Wq V, S <- S V (columns U_k sigma_k), stored as Rxi S V for Xn
    dlr::launch_svd(s, r, I->Ra, I->Vsvd, I->Sn, I->status, I->Rxi);
    dlr::launch_rmul(s, nq, r, I->Wq, I->Vsvd, I->W);
    if (I->side) hip_check(hipStreamWaitEvent(s, I->ev_join, 0), "wait");
    std::swap(I->X, I->Xn);
    std::swap(I->S, I->Sn);
    if (!I->capturing) hip_check(hipEventRecord(I->ev[1], s), "event");
}

template <typename TS>
void phase_end(dlr_instance* I) {
    phase_end_a<TS>(I);
    phase_end_b<TS>(I);
}

// energy, DEIM margins and weights into pinned memory behind the step; the status check's
// stream synchronisation completes them (one host round trip per step)
void step_publish(dlr_instance* I, unsigned seq = 0) {
    publish(I, I->stream, kPinnedNorm, I->energy_out, 2, I->margins, I->r, I->cw, I->r, 4, seq);
}

// After the stream has passed step_publish.
dlr_status step_read(dlr_instance* I, bool timed_sweeps, unsigned seq = 0) {
    const int r = I->r;
    double* hf = I->h_norm + kPinnedNorm;
    const dlr_status st = check_device_status(I, true, seq);
    if (st != DLR_OK) return st;
    const double en = hf[0];
    I->stats.outflow = hf[1];
    I->stats.inflow = I->inflow_power;
    I->stats.source = I->source_power;
    const std::vector<double> marg(hf + 2, hf + 2 + r), cwv(hf + 2 + r, hf + 2 + 2 * r);
    float step_ms = 0.f;   // graph-recorded steps are not timed per instance
    if (!I->device_si && !I->untimed) {
        if (seq) hip_check(hipEventSynchronize(I->ev[1]), "sync");   // ahead of the publish: done already
        hip_check(hipEventElapsedTime(&step_ms, I->ev[0], I->ev[1]), "elapsed");
    }
    I->stats.si_iters = I->si_it;
    I->stats.energy = en;
    I->stats.deim_min_margin = *std::min_element(marg.begin(), marg.end());
    double sa_ = 0.0;
    for (double v : cwv) sa_ += std::fabs(v);
    I->stats.sum_abs_cw_over_4pi = sa_ / dlr::kFourPi;
    I->stats.sweep_ms = timed_sweeps ? I->sweep_ms_acc : 0.f;
    I->stats.si_ms = timed_sweeps ? I->si_ms_acc : 0.f;
    I->stats.svd_sweeps = I->h_status[2];   // written by the SVD kernel of this step
    I->stats.step_ms = step_ms;
    I->s_is_usigma = true;
    I->have_sel = true;
    ++I->steps_done;
    I->stats.steps_done = I->steps_done;
    return DLR_OK;
}


// Source iterations decided on the device, K of them queued at once.  The scalar-flux pass of each
// raises the control flag when the iteration has converged, gone non-finite or reached its limit, and
// the sweeps, flux passes and DSA corrections queued behind it then return at once; the host waits
// once, reads the flag, and goes on by its own decisions if K iterations were not enough.  The device
// takes the host loop's decisions (the same test on the same residual), so the results are those of
// the host loop.  Each iteration is timed as in the host loop; the ones that did not run are left out.
// With `ahead`, the first part of the step's end (phase_end_a, which writes only scratch) is queued
// behind them before the host looks, so the GPU is not idle while it does; if the iteration turns out
// not to have converged, that part is queued again later and the status bits it may have raised on
// the unconverged data are cleared (the status word read before it was clean).
template <typename TS>
dlr_status si_queue(dlr_instance* I, int K, bool ahead) {
    hipStream_t s = I->stream;
    if (I->sw_prefetch == 0) sweep_tune<TS>(I);
    I->device_si = true;
    // events: iteration k's sweep runs from ev_si[st[k]] to ev_si[sw[k]], the iteration to ev_si[en[k]];
    // without DSA the end of one iteration is the start of the next (one event fewer per iteration:
    // each event costs a few microseconds of idle GPU between the kernels around it)
    int st[kSiSpec], sw[kSiSpec], en[kSiSpec];
    int ne = 0;
    st[0] = ne;
    hip_check(hipEventRecord(I->ev_si[ne++], s), "event");
    for (int k = 0; k < K; ++k) {
        sweep_launch<TS>(I, I->sw_prefetch, I->sw_grid);
        sw[k] = ne;
        hip_check(hipEventRecord(I->ev_si[ne++], s), "event");
        si_phi<TS>(I);   // swaps the host's names of the two flux buffers
        en[k] = ne;
        hip_check(hipEventRecord(I->ev_si[ne++], s), "event");
        if (k + 1 < K) {
            if (I->dsa) {
                dsa_correct(I);
                st[k + 1] = ne;
                hip_check(hipEventRecord(I->ev_si[ne++], s), "event");
            } else {
                st[k + 1] = en[k];
            }
        }
    }
    I->device_si = false;
    // the last flux pass's norms, the status word and the control words into pinned memory
    dlr::PublishArgs pa{};
    pa.src[0] = I->norm_out; pa.n[0] = 3;
    pa.dst = I->d_h_norm;
    pa.status = I->status; pa.nstatus = 1; pa.dst_status = I->d_h_status;
    pa.isrc = I->si_flag; pa.ni = 3; pa.idst = I->d_h_status + 4;
    const unsigned seq = next_publish(I);
    pa.seq_dst = reinterpret_cast<unsigned*>(I->d_h_status + 7);
    pa.seq = seq;
    dlr::launch_publish(s, pa);
    if (ahead) phase_end_a<TS>(I);
    wait_published(I, seq);
    hip_check(hipEventSynchronize(I->ev_si[en[K - 1]]), "sync");   // ahead of the publish: done already
    const int* f = I->h_status + 4;   // stopped, iterations run, why (1 converged, 2 non-finite, 3 limit)
    const int ran = f[1];
    if (ran < 1 || ran > K) {
        I->poisoned = true;
        I->poison_code = DLR_ERR_HIP;
        return fail(DLR_ERR_HIP, "source-iteration control words out of range");
    }
    for (int k = 0; k < ran; ++k) {
        float ms = 0.f, si_ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, I->ev_si[st[k]], I->ev_si[sw[k]]), "elapsed");
        hip_check(hipEventElapsedTime(&si_ms, I->ev_si[st[k]], I->ev_si[en[k]]), "elapsed");
        I->sweep_ms_acc += ms;
        I->si_ms_acc += si_ms;
    }
    if ((K - ran) & 1) std::swap(I->phi_cur, I->phi_nxt);   // the newest flux after `ran` iterations
    I->si_it = ran;
    if (*I->h_status != 0) return check_device_status(I);
    const double rel = I->h_norm[2];
    I->stats.si_residual = rel;
    const bool rename = I->phi_cur != I->phi && !I->untimed;
    if (f[2] == 2 || (f[0] == 0 && !std::isfinite(rel))) {
        I->poisoned = true;
        I->poison_code = DLR_ERR_NONFINITE;
        return fail(DLR_ERR_NONFINITE, "non-finite scalar flux in source iteration");
    }
    if (f[2] == 1) {
        I->si_conv = true;
        if (rename) std::swap(I->phi, I->phi2);
        return DLR_OK;
    }
    if (f[2] == 3) {
        if (rename) std::swap(I->phi, I->phi2);
        I->poisoned = true;
        I->poison_code = DLR_ERR_NOT_CONVERGED;
        return fail(DLR_ERR_NOT_CONVERGED, "source iteration reached si_max_iter");
    }
    if (ahead) hip_check(hipMemsetAsync(I->status, 0, sizeof(int), s), "status reset");
    if (I->dsa) dsa_correct(I);   // the correction after the last queued iteration (host loop from here)
    return DLR_OK;
}

template <typename TS>
dlr_status step_once(dlr_instance* I) {
    phase_begin<TS>(I);
    // as many source iterations at once as the last step needed (one host wait instead of one each)
    const int K = std::min(std::min(I->si_last, kSiSpec), I->si_max_iter);
    bool ended_a = false;   // phase_end_a is queued behind the converged iteration
    if (K >= 2) {
        const dlr_status st = si_queue<TS>(I, K, true);
        if (st != DLR_OK) return st;
        ended_a = I->si_conv;
    }
    while (!I->si_conv) {
        sweep_alone<TS>(I);
        si_phi<TS>(I);
        hip_check(hipEventRecord(I->ev[4], I->stream), "event");
        hip_check(hipStreamSynchronize(I->stream), "sync");
        float ms = 0.f, si_ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, I->ev[2], I->ev[3]), "elapsed");
        hip_check(hipEventElapsedTime(&si_ms, I->ev[2], I->ev[4]), "elapsed");
        I->sweep_ms_acc += ms;
        I->si_ms_acc += si_ms;
        const dlr_status st = si_check(I);
        if (st != DLR_OK) return st;
        if (!I->si_conv && I->dsa) dsa_correct(I);
    }
    // the DEIM status was checked with the last source iteration's status word (copied after it)
    if (!ended_a) phase_end_a<TS>(I);
    phase_end_b<TS>(I);
    const unsigned seq = next_publish(I);
    step_publish(I, seq);
    // The next step's start behind the statistics: this step's end event starts it, and its
    // linearisation (step 1 on the new temperature) and selection (step 2 on the new W and S, picks
    // into sel_alt: sel keeps this step's for read-back) run while the host reads them.  Loading new
    // factors and temperature or switching DSA on makes the next step do its part again, and a forced
    // selection its selection.
    launch_linearize(I, I->stream);
    I->lin_ready = true;
    launch_selection(I, I->stream, I->sel_alt);
    I->deim_ready = true;
    const dlr_status st = step_read(I, true, seq);
    I->si_last = I->si_it;
    return st;
}

// ---------------------------------------------------------------------------------------------------------
// Plain SN step (the comparator): backward Euler with the same linearisation; the fixed source of every
// ordinate is q + psi_prev / (c dt); source iteration on phi = sum_q w_q psi_q; T from the converged phi.
template <typename TS>
void sn_phi(dlr_instance* I, const double* phi_old, double* phi_new) {
    dlr::launch_sn_phi<TS>(I->stream, I->nx, I->ny, I->ldg, I->dirs, I->dir_off, I->w, static_cast<const TS*>(I->psi),
                           I->phio, I->sig_s, phi_old, phi_new, static_cast<TS*>(I->s_e), I->partials, I->nb_phi,
                           I->counters + 0, I->norm_out);
}

template <typename TS>
dlr_status sn_step_once(dlr_instance* I) {
    hipStream_t s = I->stream;
    hip_check(hipEventRecord(I->ev[0], s), "event");
    dlr::launch_linearize(s, I->nx, I->ny, I->sigma, I->rho_cv, I->q_ext, I->T, I->dt, I->a, I->c, I->D, I->sig_s,
                          I->q, I->sig_t, I->sig_t32, I->ldg, I->q_diag);
    dlr::launch_sn_source<TS>(s, I->nq, I->ldg, I->orient, I->q_diag, static_cast<const TS*>(I->psi),
                              1.0 / (I->c * I->dt), static_cast<TS*>(I->src0));
    sn_phi<TS>(I, I->phi2, I->phi);   // start: phi of the previous step's psi, and its s_e
    I->phi_cur = I->phi;
    I->phi_nxt = I->phi2;
    I->si_it = 0;
    I->si_conv = false;
    I->sweep_ms_acc = 0.f;
    I->si_ms_acc = 0.f;
    while (!I->si_conv) {
        sweep_alone<TS>(I);
        sn_phi<TS>(I, I->phi_cur, I->phi_nxt);
        hip_check(hipEventRecord(I->ev[4], s), "event");
        std::swap(I->phi_cur, I->phi_nxt);
        publish(I, s, 0, I->norm_out, 3, nullptr, 0, nullptr, 0, 1);
        hip_check(hipStreamSynchronize(s), "sync");
        float ms = 0.f, si_ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, I->ev[2], I->ev[3]), "elapsed");
        hip_check(hipEventElapsedTime(&si_ms, I->ev[2], I->ev[4]), "elapsed");
        I->sweep_ms_acc += ms;
        I->si_ms_acc += si_ms;
        const dlr_status st = si_check(I);
        if (st != DLR_OK) return st;
        if (!I->si_conv && I->dsa) dsa_correct(I);
    }
    dlr::launch_tupdate(s, tupdate_args(I, nullptr, nullptr), I->nb_cells);
    if (I->fp32())
        dlr::launch_sn_outflow<float>(s, I->nx, I->ny, I->nq, I->ldg, I->mu, I->eta, I->w,
                                      static_cast<const float*>(I->psi), I->hx, I->hy, I->partials, 1024,
                                      I->counters + 2, I->energy_out);
    else
        dlr::launch_sn_outflow<double>(s, I->nx, I->ny, I->nq, I->ldg, I->mu, I->eta, I->w,
                                       static_cast<const double*>(I->psi), I->hx, I->hy, I->partials, 1024,
                                       I->counters + 2, I->energy_out);
    hip_check(hipEventRecord(I->ev[1], s), "event");
    double* hf = I->h_norm + kPinnedNorm;
    publish(I, s, kPinnedNorm, I->energy_out, 2, nullptr, 0, nullptr, 0, 4);
    const dlr_status st = check_device_status(I, true);
    if (st != DLR_OK) return st;
    const double en = hf[0];
    I->stats.outflow = hf[1];
    I->stats.inflow = I->inflow_power;
    I->stats.source = I->source_power;
    float step_ms = 0.f;
    hip_check(hipEventElapsedTime(&step_ms, I->ev[0], I->ev[1]), "elapsed");
    I->stats.si_iters = I->si_it;
    I->stats.energy = en;
    I->stats.deim_min_margin = 0.0;
    I->stats.sum_abs_cw_over_4pi = 1.0;
    I->stats.sweep_ms = I->sweep_ms_acc;
    I->stats.si_ms = I->si_ms_acc;
    I->stats.step_ms = step_ms;
    ++I->steps_done;
    I->stats.steps_done = I->steps_done;
    return DLR_OK;
}

// row-major cells (e = j*nx + i, the C interface) <-> column-major cells (e = i*ny + j, device)
std::vector<double> to_cm(const double* src, int nx, int ny) {
    std::vector<double> out((size_t)nx * ny);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) out[(size_t)i * ny + j] = src[(size_t)j * nx + i];
    return out;
}
void to_rm(const double* src, double* dst, int nx, int ny) {
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) dst[(size_t)j * nx + i] = src[(size_t)i * ny + j];
}

void upload(void* dst, const void* src, size_t bytes) { hip_check(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), "upload"); }
void download(void* dst, const void* src, size_t bytes) {
    hip_check(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost), "download");
}

// Mean intensity of the current factors, for E_r before the first step / after a load: beta = W^T w,
// coef = S beta, phi = X coef, on the device.
// The stored basis is orthonormal as it stands (creation, load): Rx = Rxi = I.
void reset_basis_factor(dlr_instance* I) {
    const size_t R = (size_t)I->r;
    std::vector<double> id(R * R, 0.0);
    for (size_t k = 0; k < R; ++k) id[k * R + k] = 1.0;
    upload(I->Rx, id.data(), id.size() * sizeof(double));
    upload(I->Rxi, id.data(), id.size() * sizeof(double));
}

void refresh_phi(dlr_instance* I) {
    dlr::launch_wsum(I->stream, I->nq, I->r, I->W, I->w, I->S, I->beta, I->coef);
    dlr::launch_phi_of_factors(I->stream, I->N, I->r, I->X, I->coef, I->phi);
    hip_check(hipStreamSynchronize(I->stream), "sync");
}

// Problem fields, launch shapes and the quadrature of a new instance (no device work).
void init_fields(dlr_instance* I, const dlr_problem* p, hipStream_t stream, bool sn = false, bool augment = false) {
    I->sn = sn;
    I->augment = augment && !sn;
    I->nx = p->nx; I->ny = p->ny; I->N = p->nx * p->ny; I->npol = p->n_polar; I->naz = p->n_azim;
    I->nq = p->n_polar * p->n_azim; I->r = sn ? 0 : p->rank; I->prec = p->precision;
    I->ra = I->augment ? 2 * I->r : I->r;
    I->x0 = p->x0; I->x1 = p->x1; I->y0 = p->y0; I->y1 = p->y1;
    I->hx = (p->x1 - p->x0) / p->nx; I->hy = (p->y1 - p->y0) / p->ny; I->area = I->hx * I->hy;
    I->dt = p->dt; I->c = p->c; I->a = p->a;
    I->si_tol = p->si_tol; I->si_max_iter = p->si_max_iter; I->tie = p->deim_tie_tol;
    for (int k = 0; k < 4; ++k) {
        I->bc[k] = p->bc[k];
        I->Tb[k] = p->T_b[k];
        const double t = p->T_b[k];
        I->psib[k] = (p->bc[k] == DLR_BC_INFLOW) ? p->a * p->c * t * t * t * t / dlr::kFourPi : 0.0;
    }
    I->has_qext = p->q_ext != nullptr;
    I->stream = stream;
    const int sw = dlr::sweep_waves(I->prec == DLR_FP64);
    I->nsuper = (I->nx + 64 * sw - 1) / (64 * sw);
    I->ld = ((size_t)I->N + 63) / 64 * 64;   // compact column-major cell planes (e = i * ny + j)
    I->ldg = dlr::diag_plane(I->nx, I->ny);
    I->nb_phi = std::min(((I->nx + 7) / 8) * ((I->ny + 127) / 128), 1024);
    // Gram kernel: wavefronts take 32-cell passes; two blocks per CU keep all wavefronts resident at
    // once (a second, partly filled round of wavefronts cost a third of the time) and no block is
    // launched without a pass.  The projection kernel walks 64-cell chunks, two blocks per CU.
    const int chunks = (int)std::min<long>(((long)I->N + 63) / 64, 1 << 20);
    const long passes = ((long)I->N + 31) / 32;
    I->nb_gram = (int)std::max<long>(1, std::min<long>((passes + 3) / 4, 512));
    I->nb_gram_ang = std::max(1, std::min((((int)I->nq + 31) / 32 + 3) / 4, 32));
    I->nb_proj = std::max(1, std::min(chunks, 512));
    // temperature update: four blocks per CU keep enough of the r plane loads in flight (one block per
    // CU left the kernel latency-bound), on all CUs but one per XCD.  The kernel runs beside the
    // single-workgroup SVD, whose CU has room for only two of its blocks, and workgroups are dealt
    // round-robin over the eight XCDs: with four blocks on every CU (1024) two blocks of that XCD
    // waited for a whole block's time.  (256 CUs in 8 XCDs.)
    I->nb_cells = (int)std::max<long>(1, std::min<long>(((long)I->N + 255) / 256, 4 * (256 - 8)));
    const size_t rr = (size_t)I->ra * I->ra;
    I->partials_count = std::max({(size_t)I->nb_gram * rr, (size_t)I->nb_gram_ang * rr,
                                  (size_t)I->nb_proj * (5 * rr + 5 * I->ra),
                                  (size_t)I->nb_cells * 2, (size_t)I->nb_phi * 2, (size_t)(sn ? 1024 : 0)});
    dlr::build_quadrature(I->npol, I->naz, I->h_mu, I->h_eta, I->h_w);
    // constant terms of the energy balance: the inflow power (each inflow face takes
    // w_q |Omega_q . n| B(T_b) for every entering ordinate, times its length) and the source power
    I->inflow_power = 0.0;
    for (size_t q = 0; q < I->h_mu.size(); ++q) {
        const double m = I->h_mu[q], e = I->h_eta[q], wq = I->h_w[q];
        const int sx = m > 0.0 ? 0 : 1, sy = e > 0.0 ? 2 : 3;   // side the ordinate enters through
        I->inflow_power += wq * std::fabs(m) * I->psib[sx] * (I->ny * I->hy);
        I->inflow_power += wq * std::fabs(e) * I->psib[sy] * (I->nx * I->hx);
    }
    I->source_power = 0.0;
    if (p->q_ext)
        for (long e = 0; e < (long)I->N; ++e) I->source_power += p->q_ext[e];
    I->source_power *= I->area;
}

// Device bytes of an instance's arena.
size_t arena_bytes(dlr_instance* I) {
    Arena sizing;
    I->carve(sizing);
    return sizing.used;
}

// The instance's arena (hipMalloc or the allocator hook), carved and cleared on its stream.
dlr_status allocate_instance(dlr_instance* I) {
    const size_t need = arena_bytes(I);
    if (!hook_installed()) {
        size_t free_b = 0, total_b = 0;
        hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
        if (need + (64u << 20) > free_b) return fail(DLR_ERR_OOM, "instance does not fit in free device memory");
    }
    if (!I->arena.allocate(need, I->stream)) return fail(DLR_ERR_OOM, "device allocation of the instance failed");
    I->carve(I->arena);
    hip_check(hipMemsetAsync(I->arena.base, 0, I->arena.cap, I->stream), "clear");
    if (I->deim_ctr) {
        const unsigned base = 1u << 31;
        hip_check(hipMemcpyAsync(I->deim_ctr, &base, sizeof(base), hipMemcpyHostToDevice, I->stream), "counter");
    }
    hip_check(hipStreamSynchronize(I->stream), "sync");
    return DLR_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------------------------
// Batches
struct BatchSlot {
    int64_t id = 0;
    dlr_instance* I = nullptr;
    size_t bytes = 0;
    int remaining = 0;
    bool finished = false;
    dlr_status fail_status = DLR_OK;
    std::string fail_msg;
    hipEvent_t ev = nullptr;   // slot stream -> shared sweep stream
};

struct dlr_batch_s {
    size_t budget = 0, used = 0;
    hipStream_t main = nullptr;
    std::vector<hipStream_t> pool;   // per-slot streams (slot id modulo the pool)
    std::map<int64_t, BatchSlot> slots;
    std::deque<int64_t> done;
    int64_t next_id = 1;
    // shared sweep launches: one table region per precision
    size_t cap = 0;                  // table entries per region
    char* d_table[2] = {nullptr, nullptr};
    unsigned* d_unit_end[2] = {nullptr, nullptr};
    char* h_table[2] = {nullptr, nullptr};
    unsigned* h_unit_end[2] = {nullptr, nullptr};
    unsigned* d_ticket = nullptr;
    DevMem table_mem[2], unit_end_mem[2], ticket_mem;   // device memory behind the three above
    hipEvent_t ev_main = nullptr;
    // Graph-recorded steps (a composition of slots that stays the same from one advance to the next):
    // the steps of both parities of the ping-pong buffers are recorded once, with K source
    // iterations decided on the device, and replayed until the composition changes.
    bool graphs = true;                              // allowed (dlr_batch_set_graphs)
    int max_rec = 8;                                 // most source iterations recorded per step
    hipStream_t rec = nullptr;                       // recording / replay stream
    std::vector<hipStream_t> rec_streams;            // one per slot while recording: independent chains
    hipEvent_t ev_cap = nullptr;
    DevMem gtable_mem[2], gunit_mem[2], gctr_mem, gptr_mem;
    unsigned long long* d_sweep_ctr = nullptr;      // sweep launch counter of the recorded launches
    size_t gcap = 0;                                 // entries of the recorded tables and gather arrays
    int* h_gi = nullptr;                             // pinned [4 * gcap]: flags, status per slot
    double* h_gd = nullptr;                          // pinned [gcap]: last relative change per slot
    int* d_h_gi = nullptr;
    double* d_h_gd = nullptr;
    hipGraphExec_t gx_begin[2] = {nullptr, nullptr}, gx_end[2] = {nullptr, nullptr};
    std::vector<int64_t> gkey, last_key;             // recorded composition; the previous advance's
    int gK = 0, k_hint = 2, parity = 0;
    int64_t graph_steps = 0;                         // steps advanced through the recorded graphs
};

namespace {

constexpr int kBatchStreams = 8;
constexpr size_t kRecBytes = sizeof(dlr::SweepArgs<double>);
static_assert(sizeof(dlr::SweepArgs<float>) == sizeof(dlr::SweepArgs<double>), "one record size");

void batch_reserve(dlr_batch_s* B, size_t entries) {
    if (entries <= B->cap) return;
    size_t cap = std::max<size_t>(64, B->cap);
    while (cap < entries) cap *= 2;
    hip_check(hipStreamSynchronize(B->main), "sync");   // earlier launches may still read the tables
    for (int g = 0; g < 2; ++g) {
        dev_free(B->table_mem[g]);
        dev_free(B->unit_end_mem[g]);
        B->d_table[g] = nullptr;
        B->d_unit_end[g] = nullptr;
        if (B->h_table[g]) (void)hipHostFree(B->h_table[g]);
        if (B->h_unit_end[g]) (void)hipHostFree(B->h_unit_end[g]);
        B->h_table[g] = nullptr;
        B->h_unit_end[g] = nullptr;
        if (!dev_alloc(B->table_mem[g], cap * kRecBytes, B->main) ||
            !dev_alloc(B->unit_end_mem[g], cap * sizeof(unsigned), B->main))
            throw HipError("batch table: device allocation failed");
        B->d_table[g] = static_cast<char*>(B->table_mem[g].ptr);
        B->d_unit_end[g] = static_cast<unsigned*>(B->unit_end_mem[g].ptr);
        hip_check(hipHostMalloc((void**)&B->h_table[g], cap * kRecBytes, hipHostMallocDefault), "batch table");
        hip_check(hipHostMalloc((void**)&B->h_unit_end[g], cap * sizeof(unsigned), hipHostMallocDefault),
                  "batch table");
    }
    B->cap = cap;
}

// One persistent sweep launch over the pending slots of one precision (g = 0 FP64, 1 FP32).
template <typename TS>
void batch_sweep(dlr_batch_s* B, const std::vector<BatchSlot*>& pending) {
    const int g = sizeof(TS) == 4 ? 1 : 0;
    size_t n = 0;
    unsigned acc = 0;
    for (BatchSlot* sl : pending) {
        if (sl->I->fp32() != (g == 1)) continue;
        std::memcpy(B->h_table[g] + n * kRecBytes, sl->I->h_sweep_rec.data(), kRecBytes);
        acc += (unsigned)(sl->I->nsuper * sl->I->r);
        B->h_unit_end[g][n] = acc;
        ++n;
    }
    if (n == 0) return;
    hip_check(hipMemcpyAsync(B->d_table[g], B->h_table[g], n * kRecBytes, hipMemcpyHostToDevice, B->main), "table");
    hip_check(hipMemcpyAsync(B->d_unit_end[g], B->h_unit_end[g], n * sizeof(unsigned), hipMemcpyHostToDevice, B->main),
              "table");
    dlr::SweepLaunch L{};
    L.ninst = (int)n;
    L.total_units = acc;
    L.unit_end = B->d_unit_end[g];
    L.ticket = B->d_ticket;
    L.launch_id = dlr::next_sweep_launch_id();
    L.grid_blocks = (int)std::min<unsigned>(acc, 1024u);
    dlr::launch_sweep<TS>(B->main, reinterpret_cast<const dlr::SweepArgs<TS>*>(B->d_table[g]), L);
}

void slot_fail(dlr_batch_s* B, BatchSlot* sl, dlr_status st) {
    sl->finished = true;
    sl->fail_status = st;
    sl->fail_msg = g_last_error;
    B->done.push_back(sl->id);
}

BatchSlot* find_slot(dlr_batch_s* B, int64_t id) {
    auto it = B->slots.find(id);
    return it == B->slots.end() ? nullptr : &it->second;
}

// ---------------------------------------------------------------------------------------------- recorded steps
void graph_clear(dlr_batch_s* B) {
    for (int p = 0; p < 2; ++p) {
        if (B->gx_begin[p]) (void)hipGraphExecDestroy(B->gx_begin[p]);
        if (B->gx_end[p]) (void)hipGraphExecDestroy(B->gx_end[p]);
        B->gx_begin[p] = B->gx_end[p] = nullptr;
    }
    B->gkey.clear();
    B->gK = 0;
    B->parity = 0;
}

// Tables of the recorded sweep launches and the gather arrays, for n slots.
void graph_reserve(dlr_batch_s* B, size_t n) {
    if (n <= B->gcap) return;
    size_t cap = std::max<size_t>(64, B->gcap);
    while (cap < n) cap *= 2;
    hip_check(hipStreamSynchronize(B->rec), "sync");
    for (int g = 0; g < 2; ++g) {
        dev_free(B->gtable_mem[g]);
        dev_free(B->gunit_mem[g]);
        if (!dev_alloc(B->gtable_mem[g], cap * kRecBytes, B->rec) ||
            !dev_alloc(B->gunit_mem[g], cap * sizeof(unsigned), B->rec))
            throw HipError("recorded sweep tables: device allocation failed");
    }
    dev_free(B->gptr_mem);
    if (!dev_alloc(B->gptr_mem, 3 * cap * sizeof(void*), B->rec)) throw HipError("gather table: device allocation failed");
    if (B->h_gi) (void)hipHostFree(B->h_gi);
    if (B->h_gd) (void)hipHostFree(B->h_gd);
    B->h_gi = nullptr;
    B->h_gd = nullptr;
    hip_check(hipHostMalloc((void**)&B->h_gi, 4 * cap * sizeof(int), hipHostMallocDefault), "pinned");
    hip_check(hipHostMalloc((void**)&B->h_gd, cap * sizeof(double), hipHostMallocDefault), "pinned");
    hip_check(hipHostGetDevicePointer((void**)&B->d_h_gi, B->h_gi, 0), "pinned mapping");
    hip_check(hipHostGetDevicePointer((void**)&B->d_h_gd, B->h_gd, 0), "pinned mapping");
    B->gcap = cap;
}

template <typename TS>
void graph_sweep(dlr_batch_s* B, int n, unsigned units) {
    if (n == 0) return;
    const int g = sizeof(TS) == 4 ? 1 : 0;
    dlr::SweepLaunch L{};
    L.ninst = n;
    L.total_units = units;
    L.unit_end = static_cast<const unsigned*>(B->gunit_mem[g].ptr);
    L.ticket = B->d_ticket;
    L.launch_id = 0;
    L.id_ctr = B->d_sweep_ctr;   // every replay tags its progress words apart
    L.grid_blocks = (int)std::min<unsigned>(units, 1024u);
    dlr::launch_sweep<TS>(B->rec, static_cast<const dlr::SweepArgs<TS>*>(B->gtable_mem[g].ptr), L);
}

// Record the step of the slots `act` for both parities of their ping-pong buffers: the beginning
// (Algorithm 1 steps 1-3) with K source iterations (step 4) decided on the device, then the end
// (steps 5-9) with the values the host reads.  Slots of one pool stream keep their order; the
// shared sweep launches join every slot.  Kernel launches only: no memory operation is recorded.
void graph_record(dlr_batch_s* B, const std::vector<BatchSlot*>& act, const std::vector<int64_t>& key, int K) {
    graph_clear(B);
    graph_reserve(B, act.size());
    const size_t n = act.size();
    std::vector<char> tab[2];
    std::vector<unsigned> ue[2];
    unsigned units[2] = {0u, 0u};
    std::vector<const void*> ptrs(3 * n);
    // Each slot records on a stream of its own, so that the graph holds one independent chain per
    // slot (the pool streams would chain the slots that share one).
    while (B->rec_streams.size() < n) {
        hipStream_t st = nullptr;
        hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "stream");
        B->rec_streams.push_back(st);
    }
    std::vector<hipStream_t> used, home(n);
    for (size_t k = 0; k < n; ++k) {
        home[k] = act[k]->I->stream;
        act[k]->I->stream = B->rec_streams[k];
    }
    for (size_t k = 0; k < n; ++k) {
        dlr_instance* I = act[k]->I;
        const int g = I->fp32() ? 1 : 0;
        tab[g].insert(tab[g].end(), I->h_sweep_rec.begin(), I->h_sweep_rec.end());
        units[g] += (unsigned)(I->nsuper * I->r);
        ue[g].push_back(units[g]);
        ptrs[k] = I->si_flag;
        ptrs[n + k] = I->status;
        ptrs[2 * n + k] = I->norm_out + 2;
        if (std::find(used.begin(), used.end(), I->stream) == used.end()) used.push_back(I->stream);
    }
    for (int g = 0; g < 2; ++g)
        if (!ue[g].empty()) {
            hip_check(hipMemcpy(B->gtable_mem[g].ptr, tab[g].data(), tab[g].size(), hipMemcpyHostToDevice), "table");
            hip_check(hipMemcpy(B->gunit_mem[g].ptr, ue[g].data(), ue[g].size() * sizeof(unsigned),
                                hipMemcpyHostToDevice), "table");
        }
    hip_check(hipMemcpy(B->gptr_mem.ptr, ptrs.data(), ptrs.size() * sizeof(void*), hipMemcpyHostToDevice), "table");
    const int* const* dflags = static_cast<const int* const*>(B->gptr_mem.ptr);
    const int* const* dstat = dflags + n;
    const double* const* drel = reinterpret_cast<const double* const*>(dflags + 2 * n);
    const int nd = (int)ue[0].size(), nf = (int)ue[1].size();
    auto fork = [&]() {
        hip_check(hipStreamBeginCapture(B->rec, hipStreamCaptureModeRelaxed), "begin capture");
        hip_check(hipEventRecord(B->ev_cap, B->rec), "event");
        for (hipStream_t st : used) hip_check(hipStreamWaitEvent(st, B->ev_cap, 0), "wait");
    };
    auto join = [&](hipGraphExec_t* out) {
        for (BatchSlot* sl : act) hip_check(hipStreamWaitEvent(B->rec, sl->ev, 0), "wait");
        hipGraph_t gr = nullptr;
        hip_check(hipStreamEndCapture(B->rec, &gr), "end capture");
        const hipError_t e = hipGraphInstantiate(out, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        hip_check(e, "instantiate");
    };
    for (BatchSlot* sl : act) sl->I->capturing = true;
    try {
        for (int p = 0; p < 2; ++p) {
            fork();
            for (BatchSlot* sl : act) {
                sl->I->device_si = true;
                if (sl->I->fp32()) phase_begin<float>(sl->I); else phase_begin<double>(sl->I);
                hip_check(hipEventRecord(sl->ev, sl->I->stream), "event");
            }
            for (int it = 0; it < K; ++it) {
                for (BatchSlot* sl : act) hip_check(hipStreamWaitEvent(B->rec, sl->ev, 0), "wait");
                graph_sweep<double>(B, nd, units[0]);
                graph_sweep<float>(B, nf, units[1]);
                hip_check(hipEventRecord(B->ev_main, B->rec), "event");
                for (BatchSlot* sl : act) {
                    dlr_instance* I = sl->I;
                    hip_check(hipStreamWaitEvent(I->stream, B->ev_main, 0), "wait");
                    if (I->fp32()) si_phi<float>(I); else si_phi<double>(I);
                    if (I->dsa) dsa_correct(I);
                    hip_check(hipEventRecord(sl->ev, I->stream), "event");
                }
            }
            for (BatchSlot* sl : act) hip_check(hipStreamWaitEvent(B->rec, sl->ev, 0), "wait");
            dlr::launch_gather_si(B->rec, (int)n, dflags, dstat, drel, B->d_h_gi, B->d_h_gd);
            join(&B->gx_begin[p]);
            // the end of the step; phase_end swaps the host's X/Xn and S/Sn, so the next pass records
            // the other parity and the second pass restores the present one
            fork();
            for (BatchSlot* sl : act) {
                if (sl->I->fp32()) phase_end<float>(sl->I); else phase_end<double>(sl->I);
                step_publish(sl->I);
                hip_check(hipEventRecord(sl->ev, sl->I->stream), "event");
            }
            join(&B->gx_end[p]);
        }
    } catch (...) {
        for (size_t k = 0; k < n; ++k) act[k]->I->stream = home[k];
        hipGraph_t junk = nullptr;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(B->rec, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
            (void)hipStreamEndCapture(B->rec, &junk);
        if (junk) (void)hipGraphDestroy(junk);
        for (BatchSlot* sl : act) {
            sl->I->capturing = false;
            sl->I->device_si = false;
        }
        graph_clear(B);
        throw;
    }
    for (size_t k = 0; k < n; ++k) act[k]->I->stream = home[k];
    for (BatchSlot* sl : act) {
        sl->I->capturing = false;
        sl->I->device_si = false;
    }
    B->gkey = key;
    B->gK = K;
    B->parity = 0;
}

}  // namespace

extern "C" {

dlr_status dlr_set_allocator(void* (*alloc)(size_t, void*, void*), void (*release)(void*, void*, void*), void* user) {
    if ((alloc == nullptr) != (release == nullptr))
        return fail(DLR_ERR_ARG, "alloc and release must both be set or both be NULL");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_hook.alloc = alloc;
    g_hook.release = release;
    g_hook.user = alloc ? user : nullptr;
    return DLR_OK;
}

const char* dlr_status_string(dlr_status s) {
    switch (s) {
        case DLR_OK: return "ok";
        case DLR_ERR_ARG: return "invalid argument";
        case DLR_ERR_OOM: return "out of device memory";
        case DLR_ERR_HIP: return "HIP runtime error";
        case DLR_ERR_NOT_CONVERGED: return "source iteration did not converge";
        case DLR_ERR_NONFINITE: return "non-finite values";
        case DLR_ERR_STATE: return "handle poisoned by an earlier error";
        case DLR_ERR_UNSUPPORTED: return "unsupported option";
        case DLR_ERR_NUMERIC: return "numerical breakdown";
        case DLR_ERR_TIMEOUT: return "device wait exceeded its spin limit";
    }
    return "unknown status";
}

const char* dlr_last_error(void) { return g_last_error.c_str(); }

namespace {

dlr_status create_dlr(const dlr_problem* p, void* hip_stream, dlr_handle* out, bool augment) {
    if (!out) return fail(DLR_ERR_ARG, "out is NULL");
    *out = nullptr;
    g_last_error.clear();
    const dlr_status v = validate(p);
    if (v != DLR_OK) return v;
    if (augment && (2LL * p->rank > dlr::kMaxRank || 2LL * p->rank > (long long)p->n_polar * p->n_azim ||
                    2LL * p->rank > (long long)p->nx * p->ny))
        return fail(DLR_ERR_ARG, "the augmented basis needs 2 rank <= min(64, ordinates, cells)");
    dlr_instance* I = new (std::nothrow) dlr_instance();
    if (!I) return fail(DLR_ERR_OOM, "host allocation failed");
    try {
        init_fields(I, p, static_cast<hipStream_t>(hip_stream), false, augment);
        const dlr_status am = allocate_instance(I);
        if (am != DLR_OK) {
            delete I;
            return am;
        }
        upload_sweep_record(I);
        hip_check(hipHostMalloc((void**)&I->h_norm, kPinnedDoubles * sizeof(double), hipHostMallocDefault), "pinned");
        hip_check(hipHostMalloc((void**)&I->h_status, kPinnedInts * sizeof(int), hipHostMallocDefault), "pinned");
        hip_check(hipHostGetDevicePointer((void**)&I->d_h_norm, I->h_norm, 0), "pinned mapping");
        hip_check(hipHostGetDevicePointer((void**)&I->d_h_status, I->h_status, 0), "pinned mapping");
        std::memset(I->h_status, 0, kPinnedInts * sizeof(int));
        for (auto& ev : I->ev) hip_check(hipEventCreate(&ev), "event create");
        hip_check(hipStreamCreateWithFlags(&I->side, hipStreamNonBlocking), "side stream");
        hip_check(hipEventCreateWithFlags(&I->ev_fork, hipEventDisableTiming), "event create");
        hip_check(hipEventCreateWithFlags(&I->ev_join, hipEventDisableTiming), "event create");
        for (auto& ev : I->ev_si) hip_check(hipEventCreate(&ev), "event create");
        const size_t n = I->N;
        upload(I->mu, I->h_mu.data(), I->nq * sizeof(double));
        upload(I->eta, I->h_eta.data(), I->nq * sizeof(double));
        upload(I->w, I->h_w.data(), I->nq * sizeof(double));
        upload(I->sigma, to_cm(p->sigma_a, I->nx, I->ny).data(), n * sizeof(double));
        upload(I->rho_cv, to_cm(p->rho_cv, I->nx, I->ny).data(), n * sizeof(double));
        if (p->q_ext) upload(I->q_ext, to_cm(p->q_ext, I->nx, I->ny).data(), n * sizeof(double));
        upload(I->T, to_cm(p->T_init, I->nx, I->ny).data(), n * sizeof(double));
        dlr::ProblemHost ph{I->nx, I->ny, I->r, I->hx, I->hy, I->a, I->c, p->T_init};
        std::vector<double> X, S, W;
        dlr::build_initial_factors(ph, I->h_mu, I->h_eta, I->h_w, X, S, W);
        for (int k = 0; k < I->r; ++k) {
            const std::vector<double> col = to_cm(&X[(size_t)k * n], I->nx, I->ny);
            std::copy(col.begin(), col.end(), X.begin() + (size_t)k * n);
        }
        upload(I->X, X.data(), X.size() * sizeof(double));
        upload(I->S, S.data(), S.size() * sizeof(double));
        upload(I->W, W.data(), W.size() * sizeof(double));
        reset_basis_factor(I);
        if (augment) {
            // The augmented Galerkin space takes the whole span of the old basis, so the completion
            // of the rank-one initial state is part of the method here (the plain step meets those
            // columns only through zero entries of S): X = CGS2 of [B(T_init) | 0 ...] with the
            // graded spatial monomials filling the zero columns.  Unless a monomial is (nearly)
            // dependent, that CGS2 keeps B(T_init) and the next r - 1 monomials (skipping the
            // constant when B(T_init) is constant), and its Q is the unique QR factor of that matrix:
            // formed here by Cholesky QR twice on all of the cells at once.  When a pivot flags a
            // nearly dependent column, the one-workgroup CGS2 of [B(T_init) | 0 ...] decides instead.
            bool b0_const = true;
            for (long e = 1; e < (long)n && b0_const; ++e) b0_const = p->T_init[e] == p->T_init[0];
            const int r = I->r;
            hipStream_t st = I->stream;
            hip_check(hipMemcpyAsync(I->Xn, I->X, n * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
            dlr::launch_monomials(st, I->nx, I->ny, b0_const ? 1 : 0, r - 1, I->Xn + n, n);
            dlr::launch_gram<double>(st, (long)n, r, I->Xn, n, nullptr, I->area, I->partials, I->nb_gram, I->Gm);
            dlr::launch_chol(st, r, I->Gm, I->R1, I->R1i, I->status, dlr::kStatusQrBreakdownX);
            dlr::launch_trmm<double>(st, (int)n, r, I->Xn, n, I->R1i, I->X);
            dlr::launch_gram<double>(st, (long)n, r, I->X, n, nullptr, I->area, I->partials, I->nb_gram, I->Gm);
            dlr::launch_chol(st, r, I->Gm, I->R2, I->R2i, I->status, dlr::kStatusQrBreakdownX, I->status + 3, 1e-15);
            dlr::launch_trmm_inplace(st, (int)n, r, I->X, I->R2i, I->status + 3);
            // the exact rule, on the device only when a pivot above flagged the columns
            hip_check(hipMemsetAsync(I->Va, 0, (size_t)r * n * sizeof(double), st), "clear");
            hip_check(hipMemcpyAsync(I->Va, I->Xn, n * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
            dlr::launch_cgs2<double>(st, (long)n, r, I->Va, n, nullptr, I->area, 0, I->nx, I->ny, nullptr, nullptr,
                                     I->X, I->R1, I->status, dlr::kStatusQrBreakdownX, I->status,
                                     dlr::kStatusNoCompletion);
            int st0 = 0;
            hip_check(hipMemcpyAsync(&st0, I->status, sizeof(int), hipMemcpyDeviceToHost, I->stream), "status");
            hip_check(hipStreamSynchronize(I->stream), "sync");
            if (st0 != 0) {
                dlr_destroy(I);
                return fail(DLR_ERR_NUMERIC, "no spatial completion of the initial basis");
            }
        }
        refresh_phi(I);
        I->s_is_usigma = true;   // S = diag(s, 0, ...)
        hip_check(hipDeviceSynchronize(), "sync");
    } catch (const std::exception& ex) {
        dlr_destroy(I);
        return fail(DLR_ERR_HIP, ex.what());
    }
    *out = I;
    return DLR_OK;
}

}  // namespace

dlr_status dlr_create(const dlr_problem* p, void* hip_stream, dlr_handle* out) {
    return create_dlr(p, hip_stream, out, false);
}

dlr_status dlr_create_augmented(const dlr_problem* p, void* hip_stream, dlr_handle* out) {
    return create_dlr(p, hip_stream, out, true);
}

dlr_status dlr_sn_create(const dlr_problem* p, void* hip_stream, dlr_handle* out) {
    if (!out) return fail(DLR_ERR_ARG, "out is NULL");
    *out = nullptr;
    g_last_error.clear();
    const dlr_status v = validate(p, true);
    if (v != DLR_OK) return v;
    dlr_instance* I = new (std::nothrow) dlr_instance();
    if (!I) return fail(DLR_ERR_OOM, "host allocation failed");
    try {
        init_fields(I, p, static_cast<hipStream_t>(hip_stream), true);
        const dlr_status am = allocate_instance(I);
        if (am != DLR_OK) {
            delete I;
            return am;
        }
        upload_sweep_record(I);
        hip_check(hipHostMalloc((void**)&I->h_norm, kPinnedDoubles * sizeof(double), hipHostMallocDefault), "pinned");
        hip_check(hipHostMalloc((void**)&I->h_status, kPinnedInts * sizeof(int), hipHostMallocDefault), "pinned");
        hip_check(hipHostGetDevicePointer((void**)&I->d_h_norm, I->h_norm, 0), "pinned mapping");
        hip_check(hipHostGetDevicePointer((void**)&I->d_h_status, I->h_status, 0), "pinned mapping");
        for (auto& ev : I->ev) hip_check(hipEventCreate(&ev), "event create");
        const size_t n = I->N, Q = I->nq;
        // ordinates grouped by orientation, and their isotropic inflow values
        std::vector<int> orient(Q), dirs, off(8, 0);
        std::vector<double> inx(Q), iny(Q);
        for (size_t k = 0; k < Q; ++k) {
            orient[k] = dlr::orient_of(I->h_mu[k], I->h_eta[k]);
            inx[k] = I->psib[I->h_mu[k] > 0.0 ? 0 : 1];
            iny[k] = I->psib[I->h_eta[k] > 0.0 ? 2 : 3];
        }
        for (int o = 0; o < 4; ++o) {
            off[o] = (int)dirs.size();
            for (size_t k = 0; k < Q; ++k)
                if (orient[k] == o) dirs.push_back((int)k);
        }
        off[4] = (int)dirs.size();
        upload(I->mu, I->h_mu.data(), Q * sizeof(double));
        upload(I->eta, I->h_eta.data(), Q * sizeof(double));
        upload(I->w, I->h_w.data(), Q * sizeof(double));
        upload(I->orient, orient.data(), Q * sizeof(int));
        upload(I->dirs, dirs.data(), Q * sizeof(int));
        upload(I->dir_off, off.data(), 8 * sizeof(int));
        upload(I->inflow_x, inx.data(), Q * sizeof(double));
        upload(I->inflow_y, iny.data(), Q * sizeof(double));
        upload(I->sigma, to_cm(p->sigma_a, I->nx, I->ny).data(), n * sizeof(double));
        upload(I->rho_cv, to_cm(p->rho_cv, I->nx, I->ny).data(), n * sizeof(double));
        if (p->q_ext) upload(I->q_ext, to_cm(p->q_ext, I->nx, I->ny).data(), n * sizeof(double));
        upload(I->T, to_cm(p->T_init, I->nx, I->ny).data(), n * sizeof(double));
        // every ordinate starts at the isotropic equilibrium intensity B(T_init)
        if (I->fp32())
            dlr::launch_sn_init<float>(I->stream, I->nx, I->ny, I->nq, I->ldg, I->orient, I->T, I->a, I->c,
                                       static_cast<float*>(I->psi), I->phi);
        else
            dlr::launch_sn_init<double>(I->stream, I->nx, I->ny, I->nq, I->ldg, I->orient, I->T, I->a, I->c,
                                        static_cast<double*>(I->psi), I->phi);
        hip_check(hipStreamSynchronize(I->stream), "sync");
    } catch (const std::exception& ex) {
        dlr_destroy(I);
        return fail(DLR_ERR_HIP, ex.what());
    }
    *out = I;
    return DLR_OK;
}

dlr_status dlr_step(dlr_handle h, int32_t n_steps) {
    if (!h) return fail(DLR_ERR_ARG, "handle is NULL");
    if (n_steps < 0) return fail(DLR_ERR_ARG, "n_steps must be >= 0");
    if (h->poisoned) return fail(DLR_ERR_STATE, std::string("handle poisoned: ") + dlr_status_string(h->poison_code));
    try {
        for (int k = 0; k < n_steps; ++k) {
            const dlr_status st = h->sn ? (h->fp32() ? sn_step_once<float>(h) : sn_step_once<double>(h))
                                        : (h->fp32() ? step_once<float>(h) : step_once<double>(h));
            if (st != DLR_OK) return st;
        }
    } catch (const std::exception& ex) {
        h->poisoned = true;
        h->poison_code = DLR_ERR_HIP;
        return fail(DLR_ERR_HIP, ex.what());
    }
    return DLR_OK;
}

dlr_status dlr_sync(dlr_handle h) {
    if (!h) return fail(DLR_ERR_ARG, "handle is NULL");
    const hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(DLR_ERR_HIP, hipGetErrorString(e));
    return DLR_OK;
}

dlr_status dlr_read_fields(dlr_handle h, double* E_r, double* T) {
    if (!h) return fail(DLR_ERR_ARG, "handle is NULL");
    try {
        hip_check(hipStreamSynchronize(h->stream), "sync");
        std::vector<double> buf((size_t)h->N);
        if (E_r) {
            download(buf.data(), h->phi, (size_t)h->N * sizeof(double));
            to_rm(buf.data(), E_r, h->nx, h->ny);
            for (int e = 0; e < h->N; ++e) E_r[e] /= h->c;
        }
        if (T) {
            download(buf.data(), h->T, (size_t)h->N * sizeof(double));
            to_rm(buf.data(), T, h->nx, h->ny);
        }
    } catch (const std::exception& ex) {
        return fail(DLR_ERR_HIP, ex.what());
    }
    return DLR_OK;
}

dlr_status dlr_read_factors(dlr_handle h, double* Xo, double* So, double* Wo, int32_t* selo) {
    if (!h) return fail(DLR_ERR_ARG, "handle is NULL");
    if (h->sn) return fail(DLR_ERR_UNSUPPORTED, "a plain SN handle has no factors");
    try {
        hip_check(hipStreamSynchronize(h->stream), "sync");
        const size_t n = h->N, R = h->r, Q = h->nq;
        std::vector<double> X(R * n), Ss(R * R), W(R * Q), Rx(R * R), Rxi(R * R);
        download(X.data(), h->X, X.size() * sizeof(double));
        download(Ss.data(), h->S, Ss.size() * sizeof(double));
        download(W.data(), h->W, W.size() * sizeof(double));
        download(Rx.data(), h->Rx, Rx.size() * sizeof(double));
        download(Rxi.data(), h->Rxi, Rxi.size() * sizeof(double));
        // the stored pair is (X, Ss) with the orthonormal basis X Rxi: its coupling is S = Rx Ss
        std::vector<double> S(R * R, 0.0);
        for (size_t i = 0; i < R; ++i)
            for (size_t j = 0; j < R; ++j) {
                double acc = 0.0;
                for (size_t k = 0; k < R; ++k) acc += Rx[i * R + k] * Ss[k * R + j];
                S[i * R + j] = acc;
            }
        std::vector<double> U(R * R, 0.0), sig(R, 0.0);
        if (h->s_is_usigma) {
            // S holds U Sigma column-wise: sigma_k = ||S_k||, U_k = S_k / sigma_k; zero
            // columns are completed with unit vectors orthogonalised against the others.
            for (size_t k = 0; k < R; ++k) {
                double s2 = 0.0;
                for (size_t i = 0; i < R; ++i) s2 += S[i * R + k] * S[i * R + k];
                sig[k] = std::sqrt(s2);
                if (sig[k] > 0.0)
                    for (size_t i = 0; i < R; ++i) U[i * R + k] = S[i * R + k] / sig[k];
            }
            for (size_t k = 0; k < R; ++k) {
                if (sig[k] > 0.0) continue;
                for (size_t cand = 0; cand < R; ++cand) {
                    std::vector<double> v(R, 0.0);
                    v[cand] = 1.0;
                    for (int pass = 0; pass < 2; ++pass)
                        for (size_t j = 0; j < R; ++j) {
                            if (j == k || (sig[j] == 0.0 && j > k)) continue;
                            double d = 0.0;
                            for (size_t i = 0; i < R; ++i) d += U[i * R + j] * v[i];
                            for (size_t i = 0; i < R; ++i) v[i] -= d * U[i * R + j];
                        }
                    double nv = 0.0;
                    for (double x : v) nv += x * x;
                    nv = std::sqrt(nv);
                    if (nv > 1e-8) {
                        for (size_t i = 0; i < R; ++i) U[i * R + k] = v[i] / nv;
                        break;
                    }
                }
            }
        } else {
            for (size_t k = 0; k < R; ++k) U[k * R + k] = 1.0;
        }
        if (Xo) {
            // orthonormal basis rotated to the singular vectors: X Rxi U
            std::vector<double> M(R * R, 0.0);
            for (size_t i = 0; i < R; ++i)
                for (size_t k = 0; k < R; ++k) {
                    double acc = 0.0;
                    for (size_t j = 0; j < R; ++j) acc += Rxi[i * R + j] * U[j * R + k];
                    M[i * R + k] = acc;
                }
            const size_t nx = h->nx, ny = h->ny;
            for (size_t e = 0; e < n; ++e) {
                const size_t erm = (e % ny) * nx + (e / ny);   // device cell e = i*ny + j -> j*nx + i
                for (size_t k = 0; k < R; ++k) {
                    double s = 0.0;
                    for (size_t j = 0; j < R; ++j) s += X[j * n + e] * M[j * R + k];
                    Xo[erm * R + k] = s;
                }
            }
        }
        if (So)
            for (size_t i = 0; i < R; ++i)
                for (size_t j = 0; j < R; ++j) So[i * R + j] = h->s_is_usigma ? (i == j ? sig[i] : 0.0) : S[i * R + j];
        if (Wo)
            for (size_t qq = 0; qq < Q; ++qq)
                for (size_t k = 0; k < R; ++k) Wo[qq * R + k] = W[k * Q + qq];
        if (selo) {
            if (h->have_sel) {
                std::vector<int> sv(R);
                download(sv.data(), h->sel, R * sizeof(int));
                for (size_t k = 0; k < R; ++k) selo[k] = sv[k];
            } else {
                for (size_t k = 0; k < R; ++k) selo[k] = -1;
            }
        }
    } catch (const std::exception& ex) {
        return fail(DLR_ERR_HIP, ex.what());
    }
    return DLR_OK;
}

dlr_status dlr_load_factors(dlr_handle h, const double* Xi, const double* Si, const double* Wi, const double* Ti) {
    if (!h) return fail(DLR_ERR_ARG, "handle is NULL");
    if (h->sn) return fail(DLR_ERR_UNSUPPORTED, "a plain SN handle has no factors");
    if (!Xi || !Si || !Wi || !Ti) return fail(DLR_ERR_ARG, "X, S, W and T are required");
    try {
        hip_check(hipStreamSynchronize(h->stream), "sync");
        const size_t n = h->N, R = h->r, Q = h->nq;
        std::vector<double> X(R * n), W(R * Q);
        const size_t nx = h->nx, ny = h->ny;
        for (size_t e = 0; e < n; ++e) {
            const size_t erm = (e % ny) * nx + (e / ny);
            for (size_t k = 0; k < R; ++k) X[k * n + e] = Xi[erm * R + k];
        }
        for (size_t qq = 0; qq < Q; ++qq)
            for (size_t k = 0; k < R; ++k) W[k * Q + qq] = Wi[qq * R + k];
        upload(h->X, X.data(), X.size() * sizeof(double));
        upload(h->S, Si, R * R * sizeof(double));
        upload(h->W, W.data(), W.size() * sizeof(double));
        upload(h->T, to_cm(Ti, h->nx, h->ny).data(), n * sizeof(double));
        h->lin_ready = false;   // the linearisation and selection queued behind the last step used the old state
        h->deim_ready = false;
        h->si_last = 0;
        reset_basis_factor(h);
        refresh_phi(h);
        hip_check(hipDeviceSynchronize(), "sync");
        h->s_is_usigma = false;
        h->have_sel = false;
        h->poisoned = false;
        h->poison_code = DLR_OK;
        h->steps_done = 0;
        h->stats = dlr_step_stats{};
        int zero = 0;
        upload(h->status, &zero, sizeof(int));
    } catch (const std::exception& ex) {
        return fail(DLR_ERR_HIP, ex.what());
    }
    return DLR_OK;
}

dlr_status dlr_read_stats(dlr_handle h, dlr_step_stats* out) {
    if (!h || !out) return fail(DLR_ERR_ARG, "NULL argument");
    *out = h->stats;
    out->steps_done = h->steps_done;
    out->rank = h->nsweep();
    return DLR_OK;
}

dlr_status dlr_force_selection(dlr_handle h, const int32_t* selv) {
    if (!h) return fail(DLR_ERR_ARG, "handle is NULL");
    if (h->sn) return fail(DLR_ERR_UNSUPPORTED, "a plain SN handle has no angle selection");
    if (!selv) {
        h->force_pending = false;
        return DLR_OK;
    }
    std::vector<char> seen(h->nq, 0);
    for (int k = 0; k < h->r; ++k) {
        if (selv[k] < 0 || selv[k] >= h->nq || seen[selv[k]]) return fail(DLR_ERR_ARG, "invalid forced selection");
        seen[selv[k]] = 1;
    }
    try {
        upload(h->forced, selv, h->r * sizeof(int));
    } catch (const std::exception& ex) {
        return fail(DLR_ERR_HIP, ex.what());
    }
    h->force_pending = true;
    return DLR_OK;
}

dlr_status dlr_destroy(dlr_handle h) {
    if (!h) return DLR_OK;
    if (h->stream || h->arena.base) (void)hipStreamSynchronize(h->stream);
    if (h->side) {
        (void)hipStreamSynchronize(h->side);
        (void)hipStreamDestroy(h->side);
    }
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    for (auto& ev : h->ev_si)
        if (ev) (void)hipEventDestroy(ev);
    for (auto& ev : h->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (h->h_norm) (void)hipHostFree(h->h_norm);
    if (h->h_status) (void)hipHostFree(h->h_status);
    dev_free(h->dsa_mem);
    h->arena.release();
    delete h;
    return DLR_OK;
}

dlr_status dlr_sweep_shape(dlr_handle h, int32_t* prefetch, int32_t* grid_blocks) {
    if (!h || !prefetch || !grid_blocks) return fail(DLR_ERR_ARG, "handle or outputs NULL");
    *prefetch = h->sw_prefetch;
    *grid_blocks = h->sw_grid;
    return DLR_OK;
}

dlr_status dlr_set_sweep_shape(dlr_handle h, int32_t prefetch, int32_t grid_blocks) {
    if (!h) return fail(DLR_ERR_ARG, "handle is NULL");
    if (prefetch == 0 && grid_blocks == 0) {
        h->sw_prefetch = h->sw_grid = 0;   // the tuner chooses (or its earlier choice for this shape)
        return DLR_OK;
    }
    if (!(prefetch == 2 || prefetch == 4 || (prefetch == 8 && h->fp32())))
        return fail(DLR_ERR_ARG, "prefetch must be 2 or 4 (or 8 with FP32 sweeps)");
    if (grid_blocks < 1 || grid_blocks > 65535) return fail(DLR_ERR_ARG, "grid_blocks must be in [1, 65535]");
    h->sw_prefetch = prefetch;
    h->sw_grid = grid_blocks;
    return DLR_OK;
}

dlr_status dlr_set_dsa(dlr_handle h, int32_t enable, double cg_tol, int32_t cg_max_iter) {
    if (!h) return fail(DLR_ERR_ARG, "handle is NULL");
    if (h->poisoned) return fail(DLR_ERR_STATE, "handle poisoned by an earlier device error");
    if (!enable) {
        h->dsa = false;
        return DLR_OK;
    }
    if (!(cg_tol > 0.0 && cg_tol < 1.0) || cg_max_iter < 1 || cg_max_iter > 100000)
        return fail(DLR_ERR_ARG, "need 0 < cg_tol < 1 and 1 <= cg_max_iter <= 100000");
    try {
        if (!h->dsa_mem.ptr) {
            const size_t n = (size_t)h->N, nb = (size_t)dlr::dsa_blocks(h->nx, h->ny);
            const size_t doubles = 7 * n + 2 * nb + 8 + 2;
            const size_t bytes = ((doubles * sizeof(double) + 255) & ~size_t(255)) + 256;
            hip_check(hipStreamSynchronize(h->stream), "stream sync");
            if (!dev_alloc(h->dsa_mem, bytes, h->stream)) return fail(DLR_ERR_OOM, "DSA workspace");
            double* base = static_cast<double*>(h->dsa_mem.ptr);
            h->dsa_ws = base;
            h->dsa_part = base + 7 * n;
            h->dsa_scal = h->dsa_part + 2 * nb;
            h->dsa_kappa = h->dsa_scal + 8;
            h->dsa_count = reinterpret_cast<unsigned*>(reinterpret_cast<char*>(base) + (bytes - 256));
            hip_check(hipMemsetAsync(h->dsa_count, 0, 256, h->stream), "clear");
        }
        if (h->sn)   // every ordinate with its quadrature weight
            dlr::launch_dsa_kappa(h->stream, h->nq, h->w, h->mu, h->eta, h->dsa_kappa);
        hip_check(hipStreamSynchronize(h->stream), "stream sync");
    } catch (const std::exception& ex) {
        return fail(DLR_ERR_HIP, ex.what());
    }
    h->dsa = true;
    h->dsa_tol = cg_tol;
    h->dsa_max_iter = cg_max_iter;
    h->deim_ready = false;   // a selection queued without DSA lacks the DSA coefficients of its picks
    return DLR_OK;
}

// ---------------------------------------------------------------------------------------------------------
// Batches

dlr_status dlr_batch_footprint(const dlr_problem* p, size_t* bytes) {
    if (!bytes) return fail(DLR_ERR_ARG, "bytes is NULL");
    g_last_error.clear();
    const dlr_status v = validate(p);
    if (v != DLR_OK) return v;
    dlr_instance tmp;
    init_fields(&tmp, p, nullptr);
    *bytes = arena_bytes(&tmp);
    return DLR_OK;
}

dlr_status dlr_batch_create(size_t hbm_budget, void* hip_stream, dlr_batch* out) {
    if (!out) return fail(DLR_ERR_ARG, "out is NULL");
    *out = nullptr;
    dlr_batch_s* B = new (std::nothrow) dlr_batch_s();
    if (!B) return fail(DLR_ERR_OOM, "host allocation failed");
    try {
        B->main = static_cast<hipStream_t>(hip_stream);
        if (hbm_budget == 0) {
            size_t free_b = 0, total_b = 0;
            hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
            hbm_budget = free_b > (1ull << 30) ? free_b - (1ull << 30) : 0;
        }
        B->budget = hbm_budget;
        for (int k = 0; k < kBatchStreams; ++k) {
            hipStream_t st = nullptr;
            hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "stream");
            B->pool.push_back(st);
        }
        if (!dev_alloc(B->ticket_mem, 256, B->main)) throw HipError("ticket: device allocation failed");
        B->d_ticket = static_cast<unsigned*>(B->ticket_mem.ptr);
        hip_check(hipMemsetAsync(B->d_ticket, 0, 4 * sizeof(unsigned), B->main), "ticket");
        hip_check(hipStreamSynchronize(B->main), "sync");
        hip_check(hipEventCreateWithFlags(&B->ev_main, hipEventDisableTiming), "event");
        batch_reserve(B, 64);
        // recorded steps: their own stream, and the sweep launch counter (ids from 2^31 on)
        hip_check(hipStreamCreateWithFlags(&B->rec, hipStreamNonBlocking), "stream");
        hip_check(hipEventCreateWithFlags(&B->ev_cap, hipEventDisableTiming), "event");
        if (!dev_alloc(B->gctr_mem, 256, B->rec)) throw HipError("counter: device allocation failed");
        B->d_sweep_ctr = static_cast<unsigned long long*>(B->gctr_mem.ptr);
        const unsigned long long base = 1ull << 31;
        hip_check(hipMemcpy(B->d_sweep_ctr, &base, sizeof(base), hipMemcpyHostToDevice), "counter");
    } catch (const std::exception& ex) {
        dlr_batch_destroy(B);
        return fail(DLR_ERR_HIP, ex.what());
    }
    *out = B;
    return DLR_OK;
}

dlr_status dlr_batch_admit(dlr_batch B, const dlr_problem* p, int32_t n_steps, int64_t* slot) {
    if (!B || !slot) return fail(DLR_ERR_ARG, "batch or slot is NULL");
    if (n_steps < 1) return fail(DLR_ERR_ARG, "n_steps must be >= 1");
    size_t bytes = 0;
    const dlr_status f = dlr_batch_footprint(p, &bytes);
    if (f != DLR_OK) return f;
    if (B->used + bytes > B->budget) return fail(DLR_ERR_OOM, "footprint exceeds the remaining batch budget");
    const int64_t id = B->next_id;
    dlr_handle h = nullptr;
    const dlr_status c = dlr_create(p, B->pool[(size_t)(id % kBatchStreams)], &h);
    if (c != DLR_OK) return c;
    // slots overlap with each other; they keep their phases in order on their pool stream
    if (h->side) {
        (void)hipStreamDestroy(h->side);
        h->side = nullptr;
    }
    BatchSlot sl;
    sl.id = id;
    sl.I = h;
    sl.bytes = bytes;
    sl.remaining = n_steps;
    if (hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
        dlr_destroy(h);
        return fail(DLR_ERR_HIP, "event create");
    }
    B->slots.emplace(id, sl);
    B->used += bytes;
    ++B->next_id;
    *slot = id;
    return DLR_OK;
}

dlr_status dlr_batch_advance(dlr_batch B) {
    if (!B) return fail(DLR_ERR_ARG, "batch is NULL");
    std::vector<BatchSlot*> act;
    std::vector<int64_t> key;
    for (auto& kv : B->slots)
        if (!kv.second.finished && kv.second.remaining > 0) {
            act.push_back(&kv.second);
            key.push_back(kv.first);
        }
    if (act.empty()) return DLR_OK;
    try {
        batch_reserve(B, act.size());
        // A composition seen at two advances in a row runs from recorded graphs (recorded once per
        // composition and count of source iterations); a forced selection (the parity replay) runs eagerly.
        bool forced = false;
        for (BatchSlot* sl : act) forced = forced || sl->I->force_pending;
        const bool stable = B->graphs && B->rec && !forced && key == B->last_key;
        B->last_key = key;
        const int K = std::max(1, std::min(B->k_hint, B->max_rec));
        if (!stable) {
            if (!B->gkey.empty()) graph_clear(B);
        } else if (B->gkey != key || B->gK != K) {
            graph_record(B, act, key, K);
        }
        const bool replay = stable && B->gkey == key;
        const int p = B->parity;
        std::vector<BatchSlot*> pending;
        bool broken = false;
        if (replay) {
            for (BatchSlot* sl : act) {
                dlr_instance* I = sl->I;
                I->phi_cur = I->phi;
                I->phi_nxt = I->phi2;
                I->si_it = 0;
                I->si_conv = false;
                I->sweep_ms_acc = 0.f;
                I->si_ms_acc = 0.f;
                I->force_pending = false;
                I->device_si = true;
                I->untimed = true;
            }
            hip_check(hipGraphLaunch(B->gx_begin[p], B->rec), "graph launch");
            hip_check(hipStreamSynchronize(B->rec), "sync");
            for (size_t k = 0; k < act.size(); ++k) {
                BatchSlot* sl = act[k];
                dlr_instance* I = sl->I;
                const int* f = B->h_gi + 4 * k;
                I->si_it = f[1];
                I->stats.si_residual = B->h_gd[k];
                if (f[1] & 1) std::swap(I->phi_cur, I->phi_nxt);   // the newest flux after an odd count
                dlr_status st = DLR_OK;
                if (f[3] != 0) {
                    st = check_device_status(I);
                } else if (f[2] == 2) {
                    I->poisoned = true;
                    I->poison_code = DLR_ERR_NONFINITE;
                    st = fail(DLR_ERR_NONFINITE, "non-finite scalar flux in source iteration");
                } else if (f[2] == 3) {
                    I->poisoned = true;
                    I->poison_code = DLR_ERR_NOT_CONVERGED;
                    st = fail(DLR_ERR_NOT_CONVERGED, "source iteration reached si_max_iter");
                } else if (f[2] == 1) {
                    I->si_conv = true;
                } else {
                    I->device_si = false;   // more iterations than recorded: continued below
                    hip_check(hipEventRecord(sl->ev, I->stream), "event");
                    pending.push_back(sl);
                }
                if (st != DLR_OK) {
                    slot_fail(B, sl, st);
                    broken = true;
                }
            }
        } else {
            for (BatchSlot* sl : act) {
                if (sl->I->fp32()) phase_begin<float>(sl->I); else phase_begin<double>(sl->I);
                hip_check(hipEventRecord(sl->ev, sl->I->stream), "event");
            }
            pending = act;
        }
        // source iterations on the host's decision: all of them without a recorded step, the
        // remaining ones of slots that needed more than were recorded
        while (!pending.empty()) {
            for (BatchSlot* sl : pending) hip_check(hipStreamWaitEvent(B->main, sl->ev, 0), "wait");
            batch_sweep<double>(B, pending);
            batch_sweep<float>(B, pending);
            hip_check(hipEventRecord(B->ev_main, B->main), "event");
            for (BatchSlot* sl : pending) {
                hip_check(hipStreamWaitEvent(sl->I->stream, B->ev_main, 0), "wait");
                if (sl->I->fp32()) si_phi<float>(sl->I); else si_phi<double>(sl->I);
                hip_check(hipEventRecord(sl->ev, sl->I->stream), "event");
            }
            std::vector<BatchSlot*> next;
            for (BatchSlot* sl : pending) {
                hip_check(hipEventSynchronize(sl->ev), "sync");
                const dlr_status st = si_check(sl->I);
                if (st != DLR_OK) {
                    slot_fail(B, sl, st);
                    broken = true;
                } else if (!sl->I->si_conv) {
                    if (sl->I->dsa) dsa_correct(sl->I);
                    hip_check(hipEventRecord(sl->ev, sl->I->stream), "event");
                    next.push_back(sl);
                }
            }
            pending.swap(next);
        }
        if (replay && !broken) {
            hip_check(hipGraphLaunch(B->gx_end[p], B->rec), "graph launch");
            hip_check(hipStreamSynchronize(B->rec), "sync");
            B->parity ^= 1;
            ++B->graph_steps;
            for (BatchSlot* sl : act) {
                std::swap(sl->I->X, sl->I->Xn);   // as the recorded end of the step did
                std::swap(sl->I->S, sl->I->Sn);
            }
        } else {
            if (replay) graph_clear(B);
            for (BatchSlot* sl : act)
                if (!sl->finished) {
                    if (sl->I->fp32()) phase_end<float>(sl->I); else phase_end<double>(sl->I);
                    step_publish(sl->I);
                }
        }
        int most = 1;
        for (BatchSlot* sl : act) {
            if (sl->finished) continue;
            most = std::max(most, sl->I->si_it);
            const dlr_status st = step_read(sl->I, false);
            sl->I->device_si = false;
            sl->I->untimed = false;
            if (st != DLR_OK) {
                slot_fail(B, sl, st);
                continue;
            }
            if (--sl->remaining == 0) {
                sl->finished = true;
                B->done.push_back(sl->id);
            }
        }
        for (BatchSlot* sl : act) {
            sl->I->device_si = false;
            sl->I->untimed = false;
        }
        B->k_hint = most;
    } catch (const std::exception& ex) {
        return fail(DLR_ERR_HIP, ex.what());
    }
    return DLR_OK;
}

dlr_status dlr_batch_poll(dlr_batch B, int64_t* done, int32_t cap, int32_t* n) {
    if (!B || !n || (cap > 0 && !done) || cap < 0) return fail(DLR_ERR_ARG, "bad poll arguments");
    int32_t k = 0;
    while (k < cap && !B->done.empty()) {
        done[k++] = B->done.front();
        B->done.pop_front();
    }
    *n = k;
    return DLR_OK;
}

dlr_status dlr_batch_read(dlr_batch B, int64_t slot, double* E_r, double* T) {
    if (!B) return fail(DLR_ERR_ARG, "batch is NULL");
    BatchSlot* sl = find_slot(B, slot);
    if (!sl) return fail(DLR_ERR_ARG, "no such slot");
    if (sl->fail_status != DLR_OK) return fail(sl->fail_status, sl->fail_msg);
    return dlr_read_fields(sl->I, E_r, T);
}

dlr_status dlr_batch_read_stats(dlr_batch B, int64_t slot, dlr_step_stats* out) {
    if (!B) return fail(DLR_ERR_ARG, "batch is NULL");
    BatchSlot* sl = find_slot(B, slot);
    if (!sl) return fail(DLR_ERR_ARG, "no such slot");
    return dlr_read_stats(sl->I, out);
}

dlr_status dlr_batch_release(dlr_batch B, int64_t slot) {
    if (!B) return fail(DLR_ERR_ARG, "batch is NULL");
    BatchSlot* sl = find_slot(B, slot);
    if (!sl) return fail(DLR_ERR_ARG, "no such slot");
    if (std::find(B->gkey.begin(), B->gkey.end(), slot) != B->gkey.end()) {
        if (B->rec) (void)hipStreamSynchronize(B->rec);
        graph_clear(B);
    }
    dlr_destroy(sl->I);
    if (sl->ev) (void)hipEventDestroy(sl->ev);
    B->used -= sl->bytes;
    B->slots.erase(slot);
    for (auto it = B->done.begin(); it != B->done.end(); ++it)
        if (*it == slot) {
            B->done.erase(it);
            break;
        }
    return DLR_OK;
}

dlr_status dlr_batch_usage(dlr_batch B, int32_t* active_slots, size_t* bytes_in_use) {
    if (!B) return fail(DLR_ERR_ARG, "batch is NULL");
    int32_t a = 0;
    for (auto& kv : B->slots)
        if (!kv.second.finished) ++a;
    if (active_slots) *active_slots = a;
    if (bytes_in_use) *bytes_in_use = B->used;
    return DLR_OK;
}

dlr_status dlr_batch_destroy(dlr_batch B) {
    if (!B) return DLR_OK;
    if (B->main || !B->pool.empty()) (void)hipDeviceSynchronize();
    for (auto& kv : B->slots) {
        dlr_destroy(kv.second.I);
        if (kv.second.ev) (void)hipEventDestroy(kv.second.ev);
    }
    for (int g = 0; g < 2; ++g) {
        dev_free(B->table_mem[g]);
        dev_free(B->unit_end_mem[g]);
        if (B->h_table[g]) (void)hipHostFree(B->h_table[g]);
        if (B->h_unit_end[g]) (void)hipHostFree(B->h_unit_end[g]);
    }
    dev_free(B->ticket_mem);
    graph_clear(B);
    for (int g = 0; g < 2; ++g) {
        dev_free(B->gtable_mem[g]);
        dev_free(B->gunit_mem[g]);
    }
    dev_free(B->gptr_mem);
    dev_free(B->gctr_mem);
    if (B->h_gi) (void)hipHostFree(B->h_gi);
    if (B->h_gd) (void)hipHostFree(B->h_gd);
    if (B->ev_cap) (void)hipEventDestroy(B->ev_cap);
    if (B->rec) (void)hipStreamDestroy(B->rec);
    for (hipStream_t st : B->rec_streams) (void)hipStreamDestroy(st);
    if (B->ev_main) (void)hipEventDestroy(B->ev_main);
    for (hipStream_t st : B->pool) (void)hipStreamDestroy(st);
    delete B;
    return DLR_OK;
}

dlr_status dlr_batch_set_graphs(dlr_batch B, int32_t enable) {
    if (!B) return fail(DLR_ERR_ARG, "batch is NULL");
    if (enable < 0 || enable > 64) return fail(DLR_ERR_ARG, "enable must be in [0, 64]");
    B->graphs = enable != 0;
    if (enable > 0) B->max_rec = enable == 1 ? 8 : enable;
    if (B->rec) (void)hipStreamSynchronize(B->rec);
    graph_clear(B);   // re-recorded under the new setting
    return DLR_OK;
}

dlr_status dlr_batch_graph_steps(dlr_batch B, int64_t* steps) {
    if (!B || !steps) return fail(DLR_ERR_ARG, "batch or steps is NULL");
    *steps = B->graph_steps;
    return DLR_OK;
}


// ---------------------------------------------------------------------------------------------------------
// Bilinear (Q1) DG sweep operator

}  // extern "C"

struct dlr_q1_s {
    int nx = 0, ny = 0, nd = 0, precision = 0, nsuper = 0, grid = 0;
    double hx = 0, hy = 0;
    hipStream_t stream = nullptr;
    Arena arena;
    double* mu = nullptr;
    double* eta = nullptr;
    void* edge = nullptr;
    unsigned long long* progress = nullptr;
    unsigned* ticket = nullptr;
    int* status = nullptr;
    int* h_status = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool poisoned = false;
    size_t elem() const { return precision == DLR_FP64 ? sizeof(double) : sizeof(float); }
};

namespace {

void q1_carve(dlr_q1_s* Q) {
    const size_t nd = (size_t)Q->nd;
    Q->mu = Q->arena.take<double>(nd);
    Q->eta = Q->arena.take<double>(nd);
    Q->progress = Q->arena.take<unsigned long long>(nd * Q->nsuper);
    Q->ticket = Q->arena.take<unsigned>(2);
    Q->status = Q->arena.take<int>(1);
    const size_t ne = nd * Q->nsuper * (size_t)Q->ny * 2;
    if (Q->precision == DLR_FP64)
        Q->edge = Q->arena.take<double>(ne);
    else
        Q->edge = Q->arena.take<float>(ne);
}

template <typename TS>
dlr::Q1Args<TS> q1_args(const dlr_q1_s* Q, const void* sig, const void* src, const void* inx, const void* iny,
                        void* psi) {
    dlr::Q1Args<TS> a{};
    a.nx = Q->nx; a.ny = Q->ny; a.nd = Q->nd; a.nsuper = Q->nsuper;
    a.total_units = (unsigned)(Q->nsuper * Q->nd);
    a.grid_blocks = Q->grid;
    a.hx = Q->hx; a.hy = Q->hy;
    a.mu = Q->mu; a.eta = Q->eta;
    a.sig = static_cast<const TS*>(sig);
    a.src = static_cast<const TS*>(src);
    a.inx = static_cast<const TS*>(inx);
    a.iny = static_cast<const TS*>(iny);
    a.psi = static_cast<TS*>(psi);
    a.edge = static_cast<TS*>(Q->edge);
    a.progress = Q->progress;
    a.ticket = Q->ticket;
    a.status = Q->status;
    a.spin_limit = 1u << 20;
    a.launch_id = dlr::next_sweep_launch_id();
    return a;
}

dlr_status q1_launch(dlr_q1_s* Q, const void* sig, const void* src, const void* inx, const void* iny, void* psi) {
    if (Q->poisoned) return fail(DLR_ERR_STATE, "Q1 sweep handle poisoned by an earlier device error");
    if (!sig || !src || !inx || !iny || !psi) return fail(DLR_ERR_ARG, "NULL array");
    const size_t el = Q->elem();
    auto misaligned = [](const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) != 0; };
    if (misaligned(sig, el) || misaligned(src, 4 * el) || misaligned(psi, 4 * el) || misaligned(inx, 2 * el) ||
        misaligned(iny, 2 * el))
        return fail(DLR_ERR_ARG, "misaligned array (src and psi need 4-element, inflow 2-element alignment)");
    if (Q->precision == DLR_FP64)
        dlr::launch_q1_sweep<double>(Q->stream, q1_args<double>(Q, sig, src, inx, iny, psi));
    else
        dlr::launch_q1_sweep<float>(Q->stream, q1_args<float>(Q, sig, src, inx, iny, psi));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DLR_ERR_HIP, std::string("Q1 sweep launch: ") + hipGetErrorString(e));
    return DLR_OK;
}

dlr_status q1_check(dlr_q1_s* Q) {
    hip_check(hipMemcpyAsync(Q->h_status, Q->status, sizeof(int), hipMemcpyDeviceToHost, Q->stream), "status copy");
    hip_check(hipStreamSynchronize(Q->stream), "stream sync");
    if (*Q->h_status == 0) return DLR_OK;
    Q->poisoned = true;
    return fail(DLR_ERR_TIMEOUT, "Q1 sweep: a hand-off wait exceeded its spin limit");
}

}  // namespace

extern "C" {

dlr_status dlr_q1_create(int32_t nx, int32_t ny, double hx, double hy, int32_t n_dir, const double* mu,
                         const double* eta, int32_t precision, void* hip_stream, dlr_q1* out) {
    if (!out) return fail(DLR_ERR_ARG, "out is NULL");
    *out = nullptr;
    g_last_error.clear();
    if (nx < 1 || ny < 1 || nx > (1 << 20) || ny > (1 << 20) || (int64_t)nx * ny > (int64_t(1) << 28))
        return fail(DLR_ERR_ARG, "need 1 <= nx, ny <= 2^20 and nx * ny <= 2^28");
    if (!(hx > 0.0) || !(hy > 0.0) || !std::isfinite(hx) || !std::isfinite(hy))
        return fail(DLR_ERR_ARG, "cell sizes must be positive and finite");
    if (n_dir < 1 || !mu || !eta) return fail(DLR_ERR_ARG, "need n_dir >= 1 and direction arrays");
    for (int d = 0; d < n_dir; ++d)
        if (!std::isfinite(mu[d]) || !std::isfinite(eta[d]) || (mu[d] == 0.0 && eta[d] == 0.0))
            return fail(DLR_ERR_ARG, "direction cosines must be finite and not both zero");
    if (precision != DLR_FP64 && precision != DLR_FP32_SWEEP)
        return fail(DLR_ERR_ARG, "precision must be DLR_FP64 or DLR_FP32_SWEEP");
    dlr_q1_s* Q = new (std::nothrow) dlr_q1_s;
    if (!Q) return fail(DLR_ERR_OOM, "host allocation");
    Q->nx = nx; Q->ny = ny; Q->nd = n_dir; Q->precision = precision;
    Q->hx = hx; Q->hy = hy;
    Q->nsuper = (nx + 64 * dlr::kQ1Waves - 1) / (64 * dlr::kQ1Waves);
    Q->grid = std::min(Q->nsuper * n_dir, 2048);
    Q->stream = static_cast<hipStream_t>(hip_stream);
    try {
        q1_carve(Q);   // sizing pass
        const size_t need = Q->arena.used;
        Q->arena.used = 0;
        if (!Q->arena.allocate(need, Q->stream)) {
            dlr_q1_destroy(Q);
            return fail(DLR_ERR_OOM, "device allocation of the Q1 operator failed");
        }
        q1_carve(Q);
        hip_check(hipHostMalloc(reinterpret_cast<void**>(&Q->h_status), sizeof(int)), "host status");
        for (auto& ev : Q->ev) hip_check(hipEventCreate(&ev), "event");
        hip_check(hipMemsetAsync(Q->arena.base, 0, need, Q->stream), "clear");
        hip_check(hipMemcpyAsync(Q->mu, mu, n_dir * sizeof(double), hipMemcpyHostToDevice, Q->stream), "mu");
        hip_check(hipMemcpyAsync(Q->eta, eta, n_dir * sizeof(double), hipMemcpyHostToDevice, Q->stream), "eta");
        hip_check(hipStreamSynchronize(Q->stream), "stream sync");
    } catch (const HipError& ex) {
        dlr_q1_destroy(Q);
        return fail(DLR_ERR_HIP, ex.what());
    }
    *out = Q;
    return DLR_OK;
}

dlr_status dlr_q1_sweep(dlr_q1 Q, const void* sigma_t, const void* src, const void* inflow_x, const void* inflow_y,
                        void* psi) {
    if (!Q) return fail(DLR_ERR_ARG, "NULL handle");
    return q1_launch(Q, sigma_t, src, inflow_x, inflow_y, psi);
}

dlr_status dlr_q1_sync(dlr_q1 Q) {
    if (!Q) return fail(DLR_ERR_ARG, "NULL handle");
    if (Q->poisoned) return fail(DLR_ERR_STATE, "Q1 sweep handle poisoned by an earlier device error");
    try {
        return q1_check(Q);
    } catch (const HipError& ex) {
        Q->poisoned = true;
        return fail(DLR_ERR_HIP, ex.what());
    }
}

dlr_status dlr_q1_time(dlr_q1 Q, const void* sigma_t, const void* src, const void* inflow_x, const void* inflow_y,
                       void* psi, int32_t reps, double* ms_per_sweep) {
    if (!Q) return fail(DLR_ERR_ARG, "NULL handle");
    if (reps < 1 || !ms_per_sweep) return fail(DLR_ERR_ARG, "need reps >= 1 and an output");
    try {
        hip_check(hipEventRecord(Q->ev[0], Q->stream), "event");
        for (int k = 0; k < reps; ++k) {
            const dlr_status st = q1_launch(Q, sigma_t, src, inflow_x, inflow_y, psi);
            if (st != DLR_OK) return st;
        }
        hip_check(hipEventRecord(Q->ev[1], Q->stream), "event");
        const dlr_status st = q1_check(Q);
        if (st != DLR_OK) return st;
        float ms = 0.0f;
        hip_check(hipEventElapsedTime(&ms, Q->ev[0], Q->ev[1]), "elapsed");
        *ms_per_sweep = (double)ms / reps;
    } catch (const HipError& ex) {
        Q->poisoned = true;
        return fail(DLR_ERR_HIP, ex.what());
    }
    return DLR_OK;
}

dlr_status dlr_q1_destroy(dlr_q1 Q) {
    if (!Q) return DLR_OK;
    if (Q->arena.base) (void)hipStreamSynchronize(Q->stream);
    for (auto& ev : Q->ev)
        if (ev) (void)hipEventDestroy(ev);
    if (Q->h_status) (void)hipHostFree(Q->h_status);
    Q->arena.release();
    delete Q;
    return DLR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------------------
// Q1 sweep without allocation.  The hand-off state of the sweep (unit ticket, progress words, edge
// values) lives in a static device array instead of an operator's arena.  In host code the array's
// name only stands for the symbol; its device address (one per GPU) comes from hipGetSymbolAddress
// with that GPU current and is what every kernel argument uses.
namespace {

constexpr size_t kQ1ScratchBytes = size_t(16) << 20;
constexpr size_t kQ1ScratchHead = 256;   // ticket [2] (zeroed before every launch), then progress, edges
__device__ __align__(256) unsigned char scratch[kQ1ScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

__global__ void k_zero_words(unsigned* p, int n) {
    const int i = (int)threadIdx.x;
    if (i < n) p[i] = 0u;
}

// the device address of the scratch array on the current device (resolved once per device)
dlr_status scratch_address(hipStream_t stream, void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(DLR_ERR_HIP, "hipGetDevice failed");
    if (stream) {
        int sdev = -1;
        if (hipStreamGetDevice(stream, &sdev) != hipSuccess) return fail(DLR_ERR_HIP, "hipStreamGetDevice failed");
        if (sdev != dev) return fail(DLR_ERR_ARG, "the stream belongs to another device than the current one");
    }
    if (dev < 0 || dev >= kMaxDevices) return fail(DLR_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(DLR_ERR_HIP, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DLR_OK;
}

}  // namespace

extern "C" {

dlr_status dlr_q1_sweep_noalloc(int32_t nx, int32_t ny, double hx, double hy, int32_t n_dir, const double* mu,
                                const double* eta, int32_t precision, void* hip_stream, const void* sigma_t,
                                const void* src, const void* inflow_x, const void* inflow_y, void* psi,
                                int32_t* status) {
    g_last_error.clear();
    if (nx < 1 || ny < 1 || nx > (1 << 20) || ny > (1 << 20) || (int64_t)nx * ny > (int64_t(1) << 28))
        return fail(DLR_ERR_ARG, "need 1 <= nx, ny <= 2^20 and nx * ny <= 2^28");
    if (!(hx > 0.0) || !(hy > 0.0) || !std::isfinite(hx) || !std::isfinite(hy))
        return fail(DLR_ERR_ARG, "cell sizes must be positive and finite");
    if (n_dir < 1 || !mu || !eta) return fail(DLR_ERR_ARG, "need n_dir >= 1 and direction arrays");
    if (precision != DLR_FP64 && precision != DLR_FP32_SWEEP)
        return fail(DLR_ERR_ARG, "precision must be DLR_FP64 or DLR_FP32_SWEEP");
    if (!status) return fail(DLR_ERR_ARG, "status is NULL");
    dlr_q1_s Q;   // describes the launch only: no arena, no events
    Q.nx = nx; Q.ny = ny; Q.nd = n_dir; Q.precision = precision;
    Q.hx = hx; Q.hy = hy;
    Q.nsuper = (nx + 64 * dlr::kQ1Waves - 1) / (64 * dlr::kQ1Waves);
    Q.grid = std::min(Q.nsuper * n_dir, 2048);
    Q.stream = static_cast<hipStream_t>(hip_stream);
    const size_t nprog = (size_t)n_dir * Q.nsuper;
    const size_t edge_off = (kQ1ScratchHead + nprog * sizeof(unsigned long long) + 255) & ~size_t(255);
    const size_t need = edge_off + nprog * (size_t)ny * 2 * Q.elem();
    if (need > kQ1ScratchBytes)
        return fail(DLR_ERR_ARG, "n_dir * ceil(nx / 128) * ny exceeds the static scratch of " +
                                     std::to_string(kQ1ScratchBytes >> 20) + " MiB");
    void* base = nullptr;
    const dlr_status sa = scratch_address(Q.stream, &base);
    if (sa != DLR_OK) return sa;
    char* b = static_cast<char*>(base);
    Q.ticket = reinterpret_cast<unsigned*>(b);
    Q.progress = reinterpret_cast<unsigned long long*>(b + kQ1ScratchHead);
    Q.edge = b + edge_off;
    Q.mu = const_cast<double*>(mu);
    Q.eta = const_cast<double*>(eta);
    Q.status = status;
    // the unit ticket must start at zero (a fill kernel, not a memset: the call may be captured)
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, Q.stream, Q.ticket, 2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DLR_ERR_HIP, std::string("scratch clear: ") + hipGetErrorString(e));
    // progress words carry the launch id, so stale ones from earlier calls never match
    return q1_launch(&Q, sigma_t, src, inflow_x, inflow_y, psi);
}

}  // extern "C"
