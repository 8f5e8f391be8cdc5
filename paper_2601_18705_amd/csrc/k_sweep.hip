// Upwind transport sweep for the selected directions (Algorithm 1 step 4): one
// application of the inverse of the degree-0 upwind operator plus sigma_t,
//   psi_e = (src0_e + s_e + ax psi_upwind_x + ay psi_upwind_y) / (sigma_t,e + ax + ay),
// ax = |mu|/hx, ay = |eta|/hy, for every swept direction d and cell e.
//
// Layout.  Cells are column-major, and every column of a sweep plane carries
// kColGuard spare rows above and below its data (cell (i, j) at
// i*(ny + 2 kColGuard) + kColGuard + j), so any sixteen-row segment that meets
// a column lies inside that column's padded range; consecutive planes are ld
// apart and each plane ends with a spare slot that absorbs redirected stores.
//
// Work decomposition.  In each direction's own sweep coordinates (i', j') --
// i' = i for mu > 0 else nx-1-i, likewise j' -- the grid is cut into strips of
// 64 columns, four consecutive strips forming a superstrip.  A workgroup takes
// one (superstrip S, direction d) unit with four compute wavefronts and one
// helper wavefront.  Compute wavefront w owns strip 4S + w; its lane l owns
// column i' = 64 (4S + w) + l and at step t updates row j' = t - l, so the
// x-upwind value is lane l-1's result of the previous step (a DPP wave shift)
// and the y-upwind value is the lane's own previous result.
//
// Each lane streams its own column: sixteen rows of src0, sigma_t and s_e per
// chunk as 16-byte loads issued a chunk ahead (register double-buffering),
// sixteen results per chunk as 16-byte stores.  Compute wavefronts issue these
// memory operations unconditionally (a segment that misses the column is
// redirected to the column start or to the spare slot rather than branched
// around) and exchange boundary fluxes only through LDS rings, so the compiler
// can count outstanding loads exactly and the prefetch is never drained.  The helper wavefront alone talks to the other
// workgroups: it copies the incoming edge of superstrip S-1 from global memory
// into the LDS ring of wavefront 0 and the outgoing edge of wavefront 3 to
// global memory, publishing progress words tagged with the launch id.  Units
// come from an atomic ticket in (superstrip, direction) order, so a workgroup
// only waits on a unit with a smaller ticket, which is already running.
#include "dlr_internal.h"

namespace dlr {

namespace {

constexpr int kWaves = kSweepWaves;   // compute wavefronts per workgroup
constexpr int kC = 16;                // rows per chunk
constexpr int kRing = 256;            // LDS ring length (rows)
static_assert(kC <= kColGuard, "a live segment may reach kC-1 rows past either end of its column");

template <typename TS>
struct Vec4 {
    typedef TS type __attribute__((ext_vector_type(4), aligned(sizeof(TS))));
};

template <typename TS>
__device__ __forceinline__ void load16(const TS* p, TS (&v)[kC]) {
    typedef typename Vec4<TS>::type V;
    const V* q = reinterpret_cast<const V*>(p);
#pragma unroll
    for (int c = 0; c < kC / 4; ++c) {
        const V x = q[c];
        v[4 * c + 0] = x[0];
        v[4 * c + 1] = x[1];
        v[4 * c + 2] = x[2];
        v[4 * c + 3] = x[3];
    }
}

template <typename TS>
__device__ __forceinline__ void store16(TS* p, const TS (&v)[kC]) {
    typedef typename Vec4<TS>::type V;
    V* q = reinterpret_cast<V*>(p);
#pragma unroll
    for (int c = 0; c < kC / 4; ++c) {
        V x;
        x[0] = v[4 * c + 0];
        x[1] = v[4 * c + 1];
        x[2] = v[4 * c + 2];
        x[3] = v[4 * c + 3];
        q[c] = x;
    }
}

// lane l receives lane l-1's value; lane 0 receives `first`
__device__ __forceinline__ float shift_in(float first, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, first),
                                                                  __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double shift_in(double first, double v) {
    const long long f = __builtin_bit_cast(long long, first), x = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp((int)(f & 0xffffffffll), (int)(x & 0xffffffffll), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(f >> 32), (int)(x >> 32), 0x138, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float step_value(float rhs, float sig, float axy, float ax, float ay, float left, float up) {
    const float num = fmaf(ax, left, fmaf(ay, up, rhs));
    return num * __builtin_amdgcn_rcpf(sig + axy);
}
__device__ __forceinline__ double step_value(double rhs, double sig, double axy, double ax, double ay, double left, double up) {
    const double num = fma(ax, left, fma(ay, up, rhs));
    return num / (sig + axy);
}

template <typename TS>
struct Shared {
    TS ring[kWaves + 1][kRing];   // ring[w]: left inflow of compute wave w; ring[kWaves]: outgoing edge
    int prod[kWaves + 1];         // rows published into ring[w]
    int cons[kWaves + 1];         // rows consumed from ring[w]
    int stall;
    unsigned task;
};

__device__ __forceinline__ int lds_load(int* p) { return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ __forceinline__ void lds_store(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Per-wavefront constant data of one strip.
template <typename TS>
struct Strip {
    const TS* sp;   // src0 column (row 0)
    const TS* qp;   // sigma_t column (row 0)
    const TS* ep;   // s_e column (row 0)
    TS* op;         // psi column (row 0)
    TS* trash;      // spare slot (kC elements) that absorbs redirected stores
    TS ax, ay, axy, bx, by;
    int lane, ny, nch;
    bool col_ok;
    bool REV;
};

template <typename TS, bool REV>
__device__ __forceinline__ int seg_start(const Strip<TS>& s, int m) {
    return REV ? (s.ny - kC * m + s.lane - kC) : (kC * m - s.lane);
}

// issue the loads of chunk m into buffers (unconditionally; dead segments read the padded column start)
template <typename TS, bool REV>
__device__ __forceinline__ void issue_loads(const Strip<TS>& s, int m, TS (&bs)[kC], TS (&bq)[kC], TS (&be)[kC]) {
    const int s0 = seg_start<TS, REV>(s, m);
    const bool live = s.col_ok && m < s.nch && s0 < s.ny && s0 + kC > 0;
    const int off = live ? s0 : -kColGuard;
    load16<TS>(s.sp + off, bs);
    load16<TS>(s.qp + off, bq);
    load16<TS>(s.ep + off, be);
}

// One chunk of sixteen steps.  FAST: every lane with a valid column is inside
// the column for all sixteen rows (no masking, vector stores).
template <typename TS, bool REV, bool FAST>
__device__ __forceinline__ void run_chunk(const Strip<TS>& s, int m, const TS (&bs)[kC], const TS (&bq)[kC],
                                 const TS (&be)[kC], const TS (&edgev)[kC], TS& mine, TS (&ob)[kC]) {
    const int r0 = kC * m;
#pragma unroll
    for (int k = 0; k < kC; ++k) {
        const int kk = REV ? kC - 1 - k : k;
        const TS left = shift_in(edgev[k], mine);
        const TS val = step_value(bs[kk] + be[kk], bq[kk], s.axy, s.ax, s.ay, left, mine);
        if (FAST) {
            mine = val;
        } else {
            const int jp = r0 + k - s.lane;
            mine = (s.col_ok && jp >= 0 && jp < s.ny) ? val : mine;
        }
        ob[kk] = val;
    }
    // rows of a live segment outside [0, ny) land in the column's spare rows
    const int s0 = seg_start<TS, REV>(s, m);
    const bool live = s.col_ok && (FAST || (s0 < s.ny && s0 + kC > 0));
    store16<TS>(live ? s.op + s0 : s.trash, ob);
}

template <typename TS, bool REV, int P>
__device__ __forceinline__ void compute_wave(const SweepArgs<TS>& a, Shared<TS>& sh, int S, int d, int w, int lane) {
    const int nx = a.nx, ny = a.ny;
    const int strip = S * kWaves + w;
    const double mu = a.mu[d], eta = a.eta[d];
    Strip<TS> s;
    s.ax = (TS)(fabs(mu) * a.inv_hx);
    s.ay = (TS)(fabs(eta) * a.inv_hy);
    s.axy = s.ax + s.ay;
    s.bx = (TS)a.inflow_x[d];
    s.by = (TS)a.inflow_y[d];
    s.lane = lane;
    s.ny = ny;
    s.nch = (ny + 63 + kC - 1) / kC;
    s.REV = REV;
    const int ip = strip * 64 + lane;
    s.col_ok = ip < nx;
    const int col = s.col_ok ? (mu > 0.0 ? ip : nx - 1 - ip) : 0;
    const size_t ldc = (size_t)ny + 2 * kColGuard;
    const size_t cb = (size_t)col * ldc + kColGuard;
    s.sp = a.src0 + (size_t)d * a.ld + cb;
    s.qp = a.sig_t + cb;
    s.ep = a.s_e + cb;
    s.op = a.psi + (size_t)d * a.ld + cb;
    s.trash = a.psi + (size_t)d * a.ld + (size_t)nx * ldc;   // spare slot after this plane's columns
    const bool from_ring = strip > 0;
    const bool has_next = (strip + 1) * 64 < nx;
    const int out_ring = (w < kWaves - 1) ? w + 1 : kWaves;
    const int nch = s.nch;
    // Chunk ranges: [0, m0) prologue, [m0, m1) fast, [m1, nch) epilogue, with m0 and m1 - m0
    // multiples of P.  A chunk m is fast when every lane's rows [16m - l, 16m - l + 16) lie in
    // [0, ny): m >= 4 (lane 63) and 16m + 16 <= ny (lane 0), i.e. 4 <= m < mf.
    const int m0 = (4 + P - 1) / P * P;
    const int mf = (ny >= kC) ? (ny - kC) / kC + 1 : 0;
    const int m1 = (mf > m0) ? m0 + (mf - m0) / P * P : m0;   // m1 <= mf < nch

    TS bs[P][kC], bq[P][kC], be[P][kC];
#pragma unroll
    for (int p = 0; p < P; ++p) issue_loads<TS, REV>(s, p, bs[p], bq[p], be[p]);
    TS mine = s.by;

    auto left_values = [&](int m, TS (&edgev)[kC]) {
        const int r0 = kC * m;
        if (!from_ring || r0 >= ny) {
#pragma unroll
            for (int k = 0; k < kC; ++k) edgev[k] = s.bx;
            return;
        }
        const int need = min(r0 + kC, ny);
        unsigned polls = 0;
        while (lds_load(&sh.prod[w]) < need) {
            __builtin_amdgcn_s_sleep(1);
            if (++polls > a.spin_limit) {
                sh.stall = 1;
                break;
            }
        }
#pragma unroll
        for (int k = 0; k < kC; ++k) edgev[k] = sh.ring[w][(r0 + k) & (kRing - 1)];
        lds_store(&sh.cons[w], need);
    };
    auto publish = [&](int m, const TS (&ob)[kC]) {
        if (!has_next) return;
        const int r0 = kC * m;
        const int newest = r0 + kC - 64;   // newest row written by lane 63 in this chunk
        unsigned polls = 0;
        while (newest - lds_load(&sh.cons[out_ring]) >= kRing) {   // back-pressure
            __builtin_amdgcn_s_sleep(1);
            if (++polls > a.spin_limit) {
                sh.stall = 1;
                break;
            }
        }
        if (lane == 63) {
#pragma unroll
            for (int k = 0; k < kC; ++k) {
                const int row = r0 + k - 63;
                if (row >= 0 && row < ny) sh.ring[out_ring][row & (kRing - 1)] = ob[REV ? kC - 1 - k : k];
            }
            lds_store(&sh.prod[out_ring], min(max(r0 + kC - 63, 0), ny));
        }
    };

    // prologue and epilogue: masked steps, element stores
    auto generic = [&](int mbeg, int mend) {
        for (int mb = mbeg; mb < mend; mb += P) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int m = mb + p;
                if (m >= mend) break;
                TS edgev[kC], ob[kC];
                left_values(m, edgev);
                run_chunk<TS, REV, false>(s, m, bs[p], bq[p], be[p], edgev, mine, ob);
                issue_loads<TS, REV>(s, m + P, bs[p], bq[p], be[p]);
                publish(m, ob);
            }
        }
    };
    if (m1 <= m0) {   // no full fast group: the whole strip takes the masked path
        generic(0, nch);
        return;
    }
    generic(0, m0);
    for (int mb = m0; mb < m1; mb += P) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int m = mb + p;
            TS edgev[kC], ob[kC];
            left_values(m, edgev);
            run_chunk<TS, REV, true>(s, m, bs[p], bq[p], be[p], edgev, mine, ob);
            issue_loads<TS, REV>(s, m + P, bs[p], bq[p], be[p]);
            publish(m, ob);
        }
    }
    generic(m1, nch);
}

// Helper wavefront: incoming edge (global -> ring[0]) and outgoing edge (ring[kWaves] -> global).
template <typename TS>
__device__ __forceinline__ void helper_wave(const SweepArgs<TS>& a, Shared<TS>& sh, int S, int d, int lane) {
    const int nx = a.nx, ny = a.ny;
    const bool incoming = S > 0;
    const bool outgoing = ((S + 1) * kWaves) * 64 < nx;   // the next superstrip has columns
    const TS* edge_in = incoming ? a.edge + ((size_t)d * a.nsuper + (S - 1)) * ny : nullptr;
    TS* edge_out = outgoing ? a.edge + ((size_t)d * a.nsuper + S) * ny : nullptr;
    unsigned long long* prog_in = incoming ? &a.progress[(size_t)d * a.nsuper + S - 1] : nullptr;
    unsigned long long* prog_out = outgoing ? &a.progress[(size_t)d * a.nsuper + S] : nullptr;
    const unsigned long long tag = a.launch_id << 32;
    int rin = incoming ? 0 : ny;    // rows copied into ring[0]
    int rout = outgoing ? 0 : ny;   // rows copied out of ring[kWaves]
    unsigned idle = 0;
    while (rin < ny || rout < ny) {
        bool moved = false;
        if (rin < ny) {
            const unsigned long long pv = __hip_atomic_load(prog_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int avail = (pv >> 32) == a.launch_id ? (int)(pv & 0xffffffffull) : 0;
            avail = min(avail, lds_load(&sh.cons[0]) + kRing);   // ring space
            avail = min(avail, rin + 64);
            if (avail > rin) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const int row = rin + lane;
                if (row < avail) sh.ring[0][row & (kRing - 1)] = edge_in[row];
                rin = avail;
                lds_store(&sh.prod[0], rin);
                moved = true;
            }
        }
        if (rout < ny) {
            const int avail = min(lds_load(&sh.prod[kWaves]), rout + 64);
            if (avail > rout) {
                const int row = rout + lane;
                if (row < avail) edge_out[row] = sh.ring[kWaves][row & (kRing - 1)];
                rout = avail;
                lds_store(&sh.cons[kWaves], rout);
                __hip_atomic_store(prog_out, tag | (unsigned long long)rout, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                moved = true;
            }
        }
        if (!moved) {
            __builtin_amdgcn_s_sleep(2);
            if (++idle > a.spin_limit) {
                sh.stall = 1;
                // release whatever waits on this helper so every wavefront still finishes
                if (lane == 0) {
                    lds_store(&sh.prod[0], ny);
                    lds_store(&sh.cons[kWaves], 1 << 30);
                }
                break;
            }
        } else {
            idle = 0;
        }
    }
    (void)tag;
}

template <typename TS, int P>
__global__ __launch_bounds__(64 * (kWaves + 1)) void k_sweep(SweepArgs<TS> a) {
    __shared__ Shared<TS> sh;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x == 0) sh.stall = 0;
    for (;;) {
        if (threadIdx.x == 0) sh.task = atomicAdd(&a.ticket[0], 1u);
        if (threadIdx.x <= kWaves) {
            sh.prod[threadIdx.x] = 0;
            sh.cons[threadIdx.x] = 0;
        }
        __syncthreads();
        const unsigned n = sh.task;
        if (n >= (unsigned)a.total_units) break;
        const int S = (int)(n / (unsigned)a.nd);
        const int d = (int)(n % (unsigned)a.nd);
        if (w < kWaves) {
            if ((S * kWaves + w) * 64 < a.nx) {
                if (a.eta[d] > 0.0)
                    compute_wave<TS, false, P>(a, sh, S, d, w, lane);
                else
                    compute_wave<TS, true, P>(a, sh, S, d, w, lane);
            }
        } else if ((S * kWaves) * 64 < a.nx) {
            helper_wave<TS>(a, sh, S, d, lane);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (sh.stall) atomicOr(a.status, (int)kStatusSweepStall);
        // the last workgroup to retire resets the ticket for the next launch on the stream
        const unsigned prev = atomicAdd(&a.ticket[1], 1u);
        if (prev == (unsigned)a.grid_blocks - 1u) {
            __hip_atomic_store(&a.ticket[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.ticket[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace

template <typename TS>
void launch_sweep(hipStream_t s, const SweepArgs<TS>& a) {
    constexpr int P = sizeof(TS) == 4 ? 2 : 1;
    hipLaunchKernelGGL((k_sweep<TS, P>), dim3(a.grid_blocks), dim3(64 * (kWaves + 1)), 0, s, a);
}
template void launch_sweep<double>(hipStream_t, const SweepArgs<double>&);
template void launch_sweep<float>(hipStream_t, const SweepArgs<float>&);

}  // namespace dlr
