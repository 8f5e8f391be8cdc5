// Upwind transport sweep for the selected directions (Algorithm 1 step 4): one
// application of the inverse of the degree-0 upwind operator plus sigma_t,
//   psi_e = (src0_e + s_e + ax psi_upwind_x + ay psi_upwind_y) / (sigma_t,e + ax + ay),
// ax = |mu|/hx, ay = |eta|/hy, for every swept direction d and cell e.
//
// Work decomposition.  In each direction's own sweep coordinates (i', j') --
// i' = i for mu > 0 else nx-1-i, likewise j' -- the grid is cut into strips of
// 64 columns, sweep_waves(precision) consecutive strips forming a superstrip.  A workgroup
// takes one (superstrip S, direction d) unit with one compute wavefront per
// strip and one helper wavefront.  Lane l of a compute wavefront owns column
// i' = 64 strip + l and at step t updates row j' = t - l: the x-upwind value is
// lane l-1's result of the previous step (a DPP wave shift) and the y-upwind
// value the lane's own previous result.
//
// Layout.  All sweep planes use the diagonal layout of the direction's
// orientation, in which the value of lane l at step t sits next to those of the
// other lanes at the same step: the sixteen steps of a chunk are four 16-byte
// loads per lane per plane, each a contiguous kilobyte across the wavefront
// (FP32), issued a chunk or two ahead (register double-buffering) and stored the
// same way.  Steps outside the grid (the skewed head and tail of a strip) read
// and write the layout's padding, so no memory operation is predicated.
//
// Hand-off.  Compute wavefronts exchange boundary fluxes only through LDS rings.
// The helper wavefront alone talks to other workgroups: it copies the incoming
// edge of superstrip S-1 from global memory into the ring of wavefront 0 and
// the outgoing edge of the last wavefront to global memory, publishing progress
// words tagged with the launch id.  Units come from an atomic ticket in
// (superstrip, direction) order, so a workgroup only waits on a unit with a
// smaller ticket, which is already running.
#include "dlr_internal.h"
#include "wave_ops.h"

#include <atomic>

namespace dlr {

namespace {

constexpr int kC = 16;                // rows per chunk
constexpr int kRing = 256;            // LDS ring length (rows)

template <typename TS>
struct Vec4 {
    typedef TS type __attribute__((ext_vector_type(4), aligned(sizeof(TS))));
};

// The plane pointers come from the sweep record in memory, so the compiler cannot see that they
// point to global memory and would emit flat accesses -- which also count against the LDS wait
// counter, making every wait on a ring row wait for all prefetched chunks as well.  The chunk
// loads and stores therefore go through global-address-space pointers.
#define DLR_GLOBAL __attribute__((address_space(1)))

// Chunk m of a lane: diagonal groups 4m..4m+3 at p + g*256 elements, four values each.
template <typename TS>
__device__ __forceinline__ void load_chunk(const TS* p, TS (&v)[kC]) {
    typedef typename Vec4<TS>::type V;
#pragma unroll
    for (int c = 0; c < kC / 4; ++c) {
        const V x = *(const DLR_GLOBAL V*)(p + (size_t)c * 256);
        v[4 * c + 0] = x[0];
        v[4 * c + 1] = x[1];
        v[4 * c + 2] = x[2];
        v[4 * c + 3] = x[3];
    }
}

template <typename TS>
__device__ __forceinline__ void store_chunk(TS* p, const TS (&v)[kC]) {
    typedef typename Vec4<TS>::type V;
#pragma unroll
    for (int c = 0; c < kC / 4; ++c) {
        V x;
        x[0] = v[4 * c + 0];
        x[1] = v[4 * c + 1];
        x[2] = v[4 * c + 2];
        x[3] = v[4 * c + 3];
        *(DLR_GLOBAL V*)(p + (size_t)c * 256) = x;
    }
}

__device__ __forceinline__ float step_value(float rhs, float sig, float axy, float ax, float ay, float left, float up) {
    const float num = fmaf(ax, left, fmaf(ay, up, rhs));
    return num * __builtin_amdgcn_rcpf(sig + axy);
}
__device__ __forceinline__ double step_value(double rhs, double sig, double axy, double ax, double ay, double left, double up) {
    const double num = fma(ax, left, fma(ay, up, rhs));
    return num / (sig + axy);
}

// compute wavefronts per workgroup for planes of type TS
template <typename TS>
constexpr int kWavesOf = sweep_waves(sizeof(TS) == 8);

template <typename TS>
struct Shared {
    static constexpr int kWaves = kWavesOf<TS>;
    TS ring[kWaves + 1][kRing] __attribute__((aligned(16)));   // ring[w]: left inflow of compute wave w;
                                                                // ring[kWaves]: outgoing edge; row j in slot (j+63) % kRing
    int prod[kWaves + 1];         // rows published into ring[w]
    int cons[kWaves + 1];         // rows consumed from ring[w]
    int stall;
    unsigned task;
};

// Per-wavefront constant data of one strip.
template <typename TS>
struct Strip {
    const TS* sp;   // src0: this lane's element of diagonal group 0
    const TS* qp;   // sigma_t
    const TS* ep;   // s_e
    TS* op;         // psi
    TS ax, ay, axy, bx, by;
    int lane, nch;
};

// issue the loads of chunk m (clamped to the last chunk, so a prefetch past the end stays in the plane)
template <typename TS>
__device__ __forceinline__ void issue_loads(const Strip<TS>& s, int m, TS (&bs)[kC], TS (&bq)[kC], TS (&be)[kC]) {
    const size_t off = (size_t)min(m, s.nch - 1) * (kC / 4) * 256;
    load_chunk<TS>(s.sp + off, bs);
    load_chunk<TS>(s.qp + off, bq);
    load_chunk<TS>(s.ep + off, be);
}

// One chunk of sixteen steps.  MASK: steps before the lane's first row (t < lane) keep the
// inflow value; later steps past the last row compute padding that nothing reads.
template <typename TS, bool MASK>
__device__ __forceinline__ void run_chunk(const Strip<TS>& s, int m, const TS (&bs)[kC], const TS (&bq)[kC],
                                          const TS (&be)[kC], const TS (&edgev)[kC], TS& mine, TS (&ob)[kC]) {
    const int t0 = kC * m;
#pragma unroll
    for (int k = 0; k < kC; ++k) {
        const TS left = shift_in(edgev[k], mine);
        const TS val = step_value(bs[k] + be[k], bq[k], s.axy, s.ax, s.ay, left, mine);
        if (MASK)
            mine = (t0 + k >= s.lane) ? val : mine;
        else
            mine = val;
        ob[k] = val;
    }
    store_chunk<TS>(s.op + (size_t)m * (kC / 4) * 256, ob);
}

template <typename TS, int P>
__device__ __forceinline__ void compute_wave(const SweepArgs<TS>& a, Shared<TS>& sh, int S, int d, int w, int lane) {
    constexpr int kWaves = kWavesOf<TS>;
    const int ny = a.ny;
    const int strip = S * kWaves + w;
    const double mu = a.mu[d], eta = a.eta[d];
    const int o = orient_of(mu, eta);
    const int ndg = diag_groups(ny);
    Strip<TS> s;
    s.ax = (TS)(fabs(mu) * a.inv_hx);
    s.ay = (TS)(fabs(eta) * a.inv_hy);
    s.axy = s.ax + s.ay;
    s.bx = (TS)a.inflow_x[d];
    s.by = (TS)a.inflow_y[d];
    s.lane = lane;
    s.nch = ndg / (kC / 4);
    const size_t lane_base = (size_t)strip * ndg * 256 + (size_t)lane * 4;
    s.sp = a.src0 + (size_t)d * a.ldg + lane_base;
    s.qp = a.sig_t + (size_t)o * a.ldg + lane_base;
    s.ep = a.s_e + (size_t)o * a.ldg + lane_base;
    s.op = a.psi + (size_t)d * a.ldg + lane_base;
    const bool from_ring = strip > 0;
    const bool has_next = (strip + 1) * 64 < a.nx;
    const int out_ring = (w < kWaves - 1) ? w + 1 : kWaves;
    const int nch = s.nch;
    // chunks [0, m0) carry the skewed head (masked), with m0 a multiple of P; nch >= 4 always, and
    // with P = 8 a short column (ny < 50) has fewer than m0 chunks: the head loop stops at nch
    const int m0 = (4 + P - 1) / P * P;

    TS bs[P][kC], bq[P][kC], be[P][kC];
#pragma unroll
    for (int p = 0; p < P; ++p) issue_loads<TS>(s, p, bs[p], bq[p], be[p]);
    TS mine = s.by;

    // Progress words only grow, so a stale copy is conservative: a wavefront polls the LDS word
    // only when the copy it last read does not cover what it needs.
    int known_prod = 0;   // rows published into ring[w], as last read
    int known_cons = 0;   // rows consumed from ring[out_ring], as last read
    auto left_values = [&](int m, TS (&edgev)[kC]) {
        const int r0 = kC * m;
        if (!from_ring || r0 >= ny) {
#pragma unroll
            for (int k = 0; k < kC; ++k) edgev[k] = s.bx;
            return;
        }
        const int need = min(r0 + kC, ny);
        if (known_prod < need) {   // poll only when the last word read does not cover this chunk
            unsigned polls = 0;
            for (;;) {
                known_prod = lds_load(&sh.prod[w]);
                if (known_prod >= need) break;
                __builtin_amdgcn_s_sleep(1);
                if (++polls > a.spin_limit) {
                    sh.stall = 1;
                    break;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kC; ++k) edgev[k] = sh.ring[w][(r0 + k + 63) & (kRing - 1)];
        lds_store(&sh.cons[w], need);
    };
    auto publish = [&](int m, const TS (&ob)[kC]) {
        if (!has_next) return;
        const int r0 = kC * m;
        const int newest = r0 + kC - 64;   // newest row written by lane 63 in this chunk
        if (newest - known_cons >= kRing) {   // back-pressure, re-read only when the ring may be full
            unsigned polls = 0;
            for (;;) {
                known_cons = lds_load(&sh.cons[out_ring]);
                if (newest - known_cons < kRing) break;
                __builtin_amdgcn_s_sleep(1);
                if (++polls > a.spin_limit) {
                    sh.stall = 1;
                    break;
                }
            }
        }
        if (lane == 63) {
            // row j lives in slot (j + 63) mod kRing, so lane 63's sixteen rows r0-63 .. r0-48 are
            // one aligned block; rows outside [0, ny) land in slots no pending row occupies
            typedef typename Vec4<TS>::type V;
            V* dst = reinterpret_cast<V*>(&sh.ring[out_ring][r0 & (kRing - 1)]);
#pragma unroll
            for (int c = 0; c < kC / 4; ++c) {
                V x;
                x[0] = ob[4 * c + 0];
                x[1] = ob[4 * c + 1];
                x[2] = ob[4 * c + 2];
                x[3] = ob[4 * c + 3];
                dst[c] = x;
            }
            lds_store(&sh.prod[out_ring], min(max(r0 + kC - 63, 0), ny));
        }
    };

    for (int mb = 0; mb < m0; mb += P) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int m = mb + p;
            if (P > 4 && m >= nch) break;
            TS edgev[kC], ob[kC];
            left_values(m, edgev);
            run_chunk<TS, true>(s, m, bs[p], bq[p], be[p], edgev, mine, ob);
            issue_loads<TS>(s, m + P, bs[p], bq[p], be[p]);
            publish(m, ob);
        }
    }
    // [m0, m1): whole groups of P chunks without a bound check; then the remaining < P chunks
    const int m1 = m0 + (nch - m0) / P * P;
    for (int mb = m0; mb < m1; mb += P) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int m = mb + p;
            TS edgev[kC], ob[kC];
            left_values(m, edgev);
            run_chunk<TS, false>(s, m, bs[p], bq[p], be[p], edgev, mine, ob);
            issue_loads<TS>(s, m + P, bs[p], bq[p], be[p]);
            publish(m, ob);
        }
    }
#pragma unroll
    for (int p = 0; p < P - 1; ++p) {
        const int m = m1 + p;
        if (m < nch) {
            TS edgev[kC], ob[kC];
            left_values(m, edgev);
            run_chunk<TS, false>(s, m, bs[p], bq[p], be[p], edgev, mine, ob);
            publish(m, ob);
        }
    }
}

// Cross-workgroup hand-off.  Edge values and progress words are agent-scope atomics, which are
// performed at the device coherence point instead of in an XCD's L2, so neither side needs the
// L2-wide writeback / invalidate of a release or acquire at agent scope (both would also stall
// every other wavefront sharing that L2).  The writer waits for its edge stores to complete
// before it stores the progress word; the reader loads the edge values only after it has seen
// that word (wait_vm_stores).
//
// Helper wavefront: incoming edge (global -> ring[0]) and outgoing edge (ring[kWaves] -> global).
template <typename TS>
__device__ __forceinline__ void helper_wave(const SweepArgs<TS>& a, unsigned long long launch_id, Shared<TS>& sh, int S,
                                            int d, int lane) {
    constexpr int kWaves = kWavesOf<TS>;
    const int nx = a.nx, ny = a.ny;
    const bool incoming = S > 0;
    const bool outgoing = ((S + 1) * kWaves) * 64 < nx;   // the next superstrip has columns
    // (global address space, as the chunk pointers: no flat accesses on the LDS wait counter)
    const DLR_GLOBAL TS* edge_in =
        incoming ? (const DLR_GLOBAL TS*)(a.edge + ((size_t)d * a.nsuper + (S - 1)) * ny) : nullptr;
    DLR_GLOBAL TS* edge_out = outgoing ? (DLR_GLOBAL TS*)(a.edge + ((size_t)d * a.nsuper + S) * ny) : nullptr;
    DLR_GLOBAL unsigned long long* prog_in =
        incoming ? (DLR_GLOBAL unsigned long long*)&a.progress[(size_t)d * a.nsuper + S - 1] : nullptr;
    DLR_GLOBAL unsigned long long* prog_out =
        outgoing ? (DLR_GLOBAL unsigned long long*)&a.progress[(size_t)d * a.nsuper + S] : nullptr;
    const unsigned long long tag = launch_id << 32;
    int rin = incoming ? 0 : ny;    // rows copied into ring[0]
    int rout = outgoing ? 0 : ny;   // rows copied out of ring[kWaves]
    unsigned idle = 0;
    while (rin < ny || rout < ny) {
        bool moved = false;
        if (rin < ny) {
            const unsigned long long pv = __hip_atomic_load(prog_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int avail = (pv >> 32) == (launch_id & 0xffffffffull) ? (int)(pv & 0xffffffffull) : 0;
            avail = min(avail, lds_load(&sh.cons[0]) + kRing);   // ring space
            avail = min(avail, rin + 64);
            if (avail > rin) {
                const int row = rin + lane;
                if (row < avail)
                    sh.ring[0][(row + 63) & (kRing - 1)] =
                        __hip_atomic_load(&edge_in[row], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                rin = avail;
                lds_store(&sh.prod[0], rin);
                moved = true;
            }
        }
        if (rout < ny) {
            const int avail = min(lds_load(&sh.prod[kWaves]), rout + 64);
            if (avail > rout) {
                const int row = rout + lane;
                if (row < avail)
                    __hip_atomic_store(&edge_out[row], sh.ring[kWaves][(row + 63) & (kRing - 1)], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                rout = avail;
                lds_store(&sh.cons[kWaves], rout);
                wait_vm_stores();   // the edge values are performed before the progress word
                __hip_atomic_store(prog_out, tag | (unsigned long long)rout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
__global__ __launch_bounds__(64 * (kWavesOf<TS> + 1)) void k_sweep(const SweepArgs<TS>* __restrict__ table,
                                                                  SweepLaunch L) {
    constexpr int kWaves = kWavesOf<TS>;
    __shared__ Shared<TS> sh;
    __shared__ int inst, skip;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // with a launch counter every workgroup reads the id before the last one to retire advances it
    const unsigned long long launch_id = L.id_ctr ? __hip_atomic_load(L.id_ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                                  : L.launch_id;
    for (;;) {
        if (threadIdx.x == 0) {
            sh.task = atomicAdd(&L.ticket[0], 1u);
            sh.stall = 0;
            // instance of the unit: first k with unit_end[k] > task (binary search)
            int lo = 0, hi = L.ninst - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (L.unit_end[mid] > sh.task) hi = mid; else lo = mid + 1;
            }
            inst = lo;
            const int* sk = table[lo].skip;
            skip = (sh.task < L.total_units && sk) ? __hip_atomic_load(sk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                                   : 0;
        }
        if (threadIdx.x <= kWaves) {
            sh.prod[threadIdx.x] = 0;
            sh.cons[threadIdx.x] = 0;
        }
        __syncthreads();
        const unsigned n = sh.task;
        if (n >= L.total_units) break;
        const int k = __builtin_amdgcn_readfirstlane(inst);
        const SweepArgs<TS> a = table[k];
        const unsigned local = n - (k > 0 ? L.unit_end[k - 1] : 0u);
        const int S = (int)(local / (unsigned)a.nd);
        const int d = (int)(local % (unsigned)a.nd);
        if (skip) {
            // the instance's source iteration has stopped: none of its units runs, so none waits
        } else if (w < kWaves) {
            if ((S * kWaves + w) * 64 < a.nx) compute_wave<TS, P>(a, sh, S, d, w, lane);
        } else if ((S * kWaves) * 64 < a.nx) {
            helper_wave<TS>(a, launch_id, sh, S, d, lane);
        }
        __syncthreads();
        if (threadIdx.x == 0 && sh.stall) atomicOr(a.status, (int)kStatusSweepStall);
    }
    if (threadIdx.x == 0) {
        // the last workgroup to retire resets the ticket for the next launch on the stream
        const unsigned prev = atomicAdd(&L.ticket[1], 1u);
        if (prev == (unsigned)L.grid_blocks - 1u) {
            __hip_atomic_store(&L.ticket[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&L.ticket[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (L.id_ctr) {
                // the tags compare the low 32 bits: keep those at 2^31 or above (the host's ids are below)
                unsigned long long nx = launch_id + 1ull;
                if ((nx & 0xffffffffull) < (1ull << 31)) nx += 1ull << 31;
                __hip_atomic_store(L.id_ctr, nx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

}  // namespace

template <typename TS>
void launch_sweep(hipStream_t s, const SweepArgs<TS>* table, const SweepLaunch& L, int prefetch) {
    const dim3 g(L.grid_blocks), b(64 * (kWavesOf<TS> + 1));
    if (prefetch == 2)
        hipLaunchKernelGGL((k_sweep<TS, 2>), g, b, 0, s, table, L);
    else if (prefetch == 8)
        hipLaunchKernelGGL((k_sweep<TS, 8>), g, b, 0, s, table, L);
    else
        hipLaunchKernelGGL((k_sweep<TS, 4>), g, b, 0, s, table, L);
}
template void launch_sweep<double>(hipStream_t, const SweepArgs<double>*, const SweepLaunch&, int);
template void launch_sweep<float>(hipStream_t, const SweepArgs<float>*, const SweepLaunch&, int);

// Host ids stay in [1, 2^31) (the tags compare the low 32 bits; device launch counters use the
// upper half of that range).
unsigned long long next_sweep_launch_id() {
    static std::atomic<unsigned long long> id{0};
    return (++id - 1ull) % ((1ull << 31) - 1ull) + 1ull;
}

}  // namespace dlr
