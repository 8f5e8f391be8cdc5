// Upwind transport sweep for the selected directions (Algorithm 1 step 4): one
// application of the inverse of the degree-0 upwind operator plus sigma_t,
//   psi_e = (src0_e + s_e + ax psi_upwind_x + ay psi_upwind_y) / (sigma_t,e + ax + ay),
// ax = |mu|/hx, ay = |eta|/hy, for every direction d and cell e.
//
// Work decomposition.  In each direction's own sweep coordinates (i', j') --
// i' = i for mu > 0 else nx-1-i, likewise j' -- the grid is cut into strips of
// 64 columns.  A unit of work is (strip s, direction d) and is run by one
// wavefront: lane l owns column i' = 64 s + l and at step t handles row
// j' = t - l.  The x-upwind value of lane l is lane l-1's result of the previous
// step (a lane shift), the y-upwind value is the lane's own previous result, so
// the anti-diagonal recurrence runs with no barrier at all.  Lane 0 takes its
// x-upwind value from the strip to its left, which publishes its last column in
// chunks of rows through a global edge buffer and a release-stored progress
// word tagged with the launch id.  Units are handed out through an atomic
// ticket in (strip, direction) order, so a wave only ever waits on a unit with
// a smaller ticket, i.e. one that is already running: the scheme cannot
// deadlock whatever the number of resident waves.
#include "dlr_internal.h"

namespace dlr {

namespace {

template <typename TS>
__global__ __launch_bounds__(64) void k_sweep(SweepArgs<TS> a) {
    const int lane = threadIdx.x;
    const size_t N = (size_t)a.nx * a.ny;
    for (;;) {
        unsigned n = 0;
        if (lane == 0) n = atomicAdd(&a.ticket[0], 1u);
        n = __shfl(n, 0);
        if (n >= (unsigned)a.total_units) break;
        const int s = (int)(n / (unsigned)a.nd);
        const int d = (int)(n % (unsigned)a.nd);
        const double mu = a.mu[d], eta = a.eta[d];
        const TS ax = (TS)(fabs(mu) * a.inv_hx);
        const TS ay = (TS)(fabs(eta) * a.inv_hy);
        const TS den_add = ax + ay;
        const int ip = s * 64 + lane;
        const bool col_ok = ip < a.nx;
        const int i = mu > 0.0 ? ip : a.nx - 1 - ip;
        const TS bx = (TS)a.inflow_x[d];
        const TS by = (TS)a.inflow_y[d];
        const TS* __restrict__ src = a.src0 + (size_t)d * N;
        TS* __restrict__ out = a.psi + (size_t)d * N;
        const TS* edge_in = (s > 0) ? a.edge + ((size_t)d * a.nstrips + (s - 1)) * a.ny : nullptr;
        TS* edge_out = (s + 1 < a.nstrips) ? a.edge + ((size_t)d * a.nstrips + s) * a.ny : nullptr;
        unsigned long long* prog_in = (s > 0) ? &a.progress[(size_t)d * a.nstrips + s - 1] : nullptr;
        unsigned long long* prog_out = &a.progress[(size_t)d * a.nstrips + s];
        const unsigned long long tag = a.launch_id << 32;
        TS mine = (TS)0;
        int avail = 0;
        for (int t = 0; t < a.ny + 63; ++t) {
            TS from_left = __shfl_up(mine, 1);
            if (t < a.ny) {
                if (s == 0) {
                    if (lane == 0) from_left = bx;
                } else {
                    if (t >= avail) {
                        const int need = min(t + kSweepChunk, a.ny);
                        const unsigned long long want = tag | (unsigned long long)need;
                        // Bounded wait: a producer that never publishes (a bug) ends the wait with
                        // an error flag instead of hanging the device.
                        unsigned polls = 0;
                        while (__hip_atomic_load(prog_in, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < want) {
                            __builtin_amdgcn_s_sleep(1);
                            if (++polls > a.spin_limit) {
                                if (lane == 0) atomicOr(a.status, (int)kStatusSweepStall);
                                break;
                            }
                        }
                        avail = need;
                    }
                    if (lane == 0) from_left = edge_in[t];
                }
            }
            const int jp = t - lane;
            if (col_ok && jp >= 0 && jp < a.ny) {
                const int j = eta > 0.0 ? jp : a.ny - 1 - jp;
                const size_t e = (size_t)j * a.nx + i;
                const TS up_y = (jp == 0) ? by : mine;
                const TS val = (src[e] + a.s_e[e] + ax * from_left + ay * up_y) / (a.sig_t[e] + den_add);
                out[e] = val;
                mine = val;
                if (lane == 63 && edge_out != nullptr) {
                    edge_out[jp] = val;
                    if (((jp + 1) % kSweepChunk) == 0 || jp + 1 == a.ny)
                        __hip_atomic_store(prog_out, tag | (unsigned long long)(jp + 1), __ATOMIC_RELEASE,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
    // The last wave to retire resets the ticket for the next launch on the stream.
    if (lane == 0) {
        const unsigned prev = atomicAdd(&a.ticket[1], 1u);
        if (prev == (unsigned)a.grid_waves - 1u) {
            __hip_atomic_store(&a.ticket[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.ticket[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace

template <typename TS>
void launch_sweep(hipStream_t s, const SweepArgs<TS>& a) {
    hipLaunchKernelGGL((k_sweep<TS>), dim3(a.grid_waves), dim3(64), 0, s, a);
}
template void launch_sweep<double>(hipStream_t, const SweepArgs<double>&);
template void launch_sweep<float>(hipStream_t, const SweepArgs<float>&);

}  // namespace dlr
