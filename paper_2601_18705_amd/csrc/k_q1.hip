// Upwind sweep of the bilinear (Q1) discontinuous-Galerkin discretisation of the
// transport operator (Sec. 4.4: volume matrices G_j, upwind face matrix F_d, mass
// matrices) for nd directions: in every cell the 4 x 4 system
//   (-Omega . G_K + F_out + sigma_t M_K) psi_K = M_K s_K + F_in psi_upwind
// with the upwind neighbours' traces (or the inflow data) on the inflow faces.
//
// Local solve.  In the cell's upwind frame (node ix' = 0 on the x-inflow face, iy' = 0
// on the y-inflow face) the element matrices are tensor products of the 1D ones, and
// after multiplying by the inverse 1D mass matrices the system becomes a Kronecker sum,
//   (m (K (x) I) + e (I (x) K) + s I) psi = f,   K = [[3, 1], [-3, 1]],
// with m = |mu| hy, e = |eta| hx, s = sigma_t hx hy (all scaled by a common factor), and
//   f = hx hy s_nodal + m [4, -2] (x) g_x + e g_y (x) [4, -2]
// for the inflow traces g_x (two nodes of the x-inflow face) and g_y.  Eliminating the
// ix' = 0 block leaves a 2 x 2 system alpha K + beta I for the outflow column; K
// satisfies K^2 = 4K - 6I, so both 2 x 2 inverses are closed forms with one reciprocal
// each.  Everything that depends only on sigma_t (the two reciprocals and the
// coefficients) is computed before the inflow traces arrive; the part on the sweep's
// dependency chain is 24 fused multiply-adds.
//
// Work decomposition and hand-off follow the degree-0 sweep: in each direction's sweep
// coordinates the grid is cut into strips of 64 columns, kQ1Waves strips forming a
// superstrip; a workgroup takes one (superstrip, direction) unit with one compute
// wavefront per strip and one helper wavefront.  Lane l owns column 64 strip + l and at
// step t updates row t - l; the x-inflow traces (two values) come from lane l-1's
// previous step by DPP shifts and the y-inflow traces are the lane's own previous top
// face.  Neighbouring strips exchange their two x-face values per row through LDS rings;
// the helper wavefront copies the incoming edge (the previous superstrip's, or the inflow
// data for the first superstrip) into the first ring and the outgoing edge to global
// memory, publishing progress words tagged with the launch id.
//
// Memory.  Source, sigma_t and psi use the natural layouts (cell e = j*nx + i, node
// a = ix + 2*iy).  At one step the lanes of a wavefront touch 64 different rows, so
// loading each lane's cell directly would cost one cache-line lookup per lane; instead the
// cells of a chunk of kC steps (a diagonal band) move between HBM and LDS in runs of
// consecutive cells of a row, and each step reads and writes its cell in LDS.  Band loads
// run two chunks ahead in registers; cells outside the grid are read
// at clamped addresses and never stored.
#include "dlr_internal.h"
#include "wave_ops.h"

namespace dlr {

namespace {

constexpr int kW = kQ1Waves;   // compute wavefronts per workgroup
constexpr int kC = 8;          // steps per chunk
constexpr int kP = 2;          // chunks of band loads in flight per wavefront
constexpr int kRing = 256;     // LDS ring length (rows)

template <typename TS, int N>
struct Vec {
    typedef TS type __attribute__((ext_vector_type(N), aligned(N * sizeof(TS))));
};

// The cells one chunk of a compute wavefront touches form a band: sweep rows t0-63 .. t0+kC-1
// (row rho = r - t0 + 63), kC consecutive columns of each row.  The band is moved between HBM
// and LDS by row segments -- lane l of band operation q takes position l % kC of band row
// q kBandRowsPerOp + l / kC -- so one operation touches eight short runs of consecutive cells
// instead of 64 scattered ones; each step then reads its cell from LDS at [step][lane].
constexpr int kBandRows = 64 + kC - 1;
constexpr int kBandRowsPerOp = 64 / kC;
constexpr int kBandOps = (kBandRows + kBandRowsPerOp - 1) / kBandRowsPerOp;
constexpr int kSlot = 65;   // LDS stride of a step's row of slots (conflict-free band transfers)

template <typename TS>
struct Q1Shared {
    typename Vec<TS, 2>::type ring[kW + 1][kRing];   // ring[w]: x-inflow of compute wave w; ring[kW]: outgoing
                                                      // edge; row j in slot (j + 63) % kRing
    typename Vec<TS, 2>::type lo[kW][kC * kSlot + 1];   // band of wave w, [step][lane]: nodes 0, 1 of the source
    typename Vec<TS, 2>::type hi[kW][kC * kSlot + 1];   // nodes 2, 3 (then of psi, after the step); + a spare slot
    TS sig[kW][kC * kSlot + 1];                         // sigma_t
    int prod[kW + 1];   // rows published into ring[w]
    int cons[kW + 1];   // rows consumed from ring[w]
    int stall;
    unsigned task;
};

// Per-direction constants.  The local system is scaled by 1 / (hx hy) in FP64 (so the
// source enters unscaled) and by 1 / (|mu| hy + |eta| hx) in FP32, where it keeps the
// determinants of fine meshes within single-precision range.
template <typename TS>
constexpr bool kUnitArea = sizeof(TS) == 8;

template <typename TS>
struct Dir {
    TS m, e, H;                  // |mu| hy, |eta| hx, hx hy, each times the scale
    TS m4, m2n, e4, e2n;         // 4m, -2m, 4e, -2e: inflow weights of f
    TS m3, e3, e3n, e2;          // 3m, 3e, -3e, 2e
    TS ac, bc, d0c;              // alpha = ac + 2e s, beta = bc + s (4m + s), D0 = d0c + a (4e + a)
};

template <typename TS>
__device__ __forceinline__ Dir<TS> make_dir(double mu, double eta, double hx, double hy) {
    const double mp = fabs(mu) * hy, ep = fabs(eta) * hx;
    const double sc = kUnitArea<TS> ? 1.0 / (hx * hy) : 1.0 / (mp + ep);
    const double m = mp * sc, e = ep * sc;
    Dir<TS> q;
    q.m = (TS)m;
    q.e = (TS)e;
    q.H = (TS)(hx * hy * sc);
    q.m4 = (TS)(4.0 * m);
    q.m2n = (TS)(-2.0 * m);
    q.e4 = (TS)(4.0 * e);
    q.e2n = (TS)(-2.0 * e);
    q.m3 = (TS)(3.0 * m);
    q.e3 = (TS)(3.0 * e);
    q.e3n = (TS)(-3.0 * e);
    q.e2 = (TS)(2.0 * e);
    q.ac = (TS)(e * (4.0 * e + 4.0 * m));
    q.bc = (TS)(6.0 * (m - e) * (m + e));
    q.d0c = (TS)(6.0 * e * e);
    return q;
}

__device__ __forceinline__ double rcp(double x) {
    // hardware estimate refined by two Newton steps
    double r = __builtin_amdgcn_rcp(x);
    double t = fma(-x, r, 1.0);
    r = fma(r, t, r);
    t = fma(-x, r, 1.0);
    return fma(r, t, r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Coefficients of one cell's solve that do not depend on the inflow traces.
template <typename TS>
struct CellCoef {
    TS ga, gb;                 // 3e + a, e + a
    TS c1a, c1b, c1c, c1d;     // (alpha K' + beta I) / D1 with K' = 4I - K
    TS e0a, e0b, e0c, e0d;     // (e K' + a I) / D0
};

template <typename TS>
__device__ __forceinline__ CellCoef<TS> cell_coef(const Dir<TS>& q, TS sig) {
    const TS s = kUnitArea<TS> ? sig : sig * q.H;
    const TS a = q.m3 + s;
    const TS al = fma(q.e2, s, q.ac);
    const TS be = fma(s, q.m4 + s, q.bc);
    const TS t = al + al + be;
    const TS d1 = fma(t, t, (al + al) * al);   // D1 = 2 alpha^2 + (2 alpha + beta)^2
    const TS d0 = fma(a, q.e4 + a, q.d0c);     // D0 = 6e^2 + 4ea + a^2
    TS r1, r0;
    if constexpr (kUnitArea<TS>) {
        // one reciprocal for both: 1/D1 = D0 / (D0 D1), 1/D0 = D1 / (D0 D1)
        const TS r = rcp(d0 * d1);
        r1 = d0 * r;
        r0 = d1 * r;
    } else {
        r1 = rcp(d1);
        r0 = rcp(d0);
    }
    CellCoef<TS> c;
    c.ga = a + q.e3;
    c.gb = a + q.e;
    c.c1a = (al + be) * r1;
    c.c1b = -al * r1;
    c.c1c = (TS)3 * al * r1;
    c.c1d = fma((TS)3, al, be) * r1;
    c.e0a = c.gb * r0;
    c.e0b = -q.e * r0;
    c.e0c = q.e3 * r0;
    c.e0d = c.ga * r0;
    return c;
}

// Compute wavefront w of superstrip S for direction d; O = orientation (bit 0: mu <= 0,
// bit 1: eta <= 0), so the local <-> physical node permutation is resolved at compile time.
template <typename TS, int O>
__device__ __forceinline__ void q1_compute(const Q1Args<TS>& a, Q1Shared<TS>& sh, int S, int d, int w, int lane) {
    typedef typename Vec<TS, 4>::type V4;
    typedef typename Vec<TS, 2>::type V2;
    constexpr int FX = O & 1, FY = (O >> 1) & 1;
    // physical node of local node (ix', iy')
    constexpr int A00 = FX + 2 * FY, A10 = (1 ^ FX) + 2 * FY, A01 = FX + 2 * (1 ^ FY), A11 = (1 ^ FX) + 2 * (1 ^ FY);
    const int nx = a.nx, ny = a.ny;
    const int strip = S * kW + w;
    const int colp = strip * 64 + lane;
    const bool colok = colp < nx;
    const int ic = colok ? (FX ? nx - 1 - colp : colp) : (FX ? 0 : nx - 1);
    const Dir<TS> q = make_dir<TS>(a.mu[d], a.eta[d], a.hx, a.hy);
    const size_t ncell = (size_t)nx * ny;
    const TS* srcd = a.src + (size_t)d * ncell * 4;
    TS* psid = a.psi + (size_t)d * ncell * 4;
    const bool has_next = (strip + 1) * 64 < nx;
    const int out_ring = (w < kW - 1) ? w + 1 : kW;
    const int nch = (ny + 63 + kC - 1) / kC;   // >= 64 / kC
    const int jbase = FY ? ny - 1 : 0, jsign = FY ? -1 : 1;
    const int i0 = strip * 64;
    const int bk = lane % kC, brho = lane / kC;   // position and row offset of this lane in a band operation
    typename Vec<TS, 2>::type* const slo = sh.lo[w];
    typename Vec<TS, 2>::type* const shi = sh.hi[w];
    TS* const ssig = sh.sig[w];

    // y-inflow traces of the lane's first row, local node order ix'
    const V2 yin = *reinterpret_cast<const V2*>(a.iny + ((size_t)d * nx + ic) * 2);
    TS top0 = FX ? yin[1] : yin[0], top1 = FX ? yin[0] : yin[1];
    TS rgt0 = (TS)0, rgt1 = (TS)0;   // right-face values of the previous step (to lane + 1)

    // Band geometry of this lane, the same for every chunk: operation q covers band row
    // rho = q kBandRowsPerOp + brho and strip column l = bk + 63 - rho, i.e. sweep row
    // r = kC m - 63 + rho of chunk m.  The cell index is linear in q and m; an index outside
    // the array belongs to a piece no step uses and is clamped, so loads stay in bounds.
    const int isign = FX ? -1 : 1;
    const int dq = kBandRowsPerOp * (jsign * nx - isign);
    const int dm = kC * jsign * nx;
    const int e00 = (jbase + jsign * (brho - 63)) * nx + (FX ? nx - 1 - i0 : i0) + isign * (bk + 63 - brho);
    const int emax = nx * ny - 1;
    unsigned okmask = 0;        // bit q: the piece lies in the band and its column in the grid
    int slot[kBandOps];         // LDS slot of each piece (the spare slot when outside the band)
#pragma unroll
    for (int q = 0; q < kBandOps; ++q) {
        const int rho = q * kBandRowsPerOp + brho;
        const int l = bk + 63 - rho;
        const bool inband = rho < kBandRows && l >= 0 && l < 64;
        slot[q] = inband ? bk * kSlot + l : kC * kSlot;
        okmask |= (inband && i0 + l < nx) ? 1u << q : 0u;
    }
    auto band_index = [&](int m, int q) -> unsigned {
        return (unsigned)min(max(e00 + m * dm + q * dq, 0), emax);
    };
    auto issue = [&](int m, V4 (&vs)[kBandOps], TS (&vq)[kBandOps]) {
        const int mc = min(m, nch - 1);
#pragma unroll
        for (int q = 0; q < kBandOps; ++q) {
            const unsigned e = band_index(mc, q);
            vs[q] = *reinterpret_cast<const V4*>(srcd + (size_t)e * 4);
            vq[q] = a.sig[e];
        }
    };
    auto stage = [&](const V4 (&vs)[kBandOps], const TS (&vq)[kBandOps]) {
#pragma unroll
        for (int q = 0; q < kBandOps; ++q) {
            slo[slot[q]] = V2{vs[q][0], vs[q][1]};
            shi[slot[q]] = V2{vs[q][2], vs[q][3]};
            ssig[slot[q]] = vq[q];
        }
    };
    auto flush = [&](int m) {
        V2 xv[kBandOps], yv[kBandOps];
#pragma unroll
        for (int q = 0; q < kBandOps; ++q) {
            xv[q] = slo[slot[q]];
            yv[q] = shi[slot[q]];
        }
#pragma unroll
        for (int q = 0; q < kBandOps; ++q) {
            const int r = kC * m - 63 + q * kBandRowsPerOp + brho;
            if (((okmask >> q) & 1u) && (unsigned)r < (unsigned)ny)
                *reinterpret_cast<V4*>(psid + (size_t)band_index(m, q) * 4) = V4{xv[q][0], xv[q][1], yv[q][0], yv[q][1]};
        }
    };
    auto left_values = [&](int m, V2 (&ev)[kC]) {
        const int r0 = kC * m;
        if (r0 >= ny) {
#pragma unroll
            for (int k = 0; k < kC; ++k) ev[k] = V2{(TS)0, (TS)0};
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
        for (int k = 0; k < kC; ++k) ev[k] = sh.ring[w][(r0 + k + 63) & (kRing - 1)];
        lds_store(&sh.cons[w], need);
    };
    auto publish = [&](int m, const V2 (&ob)[kC]) {
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
            // lane 63's rows r0-63 .. r0-63+kC-1 sit in slots r0 .. r0+kC-1; rows outside
            // [0, ny) land in slots no pending row occupies
#pragma unroll
            for (int k = 0; k < kC; ++k) sh.ring[out_ring][(r0 + k) & (kRing - 1)] = ob[k];
            lds_store(&sh.prod[out_ring], min(max(r0 + kC - 63, 0), ny));
        }
    };
    // MASK: chunks that contain steps before the lane's first row (t < lane), whose results
    // must not replace the y-inflow traces
    auto run_chunk = [&](int m, const V2 (&ev)[kC], V2 (&ob)[kC], auto mask_tag) {
        constexpr bool MASK = decltype(mask_tag)::value;
        // the chunk's inputs are read from LDS before any result is written back, so the
        // reads are not held behind the stores of earlier steps
        V2 xs[kC], ys[kC];
        TS gs[kC];
#pragma unroll
        for (int k = 0; k < kC; ++k) {
            xs[k] = slo[k * kSlot + lane];
            ys[k] = shi[k * kSlot + lane];
            gs[k] = ssig[k * kSlot + lane];
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
#pragma unroll
        for (int k = 0; k < kC; ++k) {
            const int t = kC * m + k;
            const CellCoef<TS> c = cell_coef<TS>(q, gs[k]);
            const V4 sv = V4{xs[k][0], xs[k][1], ys[k][0], ys[k][1]};
            const TS h00 = kUnitArea<TS> ? sv[A00] : q.H * sv[A00], h10 = kUnitArea<TS> ? sv[A10] : q.H * sv[A10];
            const TS h01 = kUnitArea<TS> ? sv[A01] : q.H * sv[A01], h11 = kUnitArea<TS> ? sv[A11] : q.H * sv[A11];
            const TS f00p = fma(q.e4, top0, h00), f10p = fma(q.e4, top1, h10);
            const TS f01p = fma(q.e2n, top0, h01), f11p = fma(q.e2n, top1, h11);
            const TS gx0 = shift_in(ev[k][0], rgt0), gx1 = shift_in(ev[k][1], rgt1);
            const TS f00 = fma(q.m4, gx0, f00p), f10 = fma(q.m2n, gx0, f10p);
            const TS f01 = fma(q.m4, gx1, f01p), f11 = fma(q.m2n, gx1, f11p);
            const TS g0 = fma(c.ga, f10, fma(q.e, f11, q.m3 * f00));
            const TS g1 = fma(q.e3n, f10, fma(c.gb, f11, q.m3 * f01));
            const TS p10 = fma(c.c1a, g0, c.c1b * g1);
            const TS p11 = fma(c.c1c, g0, c.c1d * g1);
            const TS hh0 = fma(-q.m, p10, f00), hh1 = fma(-q.m, p11, f01);
            const TS p00 = fma(c.e0a, hh0, c.e0b * hh1);
            const TS p01 = fma(c.e0c, hh0, c.e0d * hh1);
            V4 out;
            out[A00] = p00;
            out[A10] = p10;
            out[A01] = p01;
            out[A11] = p11;
            const int jp = t - lane;
            slo[k * kSlot + lane] = V2{out[0], out[1]};
            shi[k * kSlot + lane] = V2{out[2], out[3]};
            rgt0 = p10;
            rgt1 = p11;
            if (MASK) {
                const bool act = jp >= 0;
                top0 = act ? p01 : top0;
                top1 = act ? p11 : top1;
            } else {
                top0 = p01;
                top1 = p11;
            }
            ob[k] = V2{p10, p11};
        }
    };

    // Per chunk: stage its band (loaded two chunks ahead) into LDS, prefetch the band of the
    // chunk after next, run the steps, write psi back by row segments, publish the edge.
    V4 bs[kP][kBandOps];
    TS bq[kP][kBandOps];
#pragma unroll
    for (int p = 0; p < kP; ++p) issue(p, bs[p], bq[p]);
    auto chunk = [&](int m, int p, bool prefetch, auto mask_tag) {
        V2 ev[kC], ob[kC];
        left_values(m, ev);
        stage(bs[p], bq[p]);
        if (prefetch) issue(m + kP, bs[p], bq[p]);
        run_chunk(m, ev, ob, mask_tag);
        flush(m);
        publish(m, ob);
    };
    // chunks [0, m0) carry the skewed head (masked), with m0 a multiple of kP
    constexpr int m0 = (64 / kC + kP - 1) / kP * kP;
    for (int mb = 0; mb < m0; mb += kP) {
#pragma unroll
        for (int p = 0; p < kP; ++p) chunk(mb + p, p, true, std::true_type{});
    }
    const int m1 = m0 + (nch - m0) / kP * kP;
    for (int mb = m0; mb < m1; mb += kP) {
#pragma unroll
        for (int p = 0; p < kP; ++p) chunk(mb + p, p, true, std::false_type{});
    }
#pragma unroll
    for (int p = 0; p < kP - 1; ++p)
        if (m1 + p < nch) chunk(m1 + p, p, false, std::false_type{});
}

// Helper wavefront: incoming edge (the previous superstrip's published values, or the
// inflow data of the x-inflow boundary) -> ring[0], and ring[kW] -> the outgoing edge.
// Edge values and progress words are agent-scope atomics, performed at the device
// coherence point rather than in one XCD's L2; the writer waits for its edge stores
// before it stores the progress word, the reader loads edge values only after seeing it.
template <typename TS>
__device__ __forceinline__ void q1_helper(const Q1Args<TS>& a, Q1Shared<TS>& sh, int S, int d, bool fy, int lane) {
    typedef typename Vec<TS, 2>::type V2;
    const int nx = a.nx, ny = a.ny;
    const bool from_edge = S > 0;
    const bool outgoing = (S + 1) * kW * 64 < nx;
    const TS* edge_in = from_edge ? a.edge + ((size_t)d * a.nsuper + (S - 1)) * ny * 2 : nullptr;
    const TS* inflow = a.inx + (size_t)d * ny * 2;
    TS* edge_out = outgoing ? a.edge + ((size_t)d * a.nsuper + S) * ny * 2 : nullptr;
    unsigned long long* prog_in = from_edge ? &a.progress[(size_t)d * a.nsuper + S - 1] : nullptr;
    unsigned long long* prog_out = outgoing ? &a.progress[(size_t)d * a.nsuper + S] : nullptr;
    const unsigned long long tag = a.launch_id << 32;
    int rin = 0;                    // rows copied into ring[0]
    int rout = outgoing ? 0 : ny;   // rows copied out of ring[kW]
    unsigned idle = 0;
    while (rin < ny || rout < ny) {
        bool moved = false;
        if (rin < ny) {
            int avail = ny;
            if (from_edge) {
                const unsigned long long pv = __hip_atomic_load(prog_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                avail = (pv >> 32) == (a.launch_id & 0xffffffffull) ? (int)(pv & 0xffffffffull) : 0;
            }
            avail = min(avail, lds_load(&sh.cons[0]) + kRing);   // ring space
            avail = min(avail, rin + 64);
            if (avail > rin) {
                const int row = rin + lane;
                if (row < avail) {
                    V2 v;
                    if (from_edge) {
                        v[0] = __hip_atomic_load(&edge_in[2 * row], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        v[1] = __hip_atomic_load(&edge_in[2 * row + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        // sweep row -> physical row, physical node iy -> local iy'
                        const V2 x = *reinterpret_cast<const V2*>(inflow + 2 * (fy ? ny - 1 - row : row));
                        v[0] = fy ? x[1] : x[0];
                        v[1] = fy ? x[0] : x[1];
                    }
                    sh.ring[0][(row + 63) & (kRing - 1)] = v;
                }
                rin = avail;
                lds_store(&sh.prod[0], rin);
                moved = true;
            }
        }
        if (rout < ny) {
            const int avail = min(lds_load(&sh.prod[kW]), rout + 64);
            if (avail > rout) {
                const int row = rout + lane;
                if (row < avail) {
                    const V2 v = sh.ring[kW][(row + 63) & (kRing - 1)];
                    __hip_atomic_store(&edge_out[2 * row], v[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&edge_out[2 * row + 1], v[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                rout = avail;
                lds_store(&sh.cons[kW], rout);
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
                    lds_store(&sh.cons[kW], 1 << 30);
                }
                break;
            }
        } else {
            idle = 0;
        }
    }
}

template <typename TS>
__global__ __launch_bounds__(64 * (kW + 1)) void k_q1_sweep(Q1Args<TS> a) {
    __shared__ Q1Shared<TS> sh;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (;;) {
        if (threadIdx.x == 0) {
            sh.task = atomicAdd(&a.ticket[0], 1u);
            sh.stall = 0;
        }
        if (threadIdx.x <= kW) {
            sh.prod[threadIdx.x] = 0;
            sh.cons[threadIdx.x] = 0;
        }
        __syncthreads();
        const unsigned n = sh.task;
        if (n >= a.total_units) break;
        const int S = (int)(n / (unsigned)a.nd);
        const int d = (int)(n % (unsigned)a.nd);
        const int o = orient_of(a.mu[d], a.eta[d]);
        if (w < kW) {
            if ((S * kW + w) * 64 < a.nx) {
                switch (o) {
                    case 0: q1_compute<TS, 0>(a, sh, S, d, w, lane); break;
                    case 1: q1_compute<TS, 1>(a, sh, S, d, w, lane); break;
                    case 2: q1_compute<TS, 2>(a, sh, S, d, w, lane); break;
                    default: q1_compute<TS, 3>(a, sh, S, d, w, lane); break;
                }
            }
        } else {
            q1_helper<TS>(a, sh, S, d, (o & 2) != 0, lane);
        }
        __syncthreads();
        if (threadIdx.x == 0 && sh.stall) atomicOr(a.status, (int)kStatusSweepStall);
    }
    if (threadIdx.x == 0) {
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
void launch_q1_sweep(hipStream_t s, const Q1Args<TS>& a) {
    hipLaunchKernelGGL(k_q1_sweep<TS>, dim3(a.grid_blocks), dim3(64 * (kW + 1)), 0, s, a);
}
template void launch_q1_sweep<double>(hipStream_t, const Q1Args<double>&);
template void launch_q1_sweep<float>(hipStream_t, const Q1Args<float>&);

}  // namespace dlr
