// sweep2d.hip -- diamond-difference transport sweep in x-y geometry for a
// batch of instances of uneven size (the transport sweep of the S_N source
// iteration, arXiv 2509.01416 section 5.1 after Eq. 20), fused with the
// quadrature reduction to the scalar flux (Eq. 17).
//
// Per direction m and cell, with a = 2|mu|/dx, b = 2|eta|/dy:
//     psi = (Q + a psi_x_in + b psi_y_in) / (sigma_t + a + b)
//     psi_x_out = 2 psi - psi_x_in,   psi_y_out = 2 psi - psi_y_in
//     phi += w_m psi
//
// Work decomposition (one workgroup per (instance, octant, direction slice)):
//   * a lane owns one row of cells and walks it in the octant's x order; a
//     wave holds 64/R segments of R lanes, all on the same R rows, each with
//     its own D directions;
//   * lane r of a segment is one step behind lane r-1, so the y-face flux it
//     needs was produced by lane r-1 on the previous step and arrives by a
//     lane shuffle (the diagonal wavefront of the row block);
//   * when a lane finishes its row it continues with the row R above it, so
//     a segment streams through ceil(ny/R) row blocks without pipeline
//     drain; the first lane of a block receives the y-face flux of the last
//     lane of the previous block through a small LDS ring (written nx-R+1
//     steps earlier, R <= nx);
//   * the steps are processed in blocks of KB.  The (sigma_t, Q) pairs a
//     block needs (KB steps x R rows, identical for every wave) are loaded
//     cooperatively and coalesced one block ahead and staged in LDS, so the
//     HBM latency hides behind a block of compute;
//   * the W waves of the workgroup process identical cells at identical
//     steps, each for its own directions; their partial scalar fluxes are
//     combined in LDS after each block, in fixed wave order, and one partial
//     plane per (octant, slice) is written to HBM.  The planes are summed in
//     fixed order by the combine kernel, so the result is bitwise
//     reproducible (no floating-point atomics);
//   * angular fluxes never leave the chip except on boundary faces, which are
//     stored for reflective inflow (lagged one iteration) and leakage.
//   * linearly anisotropic scattering (P1, section 5.1 Eq. 25; generic
//     kernel, one direction per lane): the emission of direction m is
//     Q + mu_m Ex + eta_m Ey with Ex, Ey = 3 sigma_s1 J staged like Q, and
//     the waves also sum w mu psi and w eta psi into current planes.
#include "combine_dev.h"
#include "common.h"

namespace mdp {

constexpr int kMaxPrefetch = 4;   // staged values per thread per block
constexpr int kMaxRed = 2;        // reduced outputs per thread per block
constexpr int kMaxPos = 4;        // staging/reduction positions per helper thread
#ifndef MDP_STEP_AHEAD
#define MDP_STEP_AHEAD 6
#endif
#ifndef MDP_HELPER_SPLIT
#define MDP_HELPER_SPLIT 1
#endif
constexpr int kStepAhead = MDP_STEP_AHEAD;   // LDS read distance of the step loop (steps)

// Largest workgroup per directions-per-lane D, so that the register budget
// (512 per SIMD lane / waves per SIMD) holds D directions without spills.
template <int D>
struct SweepBounds {
    static constexpr int threads = D <= 2 ? 1024 : (D <= 4 ? 512 : 256);
};

// Global-address-space views: loads and stores through them are global_*
// instructions (counted on vmcnt only), never flat ones.
#define MDP_GLOBAL __attribute__((address_space(1)))
typedef MDP_GLOBAL float gfloat;
typedef const MDP_GLOBAL float cgfloat;

// Position of a (step, row) pair of the segment stream: u = t - row is split
// as u = kk*nx + ip; the cursor advances by whole blocks without division.
struct Cursor {
    int ip, kk;
    __device__ __forceinline__ void advance(int by, int nx) {
        ip += by;
        while (ip >= nx) { ip -= nx; ++kk; }
    }
};

// Cell of row rr at cursor c, or -1 outside the grid / before the start.
__device__ __forceinline__ int cursor_cell(Cursor c, int rr, int R, int nx,
                                           int ny, int nblk, bool xpos,
                                           bool ypos) {
    if (c.ip < 0 || c.ip >= nx || c.kk >= nblk) return -1;
    const int jp = c.kk * R + rr;
    if (jp >= ny) return -1;
    const int i = xpos ? c.ip : nx - 1 - c.ip;
    const int j = ypos ? jp : ny - 1 - jp;
    return j * nx + i;
}

// REFL: some inflow face of this launch is reflective (face loads inside the
// step loop); the vacuum instance has no global loads in the loop at all.
// KB: steps per block (a power of two); the step loop is fully unrolled.
template <int D, bool REFL, int KB, bool P1 = false>
__global__ void __launch_bounds__(SweepBounds<D>::threads)
sweep2d_kernel(const InstDesc* __restrict__ insts,
               const SweepWork* __restrict__ work,
               const DirTable* __restrict__ dt, const int* __restrict__ done,
               const int* __restrict__ iter, int use_faces, FinArgs fin) {
    extern __shared__ float smem[];
    constexpr int lkb = KB >= 16 ? 4 : (KB >= 8 ? 3 : (KB >= 4 ? 2 : (KB >= 2 ? 1 : 0)));
    static_assert((1 << lkb) == KB, "KB must be a power of two <= 16");
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int W = blockDim.x >> 6;
    const int nthreads = blockDim.x;
    const SweepWork wk = work[blockIdx.x];
    const int n = wk.inst;
    if (n < 0) return;                        // XCD alignment padding
    if (fin.pending) {   // uniform over the workgroup
        if (sweep_prologue(insts[n], n, fin, wk.oct == 0 && wk.slice == 0)) return;
    } else if (done != nullptr && done[n]) {
        return;
    }
    const InstDesc& I = insts[n];
    const int R = I.R, lr = __ffs(R) - 1;
    const int nseg = 64 >> lr, seg = lane >> lr, r = lane & (R - 1);
    const int o = wk.oct;
    const bool xpos = (o == 0 || o == 3), ypos = (o == 0 || o == 1);
    const int nx = I.nx, ny = I.ny, nf = I.nf, M = dt->M;
    const int par = (fin.pending ? fin.it : (iter != nullptr ? iter[n] : 0)) & 1;
    const size_t fstride = (size_t)4 * nf * M;
    cgfloat* __restrict__ fprev = (cgfloat*)(I.face + (size_t)par * fstride);
    gfloat* __restrict__ fcur = (gfloat*)(I.face + (size_t)(par ^ 1) * fstride);
    const int fxin = xpos ? 0 : 1, fxout = xpos ? 1 : 0;
    const int fyin = ypos ? 2 : 3, fyout = ypos ? 3 : 2;
    const bool rx = REFL && use_faces && I.bc[fxin] == 1;
    const bool ry = REFL && use_faces && I.bc[fyin] == 1;

    static_assert(!P1 || D == 1, "anisotropic emission: one direction per lane");
    constexpr int NF = P1 ? 4 : 2;    // staged fields: sigma_t, Q (, Ex, Ey)
    constexpr int NPB = P1 ? 3 : 1;   // partial sums: phi (, Jx, Jy)
    constexpr int MPF = P1 ? 2 * kMaxPrefetch : kMaxPrefetch;   // staging slots per thread
    float a[D], b[D], c[D], w[D], smu[D], seta[D];
    int mi[D], mxr[D], myr[D];
    const int nd = dt->count[o];
    const int base = wk.slice * (W * nseg * D) + (wv * nseg + seg) * D;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int kk = base + d;
        if (kk < nd) {
            const int m = dt->list[o][kk];
            a[d] = 2.0f * dt->amu[m] * I.inv_dx;
            b[d] = 2.0f * dt->aeta[m] * I.inv_dy;
            w[d] = dt->w[m];
            smu[d] = dt->mu[m];
            seta[d] = dt->eta[m];
            mi[d] = m;
            mxr[d] = dt->mirx[m];
            myr[d] = dt->miry[m];
        } else {
            a[d] = 0.f; b[d] = 0.f; w[d] = 0.f; smu[d] = 0.f; seta[d] = 0.f;
            mi[d] = -1; mxr[d] = 0; myr[d] = 0;
        }
        c[d] = a[d] + b[d];
    }
    // one direction per wave and one segment per wave (D = 1, R = 64): the
    // direction weight is applied in the cross-wave sums instead of the
    // step, as the specialised kernel does (same operations, same order)
    const bool fold = !P1 && D == 1 && nseg == 1;
    const float wm = fold ? 1.0f : w[0];
    __shared__ float wsh[16];   // weight of each wave's direction (W <= 16)
    if (tid < 16) {
        const int kk = wk.slice * W + tid;
        wsh[tid] = tid < W && kk < nd ? dt->w[dt->list[o][kk]] : 0.f;
    }

    // LDS: pbuf[NPB][2][KB][W*64+1] | sbuf[2][NF][KB][65] | ring[W][nseg][D][nx]
    //      | sink[W][D][nx] (target of the ring store of non-writing lanes).
    // The +1 pads make the block-level staging stores and reduction reads,
    // whose consecutive threads step through KB rows, conflict-free.
    const int PSTR = W * 64 + 1;
    const int PBS = 2 * KB * PSTR;   // one partial-sum buffer
    float* pbuf = smem;
    float* sbuf = smem + NPB * PBS;
    float* rings = sbuf + 2 * NF * KB * 65;
    float* ring = rings + (size_t)((wv * nseg + seg) * D) * nx;
    float* sink = rings + (size_t)W * nseg * D * nx + (size_t)wv * D * nx;
    const int nblk = (ny + R - 1) >> lr;
    const int T = nblk * nx + R - 1;
    cgfloat* __restrict__ St = (cgfloat*)I.st;
    cgfloat* __restrict__ Qb = (cgfloat*)I.Q;
    cgfloat* __restrict__ Exb = (cgfloat*)I.Ex;
    cgfloat* __restrict__ Eyb = (cgfloat*)I.Ey;
    gfloat* __restrict__ part = (gfloat*)(I.part + (size_t)(o * I.S + wk.slice) * I.cells);
    gfloat* __restrict__ partx =
        P1 ? (gfloat*)(I.partJ + (size_t)(o * I.S + wk.slice) * I.cells) : nullptr;
    gfloat* __restrict__ party =
        P1 ? (gfloat*)(I.partJ + (size_t)(I.P + o * I.S + wk.slice) * I.cells) : nullptr;

    // Staging slots of this thread: element e = (field, row, step) packed as
    // f << (lr+lkb) | rr << lkb | t2; each keeps a cursor for its (step, row).
    const int nstage = NF * KB * R;
    const int npf = (nstage + nthreads - 1) / nthreads;   // slots in use
    float pf[MPF];
    bool pv[MPF];
    Cursor sc[MPF];
#pragma unroll
    for (int jx = 0; jx < MPF; ++jx) {
        const int e = tid + jx * nthreads;
        sc[jx].ip = (e & (KB - 1)) - ((e >> lkb) & (R - 1));
        sc[jx].kk = 0;
        sc[jx].advance(0, nx);   // normalise: 0 <= ip < nx once ip >= 0
    }
    // all addresses first, then unconditional loads back to back (an empty
    // slot reads cell 0); the per-slot default is applied at store time
    auto stage_load = [&]() {
        int cells[MPF];
#pragma unroll
        for (int jx = 0; jx < MPF; ++jx) {
            if (jx >= npf) break;
            const int e = tid + jx * nthreads;
            const int rr = (e >> lkb) & (R - 1);
            const int cell = cursor_cell(sc[jx], rr, R, nx, ny, nblk, xpos, ypos);
            pv[jx] = cell >= 0 && e < nstage;
            cells[jx] = pv[jx] ? cell : 0;
            sc[jx].advance(KB, nx);
        }
#pragma unroll
        for (int jx = 0; jx < MPF; ++jx) {
            if (jx >= npf) break;
            const int e = tid + jx * nthreads;
            // field of the slot; padding slots (e >= nstage, f >= NF) read
            // cell 0 of a field that exists (Ex and Ey only with P1)
            const int f = e >> (lkb + lr);
            cgfloat* src = St;
            if (f == 1) src = Qb;
            else if (f >= 2) src = P1 ? (f == 2 ? Exb : Eyb) : Qb;
            pf[jx] = src[cells[jx]];
        }
    };
    auto stage_store = [&](int h) {
#pragma unroll
        for (int jx = 0; jx < MPF; ++jx) {
            if (jx >= npf) break;
            const int e = tid + jx * nthreads;
            if (e < nstage) {
                const int f = e >> (lkb + lr);
                const int rr = (e >> lkb) & (R - 1);
                const int t2 = e & (KB - 1);
                const float def = f == 0 ? 1.f : 0.f;
                sbuf[((h * NF + f) * KB + t2) * 65 + rr] = pv[jx] ? pf[jx] : def;
            }
        }
    };
    // Reduction slots: output e = rr << lkb | t2 of a block.
    const int nout = KB * R;
    const int nredu = (nout + nthreads - 1) / nthreads;
    Cursor rc_[kMaxRed];
#pragma unroll
    for (int jx = 0; jx < kMaxRed; ++jx) {
        const int e = tid + jx * nthreads;
        rc_[jx].ip = (e & (KB - 1)) - (e >> lkb);
        rc_[jx].kk = 0;
        rc_[jx].advance(0, nx);
    }

    // The ring of each wave segment starts with the y-inflow boundary (the
    // "row block -1"), so the first lane of a segment always takes its
    // incoming y flux from the ring: vacuum zero or the reflected face.
    for (int e = r; e < D * nx; e += R) {
        const int d = e / nx, ipc = e - d * nx;
        float v = 0.f;
#pragma unroll
        for (int dd = 0; dd < D; ++dd) {
            if (dd == d && REFL && ry && mi[dd] >= 0) {
                const int i = xpos ? ipc : nx - 1 - ipc;
                v = fprev[((size_t)fyin * nf + i) * M + myr[dd]];
            }
        }
        ring[e] = v;
    }
    stage_load();
    stage_store(0);
    __syncthreads();

    float xin[D], yo[D];
#pragma unroll
    for (int d = 0; d < D; ++d) { xin[d] = 0.f; yo[d] = 0.f; }
    const bool first = r == 0;
    // R divides ny (the planner guarantees it), so the top row of every row
    // block is lane R-1: it alone stores into the ring, the other lanes store
    // into the sink.  Before its first cell (ip < 0) lane R-1 stores into
    // column 0, which lane 0 has already read and which lane R-1 rewrites on
    // reaching it.
    float* wbase = (r == R - 1) ? ring : sink;
    int ip = -r, k = 0;   // position of this lane: cell ip of row block k

    // One wavefront step.  tt: step within the block; ld/stg: issue the next
    // block's staging loads / store them to LDS on this step.
    auto step = [&](int tt, const float* sp, float* pw, bool ld, bool stg, int half) {
        if (ld) stage_load();
        const float st = sp[tt * 65];
        const float q = sp[(KB + tt) * 65];
        const float ex = P1 ? sp[(2 * KB + tt) * 65] : 0.f;
        const float ey = P1 ? sp[(3 * KB + tt) * 65] : 0.f;
        // the first lane of every segment sits at the same (step, row 0)
        // position, so its ring column is uniform across the wave
        const int ip0 = __builtin_amdgcn_readfirstlane(ip);
        float yi[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const float ys = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                0, __builtin_bit_cast(int, yo[d]), 0x138 /* wave_shr:1 */, 0xf, 0xf, false));
            const float rv = ring[d * nx + ip0];
            yi[d] = first ? rv : ys;
        }
        const bool rowstart = ip == 0;
        if (REFL && rx && rowstart) {
            const int jp = k * R + r;
            const int j = ypos ? jp : ny - 1 - jp;
            const bool ok = k < nblk && jp < ny;
#pragma unroll
            for (int d = 0; d < D; ++d)
                xin[d] = (ok && mi[d] >= 0) ? fprev[((size_t)fxin * nf + j) * M + mxr[d]] : 0.f;
        } else {
#pragma unroll
            for (int d = 0; d < D; ++d) xin[d] = rowstart ? 0.f : xin[d];
        }
        float acc = 0.f, accx = 0.f, accy = 0.f;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const float qd = P1 ? fmaf(seta[d], ey, fmaf(smu[d], ex, q)) : q;
            const float rcp = __builtin_amdgcn_rcpf(st + c[d]);
            const float psi = fmaf(a[d], xin[d], fmaf(b[d], yi[d], qd)) * rcp;
            xin[d] = fmaf(psi, 2.0f, -xin[d]);
            yo[d] = fmaf(psi, 2.0f, -yi[d]);
            acc = fmaf(D == 1 ? wm : w[d], psi, acc);
            if constexpr (P1) {
                accx = fmaf(w[d] * smu[d], psi, accx);
                accy = fmaf(w[d] * seta[d], psi, accy);
            }
        }
        for (int off = R; off < 64; off <<= 1) {
            acc += __shfl_xor(acc, off, 64);
            if constexpr (P1) {
                accx += __shfl_xor(accx, off, 64);
                accy += __shfl_xor(accy, off, 64);
            }
        }
        pw[tt * PSTR] = acc;   // lanes of later segments land in unread slots
        if constexpr (P1) {
            pw[PBS + tt * PSTR] = accx;
            pw[2 * PBS + tt * PSTR] = accy;
        }
        // top row of the block hands its y flux to the ring
        float* wdst = wbase + max(ip, 0);
#pragma unroll
        for (int d = 0; d < D; ++d) wdst[d * nx] = yo[d];
        if (ip == nx - 1 && k < nblk) {
            const int jp = k * R + r;
            const int j = ypos ? jp : ny - 1 - jp;
#pragma unroll
            for (int d = 0; d < D; ++d)
                if (mi[d] >= 0) fcur[((size_t)fxout * nf + j) * M + mi[d]] = xin[d];
        }
        if (stg) stage_store(half ^ 1);
        __builtin_amdgcn_wave_barrier();
        ++ip;
        if (ip == nx) { ip = 0; ++k; }
    };

    for (int t0 = 0, blkno = 0; t0 < T; t0 += KB, ++blkno) {
        const int half = blkno & 1;
        const int tend = min(KB, T - t0);
        const bool more = t0 + KB < T;
        const float* sp = sbuf + half * NF * KB * 65 + r;
        float* pw = pbuf + half * KB * PSTR + wv * 64 + lane;
        if (tend == KB) {
#pragma unroll
            for (int tt = 0; tt < KB; ++tt)
                step(tt, sp, pw, tt == 0 && more, tt == KB - 1 && more, half);
        } else {
            for (int tt = 0; tt < tend; ++tt) step(tt, sp, pw, false, false, half);
        }
        __syncthreads();
        // fixed-order combine of the waves' partial fluxes for this block
#pragma unroll
        for (int jx = 0; jx < kMaxRed; ++jx) {
            if (jx >= nredu) break;
            const int e = tid + jx * nthreads;
            if (e < nout) {
                const int rr = e >> lkb;
                const int t2 = e & (KB - 1);
                const int cell = cursor_cell(rc_[jx], rr, R, nx, ny, nblk, xpos, ypos);
                if (t2 < tend && cell >= 0) {
                    const float* pb = pbuf + (size_t)(half * KB + t2) * PSTR + rr;
                    float s = 0.f;
                    if (fold) {
                        for (int v = 0; v < W; ++v) s = fmaf(wsh[v], pb[v * 64], s);
                    } else {
                        for (int v = 0; v < W; ++v) s += pb[v * 64];
                    }
                    part[cell] = s;
                    if constexpr (P1) {
                        float sx = 0.f, sy = 0.f;
                        for (int v = 0; v < W; ++v) {
                            sx += pb[PBS + v * 64];
                            sy += pb[2 * PBS + v * 64];
                        }
                        partx[cell] = sx;
                        party[cell] = sy;
                    }
                }
                rc_[jx].advance(KB, nx);
            }
        }
    }
    // the ring now holds the grid's outgoing y face of every column
    __builtin_amdgcn_wave_barrier();
    for (int e = r; e < D * nx; e += R) {
        const int d = e / nx, ipc = e - d * nx;
        const int i = xpos ? ipc : nx - 1 - ipc;
        int m = -1;
#pragma unroll
        for (int dd = 0; dd < D; ++dd)
            if (dd == d) m = mi[dd];
        if (m >= 0) fcur[((size_t)fyout * nf + i) * M + m] = ring[e];
    }
}

// ---------------------------------------------------------------------------
// Specialisation for the common shape: every instance of the launch has
// 64-row segments (R = 64: a wave is one segment; the last row block may be
// ragged), only vacuum inflow faces, KB <= nx, and either several row blocks
// with nx >= 63 + KB or one row block with nx >= ny - 1.  Lane l works on
// u = t - l = k*nx + ip, so with lane 0 at column ip0 the lane that starts a
// row on step t is the one with (l - ip0) mod nx == 0, and the y flux lane 0
// needs on step t was produced by lane 63 on step t - (nx - 63), at least
// KB + 1 steps (so in an earlier block) before.  With one row block lane 0
// only ever needs the vacuum inflow, so the ring is not updated at all, and
// a lane's second restart (step 2 nx + l) lies past the last step (nx + ny - 1), so
// the tally's x-outflow capture holds as well.  Lanes above the top row rl
// of a ragged last block compute on the staged defaults (sigma_t = 1,
// Q = 0); nothing of theirs is stored or flows down (the lane shift moves
// flux up only, and lane 63's ring values of that block are written after
// lane 0's last read of the column).  That makes every per-step LDS address
// an immediate offset from a per-block base and leaves no scalar
// bookkeeping in the step:
//   * lane 0 reads its y inflow from a ring of nx + KB entries (the first KB
//     mirrored at the end, so a block never wraps) and receives it as the
//     "old" operand of the lane shift (a lane with no source keeps it);
//   * every lane writes its y outflow to a [step] slot row of its own (per
//     wave, lane 63's and the top row's; the other lanes' rows are a sink
//     shared by the waves); after the block, lane 63's slots are copied
//     into the ring;
//   * a lane resets its x inflow to the vacuum value when it restarts
//     (restart step e = (l - ip0) mod nx precomputed per block);
//   * the LDS loads of step tt + kStepAhead are issued before the arithmetic
//     of step tt.
// The arithmetic and the reduction order are those of the generic kernel.
// WT > 0: the workgroup has exactly WT waves (the cross-wave sums are then
// fully unrolled, all loads in flight together); WT = 0: any W.
// TALLY: also store the outgoing boundary faces (for the particle balance;
// with vacuum inflow nothing else reads them), into the face set of the
// current parity: a lane captures the x outflow of its finished row when it
// restarts, and the 64 rows of a block are stored together after the block
// in which lane 63 restarted (lane 0 restarts only nx - 63 > KB steps
// later); the outgoing y face is stored per block from the top row's slots.
// The source iteration runs without it and tallies once, after its last
// iteration.
// The sweep of one workgroup (instance I, octant and slice of wk) into its
// partial plane; par = face parity (the tally's face set).  Shared by the
// sweep kernel and the persistent iteration kernel.
template <int D, int KB, int WT, bool TALLY>
__device__ __forceinline__ void fast_sweep_wg(const InstDesc& I, const SweepWork wk,
                                              const DirTable* __restrict__ dt, int par,
                                              float* smem) {
    constexpr int lkb = KB >= 16 ? 4 : (KB >= 8 ? 3 : (KB >= 4 ? 2 : (KB >= 2 ? 1 : 0)));
    static_assert((1 << lkb) == KB, "KB must be a power of two <= 16");
    constexpr int R = 64, lr = 6, PST = KB + 1;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int W = WT > 0 ? WT : (int)(blockDim.x >> 6);
    const int nthreads = W * 64;
    const int o = wk.oct;
    const bool xpos = (o == 0 || o == 3), ypos = (o == 0 || o == 1);
    const int nx = I.nx, ny = I.ny, nf = I.nf, M = dt->M;
    const size_t fstride = (size_t)4 * nf * M;
    gfloat* __restrict__ fcur = (gfloat*)(I.face + (size_t)(TALLY ? par : par ^ 1) * fstride);
    const int fxout = xpos ? 1 : 0, fyout = ypos ? 3 : 2;

    float a[D], b[D], c[D], w[D];
    int mi[D];
    const int nd = dt->count[o];
    const int base = wk.slice * (W * D) + wv * D;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int kk = base + d;
        if (kk < nd) {
            const int m = dt->list[o][kk];
            a[d] = 2.0f * dt->amu[m] * I.inv_dx;
            b[d] = 2.0f * dt->aeta[m] * I.inv_dy;
            w[d] = dt->w[m];
            mi[d] = m;
        } else {
            a[d] = 0.f; b[d] = 0.f; w[d] = 0.f; mi[d] = -1;
        }
        c[d] = a[d] + b[d];
    }

    // D = 1: each wave's partial flux is its direction's psi and the
    // direction weights are applied in the cross-wave sums (one VALU
    // operation less per step); wave v of the slice holds direction
    // slice * W + v
    auto wave_w = [&](int v) {
        const int kk = wk.slice * W + v;
        return kk < nd ? dt->w[dt->list[o][kk]] : 0.f;
    };
    float wsl[WT > 0 ? WT : 1];
#pragma unroll
    for (int v = 0; v < (WT > 0 ? WT : 1); ++v) wsl[v] = wave_w(v);
    // LDS: pbuf[2][W*64][KB+1] | sbuf[2][KB/2][65 float4] | ring[W][D][nx+KB]
    //      | yob[W][2][D][KB+1] | sink[64][D][KB+1]
    // sbuf holds the (sigma_t, Q) pairs of steps 2k and 2k+1 of a row side
    // by side, one 16-byte read per lane and two steps; its 65-entry rows
    // keep the staging stores (consecutive threads step through a row's KB
    // steps) free of bank conflicts.
    constexpr int SROW = 65;
    const int RS = nx + KB;
    float* pbuf = smem;
    float4* sbuf = reinterpret_cast<float4*>(smem + 2 * W * 64 * PST);
    float* ringw = smem + 2 * W * 64 * PST + 4 * KB * SROW + (size_t)(wv * D) * RS;
    // row blocks; the last one may be ragged: its top row is lane rl, and
    // the stream ends with that lane's last cell
    const int nblk = (ny + R - 1) >> lr;
    const int rl = ny - 1 - (nblk - 1) * R;
    // y-outflow slots [step]: two rows per wave, lane 63's (the ring's
    // source) and lane rl's (the tally's y face, when rl < 63); every other
    // lane writes into a sink row of its own, shared by the waves
    float* yob0 = smem + 2 * W * 64 * PST + 4 * KB * SROW + (size_t)W * D * RS;
    float* yobw = yob0 + (size_t)(wv * 2) * D * PST;
    float* yol = lane == R - 1 ? yobw
                 : lane == rl  ? yobw + D * PST
                               : yob0 + (size_t)(W * 2 + lane) * D * PST;
    const int T = nblk * nx + rl;
    gfloat* __restrict__ part = (gfloat*)(I.part + (size_t)(o * I.S + wk.slice) * I.cells);

    // Staging and reduction positions.  A block covers KB steps x 64 rows;
    // position p = rr*KB + t2 is row rr at step t2, i.e. the cell at stream
    // position u = t0 + t2 - rr = k*nx + ip (valid for 0 <= u < nblk*nx).
    // The (sigma_t, Q) pair of a position is staged one block ahead, and its
    // W partial fluxes are summed after the block, by the same thread, so
    // one cursor per position serves both.  The cursor advances by KB per
    // block with one conditional wrap (KB < nx): the cell's byte offset then
    // moves by a uniform step, dN without a wrap and dW with one.
    //
    // The positions form KB slots of 64 (one per wave and round).  Waves v,
    // v+4, v+8, ... of a workgroup share a SIMD, so with W % 4 != 0 the
    // SIMDs of waves 0 .. W%4-1 hold one wave more than the others and set
    // the pace of the steps.  Slots go out evenly (KB / W each) and the
    // remaining KB % W first to the waves on the other SIMDs.
    const int wvu = __builtin_amdgcn_readfirstlane(wv);
    int prio = wvu;   // rank in the order slots are handed out
    {
        const int wm = W & 3, q4 = W >> 2;
        if (MDP_HELPER_SPLIT && wm != 0 && q4 > 0) {
            const int c = wvu & 3, g = wvu >> 2, H = q4 * (4 - wm);
            prio = c >= wm ? g * (4 - wm) + (c - wm) : H + g * wm + c;
        }
    }
    const int nsl = KB / W + (prio < KB % W ? 1 : 0);        // slots of this wave
    const int sbase = prio * (KB / W) + min(prio, KB % W);   // its first slot
    const bool helper = nsl > 0;
    const int isg = xpos ? 1 : -1, i0 = xpos ? 0 : nx - 1;
    const int jsg = ypos ? 1 : -1, j0 = ypos ? 0 : ny - 1;
    const int dN = 4 * isg * KB, dW = 4 * (jsg * R * nx + isg * (KB - nx));
    const char* __restrict__ Stb = reinterpret_cast<const char*>(I.st);
    const char* __restrict__ Qbb = reinterpret_cast<const char*>(I.Q);
    int cip[kMaxPos], cof[kMaxPos], clo[kMaxPos], rof[kMaxPos];
    unsigned sad[kMaxPos], rad[kMaxPos], ulim[kMaxPos];
    bool cva[kMaxPos], rva[kMaxPos];
    float pst[kMaxPos], pq[kMaxPos];
#pragma unroll
    for (int jx = 0; jx < kMaxPos; ++jx) {
        // slot sl holds rows sl, sl + KB, sl + 2 KB, ... (KB >= 8): the two
        // rows of a half-wave then sit 16 banks apart at the 17-word row
        // pitch of the partial sums, so the cross-wave sums read without
        // bank conflicts (adjacent rows would collide once per half-wave)
        const int sl = sbase + jx, t2 = lane & (KB - 1);
        const int rr = KB >= 8 ? ((lane >> lkb) * KB + sl) & (R - 1)
                               : (((sl * 64 + lane) >> lkb) & (R - 1));
        cip[jx] = t2 - rr;
        clo[jx] = rr - t2;
        cof[jx] = 4 * ((j0 + jsg * rr) * nx + i0 + isg * (t2 - rr));
        // the position's stream range: rows above rl lie outside the grid
        // in the last row block
        ulim[jx] = (unsigned)((rr <= rl ? nblk : nblk - 1) * nx);
        cva[jx] = jx < nsl && (unsigned)(t2 - rr) < ulim[jx];
        rva[jx] = false;
        rof[jx] = 0;
        sad[jx] = (unsigned)((t2 >> 1) * SROW + rr) * 16u + (unsigned)(t2 & 1) * 8u;
        rad[jx] = (unsigned)(rr * PST + t2) * 4u;
        pst[jx] = 1.f;
        pq[jx] = 0.f;
    }
    auto p_live = [&](int jx) { return jx < nsl; };
    // loads of the pairs at the cursor (block t0c)
    auto stage_load = [&]() {
#pragma unroll
        for (int jx = 0; jx < kMaxPos; ++jx) {
            if (!p_live(jx)) break;
            if (cva[jx]) {
                pst[jx] = *(cgfloat*)((const MDP_GLOBAL char*)Stb + (unsigned)cof[jx]);
                pq[jx] = *(cgfloat*)((const MDP_GLOBAL char*)Qbb + (unsigned)cof[jx]);
            }
        }
    };
    auto stage_store = [&](int h) {
#pragma unroll
        for (int jx = 0; jx < kMaxPos; ++jx) {
            if (!p_live(jx)) break;
            float2* dst = reinterpret_cast<float2*>(reinterpret_cast<char*>(sbuf) +
                                                    sad[jx] + (unsigned)(h * KB * SROW * 8));
            *dst = make_float2(cva[jx] ? pst[jx] : 1.f, cva[jx] ? pq[jx] : 0.f);
        }
    };
    // keep the cursor of the block just staged for its reduction, then move
    // it one block on (to the block starting at t0n)
    auto advance = [&](int t0n) {
#pragma unroll
        for (int jx = 0; jx < kMaxPos; ++jx) {
            if (!p_live(jx)) break;
            rof[jx] = cof[jx];
            rva[jx] = cva[jx];
            int ip = cip[jx] + KB;
            const bool wrap = ip >= nx;
            cip[jx] = wrap ? ip - nx : ip;
            cof[jx] += wrap ? dW : dN;
            cva[jx] = (unsigned)(t0n - clo[jx]) < ulim[jx];
        }
    };

    // vacuum y inflow: the ring (with its mirror) starts at zero
    for (int e = lane; e < D * RS; e += 64) ringw[e] = 0.f;
    stage_load();
    stage_store(0);
    __syncthreads();

    float xin[D], yo[D], xs[D];
#pragma unroll
    for (int d = 0; d < D; ++d) { xin[d] = 0.f; yo[d] = 0.f; xs[d] = 0.f; }
    auto flush_x = [&](int kb) {
        const int jp = kb * R + lane;
        const int j = ypos ? jp : ny - 1 - jp;
        if (jp < ny) {
#pragma unroll
            for (int d = 0; d < D; ++d)
                if (mi[d] >= 0) fcur[((size_t)fxout * nf + j) * M + mi[d]] = xs[d];
        }
    };
    // lane mod nx: a lane's row starts are the steps t with t = lane (mod
    // nx); equal to lane unless a grid narrower than 64 is one row block
    const int lmod = lane < nx ? lane : lane % nx;
    int kflush = 0;

    // one step: e = this lane's restart step in the block; (st, q, rv) were
    // loaded on an earlier step; returns this lane's weighted flux sum (the
    // y outflows are left in yo)
    auto math = [&](int tt, int e, float st, float q, const float* rv) {
        float yi[D];
#pragma unroll
        for (int d = 0; d < D; ++d)
            yi[d] = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
                __builtin_bit_cast(int, rv[d]), __builtin_bit_cast(int, yo[d]),
                0x138 /* wave_shr:1 */, 0xf, 0xf, false));
        const bool rs = e == tt;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if constexpr (TALLY) xs[d] = rs ? xin[d] : xs[d];
            xin[d] = rs ? 0.f : xin[d];
        }
        float acc = 0.f;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const float rcp = __builtin_amdgcn_rcpf(st + c[d]);
            const float psi = fmaf(a[d], xin[d], fmaf(b[d], yi[d], q)) * rcp;
            xin[d] = fmaf(psi, 2.0f, -xin[d]);
            yo[d] = fmaf(psi, 2.0f, -yi[d]);
            if constexpr (D == 1) acc = psi;   // weight applied in the sums
            else acc = fmaf(w[d], psi, acc);
        }
        return acc;
    };

    int ip0b = 0;                                  // lane 0's column at tt = 0
    for (int t0 = 0, blkno = 0; t0 < T; t0 += KB, ++blkno) {
        const int half = blkno & 1;
        const int tend = min(KB, T - t0);
        const bool more = t0 + KB < T;
        int e = lmod - ip0b;
        if (e < 0) e += nx;                        // restart step of this lane
        const float4* sp = sbuf + half * (KB / 2) * SROW + lane;   // step pair k: sp[k*SROW]
        float* pw = pbuf + ((size_t)(half * W + wv) * 64 + lane) * PST;
        const float* rg = ringw + ip0b;            // ring column of step tt: rg[d*RS + tt]
        if (tend == KB) {
            // LDS traffic goes in pairs of steps: one 16-byte read of both
            // steps' (sigma_t, Q), one two-word read of their ring values,
            // and after the odd step one two-word write each of the flux
            // sums and the y outflows.  The reads of steps tt + A, tt + A + 1
            // are issued before the arithmetic of step tt (A = kStepAhead),
            // so their latency hides behind A steps of this wave.
            constexpr int A = kStepAhead < KB ? kStepAhead : KB;
            static_assert(KB >= 2 && A % 2 == 0, "steps go in pairs");
            float4 sq[A / 2 + 1];
            float rv[A + 2][D];
            float accp = 0.f, yop[D];
#pragma unroll
            for (int k = 0; k < A / 2; ++k) sq[k] = sp[k * SROW];
#pragma unroll
            for (int k = 0; k < A; ++k) {
#pragma unroll
                for (int d = 0; d < D; ++d) rv[k][d] = rg[d * RS + k];
            }
#pragma unroll
            for (int tt = 0; tt < KB; ++tt) {
                const bool odd = tt & 1;
                if (tt == 0) {
                    advance(t0 + KB);
                    if (more) stage_load();
                }
                if (!odd && tt + A < KB) {
                    sq[A / 2] = sp[((tt + A) >> 1) * SROW];
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        rv[A][d] = rg[d * RS + tt + A];
                        rv[A + 1][d] = rg[d * RS + tt + A + 1];
                    }
                }
                const float acc = math(tt, e, odd ? sq[0].z : sq[0].x,
                                       odd ? sq[0].w : sq[0].y, rv[0]);
                if (odd) {
                    pw[tt - 1] = accp;
                    pw[tt] = acc;
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        yol[d * PST + tt - 1] = yop[d];
                        yol[d * PST + tt] = yo[d];
                    }
                } else {
                    accp = acc;
#pragma unroll
                    for (int d = 0; d < D; ++d) yop[d] = yo[d];
                }
                if (tt == KB - 1 && more) stage_store(half ^ 1);
                // a scheduling fence after each pair keeps the reads where
                // they are written above (the scheduler otherwise moves some
                // of them next to their uses)
                if (odd) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 0; k <= A; ++k) {
#pragma unroll
                    for (int d = 0; d < D; ++d) rv[k][d] = rv[k + 1][d];
                }
                if (odd) {
#pragma unroll
                    for (int k = 0; k < A / 2; ++k) sq[k] = sq[k + 1];
                }
            }
        } else {
            advance(t0 + KB);
            for (int tt = 0; tt < tend; ++tt) {
                float rv[D];
#pragma unroll
                for (int d = 0; d < D; ++d) rv[d] = rg[d * RS + tt];
                const float4 sq = sp[(tt >> 1) * SROW];
                const bool odd = tt & 1;
                pw[tt] = math(tt, e, odd ? sq.z : sq.x, odd ? sq.w : sq.y, rv);
#pragma unroll
                for (int d = 0; d < D; ++d) yol[d * PST + tt] = yo[d];
            }
        }
        // lane 63's y outflow of this block into the ring (and its mirror);
        // its column ip0b + j - 63 lies in [-63, nx - 49].  One row block:
        // nothing reads the ring again.
        if (nblk > 1) {
            const int j = lane;
            if (j < tend && t0 + j >= R - 1) {
                int col = ip0b + j - (R - 1);
                if (col < 0) col += nx;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const float v = yobw[d * PST + j];
                    ringw[d * RS + col] = v;
                    if (col < KB) ringw[d * RS + nx + col] = v;
                }
            }
        }
        if constexpr (TALLY) {
            // lane 63 restarted in this block: the x outflow of the previous
            // row block is complete (lane 0 restarts nx - 63 > KB steps
            // later).  Only grids of several row blocks (nx >= 63 + KB) get
            // here: lane 63 restarts at step nx + 63 at the earliest.
            int e63 = (R - 1) - ip0b;
            if (e63 < 0) e63 += nx;
            if (e63 < tend && t0 + e63 >= nx + R - 1) flush_x(kflush++);
            // the grid's outgoing y face: lane rl's y outflow in the last
            // row block
            const int j = lane;
            const int col = t0 + j - rl - (nblk - 1) * nx;
            if (j < tend && col >= 0 && col < nx) {
                const int i = xpos ? col : nx - 1 - col;
#pragma unroll
                for (int d = 0; d < D; ++d)
                    if (mi[d] >= 0)
                        fcur[((size_t)fyout * nf + i) * M + mi[d]] =
                            yobw[(rl == R - 1 ? 0 : D * PST) + d * PST + j];
            }
        }
        ip0b += KB;
        if (ip0b >= nx) ip0b -= nx;
        __syncthreads();
        // fixed-order sums of the waves' partial fluxes of this block (all
        // partial loads of a thread first)
        if (helper) {
            const unsigned hoff = (unsigned)(half * W * 64 * PST) * 4u;
            if constexpr (WT > 0) {
                float vals[kMaxPos][WT];
#pragma unroll
                for (int jx = 0; jx < kMaxPos; ++jx) {
                    if (!p_live(jx)) break;
                    const float* pb = reinterpret_cast<const float*>(
                        reinterpret_cast<const char*>(pbuf) + rad[jx] + hoff);
#pragma unroll
                    for (int v = 0; v < WT; ++v) vals[jx][v] = pb[(size_t)v * 64 * PST];
                }
#pragma unroll
                for (int jx = 0; jx < kMaxPos; ++jx) {
                    if (!p_live(jx)) break;
                    if (rva[jx]) {
                        float s = 0.f;
#pragma unroll
                        for (int v = 0; v < WT; ++v) {
                            if constexpr (D == 1) s = fmaf(wsl[v], vals[jx][v], s);
                            else s += vals[jx][v];
                        }
                        *(gfloat*)((MDP_GLOBAL char*)part + (unsigned)rof[jx]) = s;
                    }
                }
            } else {
#pragma unroll
                for (int jx = 0; jx < kMaxPos; ++jx) {
                    if (!p_live(jx)) break;
                    if (rva[jx]) {
                        const float* pb = reinterpret_cast<const float*>(
                            reinterpret_cast<const char*>(pbuf) + rad[jx] + hoff);
                        float s = 0.f;
#pragma unroll 4
                        for (int v = 0; v < W; ++v) {
                            if constexpr (D == 1) s = fmaf(wave_w(v), pb[(size_t)v * 64 * PST], s);
                            else s += pb[(size_t)v * 64 * PST];
                        }
                        *(gfloat*)((MDP_GLOBAL char*)part + (unsigned)rof[jx]) = s;
                    }
                }
            }
        }
    }
    if constexpr (TALLY) {
        // the top lane rl ends the stream and never restarts after its last
        // row (the lanes below it restarted after theirs): capture, then
        // store the x outflow of the last row block
#pragma unroll
        for (int d = 0; d < D; ++d) xs[d] = lane == rl ? xin[d] : xs[d];
        flush_x(nblk - 1);
    }
}

template <int D, int KB, int WT, bool TALLY>
__global__ void __launch_bounds__(WT > 0 ? WT * 64 : SweepBounds<D>::threads)
sweep2d_fast_kernel(const InstDesc* __restrict__ insts,
                    const SweepWork* __restrict__ work,
                    const DirTable* __restrict__ dt, const int* __restrict__ done,
                    const int* __restrict__ iter, FinArgs fin) {
    extern __shared__ float smem[];
    const SweepWork wk = work[blockIdx.x];
    const int n = wk.inst;
    if (n < 0) return;
    if (fin.pending) {
        if (sweep_prologue(insts[n], n, fin, wk.oct == 0 && wk.slice == 0)) return;
    } else if (done != nullptr && done[n]) {
        return;
    }
    const int par = (fin.pending ? fin.it : (iter != nullptr ? iter[n] : 0)) & 1;
    fast_sweep_wg<D, KB, WT, TALLY>(insts[n], wk, dt, par, smem);
}

// ------------------------------------------------ persistent iteration --
// Several source iterations in one launch for the specialised sweep with
// one direction per lane: the workgroups of an
// instance sweep, meet at a barrier, combine their share of the instance's
// blocks of cells (combine_dev.h), meet again and evaluate the convergence
// test of the iteration, exactly as the finalize kernel does; an instance
// whose test stops it leaves the loop in all its workgroups at once (they
// read the same partial sums).  The launch is cooperative, so every
// workgroup is resident; no instance waits on another.  Results, iteration
// counts and statuses equal those of the sweep / combine / finalize
// launches.

// Barrier of the G workgroups of instance n: the counter reaches `target`
// when all of them have arrived `target / G` times.  The wait polls with a
// short sleep; it gives up after spin_limit polls (setting the flag), or as
// soon as another workgroup has set it.  Returns false after a time-out
// anywhere (the caller leaves: every later wait would give up as well).
__device__ __forceinline__ bool inst_barrier(int* bar, int target, int* err, int spin_limit,
                                             int* ok_lds) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");   // the workgroup's writes
        __hip_atomic_fetch_add(bar, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int spins = 0, ok = 1;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > spin_limit) {
                atomicOr(err, 1);
                ok = 0;
                break;
            }
            if ((spins & 63) == 0 &&
                __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the other workgroups' writes
        *ok_lds = ok;
    }
    __syncthreads();
    return *ok_lds != 0;
}

// The convergence test of iteration l of instance n (the finalize kernel's
// arithmetic and summation order); the designated workgroup records it.
// Returns true when the instance stops.
__device__ __forceinline__ bool persist_test(const InstDesc& I, int n, int l,
                                             const PersistArgs& pa, bool designated) {
    const IterState& st = pa.st;
    if (!tested_iteration(l, pa.norm_kind)) {
        if (designated && threadIdx.x == 0) st.iter[n] = l;
        return false;
    }
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < I.nred; ++b) {
        const double2 v = pa.red[I.red0 + b];
        if (pa.norm_kind != 1) { s1 += v.x; s2 += v.y; }
        else s1 = fmax(s1, v.x);
    }
    double r;
    if (pa.norm_kind != 1)
        r = s2 > 0.0 ? sqrt(s1 / s2) : (s1 == 0.0 ? 0.0 : INFINITY);
    else
        r = s1;
    const int slot = history_slot(l, pa.norm_kind);
    const double r_prev = st.rhist[2 * n + (slot ^ 1)];
    const bool bad = !isfinite(s1) || !isfinite(s2);
    const bool conv = !bad && stop_test(r, r_prev, pa.tol, pa.norm_kind);
    if (designated && threadIdx.x == 0) {
        st.resid[n] = r;
        st.rhist[2 * n + slot] = r;
        st.iter[n] = l;
        if (bad) {
            st.status[n] = -4;
            st.done[n] = 1;
        } else if (conv) {
            st.status[n] = 0;
            st.done[n] = 1;
        }
    }
    return bad || conv;
}

template <int KB, int WT>
__global__ void __launch_bounds__(WT > 0 ? WT * 64 : SweepBounds<1>::threads)
si_persistent_kernel(const InstDesc* __restrict__ insts, const SweepWork* __restrict__ work,
                     const DirTable* __restrict__ dt, PersistArgs pa) {
    extern __shared__ float smem[];
    const SweepWork wk = work[blockIdx.x];
    const int n = wk.inst;
    if (n < 0 || pa.st.done[n]) return;
    const InstDesc& I = insts[n];
    const int G = 4 * I.S;                    // workgroups of the instance
    const int rank = wk.oct * I.S + wk.slice;
    double* r1 = reinterpret_cast<double*>(smem);   // combine reduction (after the sweep)
    double* r2 = r1 + kCombineThreads;
    __shared__ int ok_lds;
    int phase = 2 * pa.it0;                   // barrier phases the instance has completed
    for (int it = 0; it < pa.k; ++it) {
        const int l = pa.it0 + it + 1;
        fast_sweep_wg<1, KB, WT, false>(I, wk, dt, 0, smem);
        if (!inst_barrier(pa.bar + n, G * ++phase, pa.err, pa.spin_limit, &ok_lds)) return;
        // the error-bound rule measures the change against the snapshot on
        // its tested iterations only
        const int mode = pa.norm_kind != 2 ? 0 : (l % kStopStride == 0 ? 2 : 3);
        for (int j = rank; j < I.nred; j += G)
            combine_block(I, j * kCombineChunk, I.red0 + j, pa.red, mode, pa.norm_kind, dt,
                          (int)threadIdx.x, (int)blockDim.x, r1, r2);
        if (!inst_barrier(pa.bar + n, G * ++phase, pa.err, pa.spin_limit, &ok_lds)) return;
        if (persist_test(I, n, l, pa, rank == 0)) break;
    }
}

bool persistent_supported(int D, int W, int KB) {
    return D == 1 && W >= 1 && 64 * W <= SweepBounds<1>::threads &&
           (KB == 16 || KB == 8 || KB == 4 || KB == 2);
}

template <int KB, int WT>
static const void* persist_fn() {
    return reinterpret_cast<const void*>(&si_persistent_kernel<KB, WT>);
}
template <int WT>
static const void* persist_fn_kb(int KB) {
    switch (KB) {
        case 16: return persist_fn<16, WT>();
        case 8: return persist_fn<8, WT>();
        case 4: return persist_fn<4, WT>();
        default: return persist_fn<2, WT>();
    }
}
// the fixed wave counts of the sweep kernel (9, 10), any other count through
// the dynamic variant
static const void* persist_kernel(int W, int KB) {
    if (W == 9) return persist_fn_kb<9>(KB);
    if (W == 10) return persist_fn_kb<10>(KB);
    return persist_fn_kb<0>(KB);
}

// Whether nwork workgroups of this shape are resident at once on `device`
// (the cooperative launch requires it).
bool persistent_fits(int W, int KB, size_t lds, int nwork, int device) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persist_kernel(W, KB), 64 * W,
                                                     lds) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) !=
            hipSuccess)
        return false;
    return (long long)per_cu * cus >= nwork;
}

hipError_t launch_persistent(int W, int KB, size_t lds, int nwork, const InstDesc* insts,
                             const SweepWork* work, const DirTable* dt, const PersistArgs& pa,
                             hipStream_t s) {
    PersistArgs a = pa;
    void* args[] = {(void*)&insts, (void*)&work, (void*)&dt, (void*)&a};
    return hipLaunchCooperativeKernel(persist_kernel(W, KB), dim3(nwork), dim3(64 * W), args,
                                      (unsigned)lds, s);
}

// Host launcher; returns false for an unsupported (D, KB).
template <int D, int KB, bool P1 = false>
static void launch_dk(bool refl, dim3 grid, dim3 block, size_t lds,
                      hipStream_t s, const InstDesc* insts,
                      const SweepWork* work, const DirTable* dt,
                      const int* done, const int* iter, int use_faces, const FinArgs& fin) {
    if (refl)
        hipLaunchKernelGGL((sweep2d_kernel<D, true, KB, P1>), grid, block, lds, s,
                           insts, work, dt, done, iter, use_faces, fin);
    else
        hipLaunchKernelGGL((sweep2d_kernel<D, false, KB, P1>), grid, block, lds, s,
                           insts, work, dt, done, iter, use_faces, fin);
}

template <int D, bool P1 = false>
static bool launch_d(int KB, bool refl, dim3 grid, dim3 block, size_t lds,
                     hipStream_t s, const InstDesc* insts,
                     const SweepWork* work, const DirTable* dt,
                     const int* done, const int* iter, int use_faces, const FinArgs& fin) {
    switch (KB) {
        case 16: launch_dk<D, 16, P1>(refl, grid, block, lds, s, insts, work, dt, done, iter, use_faces, fin); return true;
        case 8: launch_dk<D, 8, P1>(refl, grid, block, lds, s, insts, work, dt, done, iter, use_faces, fin); return true;
        case 4: launch_dk<D, 4, P1>(refl, grid, block, lds, s, insts, work, dt, done, iter, use_faces, fin); return true;
        case 2: launch_dk<D, 2, P1>(refl, grid, block, lds, s, insts, work, dt, done, iter, use_faces, fin); return true;
        default: return false;
    }
}

template <int D, int WT, bool TALLY>
static bool launch_fast_dw(int KB, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                           const InstDesc* insts, const SweepWork* work, const DirTable* dt,
                           const int* done, const int* iter, const FinArgs& fin) {
    switch (KB) {
        case 16: hipLaunchKernelGGL((sweep2d_fast_kernel<D, 16, WT, TALLY>), grid, block, lds, s, insts, work, dt, done, iter, fin); return true;
        case 8: hipLaunchKernelGGL((sweep2d_fast_kernel<D, 8, WT, TALLY>), grid, block, lds, s, insts, work, dt, done, iter, fin); return true;
        case 4: hipLaunchKernelGGL((sweep2d_fast_kernel<D, 4, WT, TALLY>), grid, block, lds, s, insts, work, dt, done, iter, fin); return true;
        case 2: hipLaunchKernelGGL((sweep2d_fast_kernel<D, 2, WT, TALLY>), grid, block, lds, s, insts, work, dt, done, iter, fin); return true;
        default: return false;
    }
}

// Wave counts compiled as constants (one direction per lane): a constant W
// unrolls the cross-wave sums and the staging loops, which a runtime W
// leaves as loops, at about 1.6 times the step time.  Each W = 2..16 is
// built with the largest block size it allows (16 from W = 4 on, 8 below),
// W = 9 and 10 (full S16 and S8 octants) with every block size; other
// block sizes, the tally sweep at W other than 9 and 10 (one launch per
// solve) and D > 1 take the runtime-W kernel.
template <int D, int WT, bool TALLY>
static bool launch_fast_const(int KB, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                              const InstDesc* insts, const SweepWork* work, const DirTable* dt,
                              const int* done, const int* iter, const FinArgs& fin) {
    constexpr int kb = WT >= 4 ? 16 : 8;
    if constexpr (WT == 9 || WT == 10)   // S16 and S8 octants: every block size
        if (KB != kb)
            return launch_fast_dw<D, WT, TALLY>(KB, grid, block, lds, s, insts, work, dt, done, iter, fin);
    if (KB != kb)
        return launch_fast_dw<D, 0, TALLY>(KB, grid, block, lds, s, insts, work, dt, done, iter, fin);
    hipLaunchKernelGGL((sweep2d_fast_kernel<D, kb, WT, TALLY>), grid, block, lds, s, insts, work,
                       dt, done, iter, fin);
    return true;
}

template <int D>
static bool launch_fast_d(int KB, dim3 grid, dim3 block, size_t lds, hipStream_t s,
                          const InstDesc* insts, const SweepWork* work, const DirTable* dt,
                          const int* done, const int* iter, bool tally, const FinArgs& fin) {
    const int W = (int)block.x / 64;
#define MDP_FAST_ARGS KB, grid, block, lds, s, insts, work, dt, done, iter, fin
    if constexpr (D == 1) {
        if (tally) {
            if (W == 9) return launch_fast_const<D, 9, true>(MDP_FAST_ARGS);
            if (W == 10) return launch_fast_const<D, 10, true>(MDP_FAST_ARGS);
        } else {
            switch (W) {
                case 2: return launch_fast_const<D, 2, false>(MDP_FAST_ARGS);
                case 3: return launch_fast_const<D, 3, false>(MDP_FAST_ARGS);
                case 4: return launch_fast_const<D, 4, false>(MDP_FAST_ARGS);
                case 5: return launch_fast_const<D, 5, false>(MDP_FAST_ARGS);
                case 6: return launch_fast_const<D, 6, false>(MDP_FAST_ARGS);
                case 7: return launch_fast_const<D, 7, false>(MDP_FAST_ARGS);
                case 8: return launch_fast_const<D, 8, false>(MDP_FAST_ARGS);
                case 9: return launch_fast_const<D, 9, false>(MDP_FAST_ARGS);
                case 10: return launch_fast_const<D, 10, false>(MDP_FAST_ARGS);
                case 11: return launch_fast_const<D, 11, false>(MDP_FAST_ARGS);
                case 12: return launch_fast_const<D, 12, false>(MDP_FAST_ARGS);
                case 13: return launch_fast_const<D, 13, false>(MDP_FAST_ARGS);
                case 14: return launch_fast_const<D, 14, false>(MDP_FAST_ARGS);
                case 15: return launch_fast_const<D, 15, false>(MDP_FAST_ARGS);
                case 16: return launch_fast_const<D, 16, false>(MDP_FAST_ARGS);
                default: break;
            }
        }
    }
    return tally ? launch_fast_dw<D, 0, true>(MDP_FAST_ARGS)
                 : launch_fast_dw<D, 0, false>(MDP_FAST_ARGS);
#undef MDP_FAST_ARGS
}

bool launch_sweep2d_fast(int D, int nwork, int W, int KB, size_t lds_bytes,
                         const InstDesc* insts, const SweepWork* work, const DirTable* dt,
                         const int* done, const int* iter, bool tally, const FinArgs& fin,
                         hipStream_t s) {
    dim3 grid(nwork), block(64 * W);
    switch (D) {
        case 1: return launch_fast_d<1>(KB, grid, block, lds_bytes, s, insts, work, dt, done, iter, tally, fin);
        case 2: return launch_fast_d<2>(KB, grid, block, lds_bytes, s, insts, work, dt, done, iter, tally, fin);
        case 3: return launch_fast_d<3>(KB, grid, block, lds_bytes, s, insts, work, dt, done, iter, tally, fin);
        case 4: return launch_fast_d<4>(KB, grid, block, lds_bytes, s, insts, work, dt, done, iter, tally, fin);
        default: return false;
    }
}

size_t sweep2d_fast_lds_bytes(int W, int KB, int D, int max_nx) {
    return sizeof(float) * ((size_t)2 * W * 64 * (KB + 1) + (size_t)4 * KB * 65 +
                            (size_t)W * D * (max_nx + KB) + (size_t)(2 * W + 64) * D * (KB + 1));
}

bool launch_sweep2d(int D, bool refl, int nwork, int W, int KB,
                    size_t lds_bytes, const InstDesc* insts,
                    const SweepWork* work, const DirTable* dt, const int* done,
                    const int* iter, int use_faces, const FinArgs& fin, hipStream_t s,
                    bool p1) {
    dim3 grid(nwork), block(64 * W);
    if (p1)
        return D == 1 && launch_d<1, true>(KB, refl, grid, block, lds_bytes, s, insts, work, dt,
                                           done, iter, use_faces, fin);
    switch (D) {
        case 1: return launch_d<1>(KB, refl, grid, block, lds_bytes, s, insts, work, dt, done, iter, use_faces, fin);
        case 2: return launch_d<2>(KB, refl, grid, block, lds_bytes, s, insts, work, dt, done, iter, use_faces, fin);
        case 3: return launch_d<3>(KB, refl, grid, block, lds_bytes, s, insts, work, dt, done, iter, use_faces, fin);
        case 4: return launch_d<4>(KB, refl, grid, block, lds_bytes, s, insts, work, dt, done, iter, use_faces, fin);
        case 6: return launch_d<6>(KB, refl, grid, block, lds_bytes, s, insts, work, dt, done, iter, use_faces, fin);
        case 9: return launch_d<9>(KB, refl, grid, block, lds_bytes, s, insts, work, dt, done, iter, use_faces, fin);
        default: return false;
    }
}

size_t sweep2d_lds_bytes(int W, int KB, int D, int max_nseg_nx, int max_nx, bool p1) {
    // + 16: the kernel's static table of wave weights
    const size_t npb = p1 ? 3 : 1, nf = p1 ? 4 : 2;
    return sizeof(float) * (npb * 2 * KB * (W * 64 + 1) + 2 * nf * KB * 65 +
                            (size_t)W * D * max_nseg_nx + (size_t)W * D * max_nx + 16);
}

// Whether the generic kernel's per-thread staging and reduction slots hold
// a block of KB steps of R rows with W waves (checked before every launch).
bool sweep2d_generic_fits(int W, int KB, int R, bool p1) {
    const int nf = p1 ? 4 : 2, mpf = p1 ? 2 * kMaxPrefetch : kMaxPrefetch;
    return nf * KB * R <= mpf * 64 * W && KB * R <= kMaxRed * 64 * W;
}

// Largest block size whose staging fits kMaxPrefetch values and whose
// reduction fits kMaxRed outputs per thread.
int sweep2d_max_kb(int W, int R, bool p1) {
    const int nf = p1 ? 4 : 2, mpf = p1 ? 2 * kMaxPrefetch : kMaxPrefetch;
    int kb = 16;
    while (kb > 1 && (nf * kb * R > mpf * 64 * W || kb * R > kMaxRed * 64 * W))
        kb >>= 1;
    return kb;
}



// Largest block size of the specialised kernel: a wave holds at most
// kMaxPos staging / reduction slots of 64 positions.
int sweep2d_fast_max_kb(int W) {
    int kb = 16;
    while (kb > 1 && kb > kMaxPos * W) kb >>= 1;
    return kb;
}

// Largest W (waves per workgroup) the kernel for D supports.
int sweep2d_max_w(int D) {
    switch (D) {
        case 1: return SweepBounds<1>::threads / 64;
        case 2: return SweepBounds<2>::threads / 64;
        case 3: return SweepBounds<3>::threads / 64;
        case 4: return SweepBounds<4>::threads / 64;
        case 6: return SweepBounds<6>::threads / 64;
        case 9: return SweepBounds<9>::threads / 64;
        default: return 1;
    }
}

}  // namespace mdp
