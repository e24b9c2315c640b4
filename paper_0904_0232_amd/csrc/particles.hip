// Particle kernels (FP64): gather + RK4 push (Sec. 3.3), zigzag current
// deposition with curved face weights (Sec. 4), removal, and loading with the
// mass-shell solve (Sec. 2.1).  One thread per particle slot, SoA storage, so
// a wavefront of 64 lanes reads 64 consecutive doubles per component.
#include "grpic_dev.h"
#include "grpic_impl.h"

namespace grpic {

// Wavefront min / max (DPP reductions of the device library); the result is
// the same in every lane.
__device__ __forceinline__ int wave_min(int v) { return __ockl_wfred_min_i32(v); }
__device__ __forceinline__ int wave_max(int v) { return __ockl_wfred_max_i32(v); }

// Add a per-lane count to a device counter with one atomic per wavefront:
// same-address atomics from many waves serialise across the XCDs.  Every
// lane of the wave must reach the call.
__device__ __forceinline__ void wave_count(unsigned long long *ctr, int v) {
    const int s = __ockl_wfred_add_i32(v);
    if (s != 0 && (threadIdx.x & 63) == 0) atomicAdd(ctr, (unsigned long long)s);
}


// Node tensor rows in LDS: 16 doubles per node padded to 18, so nodes one
// apart start 4 banks apart.
constexpr int kNodeStride2 = 9;  // double2 per staged node

// A block's copy of the node tensor over the node box [lo, lo + n) (x
// fastest), or use = false (the block reads global memory).
struct NodeBox {
    const double2 *lds;
    int lo[3], n[3];
    bool use;
    bool any;  // the block has a live lane
};

// L^a += sum over the 8 nodes of W_n (F_n u)^a, nodes addressed from the
// (0,0,0) node `p` with strides (in double2) si, sj, sk; the contraction with
// u is taken node by node, so only four accumulators stay live.  A node's 16
// components are read before any is used, so its eight 16-byte reads are in
// flight together instead of two at a time.
__device__ __forceinline__ void gather_rows(const double2 *p, int64_t si, int64_t sj, int64_t sk, const double w[3],
                                            const double U[4], double L[4]) {
#pragma unroll 1
    for (int q = 0; q < 4; q++) {
        const int dj = q & 1, dk = q >> 1;
        const double wyz = (dj ? w[1] : 1.0 - w[1]) * (dk ? w[2] : 1.0 - w[2]);
        const double2 *pq = p + dj * sj + dk * sk;
#pragma unroll
        for (int di = 0; di < 2; di++) {
            const double W = (di ? w[0] : 1.0 - w[0]) * wyz;
            const double2 *pn = pq + di * si;
            double2 f[8];
#pragma unroll
            for (int e = 0; e < 8; e++) f[e] = pn[e];
#pragma unroll
            for (int a = 0; a < 4; a++) {
                const double row = f[2 * a].x * U[0] + f[2 * a].y * U[1] + f[2 * a + 1].x * U[2] + f[2 * a + 1].y * U[3];
                L[a] += W * row;
            }
        }
    }
}

// Cell of a gather: floor(X) clamped to the grid (the offset is not clamped).
__device__ __forceinline__ void gather_cell(const Grid &G, const double X[3], int c[3]) {
    for (int ax = 0; ax < 3; ax++) {
        int n = G.dim(ax);
        int ci = (int)floor(X[ax]);
        c[ax] = ci < 0 ? 0 : (ci > n - 1 ? n - 1 : ci);
    }
}

// Lorentz term (q/m-free) L^a = F^a_b(X) u^b with F^a_b gathered trilinearly
// from the nodes of cell c (cloud-in-cell with sqrt(-det g) = 1, Sec. 3.3),
// from the block's LDS box when it holds the cell's nodes, else from global
// memory; the arithmetic is the same.
__device__ __forceinline__ void gather_lorentz(const Grid &G, const double *__restrict__ node, const NodeBox &B,
                                               const int c[3], const double X[3], const double U[4], double L[4]) {
    double w[3];
    for (int ax = 0; ax < 3; ax++) w[ax] = X[ax] - (double)c[ax];
    L[0] = L[1] = L[2] = L[3] = 0.0;
    bool inside = B.use;
    for (int ax = 0; ax < 3; ax++) inside = inside && c[ax] >= B.lo[ax] && c[ax] + 1 < B.lo[ax] + B.n[ax];
    if (inside) {
        const int64_t l = ((int64_t)(c[2] - B.lo[2]) * B.n[1] + (c[1] - B.lo[1])) * B.n[0] + (c[0] - B.lo[0]);
        gather_rows(B.lds + kNodeStride2 * l, kNodeStride2, kNodeStride2 * B.n[0],
                    (int64_t)kNodeStride2 * B.n[0] * B.n[1], w, U, L);
    } else {
        const int64_t sj = G.nx + 1, sk = (int64_t)(G.nx + 1) * (G.ny + 1);
        gather_rows(reinterpret_cast<const double2 *>(node) + 8 * G.node(c[0], c[1], c[2]), 8, 8 * sj, 8 * sk, w, U,
                    L);
    }
}

// du^a/dtau = (q/m) F^a_b u^b - Gamma^a_{mn} u^m u^n  (Sec. 3.3)
__device__ __forceinline__ void accel(const PushParams &P, const double *__restrict__ node, const NodeBox &B,
                                      const int c[3], double qm, const double X[3], const double U[4], double A[4]) {
    double L[4];
    gather_lorentz(P.G, node, B, c, X, U, L);
    double Gm[4] = {0.0, 0.0, 0.0, 0.0};
    if (P.h.m != 0.0) {
        KSGrad kp;
        ks_grad(P.h.m, P.h.a, X[0] - P.h.cx, X[1] - P.h.cy, X[2] - P.h.cz, kp);
        gamma_uu(kp, U, Gm);
    }
#pragma unroll
    for (int a = 0; a < 4; a++) A[a] = qm * L[a] - Gm[a];
}

// Stage time-dilation factor: PAPER = 1/2 [u4/c + sqrt((u4/c)^2 + 2 a4 dt / c)]
// (negative discriminant clamped to 0 and counted), U4 = u4/c.
__device__ __forceinline__ double stage_gamma(const PushParams &P, double u4, double a4, int &clamps) {
    double uc = u4 * P.inv_c;
    if (P.gamma_mode == 1) return uc;
    double disc = uc * uc + 4.0 * a4 * P.dt_2c;
    if (disc < 0.0) {
        disc = 0.0;
        clamps++;
    }
    return 0.5 * (uc + sqrt_nr(disc));
}

constexpr int kPushBlock = 256;
constexpr int kPushLdsNodes = 272;  // 38 KiB of padded node tensor per block, four blocks per CU
constexpr int kStageInFlight = 8;   // node pieces per thread in flight while the box is staged

// Stage, once per push, the node box of the cells the block's live lanes
// start in (cell c, nodes c .. c+1), widened by one cell on every side when
// that still fits, so the later RK4 stages (moves below a cell) usually
// gather from the same copy.  Every thread of the block calls this; it
// synchronises the block after the box reduction and after the copy.
__device__ __forceinline__ void stage_box(const Grid &G, const double *__restrict__ node, bool live, const int c[3],
                                          double2 *snode, int (*sred)[kPushBlock / 64], NodeBox &B) {
    const int tid = threadIdx.x;
    for (int ax = 0; ax < 3; ax++) {
        int a = wave_min(live ? c[ax] : (1 << 30)), b = wave_max(live ? c[ax] : -(1 << 30));
        if ((tid & 63) == 0) {
            sred[ax][tid >> 6] = a;
            sred[3 + ax][tid >> 6] = b;
        }
    }
    __syncthreads();
    int lo[2][3], n[2][3], count[2] = {1, 1};
    for (int ax = 0; ax < 3; ax++) {
        int a = sred[ax][0], b = sred[3 + ax][0];
        for (int w = 1; w < kPushBlock / 64; w++) {
            a = sred[ax][w] < a ? sred[ax][w] : a;
            b = sred[3 + ax][w] > b ? sred[3 + ax][w] : b;
        }
        if (ax == 0) B.any = b >= a;
        for (int e = 0; e < 2; e++) {  // e = 1: widened by one cell, within the nodes 0 .. dim
            const int l = a - e < 0 ? 0 : a - e;
            const int h = b + 1 + e > G.dim(ax) ? G.dim(ax) : b + 1 + e;
            lo[e][ax] = l;
            n[e][ax] = b >= a ? h - l + 1 : 0;
            count[e] = (n[e][ax] > 0 && count[e] <= kPushLdsNodes) ? count[e] * n[e][ax] : 0;
        }
    }
    // count = 0: no live lane
    const int e = (count[1] > 0 && count[1] <= kPushLdsNodes) ? 1 : 0;
    for (int ax = 0; ax < 3; ax++) {
        B.lo[ax] = lo[e][ax];
        B.n[ax] = n[e][ax];
    }
    B.use = count[e] > 0 && count[e] <= kPushLdsNodes;
    if (B.use) {
        const double2 *src = reinterpret_cast<const double2 *>(node);
        const int nb0 = B.n[0], nb01 = B.n[0] * B.n[1];
        const float inv0 = __builtin_amdgcn_rcpf((float)nb0), inv01 = __builtin_amdgcn_rcpf((float)nb01);
        // kStageInFlight pieces per thread are read before any is stored, so
        // the copy takes one or two memory round trips instead of one per piece
        const int total = count[e] * 8;
        for (int q0 = tid; q0 < total; q0 += kPushBlock * kStageInFlight) {
            double2 v[kStageInFlight];
#pragma unroll
            for (int t = 0; t < kStageInFlight; t++) {
                const int q = q0 + t * kPushBlock < total ? q0 + t * kPushBlock : total - 1;
                const int l = q >> 3, part = q & 7;
                const int lk = small_div(l, inv01), r = l - lk * nb01, lj = small_div(r, inv0), li = r - lj * nb0;
                v[t] = src[8 * G.node(B.lo[0] + li, B.lo[1] + lj, B.lo[2] + lk) + part];
            }
#pragma unroll
            for (int t = 0; t < kStageInFlight; t++) {  // a clamped slot rewrites piece total - 1 with its own value
                const int q = q0 + t * kPushBlock < total ? q0 + t * kPushBlock : total - 1;
                snode[kNodeStride2 * (q >> 3) + (q & 7)] = v[t];
            }
        }
    }
    __syncthreads();
}

// Classic RK4 in coordinate time on Y = (x, u): K_k = (u_k, A_k)/gamma_k,
// stages at dt/2, dt/2, dt, combination 1:2:2:1 over 6.
//
// The block first copies the node tensor of the (widened) box of cells its
// particles start in into LDS: cell-sorted particles of one block cover a
// few cells, so each node is read from L2/HBM once per block instead of once
// per particle and stage.  A lane whose stage cell lies outside the box reads
// global memory; no stage waits for the others.
__global__ __launch_bounds__(kPushBlock, 4) void k_push(PushParams P, Species cS, const double *__restrict__ node,
                                                     ParticlePtrs in, ParticlePtrs out,
                                                     unsigned long long *counters) {
    __shared__ double2 snode[kPushLdsNodes * kNodeStride2];
    __shared__ int sred[6][kPushBlock / 64];
    __shared__ double sqm[kMaxSpecies];
    if ((int64_t)blockIdx.x * kPushBlock >= live_bound(counters, P.n)) return;  // removed particles only
    const int tid = threadIdx.x;
    const int64_t id = (int64_t)blockIdx.x * kPushBlock + tid, idc = id < P.n ? id : P.n - 1;
    int clamps = 0;
    // the slot's species and state are read together (slots past n read
    // slot n - 1 and count as dead); q/m comes from the block's table
    const uint8_t sp_in = in.sp[idc];
    double X0[3], U0[4];
    for (int q = 0; q < 3; q++) X0[q] = in.x[q][idc];
    for (int q = 0; q < 4; q++) U0[q] = in.u[q][idc];
    if (tid == 0)
#pragma unroll
        for (int q = 0; q < kMaxSpecies; q++) sqm[q] = cS.qm[q];
    const uint8_t sp = id < P.n ? sp_in : kDead;
    const bool live = sp != kDead;
    const unsigned long long ballot = __ballot(live);
    if ((tid & 63) == 0 && ballot)
        atomicAdd(&counters[pushed_index(blockIdx.x)], (unsigned long long)__popcll(ballot));
    for (int q = 0; q < 3; q++) X0[q] = live ? X0[q] : 0.0;
    for (int q = 0; q < 4; q++) U0[q] = live ? U0[q] : 0.0;
    double Xs[3] = {X0[0], X0[1], X0[2]};
    double Us[4] = {U0[0], U0[1], U0[2], U0[3]};
    double Sx[3] = {0.0, 0.0, 0.0}, Su[4] = {0.0, 0.0, 0.0, 0.0};
    NodeBox B;
    B.lds = snode;
    {
        int c0[3];
        gather_cell(P.G, X0, c0);
        stage_box(P.G, node, live, c0, snode, sred, B);
    }
    const double qm = live ? sqm[sp] : 0.0;  // the table is written before the box's barriers
    if (tid == 0 && B.any) atomicAdd(&counters[pushed_index(blockIdx.x) + (B.use ? kPushedLds : kPushedGlobal)], 1ull);
#pragma unroll 1
    for (int st = 0; st < 4; st++) {
        int c[3];
        gather_cell(P.G, Xs, c);
        if (live) {
            double A[4];
            accel(P, node, B, c, qm, Xs, Us, A);
            double gam = stage_gamma(P, Us[3], A[3], clamps);
            double ig = rcp_nr(gam);
            double Kx[3] = {Us[0] * ig, Us[1] * ig, Us[2] * ig};
            double Ku[4] = {A[0] * ig, A[1] * ig, A[2] * ig, A[3] * ig};
            double wgt = (st == 0 || st == 3) ? 1.0 : 2.0;
            for (int q = 0; q < 3; q++) Sx[q] += wgt * Kx[q];
            for (int q = 0; q < 4; q++) Su[q] += wgt * Ku[q];
            if (st < 3) {
                double fac = (st < 2 ? 0.5 : 1.0) * P.dt;
                for (int q = 0; q < 3; q++) Xs[q] = X0[q] + fac * Kx[q];
                for (int q = 0; q < 4; q++) Us[q] = U0[q] + fac * Ku[q];
            }
        }
    }
    if (live) {
        double h6 = P.dt_6;
        for (int q = 0; q < 3; q++) out.x[q][id] = X0[q] + h6 * Sx[q];
        for (int q = 0; q < 4; q++) out.u[q][id] = U0[q] + h6 * Su[q];
    }
    wave_count(&counters[C_GAMMA_CLAMPS], clamps);
}

// ---------------------------------------------------------------------------
// Push ablations (FP64, Sec. 3.3 readings): the printed RK steps taken
// literally (RK = 1), the field tensor gathered once at x_n for all four
// stages (GATHER = 1) and the spatial-volume gather weights (WTS = 1).  They exist to measure the readings, so they gather
// from global memory without the LDS box.

// F^a_b at X from the nodes of cell c (row a at 4a .. 4a+3): trilinear
// weights (WTS = 0), or (WTS = 1, reading B) the sub-volume opposite each
// node, [X, c+1] or [c, X] per axis, times the spatial density at its
// centre, normalised by their sum.
template <int WTS>
__device__ __forceinline__ void gather_tensor(const PushParams &P, const double *__restrict__ node, const int c[3],
                                              const double X[3], double F[16]) {
    double w[3];
    for (int ax = 0; ax < 3; ax++) w[ax] = X[ax] - (double)c[ax];
    double W[8], sum = 0.0;
    for (int n = 0; n < 8; n++) {
        const int di = n & 1, dj = (n >> 1) & 1, dk = n >> 2;
        W[n] = (di ? w[0] : 1.0 - w[0]) * (dj ? w[1] : 1.0 - w[1]) * (dk ? w[2] : 1.0 - w[2]);
        if (WTS == 1 && P.h.m != 0.0) {
            const double mx = di ? 0.5 * ((double)c[0] + X[0]) : 0.5 * (X[0] + (double)c[0] + 1.0);
            const double my = dj ? 0.5 * ((double)c[1] + X[1]) : 0.5 * (X[1] + (double)c[1] + 1.0);
            const double mz = dk ? 0.5 * ((double)c[2] + X[2]) : 0.5 * (X[2] + (double)c[2] + 1.0);
            W[n] *= ks_volume_density(P.h.m, P.h.a, P.h.r_exc, mx - P.h.cx, my - P.h.cy, mz - P.h.cz);
        }
        sum += W[n];
    }
    if (WTS == 1) {
        const double inv = 1.0 / sum;
        for (int n = 0; n < 8; n++) W[n] *= inv;
    }
    for (int q = 0; q < 16; q++) F[q] = 0.0;
    for (int n = 0; n < 8; n++) {
        const double *src = node + 16 * P.G.node(c[0] + (n & 1), c[1] + ((n >> 1) & 1), c[2] + (n >> 2));
        for (int q = 0; q < 16; q++) F[q] += W[n] * src[q];
    }
}

// du^a/dtau at (X, U) with the field tensor gathered at X (GATHER = 0) or
// the one gathered at x_n (F0, GATHER = 1); Christoffel symbols at X.
template <int GATHER, int WTS>
__device__ __forceinline__ void accel_ablation(const PushParams &P, const double *__restrict__ node,
                                               const double F0[16], double qm, const double X[3], const double U[4],
                                               double A[4]) {
    double F[16];
    if (GATHER == 1) {
        for (int q = 0; q < 16; q++) F[q] = F0[q];
    } else {
        int c[3];
        gather_cell(P.G, X, c);
        gather_tensor<WTS>(P, node, c, X, F);
    }
    double Gm[4] = {0.0, 0.0, 0.0, 0.0};
    if (P.h.m != 0.0) {
        KSGrad kp;
        ks_grad(P.h.m, P.h.a, X[0] - P.h.cx, X[1] - P.h.cy, X[2] - P.h.cz, kp);
        gamma_uu(kp, U, Gm);
    }
    for (int a = 0; a < 4; a++)
        A[a] = qm * (F[4 * a] * U[0] + F[4 * a + 1] * U[1] + F[4 * a + 2] * U[2] + F[4 * a + 3] * U[3]) - Gm[a];
}

template <int RK, int GATHER, int WTS>
__global__ __launch_bounds__(kPushBlock) void k_push_ablation(PushParams P, Species cS,
                                                              const double *__restrict__ node, ParticlePtrs in,
                                                              ParticlePtrs out, unsigned long long *counters) {
    const int tid = threadIdx.x;
    const int64_t id = (int64_t)blockIdx.x * kPushBlock + tid;
    const uint8_t sp = id < P.n ? in.sp[id] : kDead;
    const bool live = sp != kDead;
    const unsigned long long ballot = __ballot(live);
    if ((tid & 63) == 0 && ballot)
        atomicAdd(&counters[pushed_index(blockIdx.x)], (unsigned long long)__popcll(ballot));
    if (!live) return;
    int clamps = 0;
    const double qm = cS.qm[sp];
    double X0[3], U0[4];
    for (int q = 0; q < 3; q++) X0[q] = in.x[q][id];
    for (int q = 0; q < 4; q++) U0[q] = in.u[q][id];
    double F0[16];
    if (GATHER == 1) {
        int c0[3];
        gather_cell(P.G, X0, c0);
        gather_tensor<WTS>(P, node, c0, X0, F0);
    }
    double Sx[3] = {0.0, 0.0, 0.0}, Su[4] = {0.0, 0.0, 0.0, 0.0};
    if (RK == 0) {
        // the default reading (as k_push): slopes (u_k, A_k)/gamma_k
        double Xs[3] = {X0[0], X0[1], X0[2]}, Us[4] = {U0[0], U0[1], U0[2], U0[3]};
        for (int st = 0; st < 4; st++) {
            double A[4];
            accel_ablation<GATHER, WTS>(P, node, F0, qm, Xs, Us, A);
            const double ig = 1.0 / stage_gamma(P, Us[3], A[3], clamps);
            const double wgt = (st == 0 || st == 3) ? 1.0 : 2.0;
            for (int q = 0; q < 3; q++) Sx[q] += wgt * (Us[q] * ig);
            for (int q = 0; q < 4; q++) Su[q] += wgt * (A[q] * ig);
            if (st < 3) {
                const double fac = (st < 2 ? 0.5 : 1.0) * P.dt;
                for (int q = 0; q < 3; q++) Xs[q] = X0[q] + fac * (Us[q] * ig);
                for (int q = 0; q < 4; q++) Us[q] = U0[q] + fac * (A[q] * ig);
            }
        }
        for (int q = 0; q < 3; q++) out.x[q][id] = X0[q] + P.dt_6 * Sx[q];
        for (int q = 0; q < 4; q++) out.u[q][id] = U0[q] + P.dt_6 * Su[q];
    } else {
        // the printed steps: averaged stage velocities ut_k = (u_n + u_k)/2,
        // x_k = x_n + ut_k dtau_{k-1}, dtau = dt/2g, dt/g, dt/g, dt/2g,
        // u_{k+1} = u_n + a_k dtau_k; sums 1:2:2:1 over 6 added to x_n, u_n
        double ut[4] = {U0[0], U0[1], U0[2], U0[3]}, uk[4] = {U0[0], U0[1], U0[2], U0[3]};
        double xk[3] = {X0[0], X0[1], X0[2]};
        double dtau_prev = 0.0;
        for (int st = 0; st < 4; st++) {
            if (st > 0) {
                for (int q = 0; q < 4; q++) ut[q] = 0.5 * (U0[q] + uk[q]);
                for (int q = 0; q < 3; q++) xk[q] = X0[q] + ut[q] * dtau_prev;
            }
            double A[4];
            accel_ablation<GATHER, WTS>(P, node, F0, qm, xk, ut, A);
            const double gam = stage_gamma(P, ut[3], A[3], clamps);
            const double dtau = (st == 0 || st == 3) ? P.dt / (2.0 * gam) : P.dt / gam;
            const double wgt = (st == 0 || st == 3) ? 1.0 : 2.0;
            for (int q = 0; q < 3; q++) Sx[q] += wgt * (ut[q] * dtau);
            for (int q = 0; q < 4; q++) Su[q] += wgt * (A[q] * dtau);
            for (int q = 0; q < 4; q++) uk[q] = U0[q] + A[q] * dtau;
            dtau_prev = dtau;
        }
        for (int q = 0; q < 3; q++) out.x[q][id] = X0[q] + Sx[q] / 6.0;
        for (int q = 0; q < 4; q++) out.u[q][id] = U0[q] + Su[q] / 6.0;
    }
    if (clamps) atomicAdd(&counters[C_GAMMA_CLAMPS], (unsigned long long)clamps);  // dead lanes have returned
}

template <int RK, int GA, int WT>
void launch_push_ablation(unsigned nb, const PushParams &P, const Species &S, const double *node, ParticlePtrs in,
                          ParticlePtrs out, unsigned long long *counters, hipStream_t s) {
    hipLaunchKernelGGL((k_push_ablation<RK, GA, WT>), dim3(nb), dim3(kPushBlock), 0, s, P, S, node, in, out,
                       counters);
}

void launch_push(const PushParams &P, const Species &S, const double *node, ParticlePtrs in, ParticlePtrs out,
                 unsigned long long *counters, hipStream_t s) {
    if (P.n <= 0) return;
    unsigned nb = (unsigned)((P.n + kPushBlock - 1) / kPushBlock);
    // modes are validated at creation: rk_mode, gather_mode, gather_weights in {0, 1}
    switch (P.rk_mode * 4 + P.gather_mode * 2 + P.gather_weights) {
    case 0: hipLaunchKernelGGL(k_push, dim3(nb), dim3(kPushBlock), 0, s, P, S, node, in, out, counters); break;
    case 1: launch_push_ablation<0, 0, 1>(nb, P, S, node, in, out, counters, s); break;
    case 2: launch_push_ablation<0, 1, 0>(nb, P, S, node, in, out, counters, s); break;
    case 3: launch_push_ablation<0, 1, 1>(nb, P, S, node, in, out, counters, s); break;
    case 4: launch_push_ablation<1, 0, 0>(nb, P, S, node, in, out, counters, s); break;
    case 5: launch_push_ablation<1, 0, 1>(nb, P, S, node, in, out, counters, s); break;
    case 6: launch_push_ablation<1, 1, 0>(nb, P, S, node, in, out, counters, s); break;
    default: launch_push_ablation<1, 1, 1>(nb, P, S, node, in, out, counters, s); break;
    }
}

// ---------------------------------------------------------------------------
// Deposition (Sec. 4).  The chord x_n -> x_{n+1} is split per axis at
//   x_r = min(min(i1,i2)+1, max(max(i1,i2), (x1+x2)/2))
// into two segments inside one cell each; a segment of displacement d adds
// FLUX^K = q d^K / dt to the four K-edges of its cell with transverse weights
// over the (I,J) face.  CURVED: area of the sub-rectangle opposite each node
// by the midpoint rule with density sqrt(g_II g_JJ - g_IJ^2) =
// sqrt(1 + f (1 - k_K^2)) (k null: k_1^2 + k_2^2 + k_3^2 = 1), normalised by
// their sum; FLAT: bilinear at the segment midpoint; both plus the exact
// segment-average term +-dI dJ / 12.  Current goes into int64 fixed point,
// so the sums do not depend on the order of the atomics.

struct DepCtx {
    Grid G;
    Hole h;
    double inv_dt;
    double jscale;
    int curved;
};

// Area density at a grid-coordinate point (24 of these per particle are
// most of the deposit's arithmetic).
__device__ __forceinline__ double area_density(const DepCtx &D, int K, double X, double Y, double Z) {
    if (D.h.m == 0.0) return 1.0;
    return ks_area_density(D.h.m, D.h.a, D.h.r_exc, K, X - D.h.cx, Y - D.h.cy, Z - D.h.cz);
}

// Destinations of the fixed-point current: straight to the global int64
// arrays, or into an LDS tile covering the block's particles.
struct GlobalAcc {
    unsigned long long *J[3];
    Grid G;
    unsigned long long *flags;
    __device__ __forceinline__ void add(int K, int i, int j, int k, long long v) const {
        fixed_add_checked(&J[K][G.g(i, j, k)], v, flags);
    }
};

struct LdsAcc {
    unsigned long long *sm;
    int lo0, lo1, lo2, bx, by, V;
    __device__ __forceinline__ void add(int K, int i, int j, int k, long long v) const {
        atomicAdd(&sm[K * V + ((k - lo2) * by + (j - lo1)) * bx + (i - lo0)], (unsigned long long)v);
    }
};

// Contributions of one segment A -> B inside `cell`, in units of the
// fixed-point current (FP64), added to v[K][bi + 2 bj] (the K-edge at
// cell + bi e_I + bj e_J, I = K+1, J = K+2).
__device__ __forceinline__ void dep_segment(const DepCtx &D, const double A[3], const double B[3], const int cell[3],
                                            double Q, double v[3][4]) {
    double d[3], mid[3];
    for (int ax = 0; ax < 3; ax++) {
        d[ax] = B[ax] - A[ax];
        mid[ax] = 0.5 * (A[ax] + B[ax]);
    }
#pragma unroll
    for (int K = 0; K < 3; K++) {
        const int I = (K + 1) % 3, J = (K + 2) % 3;
        double flux = Q * d[K] * D.inv_dt;
        if (flux == 0.0) continue;
        double t = d[I] * d[J] * (1.0 / 12.0);
        double loI = (double)cell[I], loJ = (double)cell[J];
        double w00, w10, w01, w11;
        double xi = mid[I] - loI, eta = mid[J] - loJ;
        if (!D.curved) {
            w00 = (1.0 - xi) * (1.0 - eta);
            w10 = xi * (1.0 - eta);
            w01 = (1.0 - xi) * eta;
            w11 = xi * eta;
        } else {
            double area[2][2];
            for (int bj = 0; bj < 2; bj++)
                for (int bi = 0; bi < 2; bi++) {
                    double i0 = bi ? loI : mid[I], i1 = bi ? mid[I] : loI + 1.0;
                    double j0 = bj ? loJ : mid[J], j1 = bj ? mid[J] : loJ + 1.0;
                    double P3[3];
                    P3[K] = mid[K];
                    P3[I] = 0.5 * (i0 + i1);
                    P3[J] = 0.5 * (j0 + j1);
                    area[bi][bj] = area_density(D, K, P3[0], P3[1], P3[2]) * ((i1 - i0) * (j1 - j0));
                }
            const double inv = rcp_nr(area[0][0] + area[1][0] + area[0][1] + area[1][1]);
            w00 = area[0][0] * inv;
            w10 = area[1][0] * inv;
            w01 = area[0][1] * inv;
            w11 = area[1][1] * inv;
        }
        w00 += t;
        w11 += t;
        w10 -= t;
        w01 -= t;
        double sc = flux * D.jscale;
        v[K][0] += sc * w00;
        v[K][1] += sc * w10;
        v[K][2] += sc * w01;
        v[K][3] += sc * w11;
    }
}

// Round the twelve edge sums of one cell to fixed point, add them to the
// accumulator and clear them.
template <typename Acc>
__device__ __forceinline__ void dep_flush(const Acc &acc, const int cell[3], double v[3][4]) {
#pragma unroll
    for (int K = 0; K < 3; K++) {
        const int I = (K + 1) % 3, J = (K + 2) % 3;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            {
                int id[3] = {cell[0], cell[1], cell[2]};
                id[I] += c & 1;
                id[J] += c >> 1;
                acc.add(K, id[0], id[1], id[2], fixed_rn(v[K][c]));
            }
            v[K][c] = 0.0;
        }
    }
}

// Both segments of one chord: summed in FP64 registers first when they lie
// in the same cell (two terms in a fixed order), so each particle's share of
// an edge is rounded to fixed point once and the atomic sums stay
// independent of order.
template <typename Acc>
__device__ __forceinline__ void dep_chord(const DepCtx &D, const Acc &acc, const double X1[3], const double xr[3],
                                          const double X2[3], const int c1[3], const int c2[3], double Q) {
    double v[3][4];
#pragma unroll
    for (int K = 0; K < 3; K++)
        for (int c = 0; c < 4; c++) v[K][c] = 0.0;
    dep_segment(D, X1, xr, c1, Q, v);
    if (c1[0] != c2[0] || c1[1] != c2[1] || c1[2] != c2[2]) dep_flush(acc, c1, v);
    dep_segment(D, xr, X2, c2, Q, v);
    dep_flush(acc, c2, v);
}

constexpr int kDepBlock = 256;
constexpr int kDepPPT = 4;      // particles per thread

// Particle p (0 .. kDepPPT-1) of thread tid within its block's slots: the 64
// lanes of a wave take slots kDepPPT * (kDepBlock / 64) = 16 apart.  In a
// cell-sorted block a cell holds about that many particles, so the lanes of
// one instruction add to different cells' edges instead of queueing on the
// same LDS addresses (the integer sums do not depend on the order).
__device__ __forceinline__ int dep_slot(int p, int tid) {
    return (tid & 63) * (kDepPPT * (kDepBlock / 64)) + p * (kDepBlock / 64) + (tid >> 6);
}
constexpr int kDepLds = 6656;  // int64 LDS entries of the current box (52 KiB: three blocks per CU)

// Zigzag split of one chord: relay point and the two cells; false when the
// move is longer than a cell or leaves the ghost layer.
__device__ __forceinline__ bool zigzag(const Grid &G, const double x1[3], const double x2[3], double xr[3],
                                       int c1[3], int c2[3]) {
    bool ok = true;
    for (int ax = 0; ax < 3; ax++) {
        int i1 = (int)floor(x1[ax]), i2 = (int)floor(x2[ax]);
        double lo = (double)((i1 < i2 ? i1 : i2) + 1);
        double hi = (double)(i1 > i2 ? i1 : i2);
        double mid = 0.5 * (x1[ax] + x2[ax]);
        double v = mid > hi ? mid : hi;
        xr[ax] = v < lo ? v : lo;
        c1[ax] = i1;
        c2[ax] = i2;
        int nn = G.dim(ax);
        if (c1[ax] < -1 || c1[ax] > nn || c2[ax] < -1 || c2[ax] > nn || !(fabs(x2[ax] - x1[ax]) < 1.0)) ok = false;
    }
    return ok;
}

// One block deposits kDepBlock*kDepPPT consecutive particles.  When the
// current they touch fits an LDS box (sorted particles: a few cells of one
// tile), it is summed there with int64 LDS atomics and flushed once with
// global atomics; otherwise the block writes global atomics directly.  Both
// routes add the same integers, so the result does not depend on the route
// or the order.  Removal follows the deposit of the final move.
__global__ __launch_bounds__(kDepBlock) void k_deposit(DepCtx D, Species cS, double r_rm, double rscale,
                                                       ParticlePtrs xo, ParticlePtrs xn, int64_t n, FieldPtrs F,
                                                       unsigned long long *counters) {
    __shared__ unsigned long long sm[kDepLds];
    __shared__ int sred[6][kDepBlock / 64];
    __shared__ double sQ[kMaxSpecies];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * (kDepBlock * kDepPPT);
    if (base >= live_bound(counters, n)) return;  // removed particles only
    // Every slot's chord is read at once (slots past n read slot n - 1 and
    // count as dead), so the loads are in flight together.
    uint8_t SP[kDepPPT];
    double P1[kDepPPT][3], P2[kDepPPT][3];
#pragma unroll
    for (int p = 0; p < kDepPPT; p++) {
        const int64_t id = base + dep_slot(p, tid), idc = id < n ? id : n - 1;
        const uint8_t s = xo.sp[idc];
        SP[p] = id < n ? s : kDead;
        for (int ax = 0; ax < 3; ax++) {
            P1[p][ax] = xo.x[ax][idc];
            P2[p][ax] = xn.x[ax][idc];
        }
    }
    if (tid == 0)
#pragma unroll
        for (int q = 0; q < kMaxSpecies; q++) sQ[q] = cS.charge[q];
    __syncthreads();
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
#pragma unroll
    for (int p = 0; p < kDepPPT; p++) {
        if (SP[p] != kDead) {
            double xr[3];
            int c1[3], c2[3];
            if (zigzag(D.G, P1[p], P2[p], xr, c1, c2) && sQ[SP[p]] != 0.0)
                for (int ax = 0; ax < 3; ax++) {
                    int a = c1[ax] < c2[ax] ? c1[ax] : c2[ax];
                    int b = (c1[ax] > c2[ax] ? c1[ax] : c2[ax]) + 1;
                    lo[ax] = a < lo[ax] ? a : lo[ax];
                    hi[ax] = b > hi[ax] ? b : hi[ax];
                }
        }
    }
    for (int ax = 0; ax < 3; ax++) {
        int a = wave_min(lo[ax]), b = wave_max(hi[ax]);
        if ((tid & 63) == 0) {
            sred[ax][tid >> 6] = a;
            sred[3 + ax][tid >> 6] = b;
        }
    }
    __syncthreads();
    int blo[3], bhi[3];
    for (int ax = 0; ax < 3; ax++) {
        blo[ax] = sred[ax][0];
        bhi[ax] = sred[3 + ax][0];
        for (int w = 1; w < kDepBlock / 64; w++) {
            blo[ax] = sred[ax][w] < blo[ax] ? sred[ax][w] : blo[ax];
            bhi[ax] = sred[3 + ax][w] > bhi[ax] ? sred[3 + ax][w] : bhi[ax];
        }
    }
    const bool any = bhi[0] >= blo[0];
    const int bx = any ? bhi[0] - blo[0] + 1 : 0, by = any ? bhi[1] - blo[1] + 1 : 0,
              bz = any ? bhi[2] - blo[2] + 1 : 0;
    const int64_t V64 = (int64_t)bx * by * bz;
    const bool use_lds = any && 3 * V64 <= kDepLds;
    const int V = use_lds ? (int)V64 : 0;
    if (use_lds) {
        for (int e = tid; e < 3 * V; e += kDepBlock) sm[e] = 0ull;
        __syncthreads();
    }
    if (tid == 0 && any) atomicAdd(&counters[use_lds ? C_DEP_LDS : C_DEP_GLOBAL], 1ull);
    LdsAcc la{sm, blo[0], blo[1], blo[2], bx, by, V};
    GlobalAcc ga{{F.Jint[0], F.Jint[1], F.Jint[2]}, D.G, &counters[C_FLAGS]};
    int n_horizon = 0, n_outer = 0;
    // the first chord is kept from above; the next slot's chord is read
    // while this one is deposited
    double nX1[3] = {P1[0][0], P1[0][1], P1[0][2]}, nX2[3] = {P2[0][0], P2[0][1], P2[0][2]};
#pragma unroll 1
    for (int p = 0; p < kDepPPT; p++) {
        double X1[3], X2[3];
        for (int ax = 0; ax < 3; ax++) {
            X1[ax] = nX1[ax];
            X2[ax] = nX2[ax];
        }
        if (p + 1 < kDepPPT) {
            const int64_t idn = base + dep_slot(p + 1, tid), idc = idn < n ? idn : n - 1;
            for (int ax = 0; ax < 3; ax++) {
                nX1[ax] = xo.x[ax][idc];
                nX2[ax] = xn.x[ax][idc];
            }
        }
        if (SP[p] == kDead) continue;
        int64_t id = base + dep_slot(p, tid);
        double Q = sQ[SP[p]];
        double xr[3];
        int c1[3], c2[3];
        bool ok = zigzag(D.G, X1, X2, xr, c1, c2);
        if (ok && Q != 0.0) {
            if (use_lds)
                dep_chord(D, la, X1, xr, X2, c1, c2, Q);
            else
                dep_chord(D, ga, X1, xr, X2, c1, c2, Q);
        } else if (!ok) {
            atomicOr(&counters[C_FLAGS], kFlagLongMove);
        }
        const double *x2 = X2;
        const bool inside_rm = ks_radius_below(D.h.a, x2[0] - D.h.cx, x2[1] - D.h.cy, x2[2] - D.h.cz, r_rm);
        bool outside = false;
        for (int ax = 0; ax < 3; ax++) {
            double nn = (double)D.G.dim(ax);
            if (!(x2[ax] >= 0.0 && x2[ax] < nn)) outside = true;
        }
        if (inside_rm) {
            // the removed charge stays on the nodes for the Gauss diagnostic
            int c[3];
            double w[3];
            bool inb = true;
            for (int ax = 0; ax < 3; ax++) {
                c[ax] = (int)floor(x2[ax]);
                w[ax] = x2[ax] - (double)c[ax];
                if (c[ax] < -1 || c[ax] > D.G.dim(ax)) inb = false;
            }
            if (inb && Q != 0.0) {
                double sc = Q * rscale;
                for (int dk = 0; dk < 2; dk++)
                    for (int dj = 0; dj < 2; dj++)
                        for (int di = 0; di < 2; di++) {
                            double W = (di ? w[0] : 1.0 - w[0]) * (dj ? w[1] : 1.0 - w[1]) * (dk ? w[2] : 1.0 - w[2]);
                            fixed_add_checked(&F.rho_abs[D.G.g(c[0] + di, c[1] + dj, c[2] + dk)],
                                              __double2ll_rn(sc * W), &counters[C_FLAGS]);
                        }
            }
            xo.sp[id] = kDead;
            n_horizon++;
        } else if (outside) {
            xo.sp[id] = kDead;
            n_outer++;
        }
    }
    wave_count(&counters[C_REMOVED_HORIZON], n_horizon);
    wave_count(&counters[C_REMOVED_OUTER], n_outer);
    if (use_lds) {
        __syncthreads();
        flush_box(sm, V, bx, by, blo, F.Jint, D.G, &counters[C_FLAGS]);
    }
}

void launch_deposit(const Grid &G, const Hole &h, double dt, int deposit_mode, double r_rm, double jscale,
                    double rscale, const Species &S, ParticlePtrs xold, ParticlePtrs xnew, int64_t n,
                    FieldPtrs &F, unsigned long long *counters, hipStream_t s) {
    if (n <= 0) return;
    DepCtx D;
    D.G = G;
    D.h = h;
    D.inv_dt = 1.0 / dt;
    D.jscale = jscale;
    D.curved = deposit_mode == 0;
    const int64_t per = kDepBlock * kDepPPT;
    unsigned nb = (unsigned)((n + per - 1) / per);
    hipLaunchKernelGGL(k_deposit, dim3(nb), dim3(kDepBlock), 0, s, D, S, r_rm, rscale, xold, xnew, n, F, counters);
}

// ---------------------------------------------------------------------------
// Load: future root of the mass shell from the covariant spatial components,
//   g^{44} u_4^2 + 2 (g^{4i} u_i) u_4 + g^{ij} u_i u_j + c^2 = 0,  u^4 = g^{4b} u_b > 0,
// then u^a = g^{ab} u_b.  Dropped particles (non-finite, outside the grid,
// inside r_rm) are stored as dead slots.
__device__ __forceinline__ bool load_one(const Grid &G, const Hole &h, double c, double r_rm,
                                         const double *__restrict__ xin, const double *__restrict__ ucin, int64_t n,
                                         int species, const ParticlePtrs &out, int64_t off, int64_t id) {
    double X[3] = {xin[id], xin[n + id], xin[2 * n + id]};
    double uc[3] = {ucin[id], ucin[n + id], ucin[2 * n + id]};
    bool ok = true;
    for (int ax = 0; ax < 3; ax++) {
        if (!isfinite(X[ax]) || !isfinite(uc[ax])) ok = false;
        if (!(X[ax] >= 0.0 && X[ax] < (double)G.dim(ax))) ok = false;
    }
    double U[4] = {0.0, 0.0, 0.0, c};
    if (ok) {
        double x = X[0] - h.cx, y = X[1] - h.cy, z = X[2] - h.cz;
        double f = 0.0, k[3] = {0.0, 0.0, 0.0};
        if (h.m != 0.0) {
            double r = ks_radius(h.a, x, y, z);
            if (r < r_rm) ok = false;
            if (ok) {
                KSPoint<double> p;
                ks_point(h.m, h.a, x, y, z, p);
                f = p.f;
                k[0] = p.k0;
                k[1] = p.k1;
                k[2] = p.k2;
            }
        }
        if (ok) {
            // g^{ab} = eta^{ab} - f k^a k^b, k^a = (k_1, k_2, k_3, -1)
            double ku[4] = {k[0], k[1], k[2], -1.0};
            const double eta[4] = {1.0, 1.0, 1.0, -1.0};
            double gi[4][4];
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) gi[a][b] = (a == b ? eta[a] : 0.0) - f * ku[a] * ku[b];
            double A = gi[3][3];
            double B = gi[3][0] * uc[0] + gi[3][1] * uc[1] + gi[3][2] * uc[2];
            double C = c * c;
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) C += gi[i][j] * uc[i] * uc[j];
            double disc = B * B - A * C;
            disc = disc < 0.0 ? 0.0 : disc;
            double sq = sqrt(disc);
            double u4l = (B <= 0.0) ? (sq - B) / A : -C / (sq + B);
            double ul[4] = {uc[0], uc[1], uc[2], u4l};
            for (int a = 0; a < 4; a++) U[a] = gi[a][0] * ul[0] + gi[a][1] * ul[1] + gi[a][2] * ul[2] + gi[a][3] * ul[3];
        }
    }
    int64_t o = off + id;
    for (int ax = 0; ax < 3; ax++) out.x[ax][o] = ok ? X[ax] : 0.0;
    for (int q = 0; q < 4; q++) out.u[q][o] = U[q];
    out.sp[o] = ok ? (uint8_t)species : kDead;
    return ok;
}

__global__ void k_load(Grid G, Hole h, double c, double r_rm, const double *__restrict__ xin,
                       const double *__restrict__ ucin, int64_t n, int species, ParticlePtrs out, int64_t off,
                       unsigned long long *counters) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = id < n && load_one(G, h, c, r_rm, xin, ucin, n, species, out, off, id);
    wave_count(&counters[C_LOAD_KEPT], ok ? 1 : 0);
}

void launch_load(const Grid &G, const Hole &h, double c, double r_rm, const double *xin, const double *ucin,
                 int64_t n, int species, ParticlePtrs out, int64_t offset, unsigned long long *counters,
                 hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_load, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, G, h, c, r_rm, xin, ucin, n,
                       species, out, offset, counters);
}

__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < n) p[id] = 0ull;
}

void launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
}

__global__ void k_zero3_u64(unsigned long long *p0, unsigned long long *p1, unsigned long long *p2, int64_t n) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < n) {
        p0[id] = 0ull;
        p1[id] = 0ull;
        p2[id] = 0ull;
    }
}

void launch_zero3_u64(unsigned long long *const p[3], int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero3_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p[0], p[1], p[2], n);
}

}  // namespace grpic
