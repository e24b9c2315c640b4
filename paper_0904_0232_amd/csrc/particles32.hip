// FP32-mixed particle kernels.  A particle is a packed int32 cell
// (i+1 | (j+1) << 10 | (k+1) << 20), an FP32 offset inside that cell and an
// FP32 contravariant four-velocity: 32 bytes plus the species byte.
// Gather, Lorentz term, RK4 stages and deposition weights run in FP32 on
// offsets relative to the particle's cell (so the position error does not
// grow with the grid size).  In the pusher the radius quartic is always
// solved in FP64 from the exact cell + offset, and within r_fp64
// (max(r_+ + 4 m, 1.25 r_exc)) of the hole the metric gradients and the
// Christoffel contraction are evaluated in FP64; the deposition's area
// densities are FP32 beyond r_fp64 and FP64 within it.
#include <type_traits>
#include "grpic_dev.h"
#include "grpic_impl.h"

namespace grpic {

// Wavefront min / max (DPP reductions of the device library); the result is
// the same in every lane.
__device__ __forceinline__ int wave_min32(int v) { return __ockl_wfred_min_i32(v); }
__device__ __forceinline__ int wave_max32(int v) { return __ockl_wfred_max_i32(v); }

// Add a per-lane count to a device counter with one atomic per wavefront:
// same-address atomics from many waves serialise across the XCDs.  Every
// lane of the wave must reach the call.
__device__ __forceinline__ void wave_count32(unsigned long long *ctr, int v) {
    const int s = __ockl_wfred_add_i32(v);
    if (s != 0 && (threadIdx.x & 63) == 0) atomicAdd(ctr, (unsigned long long)s);
}

__device__ __forceinline__ void hole_rel(const Hole &h, int i, int j, int k, const float X[3], double &x, double &y,
                                         double &z) {
    x = ((double)i - h.cx) + (double)X[0];
    y = ((double)j - h.cy) + (double)X[1];
    z = ((double)k - h.cz) + (double)X[2];
}

// FP32 node tensor rows in LDS: 16 floats per node padded to 20, so nodes one
// apart start 4 banks apart.
constexpr int kNode32Stride4 = 5;  // float4 per staged node

// A block's LDS copy of the FP32 node tensor over the node box [lo, lo + n)
// (x fastest), or use = false.
struct NodeBox32 {
    const float4 *lds;
    int lo[3], n[3];
    bool use;
    bool any;  // the block has a live lane
};

// L^a += sum over the 8 nodes of W_n (F_n u)^a from the (0,0,0) node p and
// strides (in float4) si, sj, sk.
__device__ __forceinline__ void gather_rows32(const float4 *p, int64_t si, int64_t sj, int64_t sk, const float w[3],
                                              const float U[4], float L[4]) {
#pragma unroll 1
    for (int q = 0; q < 4; q++) {
        const int dj = q & 1, dk = q >> 1;
        const float wyz = (dj ? w[1] : 1.0f - w[1]) * (dk ? w[2] : 1.0f - w[2]);
        const float4 *pq = p + dj * sj + dk * sk;
#pragma unroll
        for (int di = 0; di < 2; di++) {
            const float W = (di ? w[0] : 1.0f - w[0]) * wyz;
            const float4 *pn = pq + di * si;
#pragma unroll
            for (int a = 0; a < 4; a++) {
                float4 f = pn[a];
                float row = f.x * U[0] + f.y * U[1] + f.z * U[2] + f.w * U[3];
                L[a] += W * row;
            }
        }
    }
}

// Gather cell of offset X relative to cell `base`: base + floor(X), clamped
// to the grid.
__device__ __forceinline__ void gather_cell32(const Grid &G, const int base[3], const float X[3], int c[3]) {
    for (int ax = 0; ax < 3; ax++) {
        int n = G.dim(ax);
        int ci = base[ax] + (int)floorf(X[ax]);
        c[ax] = ci < 0 ? 0 : (ci > n - 1 ? n - 1 : ci);
    }
}

// L^a = F^a_b u^b gathered from the FP32 node tensor at offset X relative to
// cell `base` (X may leave [0,1) by up to a cell), from the nodes of the
// gather cell c, read from the block's LDS box when it holds the cell's nodes.
__device__ __forceinline__ void gather_lorentz32(const Grid &G, const float *__restrict__ node, const NodeBox32 &B,
                                                 const int base[3], const int c[3], const float X[3],
                                                 const float U[4], float L[4]) {
    float w[3];
    for (int ax = 0; ax < 3; ax++) w[ax] = (float)(base[ax] - c[ax]) + X[ax];
    L[0] = L[1] = L[2] = L[3] = 0.0f;
    bool inside = B.use;
    for (int ax = 0; ax < 3; ax++) inside = inside && c[ax] >= B.lo[ax] && c[ax] + 1 < B.lo[ax] + B.n[ax];
    if (inside) {
        const int64_t l = ((int64_t)(c[2] - B.lo[2]) * B.n[1] + (c[1] - B.lo[1])) * B.n[0] + (c[0] - B.lo[0]);
        gather_rows32(B.lds + kNode32Stride4 * l, kNode32Stride4, kNode32Stride4 * B.n[0],
                      (int64_t)kNode32Stride4 * B.n[0] * B.n[1], w, U, L);
    } else {
        const int64_t sj = G.nx + 1, sk = (int64_t)(G.nx + 1) * (G.ny + 1);
        gather_rows32(reinterpret_cast<const float4 *>(node) + 4 * G.node(c[0], c[1], c[2]), 4, 4 * sj, 4 * sk, w,
                      U, L);
    }
}

__device__ __forceinline__ void accel32(const PushParams &P, const Mixed &M, const float *__restrict__ node,
                                        const NodeBox32 &B, const int c[3], float qm, int i, int j, int k,
                                        const float X[3], const float U[4], float A[4]) {
    float L[4];
    const int base[3] = {i, j, k};
    gather_lorentz32(P.G, node, B, base, c, X, U, L);
    float Gm[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (P.h.m != 0.0) {
        double x, y, z;
        hole_rel(P.h, i, j, k, X, x, y, z);
        double r = ks_radius_nr(P.h.a, x, y, z);
        if (r < M.r_fp64) {
            KSGradT<double> kp;
            ks_grad_r<double>(P.h.m, P.h.a, x, y, z, r, kp);
            double Ud[4] = {U[0], U[1], U[2], U[3]}, Gd[4];
            gamma_uu<double>(kp, Ud, Gd);
            for (int a = 0; a < 4; a++) Gm[a] = (float)Gd[a];
        } else {
            KSGradT<float> kp;
            ks_grad_r<float>((float)P.h.m, (float)P.h.a, (float)x, (float)y, (float)z, (float)r, kp);
            gamma_uu<float>(kp, U, Gm);
        }
    }
#pragma unroll
    for (int a = 0; a < 4; a++) A[a] = qm * L[a] - Gm[a];
}

__device__ __forceinline__ float stage_gamma32(const PushParams &P, float u4, float a4, int &clamps) {
    float uc = u4 * (float)P.inv_c;
    if (P.gamma_mode == 1) return uc;
    float disc = uc * uc + 4.0f * a4 * (float)P.dt_2c;
    if (disc < 0.0f) {
        disc = 0.0f;
        clamps++;
    }
    return 0.5f * (uc + sqrtf(disc));
}

constexpr int kPush32Block = 256;
constexpr int kPush32LdsNodes = 448;  // 35 KB of padded FP32 node tensor per block
constexpr int kStage32InFlight = 8;    // node pieces per thread in flight while the box is staged

// Stage, once per push, the FP32 node box of the cells the block's live
// lanes start in, widened by one cell on every side when that still fits (as
// the FP64 pusher does).  Every thread of the block calls this; it
// synchronises the block after the box reduction and after the copy.
__device__ __forceinline__ void stage_box32(const Grid &G, const float *__restrict__ node, bool live, const int c[3],
                                            float4 *snode, int (*sred)[kPush32Block / 64], NodeBox32 &B) {
    const int tid = threadIdx.x;
    for (int ax = 0; ax < 3; ax++) {
        int a = wave_min32(live ? c[ax] : (1 << 30)), b = wave_max32(live ? c[ax] : -(1 << 30));
        if ((tid & 63) == 0) {
            sred[ax][tid >> 6] = a;
            sred[3 + ax][tid >> 6] = b;
        }
    }
    __syncthreads();
    int lo[2][3], n[2][3], count[2] = {1, 1};
    for (int ax = 0; ax < 3; ax++) {
        int a = sred[ax][0], b = sred[3 + ax][0];
        for (int w = 1; w < kPush32Block / 64; w++) {
            a = sred[ax][w] < a ? sred[ax][w] : a;
            b = sred[3 + ax][w] > b ? sred[3 + ax][w] : b;
        }
        if (ax == 0) B.any = b >= a;
        for (int e = 0; e < 2; e++) {  // e = 1: widened by one cell, within the nodes 0 .. dim
            const int l = a - e < 0 ? 0 : a - e;
            const int h = b + 1 + e > G.dim(ax) ? G.dim(ax) : b + 1 + e;
            lo[e][ax] = l;
            n[e][ax] = b >= a ? h - l + 1 : 0;
            count[e] = (n[e][ax] > 0 && count[e] <= kPush32LdsNodes) ? count[e] * n[e][ax] : 0;
        }
    }
    // count = 0: no live lane
    const int e = (count[1] > 0 && count[1] <= kPush32LdsNodes) ? 1 : 0;
    for (int ax = 0; ax < 3; ax++) {
        B.lo[ax] = lo[e][ax];
        B.n[ax] = n[e][ax];
    }
    B.use = count[e] > 0 && count[e] <= kPush32LdsNodes;
    if (B.use) {
        const float4 *src = reinterpret_cast<const float4 *>(node);
        const int nb0 = B.n[0], nb01 = B.n[0] * B.n[1];
        const float inv0 = __builtin_amdgcn_rcpf((float)nb0), inv01 = __builtin_amdgcn_rcpf((float)nb01);
        // N pieces per thread are read before any is stored, so the copy
        // takes one or two memory round trips instead of one per piece; small
        // boxes (up to 4 pieces per thread) read 4 at a time
        const int total = count[e] * 4;
        auto copy = [&](auto in_flight) {
            constexpr int N = decltype(in_flight)::value;
            for (int q0 = tid; q0 < total; q0 += kPush32Block * N) {
                float4 v[N];
#pragma unroll
                for (int t = 0; t < N; t++) {
                    const int q = q0 + t * kPush32Block < total ? q0 + t * kPush32Block : total - 1;
                    const int l = q >> 2, part = q & 3;
                    const int lk = small_div(l, inv01), r = l - lk * nb01, lj = small_div(r, inv0), li = r - lj * nb0;
                    v[t] = src[4 * G.node(B.lo[0] + li, B.lo[1] + lj, B.lo[2] + lk) + part];
                }
#pragma unroll
                for (int t = 0; t < N; t++) {  // a clamped slot rewrites piece total - 1 with its own value
                    const int q = q0 + t * kPush32Block < total ? q0 + t * kPush32Block : total - 1;
                    snode[kNode32Stride4 * (q >> 2) + (q & 3)] = v[t];
                }
            }
        };
        if (total <= 4 * kPush32Block)
            copy(std::integral_constant<int, 4>());
        else
            copy(std::integral_constant<int, kStage32InFlight>());
    }
    __syncthreads();
}

// The same RK4 in coordinate time as the FP64 pusher, on offsets relative
// to the particle's cell; the cell is re-based after the step.  The nodes are
// staged in LDS once per block and push, as in the FP64 pusher.
// Block `blk` of the push (particles blk * kPush32Block ...); LDS scratch
// snode and sred come from the calling kernel.  Every thread of the block
// calls this.
__device__ __forceinline__ void push32_block(const PushParams &P, const Mixed &M, const Species &cS,
                                             const float *__restrict__ node, const ParticlePtrs32 &in,
                                             const ParticlePtrs32 &out, unsigned long long *counters, int64_t blk,
                                             float4 *snode, int (*sred)[kPush32Block / 64], double *sqm) {
    if (P.n <= 0 || blk * kPush32Block >= live_bound(counters, P.n)) return;  // uniform: removed particles only
    const int tid = threadIdx.x;
    const int64_t id = blk * kPush32Block + tid, idc = id < P.n ? id : P.n - 1;
    int clamps = 0;
    // the slot's species and state are read together (slots past n read
    // slot n - 1 and count as dead); q/m comes from the block's table
    const uint8_t sp_in = in.sp[idc];
    const int32_t cell_in = in.cell[idc];
    float X0[3], U0[4];
    for (int q = 0; q < 3; q++) X0[q] = in.off[q][idc];
    for (int q = 0; q < 4; q++) U0[q] = in.u[q][idc];
    if (tid == 0)
#pragma unroll
        for (int q = 0; q < kMaxSpecies; q++) sqm[q] = cS.qm[q];
    const uint8_t sp = id < P.n ? sp_in : kDead;
    const bool alive = sp != kDead;
    const unsigned long long live = __ballot(alive);
    if ((tid & 63) == 0 && live)
        atomicAdd(&counters[pushed_index((unsigned)blk)], (unsigned long long)__popcll(live));
    int i = 0, j = 0, k = 0;
    if (alive) unpack_cell(cell_in, i, j, k);
    for (int q = 0; q < 3; q++) X0[q] = alive ? X0[q] : 0.0f;
    for (int q = 0; q < 4; q++) U0[q] = alive ? U0[q] : 0.0f;
    const int base[3] = {i, j, k};
    float Xs[3] = {X0[0], X0[1], X0[2]};
    float Us[4] = {U0[0], U0[1], U0[2], U0[3]};
    float Sx[3] = {0.0f, 0.0f, 0.0f}, Su[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    const float dt = (float)P.dt;
    NodeBox32 B;
    B.lds = snode;
    {
        int c0[3];
        gather_cell32(P.G, base, X0, c0);
        stage_box32(P.G, node, alive, c0, snode, sred, B);
    }
    const float qm = alive ? (float)sqm[sp] : 0.0f;  // the table is written before the box's barriers
    if (tid == 0 && B.any)
        atomicAdd(&counters[pushed_index((unsigned)blk) + (B.use ? kPushedLds : kPushedGlobal)], 1ull);
#pragma unroll 1
    for (int st = 0; st < 4; st++) {
        int c[3];
        gather_cell32(P.G, base, Xs, c);
        if (alive) {
            float A[4];
            accel32(P, M, node, B, c, qm, i, j, k, Xs, Us, A);
            float gam = stage_gamma32(P, Us[3], A[3], clamps);
            float ig = recip<float>(gam);
            float Kx[3] = {Us[0] * ig, Us[1] * ig, Us[2] * ig};
            float Ku[4] = {A[0] * ig, A[1] * ig, A[2] * ig, A[3] * ig};
            float wgt = (st == 0 || st == 3) ? 1.0f : 2.0f;
            for (int q = 0; q < 3; q++) Sx[q] += wgt * Kx[q];
            for (int q = 0; q < 4; q++) Su[q] += wgt * Ku[q];
            if (st < 3) {
                float fac = (st < 2 ? 0.5f : 1.0f) * dt;
                for (int q = 0; q < 3; q++) Xs[q] = X0[q] + fac * Kx[q];
                for (int q = 0; q < 4; q++) Us[q] = U0[q] + fac * Ku[q];
            }
        }
    }
    if (alive) {
        const float h6 = (float)P.dt_6;
        int cc[3] = {i, j, k};
        for (int q = 0; q < 3; q++) {
            float xo = X0[q] + h6 * Sx[q];
            float fl = floorf(xo);
            xo -= fl;
            // xo in (-2^-25, 0) gives xo - fl = 1.0f after rounding: that
            // point is the next cell's face, offset 0, so offsets stay in [0, 1)
            if (xo >= 1.0f) {
                xo = 0.0f;
                fl += 1.0f;
            }
            int nc = cc[q] + (int)fl;
            // a cell outside the ghost layer cannot be packed; the particle is
            // removed as outside by the deposition kernel either way
            nc = nc < -1 ? -1 : (nc > 1022 ? 1022 : nc);
            cc[q] = nc;
            out.off[q][id] = xo;
        }
        out.cell[id] = pack_cell(cc[0], cc[1], cc[2]);
        for (int q = 0; q < 4; q++) out.u[q][id] = U0[q] + h6 * Su[q];
    }
    wave_count32(&counters[C_GAMMA_CLAMPS], clamps);
}

__global__ __launch_bounds__(kPush32Block, 4) void k_push32(PushParams P, Mixed M, Species cS,
                                                           const float *__restrict__ node, ParticlePtrs32 in,
                                                           ParticlePtrs32 out, unsigned long long *counters) {
    __shared__ float4 snode[kPush32LdsNodes * kNode32Stride4];
    __shared__ int sred[6][kPush32Block / 64];
    __shared__ double sqm[kMaxSpecies];
    push32_block(P, M, cS, node, in, out, counters, blockIdx.x, snode, sred, sqm);
}

void launch_push32(const PushParams &P, const Mixed &M, const Species &S, const float *node, ParticlePtrs32 in,
                   ParticlePtrs32 out, unsigned long long *counters, hipStream_t s) {
    if (P.n <= 0) return;
    unsigned nb = (unsigned)((P.n + kPush32Block - 1) / kPush32Block);
    hipLaunchKernelGGL(k_push32, dim3(nb), dim3(kPush32Block), 0, s, P, M, S, node, in, out, counters);
}

// ---------------------------------------------------------------------------
// Deposition in FP32 coordinates local to the old cell (Sec. 4, same zigzag
// and weights as the FP64 kernel), int64 fixed-point accumulation.


// Area density sqrt(1 + f (1 - k_K^2)) at a point given as cell + local
// offset (O: the cell corner relative to the hole in FP32, P3: the offset).
// Beyond r_fp64 in FP32 with the hardware square root and reciprocals:
//   f (1 - k_K^2) = t g,  t = 2 m r / S4,  S4 = r^4 + a^2 z^2,
//   g = (r - z)(r + z) (K = 2)  or  r^2 (1 - q)(1 + q), q = n / Dn (K = 0, 1)
// (n, Dn as in the FP64 density).  Within r_fp64, and wherever R < |a|, in
// FP64 from the exact cell coordinates; every excision decision (r_exc <
// r_fp64) is taken there.
__device__ __forceinline__ float area_density32(const Dep32 &D, int K, const int base[3], const float O[3],
                                                const float P3[3]) {
    if (D.h.m == 0.0) return 1.0f;
    const float x = O[0] + P3[0], y = O[1] + P3[1], z = O[2] + P3[2];
    const float a = D.af, a2 = a * a, a2z2 = a2 * (z * z);
    const float b = fmaf(x, x, fmaf(y, y, z * z)) - a2;
    const float r2 = 0.5f * (b + __builtin_amdgcn_sqrtf(fmaf(b, b, 4.0f * a2z2)));
    if (b < 0.0f || r2 < D.r_fp64_sq) {
        const double xd = ((double)base[0] - D.h.cx) + (double)P3[0];
        const double yd = ((double)base[1] - D.h.cy) + (double)P3[1];
        const double zd = ((double)base[2] - D.h.cz) + (double)P3[2];
        return (float)ks_area_density(D.h.m, D.h.a, D.h.r_exc, K, xd, yd, zd);
    }
    const float r = __builtin_amdgcn_sqrtf(r2);
    const float t = D.m2 * r * __builtin_amdgcn_rcpf(fmaf(r2, r2, a2z2));
    float g;
    if (K == 2) {
        g = (r - z) * (r + z);
    } else {
        const float q = (K == 0 ? r * x - a * y : r * y + a * x) * __builtin_amdgcn_rcpf(r2 + a2);
        g = r2 * ((1.0f - q) * (1.0f + q));
    }
    return __builtin_amdgcn_sqrtf(fmaf(t, g, 1.0f));
}

struct GlobalAcc32 {
    unsigned long long *J[3];
    Grid G;
    unsigned long long *flags;
    __device__ __forceinline__ void add(int K, int i, int j, int k, long long v) const {
        fixed_add_checked(&J[K][G.g(i, j, k)], v, flags);
    }
};

struct LdsAcc32 {
    unsigned long long *sm;
    int lo0, lo1, lo2, bx, by, V;
    __device__ __forceinline__ void add(int K, int i, int j, int k, long long v) const {
        atomicAdd(&sm[K * V + ((k - lo2) * by + (j - lo1)) * bx + (i - lo0)], (unsigned long long)v);
    }
};

// One segment A -> B, local to cell `base` + `cell` (cell relative to base).
// Its contributions, in units of the fixed-point current (FP64), are added
// to v[K][bi + 2 bj] (the K-edge at base + cell + bi e_I + bj e_J).
__device__ __forceinline__ void dep_segment32(const Dep32 &D, const int base[3], const float O[3], const float A[3],
                                              const float B[3], const int cell[3], float Q, double v[3][4]) {
    float d[3], mid[3];
    for (int ax = 0; ax < 3; ax++) {
        d[ax] = B[ax] - A[ax];
        mid[ax] = 0.5f * (A[ax] + B[ax]);
    }
#pragma unroll
    for (int K = 0; K < 3; K++) {
        const int I = (K + 1) % 3, J = (K + 2) % 3;
        float flux = Q * d[K] * D.inv_dt;
        if (flux == 0.0f) continue;
        float t = d[I] * d[J] * (1.0f / 12.0f);
        float loI = (float)cell[I], loJ = (float)cell[J];
        float w00, w10, w01, w11;
        float xi = mid[I] - loI, eta = mid[J] - loJ;
        if (!D.curved) {
            w00 = (1.0f - xi) * (1.0f - eta);
            w10 = xi * (1.0f - eta);
            w01 = (1.0f - xi) * eta;
            w11 = xi * eta;
        } else {
            float area[2][2];
            for (int bj = 0; bj < 2; bj++)
                for (int bi = 0; bi < 2; bi++) {
                    float i0 = bi ? loI : mid[I], i1 = bi ? mid[I] : loI + 1.0f;
                    float j0 = bj ? loJ : mid[J], j1 = bj ? mid[J] : loJ + 1.0f;
                    float P3[3];
                    P3[K] = mid[K];
                    P3[I] = 0.5f * (i0 + i1);
                    P3[J] = 0.5f * (j0 + j1);
                    area[bi][bj] = area_density32(D, K, base, O, P3) * ((i1 - i0) * (j1 - j0));
                }
            const float inv = __builtin_amdgcn_rcpf(area[0][0] + area[1][0] + area[0][1] + area[1][1]);
            w00 = area[0][0] * inv;
            w10 = area[1][0] * inv;
            w01 = area[0][1] * inv;
            w11 = area[1][1] * inv;
        }
        w00 += t;
        w11 += t;
        w10 -= t;
        w01 -= t;
        double sc = (double)flux * D.jscale;
        v[K][0] += sc * (double)w00;
        v[K][1] += sc * (double)w10;
        v[K][2] += sc * (double)w01;
        v[K][3] += sc * (double)w11;
    }
}

// Round the twelve edge sums of cell base + cell to fixed point, add them to
// the accumulator and clear them.
template <typename Acc>
__device__ __forceinline__ void dep_flush32(const Acc &acc, const int base[3], const int cell[3], double v[3][4]) {
#pragma unroll
    for (int K = 0; K < 3; K++) {
        const int I = (K + 1) % 3, J = (K + 2) % 3;
#pragma unroll
        for (int c = 0; c < 4; c++) {
            {
                int id[3] = {base[0] + cell[0], base[1] + cell[1], base[2] + cell[2]};
                id[I] += c & 1;
                id[J] += c >> 1;
                acc.add(K, id[0], id[1], id[2], fixed_rn(v[K][c]));
            }
            v[K][c] = 0.0;
        }
    }
}

// Both segments of one chord, summed in FP64 registers first when they lie in
// the same cell (each particle's share of an edge is rounded once).
template <typename Acc>
__device__ __forceinline__ void dep_chord32(const Dep32 &D, const Acc &acc, const int base[3], const float X1[3],
                                            const float xr[3], const float X2[3], const int l1[3], const int l2[3],
                                            float Q) {
    double v[3][4];
#pragma unroll
    for (int K = 0; K < 3; K++)
        for (int c = 0; c < 4; c++) v[K][c] = 0.0;
    // the cell corner relative to the hole, exact in FP64, rounded once
    const float O[3] = {(float)((double)base[0] - D.h.cx), (float)((double)base[1] - D.h.cy),
                        (float)((double)base[2] - D.h.cz)};
    dep_segment32(D, base, O, X1, xr, l1, Q, v);
    if (l1[0] != l2[0] || l1[1] != l2[1] || l1[2] != l2[2]) dep_flush32(acc, base, l1, v);
    dep_segment32(D, base, O, xr, X2, l2, Q, v);
    dep_flush32(acc, base, l2, v);
}

// Zigzag in coordinates local to the old cell: x1 in [0,1), x2 = (cell2 -
// cell1) + off2.  Cells returned relative to the old cell; false when the
// move exceeds a cell or leaves the ghost layer.
__device__ __forceinline__ bool zigzag32(const Grid &G, const int base[3], const float x1[3], const float x2[3],
                                         float xr[3], int c1[3], int c2[3]) {
    bool ok = true;
    for (int ax = 0; ax < 3; ax++) {
        int i1 = (int)floorf(x1[ax]), i2 = (int)floorf(x2[ax]);
        float lo = (float)((i1 < i2 ? i1 : i2) + 1);
        float hi = (float)(i1 > i2 ? i1 : i2);
        float mid = 0.5f * (x1[ax] + x2[ax]);
        float v = mid > hi ? mid : hi;
        xr[ax] = v < lo ? v : lo;
        c1[ax] = i1;
        c2[ax] = i2;
        int nn = G.dim(ax);
        int g1 = base[ax] + i1, g2 = base[ax] + i2;
        if (g1 < -1 || g1 > nn || g2 < -1 || g2 > nn || !(fabsf(x2[ax] - x1[ax]) < 1.0f)) ok = false;
    }
    return ok;
}

// A chord as stored: packed old and new cells and offsets.
struct Chord32 {
    int32_t cell1, cell2;
    float off1[3], off2[3];
};
__device__ __forceinline__ void read_chord32(const ParticlePtrs32 &xo, const ParticlePtrs32 &xn, int64_t id,
                                             Chord32 &R) {
    R.cell1 = xo.cell[id];
    R.cell2 = xn.cell[id];
    for (int ax = 0; ax < 3; ax++) {
        R.off1[ax] = xo.off[ax][id];
        R.off2[ax] = xn.off[ax][id];
    }
}

// Old cell, old offset and the new position relative to the old cell.
__device__ __forceinline__ void load_chord32(const Chord32 &R, int B1[3], float X1[3], float X2[3]) {
    int c2[3];
    unpack_cell(R.cell1, B1[0], B1[1], B1[2]);
    unpack_cell(R.cell2, c2[0], c2[1], c2[2]);
    for (int ax = 0; ax < 3; ax++) {
        X1[ax] = R.off1[ax];
        X2[ax] = (float)(c2[ax] - B1[ax]) + R.off2[ax];
    }
}

constexpr int kDep32Block = 256;
constexpr int kDep32PPT = 4;

// Particle p of thread tid within its block's slots, wave lanes 16 slots
// apart (as in the FP64 deposit: lanes of one instruction in different cells).
__device__ __forceinline__ int dep32_slot(int p, int tid) {
    return (tid & 63) * (kDep32PPT * (kDep32Block / 64)) + p * (kDep32Block / 64) + (tid >> 6);
}
constexpr int kDep32Lds = 6656;  // int64 LDS entries of the current box (52 KiB: three blocks per CU)

// Block `blk` of the deposit (particles blk * kDep32Block * kDep32PPT ...);
// LDS scratch sm and sred come from the calling kernel.  Every thread of the
// block calls this.
__device__ __forceinline__ void deposit32_block(const Dep32 &D, const Species &cS, double r_rm, double rscale,
                                                const ParticlePtrs32 &xo, const ParticlePtrs32 &xn, int64_t n,
                                                const FieldPtrsT<float> &F, unsigned long long *counters, int64_t blk,
                                                unsigned long long *sm, int (*sred)[kDep32Block / 64], double *sQ) {
    const int64_t base = blk * (kDep32Block * kDep32PPT);
    if (n <= 0 || base >= live_bound(counters, n)) return;  // uniform: removed particles only
    const int tid = threadIdx.x;
    // Every slot's record is read at once (slots past n read slot n - 1 and
    // count as dead), so the loads are in flight together.
    uint8_t SP[kDep32PPT];
    Chord32 R[kDep32PPT];
#pragma unroll
    for (int p = 0; p < kDep32PPT; p++) {
        const int64_t id = base + dep32_slot(p, tid), idc = id < n ? id : n - 1;
        const uint8_t s = xo.sp[idc];
        SP[p] = id < n ? s : kDead;
        read_chord32(xo, xn, idc, R[p]);
    }
    if (tid == 0)
#pragma unroll
        for (int q = 0; q < kMaxSpecies; q++) sQ[q] = cS.charge[q];
    __syncthreads();
    int lo[3] = {1 << 30, 1 << 30, 1 << 30}, hi[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
#pragma unroll
    for (int p = 0; p < kDep32PPT; p++) {
        if (SP[p] != kDead) {
            int B1[3];
            float X1[3], X2[3];
            load_chord32(R[p], B1, X1, X2);
            float xr[3];
            int l1[3], l2[3];
            if (zigzag32(D.G, B1, X1, X2, xr, l1, l2) && sQ[SP[p]] != 0.0)
                for (int ax = 0; ax < 3; ax++) {
                    int a = B1[ax] + (l1[ax] < l2[ax] ? l1[ax] : l2[ax]);
                    int b = B1[ax] + (l1[ax] > l2[ax] ? l1[ax] : l2[ax]) + 1;
                    lo[ax] = a < lo[ax] ? a : lo[ax];
                    hi[ax] = b > hi[ax] ? b : hi[ax];
                }
        }
    }
    for (int ax = 0; ax < 3; ax++) {
        int a = wave_min32(lo[ax]), b = wave_max32(hi[ax]);
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
        for (int w = 1; w < kDep32Block / 64; w++) {
            blo[ax] = sred[ax][w] < blo[ax] ? sred[ax][w] : blo[ax];
            bhi[ax] = sred[3 + ax][w] > bhi[ax] ? sred[3 + ax][w] : bhi[ax];
        }
    }
    const bool any = bhi[0] >= blo[0];
    const int bx = any ? bhi[0] - blo[0] + 1 : 0, by = any ? bhi[1] - blo[1] + 1 : 0,
              bz = any ? bhi[2] - blo[2] + 1 : 0;
    const int64_t V64 = (int64_t)bx * by * bz;
    const bool use_lds = any && 3 * V64 <= kDep32Lds;
    const int V = use_lds ? (int)V64 : 0;
    if (use_lds) {
        for (int e = tid; e < 3 * V; e += kDep32Block) sm[e] = 0ull;
        __syncthreads();
    }
    if (tid == 0 && any) atomicAdd(&counters[use_lds ? C_DEP_LDS : C_DEP_GLOBAL], 1ull);
    LdsAcc32 la{sm, blo[0], blo[1], blo[2], bx, by, V};
    GlobalAcc32 ga{{F.Jint[0], F.Jint[1], F.Jint[2]}, D.G, &counters[C_FLAGS]};
    int n_horizon = 0, n_outer = 0;
    // the next slot's record is read while this one is deposited
    Chord32 next = R[0];
#pragma unroll 1
    for (int p = 0; p < kDep32PPT; p++) {
        const Chord32 cur = next;
        if (p + 1 < kDep32PPT) {
            const int64_t idn = base + dep32_slot(p + 1, tid);
            read_chord32(xo, xn, idn < n ? idn : n - 1, next);
        }
        if (SP[p] == kDead) continue;
        int64_t id = base + dep32_slot(p, tid);
        float Q = (float)sQ[SP[p]];
        int B1[3];
        float X1[3], X2[3];
        load_chord32(cur, B1, X1, X2);
        float xr[3];
        int l1[3], l2[3];
        bool ok = zigzag32(D.G, B1, X1, X2, xr, l1, l2);
        if (ok && Q != 0.0f) {
            if (use_lds)
                dep_chord32(D, la, B1, X1, xr, X2, l1, l2, Q);
            else
                dep_chord32(D, ga, B1, X1, xr, X2, l1, l2, Q);
        } else if (!ok) {
            atomicOr(&counters[C_FLAGS], kFlagLongMove);
        }
        // removal after the final move is deposited
        int c2[3];
        unpack_cell(cur.cell2, c2[0], c2[1], c2[2]);
        bool outside = false;
        for (int ax = 0; ax < 3; ax++)
            if (c2[ax] < 0 || c2[ax] > D.G.dim(ax) - 1) outside = true;
        float o2[3] = {cur.off2[0], cur.off2[1], cur.off2[2]};
        double x, y, z;
        hole_rel(D.h, c2[0], c2[1], c2[2], o2, x, y, z);
        if (ks_radius_below(D.h.a, x, y, z, r_rm)) {
            bool inb = true;
            for (int ax = 0; ax < 3; ax++)
                if (c2[ax] < -1 || c2[ax] > D.G.dim(ax)) inb = false;
            if (inb && Q != 0.0f) {
                double sc = sQ[SP[p]] * rscale;
                for (int dk = 0; dk < 2; dk++)
                    for (int dj = 0; dj < 2; dj++)
                        for (int di = 0; di < 2; di++) {
                            double W = (di ? (double)o2[0] : 1.0 - (double)o2[0]) *
                                       (dj ? (double)o2[1] : 1.0 - (double)o2[1]) *
                                       (dk ? (double)o2[2] : 1.0 - (double)o2[2]);
                            fixed_add_checked(&F.rho_abs[D.G.g(c2[0] + di, c2[1] + dj, c2[2] + dk)],
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
    wave_count32(&counters[C_REMOVED_HORIZON], n_horizon);
    wave_count32(&counters[C_REMOVED_OUTER], n_outer);
    if (use_lds) {
        __syncthreads();
        flush_box(sm, V, bx, by, blo, F.Jint, D.G, &counters[C_FLAGS]);
    }
}

__global__ __launch_bounds__(kDep32Block) void k_deposit32(Dep32 D, Species cS, double r_rm, double rscale,
                                                           ParticlePtrs32 xo, ParticlePtrs32 xn, int64_t n,
                                                           FieldPtrsT<float> F, unsigned long long *counters) {
    __shared__ unsigned long long sm[kDep32Lds];
    __shared__ int sred[6][kDep32Block / 64];
    __shared__ double sQ[kMaxSpecies];
    deposit32_block(D, cS, r_rm, rscale, xo, xn, n, F, counters, blockIdx.x, sm, sred, sQ);
}

Dep32 make_dep32(const Grid &G, const Hole &h, const Mixed &M, double dt, int deposit_mode, double jscale) {
    Dep32 D;
    D.G = G;
    D.h = h;
    D.r_fp64 = M.r_fp64;
    D.r_fp64_sq = (float)(M.r_fp64 * M.r_fp64);
    D.af = (float)h.a;
    D.m2 = (float)(2.0 * h.m);
    D.inv_dt = (float)(1.0 / dt);
    D.jscale = jscale;
    D.curved = deposit_mode == 0;
    return D;
}

// ---------------------------------------------------------------------------
// Serving batch: persistent push and deposit over the logical blocks of all
// active runs (the run table is in device memory).
__global__ __launch_bounds__(kPush32Block, 4) void k_batch_push32(const BatchTable *__restrict__ T) {
    __shared__ float4 snode[kPush32LdsNodes * kNode32Stride4];
    __shared__ int sred[6][kPush32Block / 64];
    __shared__ double sqm[kMaxSpecies];
    const int64_t total = T->total[BK_PUSH];
    for (int64_t lb = blockIdx.x; lb < total; lb += gridDim.x) {
        __syncthreads();  // the previous logical block is done with the LDS scratch
        const BatchRun32 &R = T->run[batch_run_of(T, BK_PUSH, lb)];
        push32_block(R.P, R.M, R.S, R.F.node, R.cur, R.nxt, R.counters, lb - R.off[BK_PUSH], snode, sred, sqm);
    }
}

__global__ __launch_bounds__(kDep32Block) void k_batch_deposit32(const BatchTable *__restrict__ T) {
    __shared__ unsigned long long sm[kDep32Lds];
    __shared__ int sred[6][kDep32Block / 64];
    __shared__ double sQ[kMaxSpecies];
    const int64_t total = T->total[BK_DEP];
    for (int64_t lb = blockIdx.x; lb < total; lb += gridDim.x) {
        __syncthreads();  // the previous logical block is done with the LDS scratch
        const BatchRun32 &R = T->run[batch_run_of(T, BK_DEP, lb)];
        deposit32_block(R.D, R.S, R.r_rm, R.rscale, R.cur, R.nxt, R.P.n, R.F, R.counters, lb - R.off[BK_DEP], sm,
                        sred, sQ);
    }
}

void launch_batch_push32(const BatchTable *table, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_push32, dim3(grid), dim3(kPush32Block), 0, s, table);
}

void launch_batch_deposit32(const BatchTable *table, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_deposit32, dim3(grid), dim3(kDep32Block), 0, s, table);
}

int64_t batch_blocks(int kind, const Grid &G, const int relax_box[6], int64_t n_slots) {
    auto up = [](int64_t a, int64_t b) { return (a + b - 1) / b; };
    switch (kind) {
    case BK_NODE: return up(G.nnodes(), kBatchBlock);
    case BK_GRID: return up(G.gsize(), kBatchBlock);
    case BK_RELAX: return up((int64_t)relax_box[3] * relax_box[4] * relax_box[5], kBatchBlock);
    case BK_PUSH: return up(n_slots, kPush32Block);
    case BK_DEP: return up(n_slots, (int64_t)kDep32Block * kDep32PPT);
    }
    return 0;
}

void launch_deposit32(const Grid &G, const Hole &h, const Mixed &M, double dt, int deposit_mode, double r_rm,
                      double jscale, double rscale, const Species &S, ParticlePtrs32 xold, ParticlePtrs32 xnew,
                      int64_t n, FieldPtrsT<float> &F, unsigned long long *counters, hipStream_t s) {
    if (n <= 0) return;
    const Dep32 D = make_dep32(G, h, M, dt, deposit_mode, jscale);
    const int64_t per = kDep32Block * kDep32PPT;
    hipLaunchKernelGGL(k_deposit32, dim3((unsigned)((n + per - 1) / per)), dim3(kDep32Block), 0, s, D, S, r_rm,
                       rscale, xold, xnew, n, F, counters);
}

// ---------------------------------------------------------------------------
// Load: FP64 mass shell (as in the FP64 form), then cell + FP32 offset.
__device__ __forceinline__ bool load_one32(const Grid &G, const Hole &h, double c, double r_rm,
                                           const double *__restrict__ xin, const double *__restrict__ ucin,
                                           int64_t n, int species, const ParticlePtrs32 &out, int64_t off,
                                           int64_t id) {
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
    int ci[3] = {0, 0, 0};
    for (int ax = 0; ax < 3; ax++) {
        double fl = ok ? floor(X[ax]) : 0.0;
        float of = ok ? (float)(X[ax] - fl) : 0.0f;
        // X just below an integer rounds to offset 1.0f: the next cell's face
        if (of >= 1.0f) {
            of = 0.0f;
            fl += 1.0;
        }
        ci[ax] = (int)fl;
        out.off[ax][o] = of;
    }
    out.cell[o] = pack_cell(ci[0], ci[1], ci[2]);
    for (int q = 0; q < 4; q++) out.u[q][o] = (float)U[q];
    out.sp[o] = ok ? (uint8_t)species : kDead;
    return ok;
}

__global__ void k_load32(Grid G, Hole h, double c, double r_rm, const double *__restrict__ xin,
                         const double *__restrict__ ucin, int64_t n, int species, ParticlePtrs32 out, int64_t off,
                         unsigned long long *counters) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = id < n && load_one32(G, h, c, r_rm, xin, ucin, n, species, out, off, id);
    wave_count32(&counters[C_LOAD_KEPT], ok ? 1 : 0);
}

void launch_load32(const Grid &G, const Hole &h, double c, double r_rm, const double *xin, const double *ucin,
                   int64_t n, int species, ParticlePtrs32 out, int64_t offset, unsigned long long *counters,
                   hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_load32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, G, h, c, r_rm, xin, ucin, n,
                       species, out, offset, counters);
}

// Widening to FP64 (x = cell + offset exactly, u converted) and back.
__global__ void k_to_f64(ParticlePtrs32 in, double *x, double *u, int64_t n) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    int c[3];
    unpack_cell(in.cell[id], c[0], c[1], c[2]);
    for (int q = 0; q < 3; q++) x[q * n + id] = (double)c[q] + (double)in.off[q][id];
    for (int q = 0; q < 4; q++) u[q * n + id] = (double)in.u[q][id];
}

__global__ void k_from_f64(const double *x, const double *u, ParticlePtrs32 out, int64_t n) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    int c[3];
    for (int q = 0; q < 3; q++) {
        double v = x[q * n + id];
        double fl = floor(v);
        float of = (float)(v - fl);
        if (of >= 1.0f) {  // offsets stay in [0, 1), as the pusher keeps them
            of = 0.0f;
            fl += 1.0;
        }
        const int ci = (int)fl;
        c[q] = ci < -1 ? -1 : (ci > 1022 ? 1022 : ci);
        // a cell outside the packable range keeps the offset from the clamped cell
        out.off[q][id] = c[q] == ci ? of : (float)(v - (double)c[q]);
    }
    out.cell[id] = pack_cell(c[0], c[1], c[2]);
    for (int q = 0; q < 4; q++) out.u[q][id] = (float)u[q * n + id];
}

void launch_to_f64(ParticlePtrs32 in, double *x, double *u, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_to_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, x, u, n);
}

void launch_from_f64(const double *x, const double *u, ParticlePtrs32 out, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_from_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, u, out, n);
}

}  // namespace grpic
