// Yee-staggered F-tensor field kernels (FP64) for the GRPIC cycle (Sec. 3).
//
// Evolved pair: B_c = (F_23, F_31, F_12)[c] at face centres (offset 1/2 in the
// two axes other than c, the magnetic shift of Sec. 3.1) and D^c = F^{c4} at
// edge centres (offset 1/2 along c, the electric shift of Sec. 3.2).  The
// magnetic half-step is the forward-difference Faraday update of Sec. 3.1;
// the electric step is the backward-difference divergence update of
// Sec. 3.2 in its continuous form, whose Christoffel terms vanish because
// det g = -1.
//
// Constitutive step (index raising/lowering): pointwise the map
// (D, B_cov) -> (-E_cov, H) is a symmetric 6x6 matrix S built from g^{-1}
// (S = I in flat space).  On the grid it is applied as
//   (-E_cov, H) = (D, B_cov) + P^T (S - I) P (D, B_cov)
// with P the average of the six components onto the nodes (1/2 of the two
// E points along c, 1/4 of the four B points) and P^T its transpose, so the
// discrete map is symmetric and reduces to Yee's identity at m = 0.
// (S - I) and g are evaluated per node in FP64 in each node pass (the metric
// is stationary) and rounded to the field type T: double for the FP64 form,
// float for the FP32-mixed form (whose field arithmetic is then FP32).
#include "grpic_dev.h"
#include "grpic_impl.h"

namespace grpic {

// Pairs: s = {23, 31, 12}, t = {14, 24, 34} (0-based: (1,2),(2,0),(0,1),(0,3),(1,3),(2,3)).
__host__ __device__ constexpr int pair_index(int A, int e) {
    return A == 0 ? (e ? 2 : 1) : A == 1 ? (e ? 0 : 2) : A == 2 ? (e ? 1 : 0) : (e ? 3 : A - 3);
}
__constant__ int kPair[6][2] = {{1, 2}, {2, 0}, {0, 1}, {0, 3}, {1, 3}, {2, 3}};

// packed symmetric 6x6: index of (i,j)
__host__ __device__ constexpr int sym6(int i, int j) {
    return (i < j ? i : j) * 6 - ((i < j ? i : j) * ((i < j ? i : j) - 1)) / 2 + ((i < j ? j : i) - (i < j ? i : j));
}

// ---------------------------------------------------------------------------
// Per node: the curvature part dS = S - I of the constitutive map (packed
// symmetric, 21 values) and the covariant metric g (packed, 10 values), in
// FP64 from the metric at the node.  The metric is stationary, but computing
// these in the node passes costs less than streaming 31 stored values per
// node through every pass.
// Variable order v = (D^0, D^1, D^2, B_0, B_1, B_2).
__device__ __forceinline__ void node_constitutive(const Hole &h, int i, int j, int k, double dS[21],
                                                  double gout[10]) {
    Sym4 g, gi;
    grid_metric(h, (double)i, (double)j, (double)k, g, gi);
    for (int q = 0; q < 10; q++) gout[q] = g.v[q];
    // M over the pairs: M[A][B] = gi^{mu al} gi^{nu be} - gi^{mu be} gi^{nu al}
    // (loops unrolled so that every index is a constant and the matrices stay
    // in registers)
    double M[6][6];
#pragma unroll
    for (int A = 0; A < 6; A++)
#pragma unroll
        for (int B = 0; B < 6; B++) {
            const int mu = pair_index(A, 0), nu = pair_index(A, 1), al = pair_index(B, 0), be = pair_index(B, 1);
            M[A][B] = gi.v[sym4(mu, al)] * gi.v[sym4(nu, be)] - gi.v[sym4(mu, be)] * gi.v[sym4(nu, al)];
        }
    // Minv = M_tt^{-1} by the adjugate
    double a00 = M[3][3], a01 = M[3][4], a02 = M[3][5];
    double a10 = M[4][3], a11 = M[4][4], a12 = M[4][5];
    double a20 = M[5][3], a21 = M[5][4], a22 = M[5][5];
    double c00 = a11 * a22 - a12 * a21, c01 = a02 * a21 - a01 * a22, c02 = a01 * a12 - a02 * a11;
    double c10 = a12 * a20 - a10 * a22, c11 = a00 * a22 - a02 * a20, c12 = a02 * a10 - a00 * a12;
    double c20 = a10 * a21 - a11 * a20, c21 = a01 * a20 - a00 * a21, c22 = a00 * a11 - a01 * a10;
    double idet = 1.0 / (a00 * c00 + a01 * c10 + a02 * c20);
    double Mi[3][3] = {{c00 * idet, c01 * idet, c02 * idet},
                       {c10 * idet, c11 * idet, c12 * idet},
                       {c20 * idet, c21 * idet, c22 * idet}};
    // S_DD = -Mi ; S_DB = Mi M_ts ; S_BB = M_ss - M_st Mi M_ts
    double SDB[3][3];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 3; q++) s += Mi[r][q] * M[3 + q][c];
            SDB[r][c] = s;
        }
    double S[6][6];
#pragma unroll
    for (int r = 0; r < 3; r++)
#pragma unroll
        for (int c = 0; c < 3; c++) {
            S[r][c] = -Mi[r][c];
            S[r][3 + c] = SDB[r][c];
            S[3 + c][r] = SDB[r][c];
            double s = M[r][c];
#pragma unroll
            for (int q = 0; q < 3; q++) s -= M[r][3 + q] * SDB[q][c];
            S[3 + r][3 + c] = s;
        }
#pragma unroll
    for (int r = 0; r < 6; r++)
#pragma unroll
        for (int c = r; c < 6; c++) dS[sym6(r, c)] = S[r][c] - (r == c ? 1.0 : 0.0);
}

// Update masks: bit c set if E_c at this index is updated, bit 3+c for B_c.
// Updated = integer axes in [1, n-1], half axes in [0, n-1], not excised.
__global__ void k_masks(Grid G, Hole h, uint8_t *__restrict__ mask) {
    int64_t gs = G.gsize();
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= gs) return;
    int i = (int)(id % G.sx) - 1;
    int64_t t = id / G.sx;
    int j = (int)(t % (G.ny + 3)) - 1;
    int k = (int)(t / (G.ny + 3)) - 1;
    int idx[3] = {i, j, k};
    uint8_t mk = 0;
    for (int kind = 0; kind < 2; kind++)
        for (int c = 0; c < 3; c++) {
            bool ok = true;
            double X[3];
            for (int ax = 0; ax < 3; ax++) {
                bool half = kind == 0 ? (ax == c) : (ax != c);
                int n = G.dim(ax);
                if (half) {
                    ok = ok && idx[ax] >= 0 && idx[ax] <= n - 1;
                    X[ax] = idx[ax] + 0.5;
                } else {
                    ok = ok && idx[ax] >= 1 && idx[ax] <= n - 1;
                    X[ax] = (double)idx[ax];
                }
            }
            if (ok && grid_excised(h, X[0], X[1], X[2])) ok = false;
            if (ok) mk |= (uint8_t)(1u << (kind * 3 + c));
        }
    mask[id] = mk;
}

// Node averages of the evolved pair.
template <typename T>
__device__ __forceinline__ void node_pair(const Grid &G, const T *const D[3], const T *const B[3], int i, int j, int k,
                                          T v[6]) {
    const T h = (T)0.5, q = (T)0.25;
    v[0] = h * (D[0][G.g(i - 1, j, k)] + D[0][G.g(i, j, k)]);
    v[1] = h * (D[1][G.g(i, j - 1, k)] + D[1][G.g(i, j, k)]);
    v[2] = h * (D[2][G.g(i, j, k - 1)] + D[2][G.g(i, j, k)]);
    v[3] = q * (B[0][G.g(i, j - 1, k - 1)] + B[0][G.g(i, j, k - 1)] + B[0][G.g(i, j - 1, k)] +
                   B[0][G.g(i, j, k)]);
    v[4] = q * (B[1][G.g(i - 1, j, k - 1)] + B[1][G.g(i, j, k - 1)] + B[1][G.g(i - 1, j, k)] +
                   B[1][G.g(i, j, k)]);
    v[5] = q * (B[2][G.g(i - 1, j - 1, k)] + B[2][G.g(i, j - 1, k)] + B[2][G.g(i - 1, j, k)] +
                   B[2][G.g(i, j, k)]);
}

template <typename T>
__device__ __forceinline__ void apply_dS(const double dS[21], const T v[6], T w[6]) {
#pragma unroll
    for (int r = 0; r < 6; r++) w[r] = (T)0;
#pragma unroll
    for (int r = 0; r < 6; r++)
#pragma unroll
        for (int c = r; c < 6; c++) {
            T s = (T)dS[sym6(r, c)];
            w[r] += s * v[c];
            if (c != r) w[c] += s * v[r];
        }
}

__device__ __forceinline__ void node_ijk(const Grid &G, int64_t id, int &i, int &j, int &k) {
    i = (int)(id % (G.nx + 1));
    int64_t t = id / (G.nx + 1);
    j = (int)(t % (G.ny + 1));
    k = (int)(t / (G.ny + 1));
}

// Per-index bodies of the field kernels.  A single run launches one thread
// per index; the serving batch runs the same bodies for the indices of many
// runs from one launch (see the batched kernels below).

// w = (S - I) P (D, B) at node id.
template <typename T>
__device__ __forceinline__ void node_w_at(const Grid &G, const Hole &h, const FieldPtrsT<T> &F, int64_t id) {
    const int64_t nn = G.nnodes();
    int i, j, k;
    node_ijk(G, id, i, j, k);
    const T *D[3] = {F.D[0], F.D[1], F.D[2]};
    const T *B[3] = {F.B[0], F.B[1], F.B[2]};
    T v[6], o[6];
    node_pair<T>(G, D, B, i, j, k, v);
    double dS[21], g[10];
    node_constitutive(h, i, j, k, dS, g);
    apply_dS<T>(dS, v, o);
    for (int q = 0; q < 6; q++) F.w[q * nn + id] = o[q];
}

__device__ __forceinline__ bool in_domain(const Grid &G, int kind, int c, int i, int j, int k) {
    int idx[3] = {i, j, k};
    for (int ax = 0; ax < 3; ax++) {
        bool half = kind == 0 ? (ax == c) : (ax != c);
        int n = G.dim(ax);
        if (idx[ax] < 0 || idx[ax] > (half ? n - 1 : n)) return false;
    }
    return true;
}

// E_cov at the in-domain E points of index id: -(D + P^T w) where updated,
// else the initial value (all three components).
template <typename T>
__device__ __forceinline__ void ecov_at(const Grid &G, const FieldPtrsT<T> &F, bool use_ref, int64_t id) {
    const int64_t nn = G.nnodes();
    int i, j, k;
    node_ijk(G, id, i, j, k);
    int64_t gi = G.g(i, j, k);
    uint8_t mk = F.mask[gi];
    int64_t n0 = G.node(i, j, k);
    int64_t step[3] = {1, (int64_t)(G.nx + 1), (int64_t)(G.nx + 1) * (G.ny + 1)};
    for (int c = 0; c < 3; c++) {
        if (!in_domain(G, 0, c, i, j, k)) continue;
        T val;
        if (use_ref && !(mk & (1u << c))) {
            val = F.E0[c][gi];
        } else {
            T corr = (T)0.5 * (F.w[c * nn + n0] + F.w[c * nn + n0 + step[c]]);
            val = -(F.D[c][gi] + corr);
        }
        F.E[c][gi] = val;
    }
}

// H at the in-domain B points of index id: B + P^T w where updated, else the
// initial value.
template <typename T>
__device__ __forceinline__ void hfield_at(const Grid &G, const FieldPtrsT<T> &F, bool use_ref, int64_t id) {
    const int64_t nn = G.nnodes();
    int i, j, k;
    node_ijk(G, id, i, j, k);
    int64_t gi = G.g(i, j, k);
    uint8_t mk = F.mask[gi];
    int64_t n0 = G.node(i, j, k);
    int64_t step[3] = {1, (int64_t)(G.nx + 1), (int64_t)(G.nx + 1) * (G.ny + 1)};
    for (int c = 0; c < 3; c++) {
        if (!in_domain(G, 1, c, i, j, k)) continue;
        T val;
        if (use_ref && !(mk & (1u << (3 + c)))) {
            val = F.H0[c][gi];
        } else {
            int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
            const T *wc = F.w + (3 + c) * nn;
            T corr = (T)0.25 * (wc[n0] + wc[n0 + step[a1]] + wc[n0 + step[a2]] + wc[n0 + step[a1] + step[a2]]);
            val = F.B[c][gi] + corr;
        }
        F.H[c][gi] = val;
    }
}

// Magnetic half-step (Sec. 3.1) for the pair (al, be) of component c:
//   Bout_c = Bin_c - h [ (E_be(x + e_al) - E_be(x)) - (E_al(x + e_be) - E_al(x)) ],  h = c dt / 2.
// Points that are not updated copy Bin (when Bin and Bout differ).
template <typename T>
__device__ __forceinline__ void bhalf_at(const Grid &G, const FieldPtrsT<T> &F, const T *const Bin[3], T hstep,
                                         int64_t id) {
    int i, j, k;
    node_ijk(G, id, i, j, k);
    int64_t gi = G.g(i, j, k);
    uint8_t mk = F.mask[gi];
    int64_t st[3] = {1, G.sx, G.sy};
    for (int c = 0; c < 3; c++) {
        if (!in_domain(G, 1, c, i, j, k)) continue;
        T b = Bin[c][gi];
        if (mk & (1u << (3 + c))) {
            int al = (c + 1) % 3, be = (c + 2) % 3;
            T d1 = F.E[be][gi + st[al]] - F.E[be][gi];
            T d2 = F.E[al][gi + st[be]] - F.E[al][gi];
            b -= (d1 - d2) * hstep;
        }
        F.B[c][gi] = b;
    }
}

// Electric step (Sec. 3.2):
//   Dout_c = Din_c + dx4 [ (4 pi / c) J_c - sum_k d_k F^{c k} ],
// F^{c,c+1} = H[c+2], F^{c,c+2} = -H[c+1], backward differences; J from the
// int64 accumulator.
template <typename T>
__device__ __forceinline__ void dstep_at(const Grid &G, const FieldPtrsT<T> &F, const T *const Din[3], T dx4,
                                         T four_pi_over_c, double inv_jscale, int64_t id) {
    int i, j, k;
    node_ijk(G, id, i, j, k);
    int64_t gi = G.g(i, j, k);
    uint8_t mk = F.mask[gi];
    int64_t st[3] = {1, G.sx, G.sy};
    for (int c = 0; c < 3; c++) {
        if (!in_domain(G, 0, c, i, j, k)) continue;
        T d = Din[c][gi];
        if (mk & (1u << c)) {
            int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            // + d_{c1} H[c2] - d_{c2} H[c1]
            T div = (F.H[c2][gi] - F.H[c2][gi - st[c1]]) - (F.H[c1][gi] - F.H[c1][gi - st[c2]]);
            T Jc = (T)((double)(long long)F.Jint[c][gi] * inv_jscale);
            d += dx4 * (four_pi_over_c * Jc - div);
        }
        F.D[c][gi] = d;
    }
}

// Relaxation layer inside the horizon: updated points with r_exc <= r < r_damp
// move toward their initial values by damp_max ((r_damp - r)/(r_damp - r_exc))^2.
// id runs over the box [i0, i0 + bx) x [j0, j0 + by) x [k0, k0 + bz).
template <typename T>
__device__ __forceinline__ void relax_at(const Grid &G, const Hole &h, const FieldPtrsT<T> &F, double r_damp,
                                         double damp_max, const int box[6], int64_t id) {
    int i = box[0] + (int)(id % box[3]);
    int64_t t = id / box[3];
    int j = box[1] + (int)(t % box[4]);
    int k = box[2] + (int)(t / box[4]);
    int64_t gi = G.g(i, j, k);
    uint8_t mk = F.mask[gi];
    for (int kind = 0; kind < 2; kind++)
        for (int c = 0; c < 3; c++) {
            if (!(mk & (1u << (kind * 3 + c)))) continue;
            double X = i + ((kind == 0 ? c == 0 : c != 0) ? 0.5 : 0.0);
            double Y = j + ((kind == 0 ? c == 1 : c != 1) ? 0.5 : 0.0);
            double Z = k + ((kind == 0 ? c == 2 : c != 2) ? 0.5 : 0.0);
            double r = ks_radius(h.a, X - h.cx, Y - h.cy, Z - h.cz);
            if (!(r < r_damp)) continue;
            double tt = (r_damp - r) / (r_damp - h.r_exc);
            double sg = damp_max * tt * tt;
            T *Fp = kind == 0 ? F.D[c] : F.B[c];
            const T *F0 = kind == 0 ? F.D0[c] : F.B0[c];
            Fp[gi] -= (T)sg * (Fp[gi] - F0[gi]);
        }
}

// Outer absorbing layer at node index id (all three components of both
// kinds): updated points closer than L to the nearest face relax toward
// their initial values by damp ((L - d)/L)^2.
template <typename T>
__device__ __forceinline__ void relax_outer_at(const Grid &G, const FieldPtrsT<T> &F, double L, double damp,
                                               int64_t id) {
    int i, j, k;
    node_ijk(G, id, i, j, k);
    int64_t gi = G.g(i, j, k);
    uint8_t mk = F.mask[gi];
    for (int kind = 0; kind < 2; kind++)
        for (int c = 0; c < 3; c++) {
            if (!(mk & (1u << (kind * 3 + c)))) continue;
            double X = i + ((kind == 0 ? c == 0 : c != 0) ? 0.5 : 0.0);
            double Y = j + ((kind == 0 ? c == 1 : c != 1) ? 0.5 : 0.0);
            double Z = k + ((kind == 0 ? c == 2 : c != 2) ? 0.5 : 0.0);
            double d = outer_distance(G, X, Y, Z);
            if (!(d < L)) continue;
            double tt = (L - d) / L;
            double sg = damp * tt * tt;
            T *Fp = kind == 0 ? F.D[c] : F.B[c];
            const T *F0 = kind == 0 ? F.D0[c] : F.B0[c];
            Fp[gi] -= (T)sg * (Fp[gi] - F0[gi]);
        }
}

// Node tensor F^a_b = F^{ag} g_{gb} from the node pair completed by S, row
// a at o[4a .. 4a+3].
template <typename T>
__device__ __forceinline__ void node_tensor_values(const Grid &G, const Hole &h, const FieldPtrsT<T> &F, int64_t id,
                                                   T o[16]) {
    int i, j, k;
    node_ijk(G, id, i, j, k);
    const T *D[3] = {F.D[0], F.D[1], F.D[2]};
    const T *B[3] = {F.B[0], F.B[1], F.B[2]};
    T v[6], w[6];
    node_pair<T>(G, D, B, i, j, k, v);
    double dS[21], gd[10];
    node_constitutive(h, i, j, k, dS, gd);
    apply_dS<T>(dS, v, w);
    // contravariant components: F^{c4} = v_D, F^{s} = v_B + w_B
    T Fu[4][4];
    for (int a = 0; a < 4; a++) Fu[a][a] = (T)0;
    T Hs[3] = {v[3] + w[3], v[4] + w[4], v[5] + w[5]};
    Fu[1][2] = Hs[0]; Fu[2][1] = -Hs[0];
    Fu[2][0] = Hs[1]; Fu[0][2] = -Hs[1];
    Fu[0][1] = Hs[2]; Fu[1][0] = -Hs[2];
    for (int c = 0; c < 3; c++) {
        Fu[c][3] = v[c];
        Fu[3][c] = -v[c];
    }
    T g[10];
    for (int q = 0; q < 10; q++) g[q] = (T)gd[q];
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++) {
            T s = (T)0;
            for (int c = 0; c < 4; c++) s += Fu[a][c] * g[sym4(c, b)];
            o[a * 4 + b] = s;
        }
}

template <typename T>
__device__ __forceinline__ void node_tensor_at(const Grid &G, const Hole &h, const FieldPtrsT<T> &F, int64_t id) {
    T o[16];
    node_tensor_values<T>(G, h, F, id, o);
    for (int q = 0; q < 16; q++) F.node[16 * id + q] = o[q];
}

// Single-run kernels: one thread per index.
template <typename T>
__global__ void k_node_w(Grid G, Hole h, FieldPtrsT<T> F) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < G.nnodes()) node_w_at<T>(G, h, F, id);
}
template <typename T>
__global__ void k_ecov(Grid G, FieldPtrsT<T> F, bool use_ref) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < G.nnodes()) ecov_at<T>(G, F, use_ref, id);
}
template <typename T>
__global__ void k_hfield(Grid G, FieldPtrsT<T> F, bool use_ref) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < G.nnodes()) hfield_at<T>(G, F, use_ref, id);
}
template <typename T>
__global__ void k_bhalf(Grid G, FieldPtrsT<T> F, const T *__restrict__ Bin0, const T *__restrict__ Bin1,
                        const T *__restrict__ Bin2, T hstep) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const T *Bin[3] = {Bin0, Bin1, Bin2};
    if (id < G.nnodes()) bhalf_at<T>(G, F, Bin, hstep, id);
}
template <typename T>
__global__ void k_dstep(Grid G, FieldPtrsT<T> F, const T *__restrict__ Din0, const T *__restrict__ Din1,
                        const T *__restrict__ Din2, T dx4, T four_pi_over_c, double inv_jscale) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const T *Din[3] = {Din0, Din1, Din2};
    if (id < G.nnodes()) dstep_at<T>(G, F, Din, dx4, four_pi_over_c, inv_jscale, id);
}
template <typename T>
__global__ void k_relax(Grid G, Hole h, FieldPtrsT<T> F, double r_damp, double damp_max, int i0, int j0, int k0,
                        int bx, int by, int bz) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int box[6] = {i0, j0, k0, bx, by, bz};
    if (id < (int64_t)bx * by * bz) relax_at<T>(G, h, F, r_damp, damp_max, box, id);
}
template <typename T>
__global__ void k_relax_outer(Grid G, FieldPtrsT<T> F, double L, double damp) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < G.nnodes()) relax_outer_at(G, F, L, damp, id);
}
// The block's nodes are contiguous in the output, 16 values each: the
// values go through LDS so that consecutive lanes store consecutive
// addresses (one thread's 16 values are 64 or 128 bytes apart from the
// next thread's).
constexpr int kNodeTensorBlock = 128;
template <typename T>
__global__ __launch_bounds__(kNodeTensorBlock) void k_node_tensor(Grid G, Hole h, FieldPtrsT<T> F) {
    __shared__ T tile[kNodeTensorBlock * 17];  // row stride 17: no bank conflicts
    const int64_t first = (int64_t)blockIdx.x * kNodeTensorBlock;
    const int64_t id = first + threadIdx.x;
    const int64_t nn = G.nnodes();
    if (id < nn) {
        T o[16];
        node_tensor_values<T>(G, h, F, id, o);
        for (int q = 0; q < 16; q++) tile[threadIdx.x * 17 + q] = o[q];
    }
    __syncthreads();
    const int64_t count = (nn - first < kNodeTensorBlock ? nn - first : kNodeTensorBlock) * 16;
    for (int e = threadIdx.x; e < count; e += kNodeTensorBlock) F.node[16 * first + e] = tile[(e >> 4) * 17 + (e & 15)];
}

// Initial fields: uniform F (contravariant or covariant B0) lowered/raised
// with the point metric at every ghosted point.
template <typename T>
__global__ void k_init_fields(Grid G, Hole h, FieldPtrsT<T> F, double b0, double b1, double b2, int covariant) {
    int64_t gs = G.gsize();
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= gs) return;
    int i = (int)(id % G.sx) - 1;
    int64_t t = id / G.sx;
    int j = (int)(t % (G.ny + 3)) - 1;
    int k = (int)(t / (G.ny + 3)) - 1;
    double Fm[4][4] = {{0, b2, -b1, 0}, {-b2, 0, b0, 0}, {b1, -b0, 0, 0}, {0, 0, 0, 0}};
    const double Bc[3] = {b0, b1, b2};
    for (int kind = 0; kind < 2; kind++)
        for (int c = 0; c < 3; c++) {
            double X = i + ((kind == 0 ? c == 0 : c != 0) ? 0.5 : 0.0);
            double Y = j + ((kind == 0 ? c == 1 : c != 1) ? 0.5 : 0.0);
            double Z = k + ((kind == 0 ? c == 2 : c != 2) ? 0.5 : 0.0);
            Sym4 g, gi;
            grid_metric(h, X, Y, Z, g, gi);
            const Sym4 &Mt = covariant ? gi : g;
            int al = kind == 1 ? kPair[c][0] : kPair[3 + c][0];
            int be = kind == 1 ? kPair[c][1] : kPair[3 + c][1];
            double v = 0.0;
            for (int mu = 0; mu < 4; mu++)
                for (int nu = 0; nu < 4; nu++) v += Mt.v[sym4(al, mu)] * Mt.v[sym4(be, nu)] * Fm[mu][nu];
            if (kind == 1)
                F.B[c][id] = (T)(covariant ? Bc[c] : v);
            else
                F.D[c][id] = (T)(covariant ? v : 0.0);
        }
}

// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T> void launch_bake(const Grid &G, const Hole &h, FieldPtrsT<T> &F, hipStream_t s) {
    hipLaunchKernelGGL(k_masks, dim3(nblk(G.gsize(), 256)), dim3(256), 0, s, G, h, F.mask);
}

template <typename T>
void launch_init_fields(const Grid &G, const Hole &h, FieldPtrsT<T> &F, const double B0[3], int covariant,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_init_fields<T>, dim3(nblk(G.gsize(), 128)), dim3(128), 0, s, G, h, F, B0[0], B0[1], B0[2],
                       covariant);
}

template <typename T>
void launch_derived(const Grid &G, const Hole &h, FieldPtrsT<T> &F, bool use_ref, bool do_e, bool do_h,
                    hipStream_t s) {
    unsigned nb = nblk(G.nnodes(), 256);
    hipLaunchKernelGGL(k_node_w<T>, dim3(nb), dim3(256), 0, s, G, h, F);
    if (do_e) hipLaunchKernelGGL(k_ecov<T>, dim3(nb), dim3(256), 0, s, G, F, use_ref);
    if (do_h) hipLaunchKernelGGL(k_hfield<T>, dim3(nb), dim3(256), 0, s, G, F, use_ref);
}

template <typename T>
void launch_bhalf(const Grid &G, FieldPtrsT<T> &F, const T *const Bin[3], double hstep, hipStream_t s) {
    hipLaunchKernelGGL(k_bhalf<T>, dim3(nblk(G.nnodes(), 256)), dim3(256), 0, s, G, F, Bin[0], Bin[1], Bin[2],
                       (T)hstep);
}

template <typename T>
void launch_dstep(const Grid &G, FieldPtrsT<T> &F, const T *const Din[3], double dx4, double fpc, double inv_jscale,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_dstep<T>, dim3(nblk(G.nnodes(), 256)), dim3(256), 0, s, G, F, Din[0], Din[1], Din[2],
                       (T)dx4, (T)fpc, inv_jscale);
}

// Copy of three field components (one launch instead of three copies).
template <typename T>
__global__ void k_save3(FieldPtrsT<T> F, int which, int64_t n) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    for (int q = 0; q < 3; q++) {
        if (which == 0)
            F.Bsave[q][id] = F.B[q][id];
        else
            F.Dsave[q][id] = F.D[q][id];
    }
}

template <typename T> void launch_save(const Grid &G, FieldPtrsT<T> &F, int which, hipStream_t s) {
    hipLaunchKernelGGL(k_save3<T>, dim3(nblk(G.gsize(), 256)), dim3(256), 0, s, F, which, G.gsize());
}

// Index box of the relaxation layer: the bounding box of the oblate region
// r < r_damp (|x|,|y| <= sqrt(r^2+a^2), |z| <= r) clipped to the grid;
// bx = by = bz = 0 when there is no layer.
void relax_box_of(const Grid &G, const Hole &h, double r_damp, double damp_max, int box[6]) {
    for (int q = 0; q < 6; q++) box[q] = 0;
    if (!(r_damp > h.r_exc) || !(damp_max > 0.0) || h.m == 0.0) return;
    double ext_xy = sqrt(r_damp * r_damp + h.a * h.a) + 1.0, ext_z = r_damp + 1.0;
    int i0 = (int)floor(h.cx - ext_xy), i1 = (int)ceil(h.cx + ext_xy);
    int j0 = (int)floor(h.cy - ext_xy), j1 = (int)ceil(h.cy + ext_xy);
    int k0 = (int)floor(h.cz - ext_z), k1 = (int)ceil(h.cz + ext_z);
    i0 = i0 < 0 ? 0 : i0; j0 = j0 < 0 ? 0 : j0; k0 = k0 < 0 ? 0 : k0;
    i1 = i1 > G.nx ? G.nx : i1; j1 = j1 > G.ny ? G.ny : j1; k1 = k1 > G.nz ? G.nz : k1;
    if (i1 < i0 || j1 < j0 || k1 < k0) return;
    box[0] = i0; box[1] = j0; box[2] = k0;
    box[3] = i1 - i0 + 1; box[4] = j1 - j0 + 1; box[5] = k1 - k0 + 1;
}

template <typename T>
void launch_relax(const Grid &G, const Hole &h, FieldPtrsT<T> &F, double r_damp, double damp_max, hipStream_t s) {
    int box[6];
    relax_box_of(G, h, r_damp, damp_max, box);
    if (box[3] == 0) return;
    hipLaunchKernelGGL(k_relax<T>, dim3(nblk((int64_t)box[3] * box[4] * box[5], 128)), dim3(128), 0, s, G, h, F,
                       r_damp, damp_max, box[0], box[1], box[2], box[3], box[4], box[5]);
}
template <typename T>
void launch_relax_outer(const Grid &G, FieldPtrsT<T> &F, double L, double damp, hipStream_t s) {
    if (!(L > 0.0) || !(damp > 0.0)) return;
    hipLaunchKernelGGL(k_relax_outer<T>, dim3(nblk(G.nnodes(), 256)), dim3(256), 0, s, G, F, L, damp);
}

// ---------------------------------------------------------------------------
// Serving batch: one persistent launch per field stage over the logical
// blocks of every active run (FP32 fields).  Stages of the fixed-point
// passes skip runs with fewer passes than `it + 1`.
template <int OP>
__global__ __launch_bounds__(kBatchBlock) void k_batch_field(const BatchTable *__restrict__ T, int it) {
    constexpr int kind = (OP == BF_SAVE_B || OP == BF_ZERO_J || OP == BF_SAVE_D) ? BK_GRID
                         : (OP == BF_RELAX ? BK_RELAX : BK_NODE);
    constexpr bool pass = OP == BF_NODE_W || OP == BF_ECOV || OP == BF_BHALF_SAVED || OP == BF_HFIELD ||
                          OP == BF_DSTEP;
    const int64_t total = T->total[kind];
    for (int64_t lb = blockIdx.x; lb < total; lb += gridDim.x) {
        const BatchRun32 &R = T->run[batch_run_of(T, kind, lb)];
        if (pass && it >= R.field_iters) continue;
        const int64_t id = (lb - R.off[kind]) * kBatchBlock + threadIdx.x;
        const Grid &G = R.G;
        const FieldPtrsT<float> &F = R.F;
        if (kind == BK_GRID) {
            if (id >= G.gsize()) continue;
            for (int q = 0; q < 3; q++) {
                if (OP == BF_SAVE_B) F.Bsave[q][id] = F.B[q][id];
                if (OP == BF_SAVE_D) F.Dsave[q][id] = F.D[q][id];
                if (OP == BF_ZERO_J) F.Jint[q][id] = 0ull;
            }
        } else if (kind == BK_RELAX) {
            if (id < (int64_t)R.relax_box[3] * R.relax_box[4] * R.relax_box[5])
                relax_at<float>(G, R.h, F, R.r_damp, R.damp_max, R.relax_box, id);
        } else {
            if (id >= G.nnodes()) continue;
            if (OP == BF_NODE_W) node_w_at<float>(G, R.h, F, id);
            if (OP == BF_ECOV) ecov_at<float>(G, F, true, id);
            if (OP == BF_HFIELD) hfield_at<float>(G, F, true, id);
            if (OP == BF_NODE_TENSOR) node_tensor_at<float>(G, R.h, F, id);
            if (OP == BF_BHALF_SAVED || OP == BF_BHALF_CUR) {
                const float *Bin[3] = {F.Bsave[0], F.Bsave[1], F.Bsave[2]};
                if (OP == BF_BHALF_CUR) {
                    Bin[0] = F.B[0];
                    Bin[1] = F.B[1];
                    Bin[2] = F.B[2];
                }
                bhalf_at<float>(G, F, Bin, R.hstep, id);
            }
            if (OP == BF_DSTEP) {
                const float *Din[3] = {F.Dsave[0], F.Dsave[1], F.Dsave[2]};
                const double dtp = (it < R.field_iters - 1) ? 0.5 * R.dt : R.dt;
                dstep_at<float>(G, F, Din, (float)(R.c * dtp), R.fpc, R.inv_jscale, id);
            }
        }
    }
}

void launch_batch_field(int op, const BatchTable *table, int it, int grid, hipStream_t s) {
    switch (op) {
#define GRPIC_BF(OP) \
    case OP: hipLaunchKernelGGL(k_batch_field<OP>, dim3(grid), dim3(kBatchBlock), 0, s, table, it); break;
        GRPIC_BF(BF_SAVE_B)
        GRPIC_BF(BF_NODE_W)
        GRPIC_BF(BF_ECOV)
        GRPIC_BF(BF_BHALF_SAVED)
        GRPIC_BF(BF_NODE_TENSOR)
        GRPIC_BF(BF_BHALF_CUR)
        GRPIC_BF(BF_ZERO_J)
        GRPIC_BF(BF_SAVE_D)
        GRPIC_BF(BF_HFIELD)
        GRPIC_BF(BF_DSTEP)
        GRPIC_BF(BF_RELAX)
#undef GRPIC_BF
    }
}

template <typename T> void launch_node_tensor(const Grid &G, const Hole &h, FieldPtrsT<T> &F, hipStream_t s) {
    hipLaunchKernelGGL(k_node_tensor<T>, dim3(nblk(G.nnodes(), kNodeTensorBlock)), dim3(kNodeTensorBlock), 0, s, G, h,
                       F);
}

#define GRPIC_FIELD_INSTANTIATE(T)                                                                          \
    template void launch_bake<T>(const Grid &, const Hole &, FieldPtrsT<T> &, hipStream_t);                 \
    template void launch_init_fields<T>(const Grid &, const Hole &, FieldPtrsT<T> &, const double *, int,   \
                                        hipStream_t);                                                       \
    template void launch_derived<T>(const Grid &, const Hole &, FieldPtrsT<T> &, bool, bool, bool,          \
                                    hipStream_t);                                                           \
    template void launch_bhalf<T>(const Grid &, FieldPtrsT<T> &, const T *const *, double, hipStream_t);    \
    template void launch_dstep<T>(const Grid &, FieldPtrsT<T> &, const T *const *, double, double, double,  \
                                  hipStream_t);                                                             \
    template void launch_relax<T>(const Grid &, const Hole &, FieldPtrsT<T> &, double, double, hipStream_t); \
    template void launch_relax_outer<T>(const Grid &, FieldPtrsT<T> &, double, double, hipStream_t);          \
    template void launch_node_tensor<T>(const Grid &, const Hole &, FieldPtrsT<T> &, hipStream_t);          \
    template void launch_save<T>(const Grid &, FieldPtrsT<T> &, int, hipStream_t);
GRPIC_FIELD_INSTANTIATE(double)
GRPIC_FIELD_INSTANTIATE(float)

}  // namespace grpic
