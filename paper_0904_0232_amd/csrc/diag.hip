// Diagnostics (FP64, deterministic): per-block tree reductions in a fixed
// order, finished on the host in block order.  Charge for the Gauss residual
// is accumulated in int64 fixed point, so it too is order-independent.
#include <vector>

#include "grpic_dev.h"
#include "grpic_impl.h"

namespace grpic {

constexpr int kDiagBlock = 256;

template <int NV>
__device__ void block_reduce(double (&v)[NV], const unsigned max_mask, double *out) {
    __shared__ double sh[NV][kDiagBlock];
    int t = threadIdx.x;
    for (int q = 0; q < NV; q++) sh[q][t] = v[q];
    __syncthreads();
    for (int s = kDiagBlock / 2; s > 0; s >>= 1) {
        if (t < s)
            for (int q = 0; q < NV; q++) {
                double a = sh[q][t], b = sh[q][t + s];
                sh[q][t] = ((max_mask >> q) & 1u) ? (a > b ? a : b) : a + b;
            }
        __syncthreads();
    }
    if (t == 0)
        for (int q = 0; q < NV; q++) out[(int64_t)blockIdx.x * NV + q] = sh[q][0];
}

// Particle sums: 0 charge, 1 energy M c (-u_4), 2 L_z, 3 max |g(u,u)+c^2|,
// 4..11 live count per species.  Also deposits the live charge on the nodes.
constexpr int kNVp = 12;
__global__ __launch_bounds__(kDiagBlock) void k_diag_particles(Grid G, Hole h, double c, double rscale, Species S,
                                                               ParticlePtrs P, int64_t n,
                                                               unsigned long long *rho, double *out) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[kNVp];
    for (int q = 0; q < kNVp; q++) v[q] = 0.0;
    if (id < n) {
        uint8_t sp = P.sp[id];
        if (sp != kDead) {
            double X[3] = {P.x[0][id], P.x[1][id], P.x[2][id]};
            double U[4] = {P.u[0][id], P.u[1][id], P.u[2][id], P.u[3][id]};
            double x = X[0] - h.cx, y = X[1] - h.cy, z = X[2] - h.cz;
            double f = 0.0, k[3] = {0.0, 0.0, 0.0};
            if (h.m != 0.0) {
                KSPoint<double> p;
                ks_point(h.m, h.a, x, y, z, p);
                f = p.f;
                k[0] = p.k0;
                k[1] = p.k1;
                k[2] = p.k2;
            }
            double ku = k[0] * U[0] + k[1] * U[1] + k[2] * U[2] + U[3];
            double ul[4] = {U[0] + f * k[0] * ku, U[1] + f * k[1] * ku, U[2] + f * k[2] * ku, -U[3] + f * ku};
            double shell = c * c + ul[0] * U[0] + ul[1] * U[1] + ul[2] * U[2] + ul[3] * U[3];
            double M = S.mass[sp];
            v[0] = S.charge[sp];
            v[1] = M * c * (-ul[3]);
            v[2] = M * (x * ul[1] - y * ul[0]);
            v[3] = fabs(shell);
            v[4 + sp] = 1.0;
            int cc[3];
            double w[3];
            for (int ax = 0; ax < 3; ax++) {
                cc[ax] = (int)floor(X[ax]);
                w[ax] = X[ax] - (double)cc[ax];
            }
            bool inb = true;
            for (int ax = 0; ax < 3; ax++)
                if (!(cc[ax] >= -1 && cc[ax] <= G.dim(ax))) inb = false;
            double sc = inb ? S.charge[sp] * rscale : 0.0;
            for (int dk = 0; dk < 2 && inb; dk++)
                for (int dj = 0; dj < 2; dj++)
                    for (int di = 0; di < 2; di++) {
                        double W = (di ? w[0] : 1.0 - w[0]) * (dj ? w[1] : 1.0 - w[1]) * (dk ? w[2] : 1.0 - w[2]);
                        atomicAdd(&rho[G.g(cc[0] + di, cc[1] + dj, cc[2] + dk)],
                                  (unsigned long long)__double2ll_rn(sc * W));
                    }
        }
    }
    block_reduce<kNVp>(v, 1u << 3, out);
}

__device__ __forceinline__ bool in_dom(const Grid &G, int kind, int c, int i, int j, int k) {
    int idx[3] = {i, j, k};
    for (int ax = 0; ax < 3; ax++) {
        bool half = kind == 0 ? (ax == c) : (ax != c);
        int n = G.dim(ax);
        if (idx[ax] < 0 || idx[ax] > (half ? n - 1 : n)) return false;
    }
    return true;
}

__device__ __forceinline__ bool relaxed_e(const Grid &G, const Hole &h, double r_damp, double damp_max, int c, int i,
                                          int j, int k) {
    if (!(r_damp > h.r_exc) || !(damp_max > 0.0) || h.m == 0.0) return false;
    double X = i + (c == 0 ? 0.5 : 0.0), Y = j + (c == 1 ? 0.5 : 0.0), Z = k + (c == 2 ? 0.5 : 0.0);
    return ks_radius(h.a, X - h.cx, Y - h.cy, Z - h.cz) < r_damp;
}

// Whether the E point c at (i, j, k) lies in the outer absorbing layer.
__device__ __forceinline__ bool outer_e(const Grid &G, double L, double damp, int c, int i, int j, int k) {
    if (!(L > 0.0) || !(damp > 0.0)) return false;
    double X = i + (c == 0 ? 0.5 : 0.0), Y = j + (c == 1 ? 0.5 : 0.0), Z = k + (c == 2 ? 0.5 : 0.0);
    return outer_distance(G, X, Y, Z) < L;
}

// Field sums over index (i,j,k) in [0,n]^3: 0 sum -E_cov D over E points,
// 1 sum B H over B points, 2 max Gauss residual at checked nodes (not in the
// inner relaxation layer or the outer absorbing layer).
constexpr int kNVf = 3;
template <typename T>
__global__ __launch_bounds__(kDiagBlock) void k_diag_fields(Grid G, Hole h, FieldPtrsT<T> F, double rscale, double r_damp,
                                                            double damp_max, double outer_layer, double outer_damp,
                                                            const unsigned long long *rho, double *out) {
    int64_t nn = G.nnodes();
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[kNVf] = {0.0, 0.0, 0.0};
    if (id < nn) {
        int i = (int)(id % (G.nx + 1));
        int64_t t = id / (G.nx + 1);
        int j = (int)(t % (G.ny + 1));
        int k = (int)(t / (G.ny + 1));
        int64_t gi = G.g(i, j, k);
        for (int c = 0; c < 3; c++) {
            if (in_dom(G, 0, c, i, j, k)) v[0] += -(double)F.E[c][gi] * (double)F.D[c][gi];
            if (in_dom(G, 1, c, i, j, k)) v[1] += (double)F.B[c][gi] * (double)F.H[c][gi];
        }
        if (i >= 1 && i <= G.nx - 1 && j >= 1 && j <= G.ny - 1 && k >= 1 && k <= G.nz - 1) {
            int64_t st[3] = {1, G.sx, G.sy};
            bool ok = true;
            double div = 0.0;
            for (int c = 0; c < 3; c++) {
                int im[3] = {i, j, k};
                im[c] -= 1;
                if (!(F.mask[gi] & (1u << c)) || !(F.mask[gi - st[c]] & (1u << c))) ok = false;
                if (relaxed_e(G, h, r_damp, damp_max, c, i, j, k) ||
                    relaxed_e(G, h, r_damp, damp_max, c, im[0], im[1], im[2]) ||
                    outer_e(G, outer_layer, outer_damp, c, i, j, k) ||
                    outer_e(G, outer_layer, outer_damp, c, im[0], im[1], im[2]))
                    ok = false;
                div += (double)F.D[c][gi] - (double)F.D[c][gi - st[c]];
            }
            if (ok) {
                double q = ((double)(long long)rho[gi] + (double)(long long)F.rho_abs[gi]) / rscale;
                v[2] = fabs(-div - 4.0 * M_PI * q);
            }
        }
    }
    block_reduce<kNVf>(v, 1u << 2, out);
}

template <typename T>
int run_diag(const Grid &G, const Hole &h, double c, double rscale, const Species &S, ParticlePtrs P, int64_t n,
             FieldPtrsT<T> &F, double r_damp, double damp_max, double outer_layer, double outer_damp,
             unsigned long long *rho_scratch, double *red_scratch, int64_t red_cap, DiagOut &out, hipStream_t s) {
    int64_t nbp = n > 0 ? (n + kDiagBlock - 1) / kDiagBlock : 0;
    int64_t nbf = (G.nnodes() + kDiagBlock - 1) / kDiagBlock;
    if (nbp * kNVp + nbf * kNVf > red_cap) return -1;
    launch_zero_u64(rho_scratch, G.gsize(), s);
    double *pp = red_scratch;
    double *pf = red_scratch + nbp * kNVp;
    if (nbp > 0)
        hipLaunchKernelGGL(k_diag_particles, dim3((unsigned)nbp), dim3(kDiagBlock), 0, s, G, h, c, rscale, S, P, n,
                           rho_scratch, pp);
    hipLaunchKernelGGL(k_diag_fields<T>, dim3((unsigned)nbf), dim3(kDiagBlock), 0, s, G, h, F, rscale, r_damp,
                       damp_max, outer_layer, outer_damp, rho_scratch, pf);
    std::vector<double> hp(nbp * kNVp), hf(nbf * kNVf);
    if (nbp > 0 && hipMemcpyAsync(hp.data(), pp, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
        return -2;
    if (hipMemcpyAsync(hf.data(), pf, hf.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return -2;
    if (hipStreamSynchronize(s) != hipSuccess) return -2;
    double acc[kNVp];
    for (int q = 0; q < kNVp; q++) acc[q] = 0.0;
    for (int64_t b = 0; b < nbp; b++)
        for (int q = 0; q < kNVp; q++) {
            double v = hp[b * kNVp + q];
            if (q == 3)
                acc[q] = v > acc[q] ? v : acc[q];
            else
                acc[q] += v;
        }
    double fa[kNVf] = {0.0, 0.0, 0.0};
    for (int64_t b = 0; b < nbf; b++)
        for (int q = 0; q < kNVf; q++) {
            double v = hf[b * kNVf + q];
            if (q == 2)
                fa[q] = v > fa[q] ? v : fa[q];
            else
                fa[q] += v;
        }
    out.charge_total = acc[0];
    out.energy_particles = acc[1];
    out.lz_particles = acc[2];
    out.shell_max = acc[3];
    for (int q = 0; q < kMaxSpecies; q++) out.n_alive[q] = (int64_t)acc[4 + q];
    out.energy_field = (fa[0] + fa[1]) / (8.0 * M_PI);
    out.gauss_max = fa[2];
    return 0;
}

template int run_diag<double>(const Grid &, const Hole &, double, double, const Species &, ParticlePtrs, int64_t,
                              FieldPtrsT<double> &, double, double, double, double, unsigned long long *, double *,
                              int64_t, DiagOut &, hipStream_t);
template int run_diag<float>(const Grid &, const Hole &, double, double, const Species &, ParticlePtrs, int64_t,
                             FieldPtrsT<float> &, double, double, double, double, unsigned long long *, double *,
                             int64_t, DiagOut &, hipStream_t);

}  // namespace grpic
