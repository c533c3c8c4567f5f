// Two-level composite Poisson solve: a coarse level over the whole domain and
// a fine level (refinement ratio 2) over a union of boxes -- the paper's
// block-structured AMR hierarchy (Sections 1 and 2: levels of boxes,
// inter-level interpolation and averaging, copies between decompositions).
//
// Unknowns are the fine cells and the coarse cells no fine box covers; a
// covered coarse cell holds the mean of its 8 children.
//  * A fine ghost across the coarse-fine boundary is the quadratic along the
//    normal through U_t and the two fine cells inward (u1, u2):
//    g = (8/15) U_t + (2/3) u1 - (1/5) u2, where U_t is the quadratic through
//    the 3x3 coarse cells around the ghost's coarse cell C in the face plane
//    (with the mixed term) taken at the ghost's offset (s_a, s_b) h0/4,
//    s = +1 on the upper half of C, -1 on the lower.
//  * Fine operator: the 7-point one with those ghosts (ghosts between fine
//    boxes copied from the neighbouring box).
//  * Coarse operator at an uncovered cell: (sum of the 6 outward gradients)
//    / h0; across a face against a covered cell the gradient is the mean of
//    the 4 fine gradients (u_i - g_i) / h1 through it, so the coarse flux is
//    the sum of the fine ones and the composite operator conserves.
//  * Cycle: nu1 fine red-black sweeps (ghosts refreshed before each colour),
//    composite residual (covered coarse cells take the mean of the fine
//    residuals), one coarse V-cycle from zero, correction of the uncovered
//    coarse cells and of the fine cells (trilinear interpolation, weights
//    27, 9, 3, 1 over 64 from the parent and its neighbours on the child's
//    side), nu2 fine sweeps, covered cells := mean of their children.
//
// Storage: the coarse level lives in one-box MultiFabs over the domain (the
// caller's coarse data is ParallelCopy'd in and out), so any coarse cell is
// one address computation away; a dense int map over the coarse cells holds
// the fine box that covers each one, or -1 - (mask of covered face
// neighbours).  The fine level lives in colour-split storage of its own:
// every fine box grown by one ghost layer, cell (i, j, k) of colour
// c = (i + j + k) & 1 in colour block c at row ((k - glo_z) G_y + (j - glo_y))
// and slot (i - glo_x) >> 1, so a colour sweep streams the other colour,
// its own right-hand side and its own writes.  When the fine boxes tile one
// rectangle the fine level is that one box (no ghosts between boxes);
// otherwise ghosts between fine boxes are copied from a per-layout list.
// The caller's fine fields are converted in (right-hand side) and out
// (solution) once per solve; the coarse-fine ghost cells are listed once
// per layout.  Fine boxes must be unions of whole coarse cells (even lower,
// odd upper corners) and lie at least 2 coarse cells inside the domain, so
// that every coarse cell a ghost or an interpolation reads is a domain cell.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "bxmg_host.h"

namespace bxmg {
namespace comp {

constexpr int kCB = 256;  // threads per block
constexpr int kKZ = 8;    // planes each thread walks (kernels that reduce norms, coarse kernels)
constexpr int kKZs = 4;   // planes each thread walks in the fine sweeps and the interpolation

// The coarse level: layout of the one-box fields and the domain.
// The coarse level: the one-box layout of its solution and right-hand side
// (F order, 1 ghost) and of the correction's colour-split level-0 arrays
// (residual = the V-cycle's right-hand side, correction = its solution).
struct CGeo {
    FBox cb;
    int dlo[3], n[3];  // coarse domain
    int per[3];
    double h0, h1;
    double ih0sq;  // 1 / h0^2
    int rlo[3], rglo[3], rG[3], rH;  // colour-split layout of the correction arrays
    long long rbase, rcs;
};

// A fine box in colour-split storage (grown by 1): colour block c of the
// box starts at base + c * cs; rows of H slots.
struct FRB {
    int lo[3], hi[3];  // valid cells
    int glo[3];        // lo - 1
    int G[3];          // edges + 2
    int H;             // slots per colour row, (G_x + 1) / 2
    int pad;
    long long base, cs;
};

__host__ __device__ __forceinline__ long long frb_at(const FRB& b, int i, int j, int k) {
    const int c = (i + j + k) & 1;
    return b.base + c * b.cs + (long long)(((k - b.glo[2]) * b.G[1] + (j - b.glo[1])) * b.H + ((i - b.glo[0]) >> 1));
}

// Coverage map entry of a coarse cell: >= 0 the fine box covering it;
// otherwise -1 - mask, bit 2 d + side of mask set when the face neighbour
// across (d, side) is covered, bit 6 when the cell lies on a domain face.
__device__ __forceinline__ int cq(const CGeo& g, int I, int J, int K) {
    return (I - g.dlo[0]) + g.n[0] * ((J - g.dlo[1]) + g.n[1] * (K - g.dlo[2]));
}

// offset of coarse cell (I, J, K) in the correction arrays
__device__ __forceinline__ long long ridx(const CGeo& g, int I, int J, int K) {
    return g.rbase + ((I + J + K) & 1) * g.rcs +
           (long long)(((K - g.rglo[2]) * g.rG[1] + (J - g.rglo[1])) * g.rH + ((I - g.rglo[0]) >> 1));
}

__device__ __forceinline__ long long fidx(const FBox& b, int i, int j, int k) {
    return b.base + (long long)((i - b.glo[0]) + b.G[0] * ((j - b.glo[1]) + b.G[1] * (k - b.glo[2])));
}

__device__ __forceinline__ void block_norms(double mx, double s2, double bad, double* __restrict__ out3) {
    __shared__ double sh[3 * (kCB / 64)];
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o));
        s2 = s2 + __shfl_xor(s2, o);
        bad = bad + __shfl_xor(bad, o);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { sh[3 * wid] = mx; sh[3 * wid + 1] = s2; sh[3 * wid + 2] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kCB / 64; ++w) { mx = fmax(mx, sh[3 * w]); s2 = s2 + sh[3 * w + 1]; bad = bad + sh[3 * w + 2]; }
        out3[0] = mx;
        out3[1] = s2;
        out3[2] = bad;
    }
}

__device__ __forceinline__ void norm_add(double rv, double& mx, double& s2, double& bad) {
    const double a = fabs(rv);
    if (!(a <= 1.7976931348623157e308)) bad += 1.0;
    else mx = fmax(mx, a);
    s2 = s2 + rv * rv;
}

// mean of the 8 children (2I.., 2J.., 2K..) of a coarse cell
__device__ __forceinline__ double mean8(const double* __restrict__ x, const FRB& B, int i, int j, int k) {
    return (((x[frb_at(B, i, j, k)] + x[frb_at(B, i + 1, j, k)]) +
             (x[frb_at(B, i, j + 1, k)] + x[frb_at(B, i + 1, j + 1, k)])) +
            ((x[frb_at(B, i, j, k + 1)] + x[frb_at(B, i + 1, j, k + 1)]) +
             (x[frb_at(B, i, j + 1, k + 1)] + x[frb_at(B, i + 1, j + 1, k + 1)]))) * 0.125;
}

// Coarse-fine ghosts.  One entry per ghost cell: x = box | d << 24 | side << 26
// (the ghost lies beyond face (d, side) of its box), y, z, w = its fine index.
__global__ void __launch_bounds__(kCB) k_cf_ghost(const int4* __restrict__ list, int n, CGeo g,
                                                  const double* __restrict__ Uc, const FRB* __restrict__ fb,
                                                  double* __restrict__ uf) {
    const int q = blockIdx.x * kCB + threadIdx.x;
    if (q >= n) return;
    const int4 r = list[q];
    const int b = r.x & 0xffffff, d = (r.x >> 24) & 3, side = (r.x >> 26) & 1;
    const int gx[3] = {r.y, r.z, r.w};
    const FRB B = fb[b];
    const int step = side ? -1 : 1;  // from the ghost into its box
    int i1[3] = {gx[0], gx[1], gx[2]}, i2[3] = {gx[0], gx[1], gx[2]};
    i1[d] += step;
    i2[d] += 2 * step;
    const int C[3] = {gx[0] >> 1, gx[1] >> 1, gx[2] >> 1};
    const int ta = d == 2 ? 0 : d + 1, tb = d == 0 ? 2 : d - 1;
    const double sa = (gx[ta] & 1) ? 1.0 : -1.0, sb = (gx[tb] & 1) ? 1.0 : -1.0;
    const long long c0 = fidx(g.cb, C[0], C[1], C[2]);
    const long long st[3] = {1, g.cb.G[0], (long long)g.cb.G[0] * g.cb.G[1]};
    const long long da_ = st[ta], db_ = st[tb];
    auto U = [&](int p, int s) { return Uc[c0 + p * da_ + s * db_]; };
    const double UC = U(0, 0);
    const double Up0 = U(1, 0), Um0 = U(-1, 0), U0p = U(0, 1), U0m = U(0, -1);
    const double da = (Up0 - Um0) * 0.125 * sa, db = (U0p - U0m) * 0.125 * sb;
    const double qa = ((Up0 + Um0) - 2.0 * UC) * (1.0 / 32.0);
    const double qb = ((U0p + U0m) - 2.0 * UC) * (1.0 / 32.0);
    const double xab = ((U(1, 1) - U(1, -1)) - (U(-1, 1) - U(-1, -1))) * (1.0 / 64.0) * (sa * sb);
    const double Ut = UC + ((da + db) + (qa + qb)) + xab;
    const double u1 = uf[frb_at(B, i1[0], i1[1], i1[2])], u2 = uf[frb_at(B, i2[0], i2[1], i2[2])];
    uf[frb_at(B, gx[0], gx[1], gx[2])] = ((8.0 / 15.0) * Ut + (2.0 / 3.0) * u1) - (1.0 / 5.0) * u2;
}

// Fine-box kernels: grid (plane blocks, plane groups, box); a thread takes
// one slot of a row of its box (the two cells sharing that slot, or the
// one of the swept colour) and walks the group's planes.
__device__ __forceinline__ int frb_slots(const FRB& B) { return ((B.hi[0] - B.glo[0]) >> 1) + 1; }

// One colour of red-black Gauss-Seidel on the fine boxes (ghosts current):
// u = (sum of the 6 neighbours - h1^2 f) / 6 at the cells of that colour.
__global__ void __launch_bounds__(kCB) k_fine_gs(CGeo g, const FRB* __restrict__ fb, double* __restrict__ u,
                                                 const double* __restrict__ f, int colour) {
    const uint3 bk = xcd_block();
    const FRB B = fb[bk.z];
    const int ns = frb_slots(B), ny = B.hi[1] - B.lo[1] + 1;
    const int t = bk.x * kCB + threadIdx.x;
    if (t >= ns * ny) return;
    const int ts = t % ns, j = B.lo[1] + t / ns;
    const int k0 = B.lo[2] + bk.y * kKZs, k1 = min(k0 + kKZs - 1, B.hi[2]);
    const long long sy = B.H, sz = (long long)B.H * B.G[1];
    const double h2 = g.h1 * g.h1;
    for (int k = k0; k <= k1; ++k) {
        const int i = B.glo[0] + 2 * ts + ((colour + B.glo[0] + j + k) & 1);
        if (i < B.lo[0] || i > B.hi[0]) continue;
        const long long row = (long long)((k - B.glo[2]) * B.G[1] + (j - B.glo[1])) * B.H;
        const long long o = B.base + (1 - colour) * B.cs + row;  // other colour, this row
        const long long c = B.base + colour * B.cs + row + ((i - B.glo[0]) >> 1);
        const long long m = o + ((i - B.glo[0]) >> 1);
        const double xm = u[o + ((i - 1 - B.glo[0]) >> 1)], xp = u[o + ((i + 1 - B.glo[0]) >> 1)];
        const double su = ((xm + xp) + (u[m - sy] + u[m + sy])) + (u[m - sz] + u[m + sz]);
        u[c] = (su - h2 * f[c]) / 6.0;
    }
}

// The sum of the 6 neighbours of fine cell (i, j, k).
__device__ __forceinline__ double nsum(const double* __restrict__ u, const FRB& B, int i, int j, int k) {
    const int c = (i + j + k) & 1;
    const long long row = (long long)((k - B.glo[2]) * B.G[1] + (j - B.glo[1])) * B.H;
    const long long o = B.base + (1 - c) * B.cs + row;
    const long long m = o + ((i - B.glo[0]) >> 1);
    const long long sy = B.H, sz = (long long)B.H * B.G[1];
    const double xm = u[o + ((i - 1 - B.glo[0]) >> 1)], xp = u[o + ((i + 1 - B.glo[0]) >> 1)];
    return ((xm + xp) + (u[m - sy] + u[m + sy])) + (u[m - sz] + u[m + sz]);
}

// The residual kernels' modes: the norms of f, the norms of the residual,
// or the norms and the residual stored.
enum { kNormsF = 0, kNormsR = 1, kStoreR = 2 };

// Fine residual r = f - L u on the valid cells, with per-block norms (max,
// sum of squares, non-finite count).
__global__ void __launch_bounds__(kCB) k_fine_resid(CGeo g, const FRB* __restrict__ fb, const double* __restrict__ u,
                                                    const double* __restrict__ f, double* __restrict__ r, int mode,
                                                    double* __restrict__ partials) {
    const uint3 bk = xcd_block();
    const FRB B = fb[bk.z];
    const int ns = frb_slots(B), ny = B.hi[1] - B.lo[1] + 1;
    const int t = bk.x * kCB + threadIdx.x;
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    if (t < ns * ny) {
        const int ts = t % ns, j = B.lo[1] + t / ns;
        const int k0 = B.lo[2] + bk.y * kKZ, k1 = min(k0 + kKZ - 1, B.hi[2]);
        const double ih2 = 1.0 / (g.h1 * g.h1);
        for (int k = k0; k <= k1; ++k)
            for (int e = 0; e < 2; ++e) {
                const int i = B.glo[0] + 2 * ts + e;
                if (i < B.lo[0] || i > B.hi[0]) continue;
                const long long c = frb_at(B, i, j, k);
                double rv = f[c];
                if (mode != kNormsF) {
                    rv = rv - (nsum(u, B, i, j, k) - 6.0 * u[c]) * ih2;
                    if (mode == kStoreR) r[c] = rv;
                }
                norm_add(rv, mx, s2, bad);
            }
    }
    const int blk = (bk.z * gridDim.y + bk.y) * gridDim.x + bk.x;
    block_norms(mx, s2, bad, partials + 3 * (long long)blk);
}

// Fine cells += trilinear interpolation of the coarse correction Ec.
__global__ void __launch_bounds__(kCB) k_fine_prolong(CGeo g, const FRB* __restrict__ fb, double* __restrict__ u,
                                                      const double* __restrict__ Ec) {
    const uint3 bk = xcd_block();
    const FRB B = fb[bk.z];
    const int ns = frb_slots(B), ny = B.hi[1] - B.lo[1] + 1;
    const int t = bk.x * kCB + threadIdx.x;
    if (t >= ns * ny) return;
    const int ts = t % ns, j = B.lo[1] + t / ns;
    const int k0 = B.lo[2] + bk.y * kKZs, k1 = min(k0 + kKZs - 1, B.hi[2]);
    const int J = j >> 1, sj = (j & 1) ? 1 : -1;
    for (int k = k0; k <= k1; ++k) {
        const int K = k >> 1, sk = (k & 1) ? 1 : -1;
        for (int e = 0; e < 2; ++e) {
            const int i = B.glo[0] + 2 * ts + e;
            if (i < B.lo[0] || i > B.hi[0]) continue;
            const int I = i >> 1, si = (i & 1) ? 1 : -1;
            const double c000 = Ec[ridx(g, I, J, K)], c100 = Ec[ridx(g, I + si, J, K)];
            const double c010 = Ec[ridx(g, I, J + sj, K)], c001 = Ec[ridx(g, I, J, K + sk)];
            const double c110 = Ec[ridx(g, I + si, J + sj, K)], c101 = Ec[ridx(g, I + si, J, K + sk)];
            const double c011 = Ec[ridx(g, I, J + sj, K + sk)], c111 = Ec[ridx(g, I + si, J + sj, K + sk)];
            const double v = (((27.0 * c000 + 9.0 * ((c100 + c010) + c001)) + 3.0 * ((c110 + c101) + c011)) + c111) *
                             (1.0 / 64.0);
            const long long c = frb_at(B, i, j, k);
            u[c] = u[c] + v;
        }
    }
}

// Caller layout <-> colour-split storage: grid (plane blocks, plane groups,
// caller box); caller box b lies in storage box map[b].
template <bool TO_FRB>
__global__ void __launch_bounds__(kCB) k_fab_frb(const FBox* __restrict__ fab, double* __restrict__ x,
                                                 const FRB* __restrict__ fb, const int* __restrict__ map,
                                                 double* __restrict__ y) {
    const uint3 bk = xcd_block();
    const FBox A = fab[bk.z];
    const FRB B = fb[map[bk.z]];
    const int nx = A.hi[0] - A.lo[0] + 1, ny = A.hi[1] - A.lo[1] + 1;
    const int t = bk.x * kCB + threadIdx.x;
    if (t >= nx * ny) return;
    const int i = A.lo[0] + t % nx, j = A.lo[1] + t / nx;
    const int k0 = A.lo[2] + bk.y * kKZ, k1 = min(k0 + kKZ - 1, A.hi[2]);
    for (int k = k0; k <= k1; ++k) {
        if constexpr (TO_FRB) y[frb_at(B, i, j, k)] = x[fidx(A, i, j, k)];
        else x[fidx(A, i, j, k)] = y[frb_at(B, i, j, k)];
    }
}

// Coarse kernels: grid (plane blocks, plane groups of kKZ) over the domain.

// The composite operator at an uncovered coarse cell with a covered face
// neighbour or on a domain face: (sum of the 6 outward gradients) / h0,
// a face against a covered cell taking the mean of the 4 fine gradients
// through it (from the fine ghosts, which must be current).
__device__ __forceinline__ double coarse_op_special(const CGeo& g, const int* __restrict__ cmap,
                                                    const double* __restrict__ Uc, const FRB* __restrict__ fb,
                                                    const double* __restrict__ uf, int I, int J, int K, int mask) {
    const int q = cq(g, I, J, K);
    const long long c = fidx(g.cb, I, J, K);
    const long long st[3] = {1, g.cb.G[0], (long long)g.cb.G[0] * g.cb.G[1]};
    const int mst[3] = {1, g.n[0], g.n[0] * g.n[1]};
    const double UI = Uc[c];
    const int X[3] = {I, J, K};
    double gr[6];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int nbd = X[d] + (side ? 1 : -1);
            double v;
            if ((mask >> (2 * d + side)) & 1) {
                // the 4 fine cells of the covered neighbour against the face
                int nb[3] = {X[0], X[1], X[2]};
                nb[d] = nbd;
                const FRB B = fb[cmap[q + (side ? mst[d] : -mst[d])]];
                const int ta = d == 2 ? 0 : d + 1, tb = d == 0 ? 2 : d - 1;
                double a[2][2];
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        int fi[3];
                        fi[d] = 2 * nb[d] + (side ? 0 : 1);
                        fi[ta] = 2 * nb[ta] + p;
                        fi[tb] = 2 * nb[tb] + s;
                        int gc[3] = {fi[0], fi[1], fi[2]};
                        gc[d] += side ? -1 : 1;
                        a[s][p] = (uf[frb_at(B, fi[0], fi[1], fi[2])] - uf[frb_at(B, gc[0], gc[1], gc[2])]) / g.h1;
                    }
                v = ((a[0][0] + a[0][1]) + (a[1][0] + a[1][1])) * 0.25;
            } else if (nbd < g.dlo[d] || nbd >= g.dlo[d] + g.n[d]) {
                if (!g.per[d]) {
                    v = (-UI - UI) / g.h0;
                } else {
                    const long long w = (long long)(side ? -(g.n[d] - 1) : (g.n[d] - 1)) * st[d];
                    v = (Uc[c + w] - UI) / g.h0;
                }
            } else {
                v = (Uc[c + (side ? st[d] : -st[d])] - UI) / g.h0;
            }
            gr[2 * d + side] = v;
        }
    return (((gr[0] + gr[1]) + (gr[2] + gr[3])) + (gr[4] + gr[5])) / g.h0;
}

// Composite residual on the coarse level, common cells: covered cells take
// the mean of the fine residuals below them, uncovered interior cells with
// no covered neighbour f - (7-point operator) (norms taken there); the other
// uncovered cells (map entries below -1) are k_coarse_resid_special's.
// mode as for k_fine_resid (Rc written only with kStoreR).
__global__ void __launch_bounds__(kCB) k_coarse_resid(CGeo g, const int* __restrict__ cmap,
                                                      const double* __restrict__ Uc, const double* __restrict__ Fc,
                                                      double* __restrict__ Rc, const FRB* __restrict__ fb,
                                                      const double* __restrict__ rf, int mode,
                                                      double* __restrict__ partials) {
    const uint3 bk = xcd_block();
    const int t = bk.x * kCB + threadIdx.x;
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    if (t < g.n[0] * g.n[1]) {
        const int I = g.dlo[0] + t % g.n[0], J = g.dlo[1] + t / g.n[0];
        const int K0 = g.dlo[2] + bk.y * kKZ, K1 = min(K0 + kKZ - 1, g.dlo[2] + g.n[2] - 1);
        const long long sy = g.cb.G[0], sz = (long long)g.cb.G[0] * g.cb.G[1];
        for (int K = K0; K <= K1; ++K) {
            const int code = cmap[cq(g, I, J, K)];
            const long long c = fidx(g.cb, I, J, K);
            if (code >= 0) {
                if (mode == kStoreR) Rc[ridx(g, I, J, K)] = mean8(rf, fb[code], 2 * I, 2 * J, 2 * K);
                continue;
            }
            if (code != -1) continue;
            double rv = Fc[c];
            if (mode != kNormsF) {
                const double UI = Uc[c];
                const double uxm = Uc[c - 1], uxp = Uc[c + 1], uym = Uc[c - sy], uyp = Uc[c + sy];
                const double uzm = Uc[c - sz], uzp = Uc[c + sz];
                rv = rv - ((((uxm - UI) + (uxp - UI)) + ((uym - UI) + (uyp - UI))) + ((uzm - UI) + (uzp - UI))) *
                              g.ih0sq;
                if (mode == kStoreR) Rc[ridx(g, I, J, K)] = rv;
            }
            norm_add(rv, mx, s2, bad);
        }
    }
    block_norms(mx, s2, bad, partials + 3 * (long long)(bk.y * gridDim.x + bk.x));
}

// Composite residual at the listed uncovered cells that have a covered face
// neighbour or lie on a domain face (entry: I, J, K, map entry), norms
// taken there.
__global__ void __launch_bounds__(kCB) k_coarse_resid_special(CGeo g, const int4* __restrict__ list, int n,
                                                              const int* __restrict__ cmap,
                                                              const double* __restrict__ Uc,
                                                              const double* __restrict__ Fc, double* __restrict__ Rc,
                                                              const FRB* __restrict__ fb,
                                                              const double* __restrict__ uf, int mode,
                                                              double* __restrict__ partials) {
    const int q = blockIdx.x * kCB + threadIdx.x;
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    if (q < n) {
        const int4 e = list[q];
        const long long c = fidx(g.cb, e.x, e.y, e.z);
        double rv = Fc[c];
        if (mode != kNormsF) {
            rv = rv - coarse_op_special(g, cmap, Uc, fb, uf, e.x, e.y, e.z, (-1 - e.w) & 63);
            if (mode == kStoreR) Rc[ridx(g, e.x, e.y, e.z)] = rv;
        }
        norm_add(rv, mx, s2, bad);
    }
    block_norms(mx, s2, bad, partials + 3 * (long long)blockIdx.x);
}

// Uc += Ec at the uncovered coarse cells.
__global__ void __launch_bounds__(kCB) k_coarse_update(CGeo g, const int* __restrict__ cmap, double* __restrict__ Uc,
                                                       const double* __restrict__ Ec) {
    const uint3 bk = xcd_block();
    const int t = bk.x * kCB + threadIdx.x;
    if (t >= g.n[0] * g.n[1]) return;
    const int I = g.dlo[0] + t % g.n[0], J = g.dlo[1] + t / g.n[0];
    const int K0 = g.dlo[2] + bk.y * kKZ, K1 = min(K0 + kKZ - 1, g.dlo[2] + g.n[2] - 1);
    for (int K = K0; K <= K1; ++K) {
        if (cmap[cq(g, I, J, K)] >= 0) continue;
        const long long c = fidx(g.cb, I, J, K);
        Uc[c] = Uc[c] + Ec[ridx(g, I, J, K)];
    }
}

// Covered coarse cells := the mean of their 8 children; grid (plane blocks,
// plane groups, fine box) over each fine box's coarse cells.
__global__ void __launch_bounds__(kCB) k_coarse_sync(CGeo g, double* __restrict__ Uc, const FRB* __restrict__ fb,
                                                     const double* __restrict__ uf) {
    const uint3 bk = xcd_block();
    const FRB B = fb[bk.z];
    const int cx = (B.hi[0] - B.lo[0] + 1) >> 1, cy = (B.hi[1] - B.lo[1] + 1) >> 1, cz = (B.hi[2] - B.lo[2] + 1) >> 1;
    const int t = bk.x * kCB + threadIdx.x;
    if (t >= cx * cy) return;
    const int I = (B.lo[0] >> 1) + t % cx, J = (B.lo[1] >> 1) + t / cx;
    const int K0 = (B.lo[2] >> 1) + bk.y * kKZ, K1 = min(K0 + kKZ - 1, (B.lo[2] >> 1) + cz - 1);
    for (int K = K0; K <= K1; ++K) Uc[fidx(g.cb, I, J, K)] = mean8(uf, B, 2 * I, 2 * J, 2 * K);
}

// ------------------------------------------------------------------ host
static unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

struct Comp {
    bxmg_ctx ctx = nullptr;
    uint64_t cba_id = 0, fba_id = 0;
    double h0 = 0.0;
    bxmg_boxarray one = nullptr;                                           // one box over the coarse domain
    bxmg_multifab Uc = nullptr, Fc = nullptr;  // over `one`, 1 ghost
    // the correction's own multigrid hierarchy over the coarse domain: its
    // level-0 arrays are the residual (right-hand side) and the correction
    std::shared_ptr<Hier> hier;
    double *Rc = nullptr, *Ec = nullptr;
    int levels = 0;
    CGeo geo{};
    // the fine level in colour-split storage: solution, right-hand side,
    // residual (one layout), its boxes, and the caller box -> storage box map
    DevBuf<double> uf, ff, rf;
    DevBuf<FRB> frb;
    DevBuf<int> fmap;
    DevBuf<GhostCopy> fx;  // ghosts between fine boxes, colour-0 ghosts first
    long long nfx = 0, nfx0 = 0;
    long long fslab = 0;  // elements per fine field
    DevBuf<int> cmap;
    DevBuf<int4> ghosts;  // coarse-fine ghosts, colour-0 ghosts first
    int nghosts = 0, nghosts0 = 0;
    DevBuf<int4> special;  // uncovered coarse cells next to a covered one or on a domain face
    int nspecial = 0;
    int nfine = 0;
    dim3 g_fine, g_fine_s, g_sync, g_coarse, g_conv;  // launch grids
    int nparts_fine = 0, nparts = 0;
    DevBuf<double> part, fn;
    double* h_norm = nullptr;  // pinned: the norms read back
    ~Comp() {
        for (bxmg_multifab m : {Uc, Fc})
            if (m) bxmg_multifab_release(m);
        if (hier) {
            (void)hipStreamSynchronize(ctx ? ctx->stream : nullptr);
            hier.reset();
        }
        if (one) bxmg_boxarray_release(one);
        const hipStream_t s = ctx ? ctx->stream : nullptr;
        for (DevBuf<double>* b : {&uf, &ff, &rf, &part, &fn}) b->release_async(s);
        frb.release_async(s);
        fmap.release_async(s);
        fx.release_async(s);
        cmap.release_async(s);
        ghosts.release_async(s);
        special.release_async(s);
        if (h_norm) {
            (void)hipStreamSynchronize(s);
            (void)hipHostFree(h_norm);
        }
    }
};

// Checks the fine layout against the coarse domain: the fine domain is the
// coarse one refined by 2 with the same boundaries, every fine box is a union
// of whole coarse cells and lies 2 coarse cells (4 fine) inside every domain
// face; index arithmetic stays in 32 bits (ghost copies address a fine field
// with 31-bit offsets).  Returns "" or the reason.
static std::string layout_error(const bxmg_ba_s* cba, const bxmg_ba_s* fba) {
    for (int d = 0; d < 3; ++d) {
        if (fba->dom.lo[d] != 2 * cba->dom.lo[d] || fba->dom.hi[d] != 2 * cba->dom.hi[d] + 1)
            return "the fine domain must be the coarse domain refined by 2";
        if (fba->per[d] != cba->per[d]) return "the fine and coarse boundaries differ";
    }
    const Box& D = cba->dom;
    if ((long long)(D.n(0) + 2) * (D.n(1) + 2) * (D.n(2) + 2) >= (1LL << 31)) return "coarse domain too large";
    if (fba->boxes.size() >= (1u << 24)) return "too many fine boxes";
    long long total = 0;
    for (const Box& B : fba->boxes) {
        for (int d = 0; d < 3; ++d) {
            if ((B.lo[d] & 1) || !(B.hi[d] & 1)) return "fine boxes must be unions of whole coarse cells";
            if (B.lo[d] < fba->dom.lo[d] + 4 || B.hi[d] > fba->dom.hi[d] - 4)
                return "fine boxes must lie 2 coarse cells inside the domain";
        }
        total += (long long)(B.n(0) + 3) * (B.n(1) + 2) * (B.n(2) + 2) + 128;
    }
    if (total >= (1LL << 31) - 1) return "fine level too large";
    return "";
}

static bxmg_multifab alloc_mf(bxmg_ctx ctx, bxmg_boxarray ba, int ng) {
    bxmg_multifab m = nullptr;
    if (bxmg_alloc_multifab(ctx, ba, 1, ng, BXMG_F64, nullptr, &m) != BXMG_OK) throw std::runtime_error(bxmg_last_error());
    return m;
}

static std::unique_ptr<Comp> build(bxmg_ctx ctx, const bxmg_ba_s* cba, const bxmg_ba_s* fba, double h0) {
    auto c = std::make_unique<Comp>();
    c->ctx = ctx;
    c->cba_id = cba->id;
    c->fba_id = fba->id;
    c->h0 = h0;
    const Box& D = cba->dom;
    const int lohi[6] = {D.lo[0], D.lo[1], D.lo[2], D.hi[0], D.hi[1], D.hi[2]};
    if (bxmg_define_boxarray_list(D.lo, D.hi, cba->bc, 1, lohi, &c->one) != BXMG_OK)
        throw std::runtime_error(bxmg_last_error());
    c->Uc = alloc_mf(ctx, c->one, 1);
    c->Fc = alloc_mf(ctx, c->one, 1);
    c->hier = hier_create(ctx, c->one, h0);
    RBox rb;
    hier_level0(c->hier.get(), &c->Ec, &c->Rc, &rb, &c->levels);
    CGeo& g = c->geo;
    for (int d = 0; d < 3; ++d) {
        g.rlo[d] = rb.lo[d];
        g.rglo[d] = rb.glo[d];
        g.rG[d] = rb.G[d];
    }
    g.rH = rb.H;
    g.rbase = rb.base;
    g.rcs = rb.cstride;
    g.cb = c->Uc->fboxes[0];
    for (int d = 0; d < 3; ++d) {
        g.dlo[d] = D.lo[d];
        g.n[d] = D.n(d);
        g.per[d] = cba->per[d];
    }
    g.h0 = h0;
    g.h1 = h0 * 0.5;
    g.ih0sq = 1.0 / (h0 * h0);
    // the fine boxes the kernels run over: one merged box when the caller's
    // boxes tile a rectangle (they are disjoint, so equal cell counts mean
    // they tile it), else the caller's boxes
    Box U = fba->boxes[0];
    long long fcells = 0;
    for (const Box& B : fba->boxes) {
        fcells += B.cells();
        for (int d = 0; d < 3; ++d) {
            U.lo[d] = std::min(U.lo[d], B.lo[d]);
            U.hi[d] = std::max(U.hi[d], B.hi[d]);
        }
    }
    const bool merged = fcells == U.cells();
    const std::vector<Box> fb = merged ? std::vector<Box>{U} : fba->boxes;
    std::vector<int> fmap(fba->boxes.size());
    for (size_t b = 0; b < fmap.size(); ++b) fmap[b] = merged ? 0 : (int)b;
    // colour-split storage of the fine boxes
    std::vector<FRB> frb;
    long long off = 0;
    for (const Box& B : fb) {
        FRB r{};
        for (int d = 0; d < 3; ++d) {
            r.lo[d] = B.lo[d];
            r.hi[d] = B.hi[d];
            r.glo[d] = B.lo[d] - 1;
            r.G[d] = B.n(d) + 2;
        }
        r.H = (r.G[0] + 1) / 2;
        r.cs = ((long long)r.H * r.G[1] * r.G[2] + 63) / 64 * 64;
        r.base = off;
        off += 2 * r.cs;
        frb.push_back(r);
    }
    c->fslab = off;
    c->nfine = (int)fb.size();
    // coverage map: covering fine box, or -1 - (mask of covered face neighbours)
    const long long nc = D.cells();
    std::vector<int> cmap((size_t)nc, -1);
    auto cidx = [&](int I, int J, int K) {
        return (size_t)(I - D.lo[0]) + (size_t)D.n(0) * ((size_t)(J - D.lo[1]) + (size_t)D.n(1) * (K - D.lo[2]));
    };
    int maxS = 1, maxnz = 1, maxPc = 1, maxnzc = 1;
    for (size_t b = 0; b < fb.size(); ++b) {
        const Box& B = fb[b];
        maxS = std::max(maxS, (((B.hi[0] - (B.lo[0] - 1)) >> 1) + 1) * B.n(1));
        maxnz = std::max(maxnz, B.n(2));
        maxPc = std::max(maxPc, (B.n(0) / 2) * (B.n(1) / 2));
        maxnzc = std::max(maxnzc, B.n(2) / 2);
        for (int K = B.lo[2] >> 1; K <= B.hi[2] >> 1; ++K)
            for (int J = B.lo[1] >> 1; J <= B.hi[1] >> 1; ++J)
                for (int I = B.lo[0] >> 1; I <= B.hi[0] >> 1; ++I) cmap[cidx(I, J, K)] = (int)b;
    }
    for (const Box& B : fb)
        for (int K = B.lo[2] >> 1; K <= B.hi[2] >> 1; ++K)
            for (int J = B.lo[1] >> 1; J <= B.hi[1] >> 1; ++J)
                for (int I = B.lo[0] >> 1; I <= B.hi[0] >> 1; ++I)
                    for (int d = 0; d < 3; ++d)
                        for (int side = 0; side < 2; ++side) {
                            // the neighbour across (d, side) of this covered cell sees it across (d, 1 - side)
                            int x[3] = {I, J, K};
                            x[d] += side ? 1 : -1;
                            int& m = cmap[cidx(x[0], x[1], x[2])];
                            if (m >= 0) continue;
                            const int mask = (-1 - m) | (1 << (2 * d + (1 - side)));
                            m = -1 - mask;
                        }
    // uncovered cells on a domain face are special too (bit 6 of the mask)
    std::vector<int4> sl;
    for (int K = D.lo[2]; K <= D.hi[2]; ++K)
        for (int J = D.lo[1]; J <= D.hi[1]; ++J)
            for (int I = D.lo[0]; I <= D.hi[0]; ++I) {
                int& m = cmap[cidx(I, J, K)];
                if (m >= 0) continue;
                const bool face = I == D.lo[0] || I == D.hi[0] || J == D.lo[1] || J == D.hi[1] || K == D.lo[2] ||
                                  K == D.hi[2];
                if (face) m = -1 - ((-1 - m) | 64);
                if (m != -1) sl.push_back(make_int4(I, J, K, m));
            }
    if (sl.size() >= (size_t)(1u << 31) - kCB) throw std::runtime_error("too many special coarse cells");
    c->nspecial = (int)sl.size();
    // face ghosts of each fine box: copies from the fine box that owns the
    // cell, or coarse-fine ghosts (their coarse cell is not covered)
    std::vector<int4> gl;
    std::vector<GhostCopy> fx[2];  // by the colour of the ghost
    for (size_t b = 0; b < fb.size(); ++b) {
        const Box& B = fb[b];
        for (int d = 0; d < 3; ++d)
            for (int side = 0; side < 2; ++side) {
                const int ta = d == 2 ? 0 : d + 1, tb = d == 0 ? 2 : d - 1;
                for (int y = B.lo[tb]; y <= B.hi[tb]; ++y)
                    for (int x = B.lo[ta]; x <= B.hi[ta]; ++x) {
                        int gx[3];
                        gx[d] = side ? B.hi[d] + 1 : B.lo[d] - 1;
                        gx[ta] = x;
                        gx[tb] = y;
                        const int o = cmap[cidx(gx[0] >> 1, gx[1] >> 1, gx[2] >> 1)];
                        if (o < 0) {
                            gl.push_back(make_int4((int)b | (d << 24) | (side << 26), gx[0], gx[1], gx[2]));
                        } else {
                            GhostCopy p;
                            p.dst = (uint32_t)frb_at(frb[b], gx[0], gx[1], gx[2]);
                            p.src = (uint32_t)frb_at(frb[o], gx[0], gx[1], gx[2]);
                            fx[(gx[0] + gx[1] + gx[2]) & 1].push_back(p);
                        }
                    }
            }
    }
    if (gl.size() >= (size_t)(1u << 31) - kCB) throw std::runtime_error("too many coarse-fine ghost cells");
    // colour 0 first: a sweep of colour c reads only the ghosts of colour 1 - c
    std::stable_partition(gl.begin(), gl.end(), [](const int4& e) { return ((e.y + e.z + e.w) & 1) == 0; });
    c->nghosts0 = (int)std::count_if(gl.begin(), gl.end(), [](const int4& e) { return ((e.y + e.z + e.w) & 1) == 0; });
    c->nfx0 = (long long)fx[0].size();
    fx[0].insert(fx[0].end(), fx[1].begin(), fx[1].end());
    c->nghosts = (int)gl.size();
    c->nfx = (long long)fx[0].size();
    const unsigned nf = (unsigned)c->nfine;
    c->g_fine = dim3(cdiv(maxS, kCB), cdiv(maxnz, kKZ), nf);
    c->g_fine_s = dim3(cdiv(maxS, kCB), cdiv(maxnz, kKZs), nf);
    c->g_sync = dim3(cdiv(maxPc, kCB), cdiv(maxnzc, kKZ), nf);
    c->g_coarse = dim3(cdiv((long long)g.n[0] * g.n[1], kCB), cdiv(g.n[2], kKZ), 1);
    int maxP = 1, maxz = 1;
    for (const Box& B : fba->boxes) {
        maxP = std::max(maxP, B.n(0) * B.n(1));
        maxz = std::max(maxz, B.n(2));
    }
    c->g_conv = dim3(cdiv(maxP, kCB), cdiv(maxz, kKZ), (unsigned)fba->boxes.size());
    c->nparts_fine = (int)(c->g_fine.x * c->g_fine.y * c->g_fine.z);
    c->nparts = c->nparts_fine + (int)(c->g_coarse.x * c->g_coarse.y) + (int)cdiv(c->nspecial, kCB);
    const hipStream_t s = ctx->stream;
    for (DevBuf<double>* b : {&c->uf, &c->ff, &c->rf}) {
        HIPCHK(hipMallocAsync((void**)&b->p, (size_t)c->fslab * sizeof(double), s));
        b->n = (size_t)c->fslab;
        HIPCHK(hipMemsetAsync(b->p, 0, (size_t)c->fslab * sizeof(double), s));
    }
    c->frb.upload_async(frb, s);
    c->fmap.upload_async(fmap, s);
    c->fx.upload_async(fx[0], s);
    c->cmap.upload_async(cmap, s);
    c->special.upload_async(sl, s);
    c->ghosts.upload_async(gl, s);
    c->part.upload_async(std::vector<double>((size_t)3 * c->nparts, 0.0), s);
    c->fn.upload_async(std::vector<double>(3, 0.0), s);
    HIPCHK(hipHostMalloc((void**)&c->h_norm, 4 * sizeof(double)));
    return c;
}

struct Cache {
    std::unique_ptr<Comp> comp;  // the last layout used
};

}  // namespace comp
}  // namespace bxmg

using namespace bxmg;

extern "C" bxmg_status bxmg_composite_solve(bxmg_ctx ctx, const bxmg_solve_params* params, bxmg_multifab phi_c,
                                            bxmg_multifab rhs_c, bxmg_multifab phi_f, bxmg_multifab rhs_f,
                                            bxmg_solve_info* info) {
    if (!ctx || !phi_c || !rhs_c || !phi_f || !rhs_f || !info) return fail(BXMG_EINVAL, "composite_solve: NULL argument");
    std::memset(info, 0, sizeof(*info));
    bxmg_solve_params P;
    if (params) P = *params;
    else bxmg_solve_params_default(&P);
    auto bad = [&](const std::string& m) {
        info->status = fail(BXMG_EINVAL, "composite_solve: " + m);
        return (bxmg_status)info->status;
    };
    if (P.nu1 < 0 || P.nu2 < 0 || P.max_cycles < 0 || P.precision != 0 || P.krylov != 0 || P.alpha != 0.0 ||
        P.prolong != 2)
        return bad("FP64 V-cycles of the Poisson operator with trilinear prolongation only "
                   "(precision 0, krylov 0, alpha 0, prolong 2)");
    for (bxmg_multifab m : {phi_c, rhs_c, phi_f, rhs_f})
        if (m->dtype != BXMG_F64) return bad("every field must be FP64");
    for (bxmg_multifab m : {phi_c, rhs_c, phi_f, rhs_f})
        if (m->ctx->device != ctx->device) return bad("fields on another device");
    const bxmg_ba_s* cba = phi_c->ba;
    const bxmg_ba_s* fba = phi_f->ba;
    if (check_field_mf(rhs_c, cba, "coarse rhs") != BXMG_OK || check_field_mf(rhs_f, fba, "fine rhs") != BXMG_OK)
        return (bxmg_status)(info->status = BXMG_EINVAL);
    if (!covers_domain(cba)) return bad("the coarse BoxArray must cover its domain");
    const std::string le = comp::layout_error(cba, fba);
    if (!le.empty()) return bad(le);
    const double h0 = (P.dx > 0) ? P.dx : 1.0 / cba->dom.n(0);
    // cached state on the context; composite solves on one context run one at a time
    std::lock_guard<std::mutex> lock(ctx->comp_mu);
    const auto t0 = std::chrono::steady_clock::now();
    try {
        HIPCHK(hipSetDevice(ctx->device));
        if (!ctx->composite) ctx->composite = std::make_shared<comp::Cache>();
        auto* cache = (comp::Cache*)ctx->composite.get();
        if (!cache->comp || cache->comp->cba_id != cba->id || cache->comp->fba_id != fba->id || cache->comp->h0 != h0) {
            cache->comp.reset();
            cache->comp = comp::build(ctx, cba, fba, h0);
        }
        comp::Comp& c = *cache->comp;
        const hipStream_t s = ctx->stream;
        const comp::CGeo& g = c.geo;
        double* Uc = (double*)c.Uc->data;
        double* Fc = (double*)c.Fc->data;
        double* Rc = c.Rc;
        double* Ec = c.Ec;
        double* uf = c.uf.p;
        double* ff = c.ff.p;
        double* rf = c.rf.p;
        const comp::FRB* fb = c.frb.p;
        double* const part_c = c.part.p + 3 * (size_t)c.nparts_fine;
        double* const part_s = part_c + 3 * (size_t)(c.g_coarse.x * c.g_coarse.y);
        const dim3 B(comp::kCB);
        auto chk = [](bxmg_status st) {
            if (st != BXMG_OK) throw std::runtime_error(bxmg_last_error());
        };
        // load: the coarse rhs into the one-box field, the fine rhs into the
        // colour-split storage; zero start on both levels
        chk(bxmg_parallel_copy(c.Fc, 0, rhs_c, 0, 1, 0, s));
        hipLaunchKernelGGL(comp::k_fab_frb<true>, c.g_conv, B, 0, s, rhs_f->d_fboxes.p, (double*)rhs_f->data, fb,
                           (const int*)c.fmap.p, ff);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemsetAsync(Uc, 0, c.Uc->bytes, s));
        HIPCHK(hipMemsetAsync(uf, 0, (size_t)c.fslab * sizeof(double), s));
        // ghosts of the fine level from the current state: all of them
        // (colours < 0), or those of the given colour only
        auto fill_fine = [&](int colour) {
            const long long x0 = colour == 1 ? c.nfx0 : 0, x1 = colour == 0 ? c.nfx0 : c.nfx;
            const int g0 = colour == 1 ? c.nghosts0 : 0, g1 = colour == 0 ? c.nghosts0 : c.nghosts;
            if (x1 > x0) HIPCHK(launch_fill_rb(s, uf, false, c.fx.p + x0, x1 - x0));
            if (g1 > g0)
                hipLaunchKernelGGL(comp::k_cf_ghost, dim3(comp::cdiv(g1 - g0, comp::kCB)), B, 0, s, c.ghosts.p + g0,
                                   g1 - g0, g, (const double*)Uc, fb, uf);
            HIPCHK(hipGetLastError());
        };
        // composite residual norms read back (mode: of f, of the residual, or
        // with the residual stored into rf / Rc)
        auto residual = [&](int mode, double* out) {
            if (mode != comp::kNormsF) fill_fine(-1);
            hipLaunchKernelGGL(comp::k_fine_resid, c.g_fine, B, 0, s, g, fb, (const double*)uf, (const double*)ff, rf,
                               mode, c.part.p);
            hipLaunchKernelGGL(comp::k_coarse_resid, c.g_coarse, B, 0, s, g, (const int*)c.cmap.p, (const double*)Uc,
                               (const double*)Fc, Rc, fb, (const double*)rf, mode, part_c);
            if (c.nspecial)
                hipLaunchKernelGGL(comp::k_coarse_resid_special, dim3(comp::cdiv(c.nspecial, comp::kCB)), B, 0, s, g,
                                   c.special.p, c.nspecial, (const int*)c.cmap.p, (const double*)Uc,
                                   (const double*)Fc, Rc, fb, (const double*)uf, mode, part_s);
            HIPCHK(hipGetLastError());
            if (!out) return;  // the residual is wanted, not its norms: no wait for the device
            HIPCHK(launch_norm_final(s, c.part.p, c.nparts, c.fn.p));
            HIPCHK(hipMemcpyAsync(c.h_norm, c.fn.p, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            out[0] = c.h_norm[2] > 0.0 ? (double)NAN : c.h_norm[0];
            out[1] = c.h_norm[1];
            out[2] = c.h_norm[2];
        };
        auto sweeps = [&](int n) {
            for (int q = 0; q < n; ++q)
                for (int col = 0; col < 2; ++col) {
                    fill_fine(1 - col);  // the sweep of colour col reads ghosts of the other colour
                    hipLaunchKernelGGL(comp::k_fine_gs, c.g_fine_s, B, 0, s, g, fb, uf, (const double*)ff, col);
                    HIPCHK(hipGetLastError());
                }
        };
        bxmg_solve_params Pc = P;
        Pc.fixed_cycles = 1;
        Pc.dx = h0;
        auto cycle = [&]() {
            sweeps(P.nu1);
            residual(comp::kStoreR, nullptr);  // the correction's right-hand side
            // coarse correction: one V-cycle from zero on the composite residual
            hier_vcycle_from_zero(ctx, c.hier.get(), Pc);
            info->levels = c.levels + 1;
            hipLaunchKernelGGL(comp::k_coarse_update, c.g_coarse, B, 0, s, g, (const int*)c.cmap.p, Uc,
                               (const double*)Ec);
            hipLaunchKernelGGL(comp::k_fine_prolong, c.g_fine_s, B, 0, s, g, fb, uf, (const double*)Ec);
            HIPCHK(hipGetLastError());
            sweeps(P.nu2);
            hipLaunchKernelGGL(comp::k_coarse_sync, c.g_sync, B, 0, s, g, Uc, fb, (const double*)uf);
            HIPCHK(hipGetLastError());
        };
        double fz[3];
        residual(comp::kNormsF, fz);
        const double fnorm = fz[0];
        info->f_inf = fnorm;
        int status = 0, cyc = 0;
        if (!(fnorm == fnorm)) {
            status = BXMG_ENONFINITE;
        } else if (fnorm > 0.0) {
            for (;; ++cyc) {
                double rn[3];
                residual(comp::kNormsR, rn);  // the stop test needs the norms only
                if (cyc < kHist) {
                    info->hist[cyc] = rn[0] / fnorm;
                    info->hist_l2[cyc] = std::sqrt(rn[1]);
                    info->nhist = cyc + 1;
                }
                info->rel_resid_inf = rn[0] / fnorm;
                info->resid_l2 = std::sqrt(rn[1]);
                if (!(rn[0] == rn[0])) { status = BXMG_ENONFINITE; break; }
                if (P.fixed_cycles > 0) {
                    if (cyc == P.fixed_cycles) break;
                } else {
                    if (rn[0] <= P.rel_tol * fnorm || rn[0] <= P.abs_tol) break;
                    if (cyc == P.max_cycles) { status = BXMG_ENOCONV; break; }
                }
                cycle();
            }
        }
        info->cycles = cyc;
        // the solutions back: coarse (covered cells: the mean of their
        // children) and the fine valid cells
        chk(bxmg_parallel_copy(phi_c, 0, c.Uc, 0, 1, 0, s));
        hipLaunchKernelGGL(comp::k_fab_frb<false>, c.g_conv, B, 0, s, phi_f->d_fboxes.p, (double*)phi_f->data, fb,
                           (const int*)c.fmap.p, uf);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
        info->status = status;
        if (status == BXMG_ENOCONV) fail(BXMG_ENOCONV, "composite_solve: max_cycles reached");
        if (status == BXMG_ENONFINITE) fail(BXMG_ENONFINITE, "composite_solve: non-finite values");
    } catch (HipError& e) {
        info->status = fail(BXMG_EDEVICE, std::string("composite_solve: ") + e.where + ": " + hipGetErrorString(e.e));
    } catch (std::exception& e) {
        info->status = fail(BXMG_EINVAL, std::string("composite_solve: ") + e.what());
    }
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return (bxmg_status)info->status;
}
