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
//    boxes by FillBoundary).
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
// neighbours).  The fine level is the caller's MultiFabs, or, when the fine
// boxes tile one rectangle, one merged box (ParallelCopy in and out) with no
// ghosts between boxes; the coarse-fine ghost cells are listed once per
// layout.
// Fine boxes must be unions of whole coarse cells (even lower, odd upper
// corners) and lie at least 2 coarse cells inside the domain, so that every
// coarse cell a ghost or an interpolation reads is a domain cell.
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
struct CGeo {
    FBox cb;           // every coarse field has this layout (one box, 1 ghost)
    int dlo[3], n[3];  // coarse domain
    int per[3];
    double h0, h1;
    double ih0sq;  // 1 / h0^2
};

// Coverage map entry of a coarse cell: >= 0 the fine box covering it;
// otherwise -1 - mask, bit 2 d + side of mask set when the face neighbour
// across (d, side) is covered.
__device__ __forceinline__ int cq(const CGeo& g, int I, int J, int K) {
    return (I - g.dlo[0]) + g.n[0] * ((J - g.dlo[1]) + g.n[1] * (K - g.dlo[2]));
}

__device__ __forceinline__ long long fidx(const FBox& b, int i, int j, int k) {
    return b.base + (long long)((i - b.glo[0]) + b.G[0] * ((j - b.glo[1]) + b.G[1] * (k - b.glo[2])));
}

// Block coordinates with consecutive logical blocks on one XCD: blocks are
// dispatched round-robin over the 8 XCDs (block p to XCD p % 8), so logical
// block (p % 8) * (N / 8) + p / 8 gives each XCD one contiguous eighth of the
// grid (x fastest, then y, then z), and its L2 serves the neighbouring rows
// and planes its stencils read.
__device__ __forceinline__ uint3 xcd_block() {
    const unsigned gx = gridDim.x, gy = gridDim.y, N = gx * gy * gridDim.z;
    const unsigned p = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned L = (N & 7) ? p : (p & 7) * (N >> 3) + (p >> 3);
    const unsigned r = L / gx;
    return make_uint3(L - r * gx, r % gy, r / gy);
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

__device__ __forceinline__ double mean8(const double* __restrict__ x, const FBox& B, int i, int j, int k) {
    const long long c = fidx(B, i, j, k), sy = B.G[0], sz = (long long)B.G[0] * B.G[1];
    return (((x[c] + x[c + 1]) + (x[c + sy] + x[c + sy + 1])) +
            ((x[c + sz] + x[c + sz + 1]) + (x[c + sz + sy] + x[c + sz + sy + 1]))) * 0.125;
}

// Coarse-fine ghosts.  One entry per ghost cell: x = box | d << 24 | side << 26
// (the ghost lies beyond face (d, side) of its box), y, z, w = its fine index.
__global__ void __launch_bounds__(kCB) k_cf_ghost(const int4* __restrict__ list, int n, CGeo g,
                                                  const double* __restrict__ Uc, const FBox* __restrict__ fu,
                                                  double* __restrict__ uf) {
    const int q = blockIdx.x * kCB + threadIdx.x;
    if (q >= n) return;
    const int4 r = list[q];
    const int b = r.x & 0xffffff, d = (r.x >> 24) & 3, side = (r.x >> 26) & 1;
    const int gx[3] = {r.y, r.z, r.w};
    const FBox B = fu[b];
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
    const double u1 = uf[fidx(B, i1[0], i1[1], i1[2])], u2 = uf[fidx(B, i2[0], i2[1], i2[2])];
    uf[fidx(B, gx[0], gx[1], gx[2])] = ((8.0 / 15.0) * Ut + (2.0 / 3.0) * u1) - (1.0 / 5.0) * u2;
}

// Fine-box kernels: grid (plane blocks, plane groups of kKZ, box); a thread
// takes one (i, j) of its box's planes (or half-row position, for the
// sweeps) and walks kKZ planes.

// One colour of red-black Gauss-Seidel on the fine boxes (ghosts current):
// u = (sum of the 6 neighbours - h1^2 f) / 6 at the cells of that colour.
__global__ void __launch_bounds__(kCB) k_fine_gs(CGeo g, const FBox* __restrict__ fu, const FBox* __restrict__ ff,
                                                 double* __restrict__ u, const double* __restrict__ f, int colour) {
    const uint3 bk = xcd_block();
    const FBox B = fu[bk.z], F = ff[bk.z];
    const int nx = B.hi[0] - B.lo[0] + 1, ny = B.hi[1] - B.lo[1] + 1;
    const int nxh = (nx + 1) >> 1;
    const int t = bk.x * kCB + threadIdx.x;
    if (t >= nxh * ny) return;
    const int tx = t % nxh, j = B.lo[1] + t / nxh;
    const int k0 = B.lo[2] + bk.y * kKZs, k1 = min(k0 + kKZs - 1, B.hi[2]);
    const long long sy = B.G[0], sz = (long long)B.G[0] * B.G[1];
    const double h2 = g.h1 * g.h1;
    for (int k = k0; k <= k1; ++k) {
        const int i = B.lo[0] + 2 * tx + ((B.lo[0] + j + k + colour) & 1);
        if (i > B.hi[0]) continue;
        const long long c = fidx(B, i, j, k);
        const double su = ((u[c - 1] + u[c + 1]) + (u[c - sy] + u[c + sy])) + (u[c - sz] + u[c + sz]);
        u[c] = (su - h2 * f[fidx(F, i, j, k)]) / 6.0;
    }
}

// Fine residual r = f - L u on the valid cells (or the norms of f only),
// with per-block norms (max, sum of squares, non-finite count).
__global__ void __launch_bounds__(kCB) k_fine_resid(CGeo g, const FBox* __restrict__ fu, const FBox* __restrict__ ff,
                                                    const FBox* __restrict__ fr, const double* __restrict__ u,
                                                    const double* __restrict__ f, double* __restrict__ r, int fonly,
                                                    double* __restrict__ partials) {
    const uint3 bk = xcd_block();
    const FBox B = fu[bk.z], F = ff[bk.z], R = fr[bk.z];
    const int nx = B.hi[0] - B.lo[0] + 1, ny = B.hi[1] - B.lo[1] + 1;
    const int t = bk.x * kCB + threadIdx.x;
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    if (t < nx * ny) {
        const int i = B.lo[0] + t % nx, j = B.lo[1] + t / nx;
        const int k0 = B.lo[2] + bk.y * kKZ, k1 = min(k0 + kKZ - 1, B.hi[2]);
        const long long sy = B.G[0], sz = (long long)B.G[0] * B.G[1];
        const double ih2 = 1.0 / (g.h1 * g.h1);
        for (int k = k0; k <= k1; ++k) {
            double rv = f[fidx(F, i, j, k)];
            if (!fonly) {
                const long long c = fidx(B, i, j, k);
                const double su = ((u[c - 1] + u[c + 1]) + (u[c - sy] + u[c + sy])) + (u[c - sz] + u[c + sz]);
                rv = rv - (su - 6.0 * u[c]) * ih2;
                r[fidx(R, i, j, k)] = rv;
            }
            norm_add(rv, mx, s2, bad);
        }
    }
    const int blk = (bk.z * gridDim.y + bk.y) * gridDim.x + bk.x;
    block_norms(mx, s2, bad, partials + 3 * (long long)blk);
}

// Fine cells += trilinear interpolation of the coarse correction Ec.
__global__ void __launch_bounds__(kCB) k_fine_prolong(CGeo g, const FBox* __restrict__ fu, double* __restrict__ u,
                                                      const double* __restrict__ Ec) {
    const uint3 bk = xcd_block();
    const FBox B = fu[bk.z];
    const int nx = B.hi[0] - B.lo[0] + 1, ny = B.hi[1] - B.lo[1] + 1;
    const int t = bk.x * kCB + threadIdx.x;
    if (t >= nx * ny) return;
    const int i = B.lo[0] + t % nx, j = B.lo[1] + t / nx;
    const int k0 = B.lo[2] + bk.y * kKZs, k1 = min(k0 + kKZs - 1, B.hi[2]);
    const int I = i >> 1, J = j >> 1;
    const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1;
    const long long sy = g.cb.G[0], sz = (long long)g.cb.G[0] * g.cb.G[1];
    for (int k = k0; k <= k1; ++k) {
        const int K = k >> 1, sk = (k & 1) ? 1 : -1;
        const long long e = fidx(g.cb, I, J, K), ex = si, ey = sj * sy, ez = sk * sz;
        const double c000 = Ec[e], c100 = Ec[e + ex], c010 = Ec[e + ey], c001 = Ec[e + ez];
        const double c110 = Ec[e + ex + ey], c101 = Ec[e + ex + ez], c011 = Ec[e + ey + ez];
        const double c111 = Ec[e + ex + ey + ez];
        const double v = (((27.0 * c000 + 9.0 * ((c100 + c010) + c001)) + 3.0 * ((c110 + c101) + c011)) + c111) *
                         (1.0 / 64.0);
        const long long c = fidx(B, i, j, k);
        u[c] = u[c] + v;
    }
}

// Component 0 of every fine box, valid and ghost cells, := 0.
__global__ void __launch_bounds__(kCB) k_fine_zero(const FBox* __restrict__ fu, double* __restrict__ u) {
    const uint3 bk = xcd_block();
    const FBox B = fu[bk.z];
    const int P = B.G[0] * B.G[1];
    const int t = bk.x * kCB + threadIdx.x;
    if (t >= P) return;
    for (int k = bk.y * kKZ; k < min(bk.y * kKZ + kKZ, B.G[2]); ++k) u[B.base + (long long)k * P + t] = 0.0;
}

// Coarse kernels: grid (plane blocks, plane groups of kKZ) over the domain.

// Composite residual on the coarse level: uncovered cells f - Lc u (norms
// taken there), covered cells the mean of the fine residuals below them
// (fonly: the norms of f at the uncovered cells, Rc untouched).  The fine
// ghosts of the current state must be in place (the flux-matched faces
// read them).
__global__ void __launch_bounds__(kCB) k_coarse_resid(CGeo g, const int* __restrict__ cmap,
                                                      const double* __restrict__ Uc, const double* __restrict__ Fc,
                                                      double* __restrict__ Rc, const FBox* __restrict__ fu,
                                                      const double* __restrict__ uf, const FBox* __restrict__ fr,
                                                      const double* __restrict__ rf, int fonly,
                                                      double* __restrict__ partials) {
    const uint3 bk = xcd_block();
    const int t = bk.x * kCB + threadIdx.x;
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    if (t < g.n[0] * g.n[1]) {
        const int I = g.dlo[0] + t % g.n[0], J = g.dlo[1] + t / g.n[0];
        const int K0 = g.dlo[2] + bk.y * kKZ, K1 = min(K0 + kKZ - 1, g.dlo[2] + g.n[2] - 1);
        const long long st[3] = {1, g.cb.G[0], (long long)g.cb.G[0] * g.cb.G[1]};
        const int mst[3] = {1, g.n[0], g.n[0] * g.n[1]};
        for (int K = K0; K <= K1; ++K) {
            const int q = cq(g, I, J, K);
            const long long c = fidx(g.cb, I, J, K);
            // every load of the common case issued before the first branch
            // (the ghost layer keeps the neighbour loads of boundary cells in
            // bounds)
            const int code = cmap[q];
            double rv = Fc[c];
            const double UI = Uc[c];
            const double uxm = Uc[c - 1], uxp = Uc[c + 1], uym = Uc[c - st[1]], uyp = Uc[c + st[1]];
            const double uzm = Uc[c - st[2]], uzp = Uc[c + st[2]];
            if (code >= 0) {
                if (!fonly) Rc[c] = mean8(rf, fr[code], 2 * I, 2 * J, 2 * K);
                continue;
            }
            const bool inner = code == -1 && I > g.dlo[0] && I < g.dlo[0] + g.n[0] - 1 && J > g.dlo[1] &&
                               J < g.dlo[1] + g.n[1] - 1 && K > g.dlo[2] && K < g.dlo[2] + g.n[2] - 1;
            if (!fonly && inner) {
                // no covered neighbour, no domain face: the 7-point operator
                rv = rv - ((((uxm - UI) + (uxp - UI)) + ((uym - UI) + (uyp - UI))) + ((uzm - UI) + (uzp - UI))) *
                              g.ih0sq;
                Rc[c] = rv;
            } else if (!fonly) {
                const int mask = -1 - code;
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
                            const FBox B = fu[cmap[q + (side ? mst[d] : -mst[d])]];
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
                                    const long long o = fidx(B, fi[0], fi[1], fi[2]);
                                    const long long gs = side ? -1 : 1;
                                    const long long step = d == 0 ? gs : (d == 1 ? gs * B.G[0] : gs * B.G[0] * B.G[1]);
                                    a[s][p] = (uf[o] - uf[o + step]) / g.h1;
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
                rv = rv - (((gr[0] + gr[1]) + (gr[2] + gr[3])) + (gr[4] + gr[5])) / g.h0;
                Rc[c] = rv;
            }
            norm_add(rv, mx, s2, bad);
        }
    }
    block_norms(mx, s2, bad, partials + 3 * (long long)(bk.y * gridDim.x + bk.x));
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
        Uc[c] = Uc[c] + Ec[c];
    }
}

// Covered coarse cells := the mean of their 8 children; grid (plane blocks,
// plane groups, fine box) over each fine box's coarse cells.
__global__ void __launch_bounds__(kCB) k_coarse_sync(CGeo g, double* __restrict__ Uc, const FBox* __restrict__ fu,
                                                     const double* __restrict__ uf) {
    const uint3 bk = xcd_block();
    const FBox B = fu[bk.z];
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
    bxmg_multifab Uc = nullptr, Fc = nullptr, Rc = nullptr, Ec = nullptr;  // over `one`, 1 ghost
    bxmg_multifab Rf = nullptr;                                            // fine residual
    // Merged fine level: when the fine boxes tile one rectangle, the fine
    // level runs as that one box (solution with 1 ghost, right-hand side),
    // loaded and returned by ParallelCopy; there are then no ghosts between
    // fine boxes and every ghost is a coarse-fine one.
    bxmg_boxarray fone = nullptr;
    bxmg_multifab Uf = nullptr, Ff = nullptr;
    CGeo geo{};
    DevBuf<int> cmap;
    DevBuf<int4> ghosts;
    int nghosts = 0;
    int nfine = 0;
    dim3 g_fine, g_fine_s, g_fine_gs, g_sync, g_coarse;  // launch grids
    int nparts_fine = 0, nparts = 0;
    DevBuf<double> part, fn;
    double* h_norm = nullptr;  // pinned: the norms read back
    ~Comp() {
        for (bxmg_multifab m : {Uc, Fc, Rc, Ec, Rf, Uf, Ff})
            if (m) bxmg_multifab_release(m);
        if (one) bxmg_boxarray_release(one);
        if (fone) bxmg_boxarray_release(fone);
        const hipStream_t s = ctx ? ctx->stream : nullptr;
        cmap.release_async(s);
        ghosts.release_async(s);
        part.release_async(s);
        fn.release_async(s);
        if (h_norm) {
            (void)hipStreamSynchronize(s);
            (void)hipHostFree(h_norm);
        }
    }
};

// Checks the fine layout against the coarse domain: the fine domain is the
// coarse one refined by 2 with the same boundaries, every fine box is a union
// of whole coarse cells and lies 2 coarse cells (4 fine) inside every domain
// face; index arithmetic stays in 32 bits.  Returns "" or the reason.
static std::string layout_error(const bxmg_ba_s* cba, const bxmg_ba_s* fba) {
    for (int d = 0; d < 3; ++d) {
        if (fba->dom.lo[d] != 2 * cba->dom.lo[d] || fba->dom.hi[d] != 2 * cba->dom.hi[d] + 1)
            return "the fine domain must be the coarse domain refined by 2";
        if (fba->per[d] != cba->per[d]) return "the fine and coarse boundaries differ";
    }
    const Box& D = cba->dom;
    if ((long long)(D.n(0) + 2) * (D.n(1) + 2) * (D.n(2) + 2) >= (1LL << 31)) return "coarse domain too large";
    if (fba->boxes.size() >= (1u << 24)) return "too many fine boxes";
    for (const Box& B : fba->boxes) {
        for (int d = 0; d < 3; ++d) {
            if ((B.lo[d] & 1) || !(B.hi[d] & 1)) return "fine boxes must be unions of whole coarse cells";
            if (B.lo[d] < fba->dom.lo[d] + 4 || B.hi[d] > fba->dom.hi[d] - 4)
                return "fine boxes must lie 2 coarse cells inside the domain";
        }
        if ((long long)(B.n(0) + 8) * (B.n(1) + 8) * (B.n(2) + 8) >= (1LL << 31)) return "fine box too large";
    }
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
    c->Rc = alloc_mf(ctx, c->one, 1);
    c->Ec = alloc_mf(ctx, c->one, 1);
    // the fine level: one merged box when the caller's fine boxes tile a
    // rectangle (they are disjoint, so equal cell counts mean they tile it)
    Box U = fba->boxes[0];
    long long fcells = 0;
    for (const Box& B : fba->boxes) {
        fcells += B.cells();
        for (int d = 0; d < 3; ++d) {
            U.lo[d] = std::min(U.lo[d], B.lo[d]);
            U.hi[d] = std::max(U.hi[d], B.hi[d]);
        }
    }
    std::vector<Box> fb;  // the boxes the kernels run over
    if (fcells == U.cells() && fba->boxes.size() > 1) {
        const int ul[6] = {U.lo[0], U.lo[1], U.lo[2], U.hi[0], U.hi[1], U.hi[2]};
        if (bxmg_define_boxarray_list(fba->dom.lo, fba->dom.hi, fba->bc, 1, ul, &c->fone) != BXMG_OK)
            throw std::runtime_error(bxmg_last_error());
        c->Uf = alloc_mf(ctx, c->fone, 1);
        c->Ff = alloc_mf(ctx, c->fone, 0);
        c->Rf = alloc_mf(ctx, c->fone, 0);
        fb.push_back(U);
    } else {
        bxmg_boxarray fcopy = nullptr;
        std::vector<int32_t> fl;
        for (const Box& B : fba->boxes)
            for (int v : {B.lo[0], B.lo[1], B.lo[2], B.hi[0], B.hi[1], B.hi[2]}) fl.push_back(v);
        if (bxmg_define_boxarray_list(fba->dom.lo, fba->dom.hi, fba->bc, (int32_t)fba->boxes.size(), fl.data(),
                                      &fcopy) != BXMG_OK)
            throw std::runtime_error(bxmg_last_error());
        c->Rf = alloc_mf(ctx, fcopy, 0);
        bxmg_boxarray_release(fcopy);  // the MultiFab keeps its reference
        fb = fba->boxes;
    }
    CGeo& g = c->geo;
    g.cb = c->Uc->fboxes[0];
    for (int d = 0; d < 3; ++d) {
        g.dlo[d] = D.lo[d];
        g.n[d] = D.n(d);
        g.per[d] = cba->per[d];
    }
    g.h0 = h0;
    g.h1 = h0 * 0.5;
    g.ih0sq = 1.0 / (h0 * h0);
    // coverage map: covering fine box, or -1 - (mask of covered face neighbours)
    const long long nc = D.cells();
    std::vector<int> cmap((size_t)nc, -1);
    auto cidx = [&](int I, int J, int K) {
        return (size_t)(I - D.lo[0]) + (size_t)D.n(0) * ((size_t)(J - D.lo[1]) + (size_t)D.n(1) * (K - D.lo[2]));
    };
    c->nfine = (int)fb.size();
    int maxP = 1, maxPh = 1, maxnz = 1, maxPc = 1, maxnzc = 1;
    for (size_t b = 0; b < fb.size(); ++b) {
        const Box& B = fb[b];
        maxP = std::max(maxP, B.n(0) * B.n(1));
        maxPh = std::max(maxPh, ((B.n(0) + 1) / 2) * B.n(1));
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
                            // the neighbour N across (d, side) of this covered cell sees it across (d, 1 - side)
                            int x[3] = {I, J, K};
                            x[d] += side ? 1 : -1;
                            int& m = cmap[cidx(x[0], x[1], x[2])];
                            if (m >= 0) continue;
                            const int mask = (-1 - m) | (1 << (2 * d + (1 - side)));
                            m = -1 - mask;
                        }
    // coarse-fine ghosts: face ghosts of each fine box whose coarse cell no
    // fine box covers (the others are fine cells, filled by FillBoundary)
    std::vector<int4> gl;
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
                        if (cmap[cidx(gx[0] >> 1, gx[1] >> 1, gx[2] >> 1)] >= 0) continue;
                        gl.push_back(make_int4((int)b | (d << 24) | (side << 26), gx[0], gx[1], gx[2]));
                    }
            }
    }
    if (gl.size() >= (size_t)(1u << 31) - kCB) throw std::runtime_error("too many coarse-fine ghost cells");
    c->nghosts = (int)gl.size();
    const unsigned nf = (unsigned)std::max(1, c->nfine);
    c->g_fine = dim3(cdiv(maxP, kCB), cdiv(maxnz, kKZ), nf);
    c->g_fine_s = dim3(cdiv(maxP, kCB), cdiv(maxnz, kKZs), nf);
    c->g_fine_gs = dim3(cdiv(maxPh, kCB), cdiv(maxnz, kKZs), nf);
    c->g_sync = dim3(cdiv(maxPc, kCB), cdiv(maxnzc, kKZ), nf);
    c->g_coarse = dim3(cdiv((long long)g.n[0] * g.n[1], kCB), cdiv(g.n[2], kKZ), 1);
    c->nparts_fine = c->nfine ? (int)(c->g_fine.x * c->g_fine.y * c->g_fine.z) : 0;
    c->nparts = c->nparts_fine + (int)(c->g_coarse.x * c->g_coarse.y);
    const hipStream_t s = ctx->stream;
    c->cmap.upload_async(cmap, s);
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
    if (phi_f->ng < 1) return bad("the fine solution needs nghost >= 1");
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
        double* Rc = (double*)c.Rc->data;
        double* Ec = (double*)c.Ec->data;
        const bool merged = c.Uf != nullptr;
        bxmg_multifab mu = merged ? c.Uf : phi_f, mf = merged ? c.Ff : rhs_f;
        double* uf = (double*)mu->data;
        const double* ff = (const double*)mf->data;
        double* rf = (double*)c.Rf->data;
        const FBox* fu = mu->d_fboxes.p;
        const FBox* fF = mf->d_fboxes.p;
        const FBox* fR = c.Rf->d_fboxes.p;
        const unsigned nfb = (unsigned)c.nfine;
        double* const part_c = c.part.p + 3 * (size_t)c.nparts_fine;
        // k_fine_zero covers the grown fine boxes
        int maxPG = 1, maxGz = 1;
        for (const FBox& B : mu->fboxes) {
            maxPG = std::max(maxPG, B.G[0] * B.G[1]);
            maxGz = std::max(maxGz, B.G[2]);
        }
        const dim3 g_zero(comp::cdiv(maxPG, comp::kCB), comp::cdiv(maxGz, comp::kKZ), std::max(1u, nfb));
        auto chk = [](bxmg_status st) {
            if (st != BXMG_OK) throw std::runtime_error(bxmg_last_error());
        };
        // load: coarse rhs into the one-box field, zero start on both levels
        chk(bxmg_parallel_copy(c.Fc, 0, rhs_c, 0, 1, 0, s));
        if (merged) chk(bxmg_parallel_copy(c.Ff, 0, rhs_f, 0, 1, 0, s));
        HIPCHK(hipMemsetAsync(Uc, 0, c.Uc->bytes, s));
        if (nfb) hipLaunchKernelGGL(comp::k_fine_zero, g_zero, dim3(comp::kCB), 0, s, fu, uf);
        HIPCHK(hipGetLastError());
        auto fill_fine = [&]() {
            if (!nfb) return;
            if (!merged) chk(bxmg_fill_boundary(phi_f, 0, 1, 1, s));
            if (c.nghosts)
                hipLaunchKernelGGL(comp::k_cf_ghost, dim3(comp::cdiv(c.nghosts, comp::kCB)), dim3(comp::kCB), 0, s,
                                   c.ghosts.p, c.nghosts, g, (const double*)Uc, fu, uf);
            HIPCHK(hipGetLastError());
        };
        // composite residual (fonly: norms of f) into Rf / Rc, norms read back
        auto residual = [&](bool fonly, double out[3]) {
            if (!fonly) fill_fine();
            if (nfb)
                hipLaunchKernelGGL(comp::k_fine_resid, c.g_fine, dim3(comp::kCB), 0, s, g, fu, fF, fR,
                                   (const double*)uf, ff, rf, (int)fonly, c.part.p);
            hipLaunchKernelGGL(comp::k_coarse_resid, c.g_coarse, dim3(comp::kCB), 0, s, g, (const int*)c.cmap.p,
                               (const double*)Uc, (const double*)Fc, Rc, fu, (const double*)uf, fR,
                               (const double*)rf, (int)fonly, part_c);
            HIPCHK(hipGetLastError());
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
                    fill_fine();
                    if (nfb)
                        hipLaunchKernelGGL(comp::k_fine_gs, c.g_fine_gs, dim3(comp::kCB), 0, s, g, fu, fF, uf, ff,
                                           col);
                    HIPCHK(hipGetLastError());
                }
        };
        bxmg_solve_params Pc = P;
        Pc.fixed_cycles = 1;
        Pc.dx = h0;
        auto cycle = [&]() {
            sweeps(P.nu1);
            double rn[3];
            residual(false, rn);
            // coarse correction: one V-cycle from zero on the composite residual
            int nlev = 0;
            chk(vcycle_from_zero(ctx, Pc, c.Ec, c.Rc, &nlev));
            info->levels = nlev + 1;
            hipLaunchKernelGGL(comp::k_coarse_update, c.g_coarse, dim3(comp::kCB), 0, s, g, (const int*)c.cmap.p, Uc,
                               (const double*)Ec);
            if (nfb)
                hipLaunchKernelGGL(comp::k_fine_prolong, c.g_fine_s, dim3(comp::kCB), 0, s, g, fu, uf,
                                   (const double*)Ec);
            HIPCHK(hipGetLastError());
            sweeps(P.nu2);
            if (nfb)
                hipLaunchKernelGGL(comp::k_coarse_sync, c.g_sync, dim3(comp::kCB), 0, s, g, Uc, fu, (const double*)uf);
            HIPCHK(hipGetLastError());
        };
        double fz[3];
        residual(true, fz);
        const double fnorm = fz[0];
        info->f_inf = fnorm;
        int status = 0, cyc = 0;
        if (!(fnorm == fnorm)) {
            status = BXMG_ENONFINITE;
        } else if (fnorm > 0.0) {
            for (;; ++cyc) {
                double rn[3];
                residual(false, rn);
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
        // the coarse solution (covered cells: the mean of their children) back
        chk(bxmg_parallel_copy(phi_c, 0, c.Uc, 0, 1, 0, s));
        if (merged) chk(bxmg_parallel_copy(phi_f, 0, c.Uf, 0, 1, 0, s));
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
