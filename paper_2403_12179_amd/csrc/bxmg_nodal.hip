// Nodal-centred Poisson solver (the framework's other linear-solver family,
// paper Section 2): V-cycles over node-centred data of the whole domain.
//
// On a domain of n_d cells of width h per direction the nodes sit at
// x = i h, i = 0 .. n_d.  The caller's arrays are F-order over the
// (n_0+1)(n_1+1)(n_2+1) nodes; every level is held colour-split inside the
// solver: node (i, j, k) of colour c = (i + j + k) & 1 in colour block c,
// row k (n_1+1) + j, slot i >> 1 (rows of (n_0+2)/2 slots), so a colour
// sweep streams the other colour, its own right-hand side and its own
// writes.  A homogeneous-Dirichlet
// direction keeps its boundary nodes at 0 (they are not unknowns); in a
// periodic direction node n_d is node 0: the kernels read neighbours
// through the wrapped index, and the copies n_d are refreshed only in the
// solution handed back.  Operator (L u)_i = (sum of the 6 neighbours - 6 u_i)
// / h^2; red-black Gauss-Seidel on node parity; full-weighting restriction
// (weights 1/2 at the node, 1/4 at +-1 per direction); trilinear
// prolongation; FP64 CG bottom in one workgroup.  Coarse node I is fine node
// 2I; levels halve while every n_d is even and > 2.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "bxmg_host.h"

namespace bxmg {
namespace nodal {

struct NLev {
    int n[3];    // cells per direction (nodes 0..n)
    int per[3];
    double h;
    long long size;   // nodes, (n0+1)(n1+1)(n2+1)
    int H;            // slots per colour row, (n0+2)/2
    long long cs;     // colour block stride (elements)
    long long alloc;  // elements of a level array, 2 cs
};

// offset of node (i, j, k) in the colour-split level array
__host__ __device__ inline long long nidx(const NLev& L, int i, int j, int k) {
    return ((i + j + k) & 1) * L.cs + (long long)((k * (L.n[1] + 1) + j) * L.H + (i >> 1));
}

// node (i, j, k) of the g-th node in F order (x fastest)
__device__ __forceinline__ void coords(const NLev& L, long long g, int& i, int& j, int& k) {
    const int nx = L.n[0] + 1, ny = L.n[1] + 1;
    const long long r = g / nx;
    i = (int)(g - r * nx);
    j = (int)(r % ny);
    k = (int)(r / ny);
}

__device__ __forceinline__ bool unknown(const NLev& L, int i, int j, int k) {
    const int c[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d)
        if (L.per[d] ? c[d] == L.n[d] : (c[d] == 0 || c[d] == L.n[d])) return false;
    return true;
}

__device__ __forceinline__ int wrap(const NLev& L, int d, int c) {
    if (!L.per[d]) return c;
    return c < 0 ? c + L.n[d] : (c >= L.n[d] ? c - L.n[d] : c);
}

// sum of the 6 neighbours, ((x- + x+) + (y- + y+)) + (z- + z+)
__device__ __forceinline__ double nsum(const NLev& L, const double* __restrict__ u, int i, int j, int k) {
    const double xm = u[nidx(L, wrap(L, 0, i - 1), j, k)], xp = u[nidx(L, wrap(L, 0, i + 1), j, k)];
    const double ym = u[nidx(L, i, wrap(L, 1, j - 1), k)], yp = u[nidx(L, i, wrap(L, 1, j + 1), k)];
    const double zm = u[nidx(L, i, j, wrap(L, 2, k - 1))], zp = u[nidx(L, i, j, wrap(L, 2, k + 1))];
    return ((xm + xp) + (ym + yp)) + (zm + zp);
}

__device__ __forceinline__ void block_sum2(double& a, double& b, double* sh) {
    for (int o = 32; o > 0; o >>= 1) {
        a = a + __shfl_xor(a, o);
        b = b + __shfl_xor(b, o);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) { sh[2 * wid] = a; sh[2 * wid + 1] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        a = sh[0];
        b = sh[1];
        for (int w = 1; w < nw; ++w) { a = a + sh[2 * w]; b = b + sh[2 * w + 1]; }
    }
}

constexpr int kNB = 256;

// Level kernels walk planes: grid (plane blocks, plane groups), a thread
// takes one (x, y) position of its planes.  Interior nodes read their six
// neighbours directly (x from the other colour's slots (i -+ 1) >> 1, y and z
// from the other colour's rows at slot i >> 1); the others go through the
// wrapped index.
constexpr int kKZ = 8;

// the six neighbours of interior node (i, j, k), ((x- + x+) + (y- + y+)) + (z- + z+)
__device__ __forceinline__ double nsum_in(const NLev& L, const double* __restrict__ u, int i, int j, int k) {
    const int c = (i + j + k) & 1;
    const long long o = (1 - c) * L.cs + (long long)((k * (L.n[1] + 1) + j) * L.H);
    const long long m = o + (i >> 1), sy = L.H, sz = (long long)L.H * (L.n[1] + 1);
    return ((u[o + ((i - 1) >> 1)] + u[o + ((i + 1) >> 1)]) + (u[m - sy] + u[m + sy])) + (u[m - sz] + u[m + sz]);
}

// no neighbour through a wrap: in a periodic direction node n_d - 1 reads
// node 0 through the wrapped index (the copy n_d is refreshed only at the
// end), so it is not interior
__device__ __forceinline__ bool interior(const NLev& L, int i, int j, int k) {
    return i > 0 && i < L.n[0] - L.per[0] && j > 0 && j < L.n[1] - L.per[1] && k > 0 && k < L.n[2] - L.per[2];
}

// one colour: a thread per colour node of a row position (i = 2t + parity)
__global__ void __launch_bounds__(kNB) k_nd_gs(NLev L, double* __restrict__ u, const double* __restrict__ f,
                                              int colour, int kz) {
    const uint3 bk = xcd_block();
    const int hx = (L.n[0] + 2) / 2, ny = L.n[1] + 1;
    const int t = bk.x * kNB + threadIdx.x;
    if (t >= hx * ny) return;
    const int tx = t % hx, j = t / hx;
    const int k0 = bk.y * kz, k1 = min(k0 + kz - 1, L.n[2]);
    const double h2 = L.h * L.h;
    for (int k = k0; k <= k1; ++k) {
        const int i = 2 * tx + ((colour - j - k) & 1);
        if (i > L.n[0] || !unknown(L, i, j, k)) continue;
        const long long q = nidx(L, i, j, k);
        const double su = interior(L, i, j, k) ? nsum_in(L, u, i, j, k) : nsum(L, u, i, j, k);
        u[q] = (su - h2 * f[q]) / 6.0;
    }
}

// r = f - L u at the unknowns, 0 at the other nodes; partial (max, sum r^2,
// non-finite count) per block
__global__ void __launch_bounds__(kNB) k_nd_resid(NLev L, const double* __restrict__ u,
                                                 const double* __restrict__ f, double* __restrict__ r,
                                                 double* __restrict__ partials, int kz) {
    __shared__ double sh[3 * (kNB / 64)];
    const uint3 bk = xcd_block();
    const int hx = (L.n[0] + 2) / 2, ny = L.n[1] + 1;
    const int t = bk.x * kNB + threadIdx.x;
    const double ih2 = 1.0 / (L.h * L.h);
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    if (t < hx * ny) {
        // a thread per row slot, the node of each colour in it
        const int tx = t % hx, j = t / hx;
        const int k0 = bk.y * kz, k1 = min(k0 + kz - 1, L.n[2]);
        for (int k = k0; k <= k1; ++k)
          for (int c = 0; c < 2; ++c) {
            const int i = 2 * tx + ((c - j - k) & 1);
            if (i > L.n[0]) continue;
            const long long q = nidx(L, i, j, k);
            double rv = 0.0;
            if (unknown(L, i, j, k)) {
                const double su = interior(L, i, j, k) ? nsum_in(L, u, i, j, k) : nsum(L, u, i, j, k);
                rv = f[q] - (su - 6.0 * u[q]) * ih2;
                const double a = fabs(rv);
                if (!(a <= 1.7976931348623157e308)) bad += 1.0;
                else mx = fmax(mx, a);
                s2 = s2 + rv * rv;
            }
            r[q] = rv;
          }
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o));
        s2 = s2 + __shfl_xor(s2, o);
        bad = bad + __shfl_xor(bad, o);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { sh[3 * wid] = mx; sh[3 * wid + 1] = s2; sh[3 * wid + 2] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kNB / 64; ++w) { mx = fmax(mx, sh[3 * w]); s2 = s2 + sh[3 * w + 1]; bad = bad + sh[3 * w + 2]; }
        const int blk = bk.y * gridDim.x + bk.x;
        partials[3 * blk] = mx;
        partials[3 * blk + 1] = s2;
        partials[3 * blk + 2] = bad;
    }
}

// norms of f over the unknowns (max, sum of squares, non-finite count)
__global__ void __launch_bounds__(kNB) k_nd_fnorm(NLev L, const double* __restrict__ f,
                                                 double* __restrict__ partials) {
    __shared__ double sh[3 * (kNB / 64)];
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < L.size;
         g += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        coords(L, g, i, j, k);
        if (!unknown(L, i, j, k)) continue;
        const long long q = nidx(L, i, j, k);
        const double a = fabs(f[q]);
        if (!(a <= 1.7976931348623157e308)) bad += 1.0;
        else mx = fmax(mx, a);
        s2 = s2 + f[q] * f[q];
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o));
        s2 = s2 + __shfl_xor(s2, o);
        bad = bad + __shfl_xor(bad, o);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { sh[3 * wid] = mx; sh[3 * wid + 1] = s2; sh[3 * wid + 2] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kNB / 64; ++w) { mx = fmax(mx, sh[3 * w]); s2 = s2 + sh[3 * w + 1]; bad = bad + sh[3 * w + 2]; }
        partials[3 * blockIdx.x] = mx;
        partials[3 * blockIdx.x + 1] = s2;
        partials[3 * blockIdx.x + 2] = bad;
    }
}

// full weighting onto the coarse unknowns (0 at the other coarse nodes), in
// the order z, then y, then x offsets; the coarse u is zeroed on the way
__global__ void __launch_bounds__(kNB) k_nd_restrict(NLev F, const double* __restrict__ r, NLev C,
                                                    double* __restrict__ fc, double* __restrict__ uc, int kz) {
    const uint3 bk = xcd_block();
    const int nx = C.n[0] + 1, ny = C.n[1] + 1;
    const int t = bk.x * kNB + threadIdx.x;
    if (t >= nx * ny) return;
    const int I = t % nx, J = t / nx;
    const int K0 = bk.y * kz, K1 = min(K0 + kz - 1, C.n[2]);
    const double w[3] = {0.25, 0.5, 0.25};
    for (int K = K0; K <= K1; ++K) {
        const long long q = nidx(C, I, J, K);
        double s = 0.0;
        if (unknown(C, I, J, K)) {
            for (int c = -1; c <= 1; ++c)
                for (int b = -1; b <= 1; ++b)
                    for (int a = -1; a <= 1; ++a) {
                        const int i = wrap(F, 0, 2 * I + a), j = wrap(F, 1, 2 * J + b), k = wrap(F, 2, 2 * K + c);
                        s = s + ((w[a + 1] * w[b + 1]) * w[c + 1]) * r[nidx(F, i, j, k)];
                    }
        }
        fc[q] = s;
        uc[q] = 0.0;
    }
}

// u_f += P e at the fine unknowns: fine node 2I + o takes the mean of the
// coarse nodes I + o' (o' <= o), summed z, y, x
__global__ void __launch_bounds__(kNB) k_nd_prolong(NLev C, const double* __restrict__ e, NLev F,
                                                   double* __restrict__ u) {
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < F.size;
         g += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        coords(F, g, i, j, k);
        if (!unknown(F, i, j, k)) continue;
        const long long q = nidx(F, i, j, k);
        const int I[3] = {i >> 1, j >> 1, k >> 1}, o[3] = {i & 1, j & 1, k & 1};
        double s = 0.0;
        int cnt = 0;
        for (int cz = 0; cz <= o[2]; ++cz)
            for (int cy = 0; cy <= o[1]; ++cy)
                for (int cx = 0; cx <= o[0]; ++cx) {
                    s = s + e[nidx(C, wrap(C, 0, I[0] + cx), wrap(C, 1, I[1] + cy), wrap(C, 2, I[2] + cz))];
                    ++cnt;
                }
        u[q] = u[q] + s / (double)cnt;
    }
}

// the periodic copies n_d take the values of their nodes 0
__global__ void __launch_bounds__(kNB) k_nd_copies(NLev L, double* __restrict__ u) {
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < L.size;
         g += (long long)gridDim.x * blockDim.x) {
        int c[3];
        coords(L, g, c[0], c[1], c[2]);
        const long long q = nidx(L, c[0], c[1], c[2]);
        bool copy = false;
        for (int d = 0; d < 3; ++d)
            if (L.per[d] && c[d] == L.n[d]) { c[d] = 0; copy = true; }
        if (copy) u[q] = u[nidx(L, c[0], c[1], c[2])];
    }
}

// u -= mean over the unknowns, two passes: the sum (fixed per-block order,
// then block 0 adds the block sums in order), then the subtraction
__global__ void __launch_bounds__(kNB) k_nd_sum(NLev L, const double* __restrict__ u, double* __restrict__ part) {
    __shared__ double sh[2 * (kNB / 64)];
    double s = 0.0, c = 0.0;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < L.size;
         g += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        coords(L, g, i, j, k);
        if (unknown(L, i, j, k)) { s = s + u[nidx(L, i, j, k)]; c = c + 1.0; }
    }
    block_sum2(s, c, sh);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = s; part[2 * blockIdx.x + 1] = c; }
}
__global__ void __launch_bounds__(kNB) k_nd_sub(NLev L, double* __restrict__ u, const double* __restrict__ part,
                                               int nparts) {
    double s = 0.0, c = 0.0;
    for (int b = 0; b < nparts; ++b) { s = s + part[2 * b]; c = c + part[2 * b + 1]; }
    const double m = s / c;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < L.size;
         g += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        coords(L, g, i, j, k);
        if (unknown(L, i, j, k)) {
            const long long q = nidx(L, i, j, k);
            u[q] = u[q] - m;
        }
    }
}

// Bottom: FP64 CG on the unknowns in one workgroup, vectors in device
// memory (levels of a few thousand nodes, colour-split like the others);
// fully periodic: right-hand side and solution projected to mean 0.  rtol
// on the L2 norm, at most 4 N iterations.
constexpr int kNBot = 1024;
__global__ void __launch_bounds__(kNBot) k_nd_bottom(NLev L, double* __restrict__ x, const double* __restrict__ f,
                                                    double* __restrict__ r, double* __restrict__ p,
                                                    double* __restrict__ q, double rtol, int* __restrict__ iters) {
    __shared__ double sh[2 * (kNBot / 64)];
    __shared__ double bc[2];
    const long long N = L.size;
    const bool sing = L.per[0] && L.per[1] && L.per[2];
    const double ih2 = 1.0 / (L.h * L.h);
    // sum over unknowns of a*b (or of a, with b == nullptr), broadcast
    auto dot = [&](const double* a, const double* b, double& cnt) {
        double s = 0.0, c = 0.0;
        for (long long g = threadIdx.x; g < N; g += blockDim.x) {
            int i, j, k;
            coords(L, g, i, j, k);
            if (!unknown(L, i, j, k)) continue;
            const long long o = nidx(L, i, j, k);
            s = s + (b ? a[o] * b[o] : a[o]);
            c = c + 1.0;
        }
        block_sum2(s, c, sh);
        if (threadIdx.x == 0) { bc[0] = s; bc[1] = c; }
        __syncthreads();
        cnt = bc[1];
        const double v = bc[0];
        __syncthreads();
        return v;
    };
    for (long long g = threadIdx.x; g < N; g += blockDim.x) {
        int i, j, k;
        coords(L, g, i, j, k);
        const long long o = nidx(L, i, j, k);
        r[o] = unknown(L, i, j, k) ? f[o] : 0.0;
        x[o] = 0.0;
    }
    __syncthreads();
    double cnt;
    if (sing) {
        const double m = dot(r, nullptr, cnt) / cnt;
        for (long long g = threadIdx.x; g < N; g += blockDim.x) {
            int i, j, k;
            coords(L, g, i, j, k);
            if (unknown(L, i, j, k)) {
                const long long o = nidx(L, i, j, k);
                r[o] = r[o] - m;
            }
        }
        __syncthreads();
    }
    for (long long g = threadIdx.x; g < N; g += blockDim.x) {
        int i, j, k;
        coords(L, g, i, j, k);
        const long long o = nidx(L, i, j, k);
        p[o] = r[o];
    }
    __syncthreads();
    double rs = dot(r, r, cnt);
    const double rs0 = rs;
    int it = 0;
    const long long maxit = 4 * (long long)cnt;
    if (rs0 != 0.0) {
        while (it < maxit) {
            for (long long g = threadIdx.x; g < N; g += blockDim.x) {
                int i, j, k;
                coords(L, g, i, j, k);
                const long long o = nidx(L, i, j, k);
                q[o] = unknown(L, i, j, k) ? (nsum(L, p, i, j, k) - 6.0 * p[o]) * ih2 : 0.0;
            }
            __syncthreads();
            const double alpha = rs / dot(p, q, cnt);
            for (long long g = threadIdx.x; g < N; g += blockDim.x) {
                int i, j, k;
                coords(L, g, i, j, k);
                if (!unknown(L, i, j, k)) continue;
                const long long o = nidx(L, i, j, k);
                x[o] = x[o] + alpha * p[o];
                r[o] = r[o] - alpha * q[o];
            }
            __syncthreads();
            const double rsn = dot(r, r, cnt);
            ++it;
            if (sqrt(rsn) <= rtol * sqrt(rs0)) break;
            const double beta = rsn / rs;
            for (long long g = threadIdx.x; g < N; g += blockDim.x) {
                int i, j, k;
                coords(L, g, i, j, k);
                if (unknown(L, i, j, k)) {
                    const long long o = nidx(L, i, j, k);
                    p[o] = r[o] + beta * p[o];
                }
            }
            __syncthreads();
            rs = rsn;
        }
        if (sing) {
            const double m = dot(x, nullptr, cnt) / cnt;
            for (long long g = threadIdx.x; g < N; g += blockDim.x) {
                int i, j, k;
                coords(L, g, i, j, k);
                if (unknown(L, i, j, k)) {
                    const long long o = nidx(L, i, j, k);
                    x[o] = x[o] - m;
                }
            }
        }
    }
    if (threadIdx.x == 0 && iters) *iters = it;
}

// Caller F-order node array <-> colour-split level array.
template <bool TO_SPLIT>
__global__ void __launch_bounds__(kNB) k_nd_convert(NLev L, double* __restrict__ fo, double* __restrict__ sp) {
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < L.size;
         g += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        coords(L, g, i, j, k);
        if constexpr (TO_SPLIT) sp[nidx(L, i, j, k)] = fo[g];
        else fo[g] = sp[nidx(L, i, j, k)];
    }
}

inline unsigned nblocks(long long n) { return (unsigned)std::min<long long>((n + kNB - 1) / kNB, 8192); }

// Planes each thread walks on a level: up to kmax, fewer where the level
// would otherwise give fewer than 2048 blocks.
inline int plane_depth(const NLev& L, bool half, int kmax) {
    const long long row = half ? (L.n[0] + 2) / 2 : L.n[0] + 1;
    const long long gx = (row * (L.n[1] + 1) + kNB - 1) / kNB;
    const long long kz = (gx * (L.n[2] + 1)) / 2048;
    return (int)std::max(1LL, std::min<long long>(kmax, kz));
}
// grid of the plane-walking kernels over the nodes of a level (half rows
// for the sweeps), kz planes per thread
inline dim3 plane_grid(const NLev& L, bool half, int kz) {
    const long long row = half ? (L.n[0] + 2) / 2 : L.n[0] + 1;
    return dim3((unsigned)((row * (L.n[1] + 1) + kNB - 1) / kNB), (unsigned)((L.n[2] + 1 + kz - 1) / kz), 1);
}
inline int plane_blocks(const NLev& L, bool half, int kz) {
    const dim3 g = plane_grid(L, half, kz);
    return (int)(g.x * g.y);
}
constexpr int kKZr = kKZ;  // residual
constexpr int kKZt = 2;    // transfers

// The nodal hierarchy of one geometry, cached on the context.
struct NHier {
    std::vector<NLev> L;
    std::vector<DevBuf<double>> u, f, r;
    DevBuf<double> part, bp, bq, fn;
    DevBuf<int> iters;
    std::string key;
};

struct NCache {
    std::vector<std::unique_ptr<NHier>> h;  // most recent last
};

static NHier* get(bxmg_ctx ctx, const bxmg_ba_s* ba, double h0) {
    if (!ctx->nodal) ctx->nodal = std::make_shared<NCache>();
    NCache& C = *std::static_pointer_cast<NCache>(ctx->nodal);
    std::string key;
    auto put = [&](long long v) { key.append((const char*)&v, sizeof v); };
    long long hb;
    std::memcpy(&hb, &h0, sizeof hb);
    put(hb);
    for (int d = 0; d < 3; ++d) { put(ba->dom.n(d)); put(ba->per[d]); }
    for (size_t q = 0; q < C.h.size(); ++q)
        if (C.h[q]->key == key) return C.h[q].get();
    auto H = std::make_unique<NHier>();
    H->key = key;
    NLev l;
    for (int d = 0; d < 3; ++d) { l.n[d] = ba->dom.n(d); l.per[d] = ba->per[d]; }
    l.h = h0;
    for (;;) {
        l.size = (long long)(l.n[0] + 1) * (l.n[1] + 1) * (l.n[2] + 1);
        l.H = (l.n[0] + 2) / 2;
        l.cs = ((long long)l.H * (l.n[1] + 1) * (l.n[2] + 1) + 63) / 64 * 64;
        l.alloc = 2 * l.cs;
        H->L.push_back(l);
        bool more = true;
        for (int d = 0; d < 3; ++d)
            if (l.n[d] % 2 || l.n[d] <= 2) more = false;
        if (!more) break;
        for (int d = 0; d < 3; ++d) l.n[d] /= 2;
        l.h *= 2.0;
    }
    const NLev& B = H->L.back();
    if (B.size > 4096 * 8) throw std::runtime_error("nodal: bottom level too large");
    if (H->L[0].alloc >= (1LL << 31)) throw std::runtime_error("nodal: more than 2^31 nodes");
    const size_t nl = H->L.size();
    H->u.resize(nl);
    H->f.resize(nl);
    H->r.resize(nl);
    for (size_t q = 0; q < nl; ++q) {
        H->u[q].alloc(H->L[q].alloc);
        H->f[q].alloc(H->L[q].alloc);
        H->r[q].alloc(H->L[q].alloc);
    }
    int np = 8192;
    for (const NLev& l : H->L) np = std::max(np, plane_blocks(l, true, plane_depth(l, true, kKZr)));
    H->part.alloc(3 * (size_t)np);
    H->bp.alloc(B.alloc);
    H->bq.alloc(B.alloc);
    H->fn.alloc(3);
    H->iters.alloc(1);
    if (C.h.size() >= 4) C.h.erase(C.h.begin());
    C.h.push_back(std::move(H));
    return C.h.back().get();
}

static void vcycle(NHier& H, size_t l, hipStream_t s, int nu1, int nu2, double brtol) {
    const NLev& L = H.L[l];
    if (l + 1 == H.L.size()) {
        hipLaunchKernelGGL(k_nd_bottom, dim3(1), dim3(kNBot), 0, s, L, H.u[l].p, H.f[l].p, H.r[l].p, H.bp.p, H.bq.p,
                           brtol, H.iters.p);
        HIPCHK(hipGetLastError());
        return;
    }
    const int kg = plane_depth(L, true, kKZ), kr = plane_depth(L, true, kKZr);
    const dim3 gb = plane_grid(L, true, kg);
    for (int q = 0; q < nu1; ++q)
        for (int c = 0; c < 2; ++c)
            hipLaunchKernelGGL(k_nd_gs, gb, dim3(kNB), 0, s, L, H.u[l].p, H.f[l].p, c, kg);
    hipLaunchKernelGGL(k_nd_resid, plane_grid(L, true, kr), dim3(kNB), 0, s, L, H.u[l].p, H.f[l].p, H.r[l].p,
                       H.part.p, kr);
    const NLev& C = H.L[l + 1];
    const int kc = plane_depth(C, false, kKZt);
    hipLaunchKernelGGL(k_nd_restrict, plane_grid(C, false, kc), dim3(kNB), 0, s, L, H.r[l].p, C, H.f[l + 1].p,
                       H.u[l + 1].p, kc);
    vcycle(H, l + 1, s, nu1, nu2, brtol);
    hipLaunchKernelGGL(k_nd_prolong, dim3(nblocks(L.size)), dim3(kNB), 0, s, C, H.u[l + 1].p, L, H.u[l].p);
    for (int q = 0; q < nu2; ++q)
        for (int c = 0; c < 2; ++c)
            hipLaunchKernelGGL(k_nd_gs, gb, dim3(kNB), 0, s, L, H.u[l].p, H.f[l].p, c, kg);
    HIPCHK(hipGetLastError());
}

}  // namespace nodal
}  // namespace bxmg

using namespace bxmg;

extern "C" bxmg_status bxmg_nodal_solve(bxmg_ctx ctx, const bxmg_solve_params* params, bxmg_boxarray ba,
                                        double* phi, const double* rhs, bxmg_solve_info* info) {
    if (!ctx || !ba || !phi || !rhs || !info) return fail(BXMG_EINVAL, "nodal_solve: NULL argument");
    std::memset(info, 0, sizeof(*info));
    bxmg_solve_params P;
    if (params) P = *params;
    else bxmg_solve_params_default(&P);
    if (P.nu1 < 0 || P.nu2 < 0 || P.max_cycles < 0 || P.precision != 0 || P.krylov != 0 || P.alpha != 0.0) {
        info->status = fail(BXMG_EINVAL, "nodal_solve: FP64 V-cycles of the Poisson operator only "
                                         "(precision 0, krylov 0, alpha 0)");
        return (bxmg_status)info->status;
    }
    const double h = (P.dx > 0) ? P.dx : 1.0 / ba->dom.n(0);
    std::lock_guard<std::mutex> lock(ctx->mu);
    const auto t0 = std::chrono::steady_clock::now();
    try {
        HIPCHK(hipSetDevice(ctx->device));
        nodal::NHier* H = nodal::get(ctx, ba, h);
        const hipStream_t s = ctx->stream;
        const nodal::NLev& L0 = H->L[0];
        info->levels = (int)H->L.size();
        const unsigned nb = nodal::nblocks(L0.size);
        // the caller's arrays into the colour-split level arrays
        HIPCHK(hipMemsetAsync(H->u[0].p, 0, L0.alloc * sizeof(double), s));
        HIPCHK(hipMemsetAsync(H->f[0].p, 0, L0.alloc * sizeof(double), s));
        hipLaunchKernelGGL(nodal::k_nd_convert<true>, dim3(nb), dim3(nodal::kNB), 0, s, L0, phi, H->u[0].p);
        hipLaunchKernelGGL(nodal::k_nd_convert<true>, dim3(nb), dim3(nodal::kNB), 0, s, L0, (double*)rhs, H->f[0].p);
        HIPCHK(hipGetLastError());
        const int kr0 = nodal::plane_depth(L0, true, nodal::kKZr);
        // norms reduced on the device and read back: of f (fonly) or of the
        // residual of the current iterate
        auto norms = [&](bool fonly, double out[3]) {
            if (fonly)
                hipLaunchKernelGGL(nodal::k_nd_fnorm, dim3(nb), dim3(nodal::kNB), 0, s, L0, H->f[0].p, H->part.p);
            else
                hipLaunchKernelGGL(nodal::k_nd_resid, nodal::plane_grid(L0, true, kr0), dim3(nodal::kNB), 0, s, L0,
                                   H->u[0].p, H->f[0].p, H->r[0].p, H->part.p, kr0);
            HIPCHK(hipGetLastError());
            HIPCHK(launch_norm_final(s, H->part.p, fonly ? (int)nb : nodal::plane_blocks(L0, true, kr0), H->fn.p));
            HIPCHK(hipMemcpyAsync(ctx->h_norm, H->fn.p, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            out[0] = ctx->h_norm[2] > 0.0 ? (double)NAN : ctx->h_norm[0];
            out[1] = ctx->h_norm[1];
            out[2] = ctx->h_norm[2];
        };
        double fz[3];
        norms(true, fz);
        const double fnorm = fz[0];
        info->f_inf = fnorm;
        int status = 0, cyc = 0;
        if (!(fnorm == fnorm)) {
            status = BXMG_ENONFINITE;
        } else if (fnorm > 0.0) {
            for (;; ++cyc) {
                double rn[3];
                norms(false, rn);
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
                nodal::vcycle(*H, 0, s, P.nu1, P.nu2, P.bottom_rtol);
            }
        } else {
            HIPCHK(hipMemsetAsync(H->u[0].p, 0, L0.alloc * sizeof(double), s));  // f == 0: u = 0
        }
        info->cycles = cyc;
        if (status == 0) {
            if (L0.per[0] && L0.per[1] && L0.per[2]) {
                hipLaunchKernelGGL(nodal::k_nd_sum, dim3(nb), dim3(nodal::kNB), 0, s, L0, H->u[0].p, H->part.p);
                hipLaunchKernelGGL(nodal::k_nd_sub, dim3(nb), dim3(nodal::kNB), 0, s, L0, H->u[0].p, H->part.p,
                                   (int)nb);
            }
            hipLaunchKernelGGL(nodal::k_nd_copies, dim3(nodal::nblocks(L0.size)), dim3(nodal::kNB), 0, s, L0,
                               H->u[0].p);
            HIPCHK(hipGetLastError());
            hipLaunchKernelGGL(nodal::k_nd_convert<false>, dim3(nb), dim3(nodal::kNB), 0, s, L0, phi, H->u[0].p);
            HIPCHK(hipGetLastError());
        }
        HIPCHK(hipStreamSynchronize(s));
        info->status = status;
        if (status == BXMG_ENOCONV) fail(BXMG_ENOCONV, "nodal_solve: max_cycles reached");
        if (status == BXMG_ENONFINITE) fail(BXMG_ENONFINITE, "nodal_solve: non-finite values");
    } catch (HipError& e) {
        info->status = fail(BXMG_EDEVICE, std::string("nodal_solve: ") + e.where + ": " + hipGetErrorString(e.e));
    } catch (std::exception& e) {
        info->status = fail(BXMG_EINVAL, std::string("nodal_solve: ") + e.what());
    }
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return (bxmg_status)info->status;
}
