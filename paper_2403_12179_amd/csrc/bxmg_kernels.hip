// HIP kernels of the multigrid path, written for gfx950 (wave64, 256 CUs in
// 8 XCDs).
//
// Every stage is one fused launch over all boxes of a level (the fused
// multi-box launch of the paper, Section 3.2): the host cuts each box into
// tiles and one block works one tile, so 512 boxes of 32^3 run as one grid,
// like one 256^3 box.  A block reads its tile descriptor once; threads find
// their cells with shifts and masks only, and walk ZC planes in z.  Blocks
// are dispatched round-robin over the 8 XCDs, so the block -> tile map gives
// each XCD a contiguous run of tiles: neighbouring tiles then share that
// XCD's L2 for their halo rows.
//
// Level data uses a colour-split ("red-black") layout: the cells of one
// colour of a box row are contiguous, so a half-sweep streams only the colour
// it reads (the other one) plus the right-hand side of the colour it writes,
// 1.5 arrays per half-sweep.  All stages are bandwidth-bound (<= 0.5 flop per
// byte): no matrix cores.
//
// Floating point: built with -ffp-contract=off; every expression below
// fixes its operation order, so results are reproducible run to run.
#include <hip/hip_runtime.h>
#include <type_traits>

#include <algorithm>

#include "bxmg_internal.h"

#include <mutex>

namespace bxmg {

// ----------------------------------------------------------------- helpers
// The tag holding region cell g: the last tag whose prefix is <= g.  With
// hints (the tag of the first cell of every block of kBlock cells, plus
// ntags - 1 at the end) the search starts from the block's own range.
__device__ __forceinline__ int find_tag(const Tag* __restrict__ t, int n, long long g,
                                        const int* __restrict__ hints = nullptr) {
    int lo = 0, hi = n - 1;
    if (hints) {
        lo = hints[blockIdx.x];
        hi = hints[blockIdx.x + 1];
    }
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (t[mid].prefix <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Region coordinates of cell loc of tag t (32-bit divisions when they fit).
__device__ __forceinline__ void tag_xyz(const Tag& t, long long loc, int& x, int& y, int& z) {
    if (loc < 0x7fffffffLL) {
        const unsigned l = (unsigned)loc, n0 = (unsigned)t.n[0], n1 = (unsigned)t.n[1];
        const unsigned q = l / n0;
        x = (int)(l - q * n0);
        y = (int)(q % n1);
        z = (int)(q / n1);
    } else {
        x = (int)(loc % t.n[0]);
        y = (int)((loc / t.n[0]) % t.n[1]);
        z = (int)(loc / ((long long)t.n[0] * t.n[1]));
    }
}

__device__ __forceinline__ long long rb_row(const RBox& b, int c, int j, int k) {
    return b.base + (long long)c * b.cstride + ((long long)(k - b.glo[2]) * b.G[1] + (j - b.glo[1])) * b.H;
}

__device__ __forceinline__ long long rb_idx(const RBox& b, int i, int j, int k) {
    return rb_row(b, (i + j + k) & 1, j, k) + ((i - b.glo[0]) >> 1);
}

// rb_idx relative to the box start, 32-bit (boxes small enough for buffer addressing)
__device__ __forceinline__ int rb_off(const RBox& B, int i, int j, int k) {
    return ((i + j + k) & 1) * (int)B.cstride + ((k - B.glo[2]) * B.G[1] + (j - B.glo[1])) * B.H + ((i - B.glo[0]) >> 1);
}

__device__ __forceinline__ long long fab_idx(const FBox& b, int i, int j, int k) {
    return b.base + (long long)(i - b.glo[0]) + (long long)b.G[0] * ((long long)(j - b.glo[1]) + (long long)b.G[1] * (k - b.glo[2]));
}

template <class T>
__device__ __forceinline__ T harm(T a, T b) {
    return (a * b) * T(2) / (a + b);
}

// alpha h^2: the Helmholtz term's addition to the stencil's diagonal weight
// sb (an exact zero for Poisson)
template <class T>
__device__ __forceinline__ T diag_shift(const RBox& B) {
    return (T)(B.a * (B.h * B.h));
}

// Block -> tile: XCD x (= block % 8) receives tiles [x*n/8, (x+1)*n/8),
// walked upwards, or downwards when rev != 0.  Consecutive launches over a
// level alternate the direction, so each starts on the data the previous
// one touched last, while it is still in the memory-side cache.
__device__ __forceinline__ int tile_index(int rev) {
    const int nb = gridDim.x, b = blockIdx.x;
    if ((nb & 7) == 0) {
        const int per = nb >> 3, q = b >> 3;
        return (b & 7) * per + (rev ? per - 1 - q : q);
    }
    return rev ? nb - 1 - b : b;
}

struct TileThread {
    int x, y, z0, dz;  // box-relative x and y, first z and z step
};

__device__ __forceinline__ TileThread tile_thread(const Tile& tl) {
    const int tid = threadIdx.x;
    TileThread r;
    r.x = tl.x0 + (tid & ((1 << tl.lx) - 1));
    r.y = tl.y0 + ((tid >> tl.lx) & ((1 << tl.ly) - 1));
    r.z0 = tl.z0 + (tid >> (tl.lx + tl.ly));
    r.dz = 1 << tl.lz;
    return r;
}

// x index of the colour-c cell number t of row (j, k) of box B
__device__ __forceinline__ int colour_i(const RBox& B, int t, int j, int k, int c) {
    return B.lo[0] + 2 * t + ((c - B.lo[0] - j - k) & 1);
}

// Stencil sums of one cell: su = sum_faces beta*u_nb, sb = sum_faces beta,
// in the fixed order ((x- + x+) + (y- + y+)) + (z- + z+).  Neighbours across
// a box face are read from the box's ghost cells.
//   MODE 0: constant coefficient; 1: level 0, faces = harmonic means of the
//   cell beta (same layout as u); 2: coarse level, global face arrays.
// The stencil is split into gather (every load of one cell) and sums (the
// arithmetic), so kernels can issue the loads of several cells before any
// arithmetic or store: more memory requests in flight per thread.
template <class T>
struct Nbr {
    T xm, xp, ym, yp, zm, zp;        // u at the 6 face neighbours
    T c;                             // u at the cell (if gathered)
    T bxm, bxp, bym, byp, bzm, bzp;  // MODE 1: beta at the neighbours; MODE 2: face coefficients
    T bc;                            // MODE 1: beta at the cell
};

// Loads of cell (i,j,k); returns its element index.  CENTRE: also u there.
// skip_zm: the z- neighbour (u, and cell beta in MODE 1) is already in n
// (carried from the plane below by a thread walking planes 2 apart).
template <class T, int MODE, bool CENTRE>
__device__ __forceinline__ long long gather(const T* __restrict__ u, const T* __restrict__ beta,
                                            const FaceArrays<T>& fa, const RBox& B, int i, int j, int k, Nbr<T>& n,
                                            bool skip_zm = false) {
    const int c = (i + j + k) & 1;
    const long long rc = rb_row(B, c, j, k);
    const long long ro = rb_row(B, c ^ 1, j, k);
    const long long Hy = B.H, Hz = (long long)B.H * B.G[1];
    const int m = (i - B.glo[0]) >> 1;
    const int mxm = (i - 1 - B.glo[0]) >> 1, mxp = (i + 1 - B.glo[0]) >> 1;
    const long long idx = rc + m;
    n.xm = u[ro + mxm];
    n.xp = u[ro + mxp];
    n.ym = u[ro - Hy + m];
    n.yp = u[ro + Hy + m];
    if (!skip_zm) n.zm = u[ro - Hz + m];
    n.zp = u[ro + Hz + m];
    if constexpr (CENTRE) n.c = u[idx];
    if constexpr (MODE == 1) {
        n.bc = beta[idx];
        n.bxm = beta[ro + mxm];
        n.bxp = beta[ro + mxp];
        n.bym = beta[ro - Hy + m];
        n.byp = beta[ro + Hy + m];
        if (!skip_zm) n.bzm = beta[ro - Hz + m];
        n.bzp = beta[ro + Hz + m];
    } else if constexpr (MODE == 2) {
        const int x = i - fa.dlo[0], y = j - fa.dlo[1], z = k - fa.dlo[2];
        const int nx = fa.n[0], ny = fa.n[1];
        const long long ix = (long long)x + (long long)(nx + 1) * ((long long)y + (long long)ny * z);
        const long long iy = (long long)x + (long long)nx * ((long long)y + (long long)(ny + 1) * z);
        const long long iz = (long long)x + (long long)nx * ((long long)y + (long long)ny * z);
        n.bxm = fa.c[0][ix];
        n.bxp = fa.c[0][ix + 1];
        n.bym = fa.c[1][iy];
        n.byp = fa.c[1][iy + nx];
        n.bzm = fa.c[2][iz];
        n.bzp = fa.c[2][iz + (long long)nx * ny];
    }
    return idx;
}

// su = sum_faces beta*u_nb, sb = sum_faces beta, each in the fixed order
// ((x- + x+) + (y- + y+)) + (z- + z+).
//   MODE 0: constant coefficient; 1: level 0, faces = harmonic means of the
//   cell beta (same layout as u); 2: coarse level, global face arrays.
template <class T, int MODE>
__device__ __forceinline__ void sums(const Nbr<T>& n, T& su, T& sb) {
    if constexpr (MODE == 0) {
        su = ((n.xm + n.xp) + (n.ym + n.yp)) + (n.zm + n.zp);
        sb = T(6);
    } else {
        T bxm, bxp, bym, byp, bzm, bzp;
        if constexpr (MODE == 1) {
            bxm = harm(n.bxm, n.bc);
            bxp = harm(n.bc, n.bxp);
            bym = harm(n.bym, n.bc);
            byp = harm(n.bc, n.byp);
            bzm = harm(n.bzm, n.bc);
            bzp = harm(n.bc, n.bzp);
        } else {
            bxm = n.bxm;
            bxp = n.bxp;
            bym = n.bym;
            byp = n.byp;
            bzm = n.bzm;
            bzp = n.bzp;
        }
        sb = ((bxm + bxp) + (bym + byp)) + (bzm + bzp);
        su = ((bxm * n.xm + bxp * n.xp) + (bym * n.ym + byp * n.yp)) + (bzm * n.zm + bzp * n.zp);
    }
}

// Stencil sums of one cell: neighbours across a box face are read from the
// box's ghost cells.
template <class T, int MODE>
__device__ __forceinline__ void stencil(const T* __restrict__ u, const T* __restrict__ beta, const FaceArrays<T>& fa,
                                        const RBox& B, int i, int j, int k, T& su, T& sb, T& uc, long long& idx) {
    Nbr<T> n;
    idx = gather<T, MODE, true>(u, beta, fa, B, i, j, k, n);
    uc = n.c;
    sums<T, MODE>(n, su, sb);
    sb = sb + diag_shift<T>(B);
}

// Raw-buffer access to the colour blocks of one box: a resource descriptor
// (box start, size) in scalar registers and 32-bit offsets per lane, instead
// of 64-bit addresses.  The hardware bounds-checks every access against the
// box: a read past its end returns 0 and a write there is dropped.
constexpr int kBufferDword3 = 0x00020000;  // raw buffer, gfx9 data format
// A byte offset beyond every box resource (their sizes stay below 2^31 bytes).
constexpr int kOffPastBox = (int)0x80000000u;

template <class T>
struct BoxRes;

template <>
struct BoxRes<double> {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ BoxRes(const double* base, long long nelem)
        : r(__builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(nelem * 8), kBufferDword3)) {}
    __device__ __forceinline__ double ld(int e) const {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, e * 8, 0, 0));
    }
    // element e, or (skip) an offset past every box: the hardware returns 0
    // without a memory access, so the load needs no branch around it
    __device__ __forceinline__ double ld_unless(int e, bool skip) const {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, skip ? kOffPastBox : e * 8, 0, 0));
    }
    __device__ __forceinline__ void st(int e, double v) const {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, e * 8, 0, 0);
    }
};

template <>
struct BoxRes<float> {
    __amdgpu_buffer_rsrc_t r;
    __device__ __forceinline__ BoxRes(const float* base, long long nelem)
        : r(__builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(nelem * 4), kBufferDword3)) {}
    __device__ __forceinline__ float ld(int e) const {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, e * 4, 0, 0));
    }
    __device__ __forceinline__ float ld_unless(int e, bool skip) const {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, skip ? kOffPastBox : e * 4, 0, 0));
    }
    __device__ __forceinline__ void st(int e, float v) const {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, e * 4, 0, 0);
    }
};

// gather() through box resources; offsets relative to the box start
template <class T, int MODE, bool CENTRE>
__device__ __forceinline__ int gather_res(const BoxRes<T>& U, const BoxRes<T>& Bt, const FaceArrays<T>& fa,
                                          const RBox& B, int i, int j, int k, Nbr<T>& n, bool skip_zm = false,
                                          const BoxRes<T>* F = nullptr, T* fv = nullptr, int* nbo = nullptr) {
    const int c = (i + j + k) & 1;
    const int row = ((k - B.glo[2]) * B.G[1] + (j - B.glo[1])) * B.H;
    const int cs = (int)B.cstride;
    const int rc = c * cs + row, ro = (c ^ 1) * cs + row;
    const int Hy = B.H, Hz = B.H * B.G[1];
    const int m = (i - B.glo[0]) >> 1;
    const int mxm = (i - 1 - B.glo[0]) >> 1, mxp = (i + 1 - B.glo[0]) >> 1;
    const int idx = rc + m;
    if (F) *fv = F->ld(idx);  // first, so every load of the cell leaves together
    n.xm = U.ld(ro + mxm);
    n.xp = U.ld(ro + mxp);
    n.ym = U.ld(ro - Hy + m);
    n.yp = U.ld(ro + Hy + m);
    // branch-free: a branch here would make the wave wait for every load
    // issued so far before issuing the rest
    const T zm = U.ld_unless(ro - Hz + m, skip_zm);
    n.zp = U.ld(ro + Hz + m);
    if constexpr (CENTRE) n.c = U.ld(idx);
    if constexpr (MODE == 1) {
        n.bc = Bt.ld(idx);
        n.bxm = Bt.ld(ro + mxm);
        n.bxp = Bt.ld(ro + mxp);
        n.bym = Bt.ld(ro - Hy + m);
        n.byp = Bt.ld(ro + Hy + m);
        const T bzm = Bt.ld_unless(ro - Hz + m, skip_zm);
        n.bzm = skip_zm ? n.bzm : bzm;
        n.bzp = Bt.ld(ro + Hz + m);
    } else if constexpr (MODE == 2) {
        const int x = i - fa.dlo[0], y = j - fa.dlo[1], z = k - fa.dlo[2];
        const int nx = fa.n[0], ny = fa.n[1];
        const long long ix = (long long)x + (long long)(nx + 1) * ((long long)y + (long long)ny * z);
        const long long iy = (long long)x + (long long)nx * ((long long)y + (long long)(ny + 1) * z);
        const long long iz = (long long)x + (long long)nx * ((long long)y + (long long)ny * z);
        n.bxm = fa.c[0][ix];
        n.bxp = fa.c[0][ix + 1];
        n.bym = fa.c[1][iy];
        n.byp = fa.c[1][iy + nx];
        n.bzm = fa.c[2][iz];
        n.bzp = fa.c[2][iz + (long long)nx * ny];
    }
    n.zm = skip_zm ? n.zm : zm;
    if (nbo) {  // the 6 neighbours' offsets, x-, x+, y-, y+, z-, z+ (face order)
        nbo[0] = ro + mxm;
        nbo[1] = ro + mxp;
        nbo[2] = ro - Hy + m;
        nbo[3] = ro + Hy + m;
        nbo[4] = ro - Hz + m;
        nbo[5] = ro + Hz + m;
    }
    return idx;
}


// Ghost exchange fused into a producer: cell (i,j,k) of box B just took value
// v; write v into every face ghost cell that mirrors it -- the ghost of the
// neighbouring box across each face the cell lies on (periodic images
// included) and, across a homogeneous-Dirichlet domain face, -v into the
// box's own ghost beyond it.  Exactly the values a ghost refresh would copy.
template <class T>
__device__ __forceinline__ void push_ghosts(T* __restrict__ u, const RBox* __restrict__ boxes, const RBox& B, int i,
                                            int j, int k, T v) {
    const int c[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            if (c[d] != (side ? B.hi[d] : B.lo[d])) continue;
            const int q = 2 * d + side;
            const int nb = B.nb[q];
            int t[3] = {i, j, k};
            if (nb >= 0) {
                t[d] += B.shift[q];
                u[rb_idx(boxes[nb], t[0], t[1], t[2])] = v;
            } else {
                t[d] += side ? 1 : -1;
                u[rb_idx(B, t[0], t[1], t[2])] = -v;
            }
        }
}

// The face ghost cells that mirror cell (i,j,k) of box B (the targets of
// push_ghosts), set to +0: with the cell zeroed, what a ghost refresh would
// leave there, except that a Dirichlet ghost gets +0 rather than -0, as a
// zeroed level holds everywhere.
template <class T>
__device__ __forceinline__ void zero_ghosts(T* __restrict__ u, const RBox* __restrict__ boxes, const RBox& B, int i,
                                            int j, int k) {
    const int c[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            if (c[d] != (side ? B.hi[d] : B.lo[d])) continue;
            const int q = 2 * d + side;
            const int nb = B.nb[q];
            int t[3] = {i, j, k};
            if (nb >= 0) {
                t[d] += B.shift[q];
                u[rb_idx(boxes[nb], t[0], t[1], t[2])] = T(0);
            } else {
                t[d] += side ? 1 : -1;
                u[rb_idx(B, t[0], t[1], t[2])] = T(0);
            }
        }
}

// Fixed-tree block reduction of (max, sum, sum): wave64 butterflies, then
// the 4 wave results in order.  The result is valid in thread 0.
__device__ __forceinline__ void block_reduce3(double& mx, double& s2, double& bad, double* sh) {
    for (int o = 32; o > 0; o >>= 1) {
        const double a = __shfl_xor(mx, o), b = __shfl_xor(s2, o), c = __shfl_xor(bad, o);
        mx = fmax(mx, a);
        s2 = s2 + b;
        bad = bad + c;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { sh[3 * wid] = mx; sh[3 * wid + 1] = s2; sh[3 * wid + 2] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        mx = sh[0]; s2 = sh[1]; bad = sh[2];
        for (int w = 1; w < nw; ++w) { mx = fmax(mx, sh[3 * w]); s2 = s2 + sh[3 * w + 1]; bad = bad + sh[3 * w + 2]; }
    }
}

__device__ __forceinline__ void acc_norm(double rv, double& mx, double& s2, double& bad) {
    const double a = fabs(rv);
    if (!(a <= 1.7976931348623157e308)) bad += 1.0;  // NaN or Inf
    else mx = fmax(mx, a);
    s2 = s2 + rv * rv;
}

// -------------------------------------------------------------- ghost fill
// Level ghost cells: one precomputed (dst, src) pair per cell.
template <class T>
__global__ void __launch_bounds__(kBlock) k_fill_rb(T* __restrict__ data, const GhostCopy* __restrict__ list, long long n,
                                                   const int* __restrict__ active) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n || (active && !active[0])) return;
    const GhostCopy p = list[g];
    const T v = data[p.src & 0x7fffffffu];
    data[p.dst] = (p.src >> 31) ? -v : v;
}

// Caller MultiFabs (F-order, several components): region tags.
template <class T>
__global__ void __launch_bounds__(kBlock) k_fill_fab(T* __restrict__ data, const FBox* __restrict__ boxes,
                                                    const Tag* __restrict__ tags, int ntags, long long ncells,
                                                    int comp0, int ncomp, const int* __restrict__ hints) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    auto cell = [&](const Tag& t) {
        int x, y, z;
        tag_xyz(t, g - t.prefix, x, y, z);
        const int di = t.dlo[0] + x, dj = t.dlo[1] + y, dk = t.dlo[2] + z;
        const int si = t.sgn[0] * di + t.soff[0], sj = t.sgn[1] * dj + t.soff[1], sk = t.sgn[2] * dk + t.soff[2];
        const FBox sb = boxes[t.sbox], db = boxes[t.dbox];
        const long long s0 = fab_idx(sb, si, sj, sk), d0 = fab_idx(db, di, dj, dk);
        for (int n = comp0; n < comp0 + ncomp; ++n) {
            T v = data[s0 + n * sb.cs];
            if (t.neg) v = -v;
            data[d0 + n * db.cs] = v;
        }
    };
    // a block inside one region: its tag and boxes are the same for every
    // lane (scalar loads)
    if (hints && hints[blockIdx.x] == hints[blockIdx.x + 1]) {
        const Tag t = tags[hints[blockIdx.x]];
        if (g < ncells) cell(t);
        return;
    }
    if (g >= ncells) return;
    cell(tags[find_tag(tags, ntags, g, hints)]);
}

// ParallelCopy: region tags between two MultiFabs (destination box dbox,
// source box sbox, source cell = dst cell + soff), components
// [scomp, scomp+n) into [dcomp, dcomp+n).
template <class T>
__global__ void __launch_bounds__(kBlock) k_copy_fab(T* __restrict__ dst, const FBox* __restrict__ dboxes,
                                                    const T* __restrict__ src, const FBox* __restrict__ sboxes,
                                                    const Tag* __restrict__ tags, int ntags, long long ncells,
                                                    int dcomp, int scomp, int ncomp, const int* __restrict__ hints) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    auto cell = [&](const Tag& t) {
        int x, y, z;
        tag_xyz(t, g - t.prefix, x, y, z);
        const int di = t.dlo[0] + x, dj = t.dlo[1] + y, dk = t.dlo[2] + z;
        const FBox sb = sboxes[t.sbox], db = dboxes[t.dbox];
        const long long s0 = fab_idx(sb, di + t.soff[0], dj + t.soff[1], dk + t.soff[2]), d0 = fab_idx(db, di, dj, dk);
        for (int n = 0; n < ncomp; ++n) dst[d0 + (dcomp + n) * db.cs] = src[s0 + (scomp + n) * sb.cs];
    };
    if (hints && hints[blockIdx.x] == hints[blockIdx.x + 1]) {
        const Tag t = tags[hints[blockIdx.x]];
        if (g < ncells) cell(t);
        return;
    }
    if (g >= ncells) return;
    cell(tags[find_tag(tags, ntags, g, hints)]);
}

// push_ghosts() on a one-box level addressed through its buffer resource: a
// face neighbour >= 0 is the box itself (its periodic image, the cell
// shifted by the period), and across a Dirichlet face the ghost to write is
// the neighbour the stencil just read, whose offset nbo[face] is at hand.
template <class T>
__device__ __forceinline__ void push_self(const BoxRes<T>& U, const RBox& B, int i, int j, int k, T v,
                                          const int* nbo) {
    const int c[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            if (c[d] != (side ? B.hi[d] : B.lo[d])) continue;
            const int q = 2 * d + side;
            if (B.nb[q] >= 0) {
                int t[3] = {i, j, k};
                t[d] += B.shift[q];
                U.st(rb_off(B, t[0], t[1], t[2]), v);
            } else {
                U.st(nbo[q], -v);
            }
        }
}

// Whether cell (i,j,k) of a pushing level lies on a face of its box that is
// a homogeneous-Dirichlet domain face (no neighbour box there).
__device__ __forceinline__ bool on_dirichlet_face(const RBox& B, int i, int j, int k) {
    return (i == B.lo[0] && B.nb[0] < 0) || (i == B.hi[0] && B.nb[1] < 0) || (j == B.lo[1] && B.nb[2] < 0) ||
           (j == B.hi[1] && B.nb[3] < 0) || (k == B.lo[2] && B.nb[4] < 0) || (k == B.hi[2] && B.nb[5] < 0);
}

// The neighbour values of cell (i,j,k) that are its own ghosts beyond a
// Dirichlet face (they mirror the cell itself), set to g.
template <class T>
__device__ __forceinline__ void dirichlet_self(const RBox& B, int i, int j, int k, T g, Nbr<T>& n) {
    if (i == B.lo[0] && B.nb[0] < 0) n.xm = g;
    if (i == B.hi[0] && B.nb[1] < 0) n.xp = g;
    if (j == B.lo[1] && B.nb[2] < 0) n.ym = g;
    if (j == B.hi[1] && B.nb[3] < 0) n.yp = g;
    if (k == B.lo[2] && B.nb[4] < 0) n.zm = g;
    if (k == B.hi[2] && B.nb[5] < 0) n.zp = g;
}

// ---------------------------------------------------- red-black smoothing
// One colour: u_c = (su - h^2 f) / sb.  Reads only the other colour of u.
// NORM: also the residual f - (su - sb u_c) / h^2 of each updated cell, in
// norms per tile (partials[3 tile] = max |r|, sum r^2, non-finite count):
// after the last colour-1 sweep of a V-cycle the colour-0 cells it read are
// final.  A cell on a Dirichlet face read its own ghost before this sweep
// refreshed it; its residual is formed again with the refreshed ghost, so
// every value is bitwise what k_resid computes for the stored iterate.
// PUSH: 0 none; 1 push_ghosts; 2 push_self (one-box level, RES).
template <class T, int MODE, int PUSH, bool RES, bool NORM>
__global__ void __launch_bounds__(kBlock) k_gs(Grid g, T* __restrict__ u, const T* __restrict__ f,
                                              const T* __restrict__ beta, const FaceArrays<T>* __restrict__ fat,
                                              int colour, double* __restrict__ partials) {
    __shared__ double sh[NORM ? 3 * (kBlock / 64) : 1];
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    const int tix = tile_index(g.rev);
    const Tile tl = g.tiles[tix];
    const RBox B = g.boxes[tl.box];
    if (g.active && !g.active[B.pid]) return;  // the whole workgroup
    FaceArrays<T> fa;
    if constexpr (MODE == 2) fa = fat[B.pid];
    const T h2 = (T)(B.h * B.h);
    const T ih2 = (T)(1.0 / (B.h * B.h));
    const T dg = diag_shift<T>(B);
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    const long long ne = 2 * B.cstride;
    const BoxRes<T> U(u + B.base, ne), F(f + B.base, ne), Bt((MODE == 1 ? beta : f) + B.base, ne);
    if (j <= B.hi[1]) {
        // Walking planes 2 apart, a thread's cell keeps its x position (same
        // colour parity), so the z+ neighbour of one plane is the z- neighbour
        // of the next: kept in registers instead of loaded again (one load of seven).
        const bool walk2 = th.dz == 2;
        T carry_u = T(0), carry_b = T(0);
        bool carry = false;
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int k = B.lo[2] + th.z0 + z * th.dz;
            const int i = colour_i(B, th.x, j, k, colour);
            if (k > B.hi[2]) break;
            if (i > B.hi[0]) {  // only where the walk changes the cell's parity
                carry = false;
                continue;
            }
            Nbr<T> nb;
            nb.zm = carry_u;
            nb.bzm = carry_b;
            long long idx;
            T fv;
            int nbo[6];
            if constexpr (RES) {
                idx = gather_res<T, MODE, false>(U, Bt, fa, B, i, j, k, nb, carry, &F, &fv, PUSH == 2 ? nbo : nullptr);
            } else {
                idx = gather<T, MODE, false>(u, beta, fa, B, i, j, k, nb, carry);
                fv = f[idx];
            }
            T su, sb;
            sums<T, MODE>(nb, su, sb);
            sb = sb + dg;
            const T v = (su - h2 * fv) / sb;
            if constexpr (RES) U.st((int)idx, v);
            else u[idx] = v;
            if constexpr (PUSH == 1) push_ghosts(u, g.boxes, B, i, j, k, v);
            if constexpr (PUSH == 2) push_self(U, B, i, j, k, v, nbo);
            if constexpr (NORM) {
                // su read the ghost beyond a Dirichlet face before the push
                // replaced it (-u_old -> -v); the residual of the stored
                // iterate takes the refreshed value, summed in the same order
                T sr = su;
                if (on_dirichlet_face(B, i, j, k)) {
                    Nbr<T> nr = nb;
                    dirichlet_self(B, i, j, k, -v, nr);
                    T sbr;
                    sums<T, MODE>(nr, sr, sbr);
                }
                acc_norm((double)(fv - (sr - sb * v) * ih2), mx, s2, bad);
            }
            carry = walk2;
            carry_u = nb.zp;
            if constexpr (MODE == 1) carry_b = nb.bzp;
        }
    }
    if constexpr (NORM) {
        block_reduce3(mx, s2, bad, sh);
        if (threadIdx.x == 0) {
            partials[3 * tix] = mx;
            partials[3 * tix + 1] = s2;
            partials[3 * tix + 2] = bad;
        }
    }
}

// ---------------------------------------------------------------- residual
// r = f - (su - sb u) / h^2 on both colours; optional store of r (same type
// and layout) or of float(r) (mixed precision); fused norms per block.
// COLS: bit c set = colour c's cells (3: all; 1: colour 0 only, when a
// fused colour-1 sweep has taken the colour-1 residuals).
template <class T, int MODE, class R, bool RES, int COLS>
__global__ void __launch_bounds__(kBlock) k_resid(Grid g, const T* __restrict__ u, const T* __restrict__ f,
                                                 const T* __restrict__ beta, const FaceArrays<T>* __restrict__ fat,
                                                 R* __restrict__ r, double* __restrict__ partials,
                                                 const int* __restrict__ nonzero) {
    __shared__ double sh[3 * (kBlock / 64)];
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    const int tix = tile_index(g.rev);
    const Tile tl = g.tiles[tix];
    const RBox B = g.boxes[tl.box];
    if (g.active && !g.active[B.pid]) return;
    FaceArrays<T> fa;
    if constexpr (MODE == 2) fa = fat[B.pid];
    const T ih2 = (T)(1.0 / (B.h * B.h));
    const T dg = diag_shift<T>(B);
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    const long long ne = 2 * B.cstride;
    const BoxRes<T> U(u + B.base, ne), F(f + B.base, ne), Bt((MODE == 1 ? beta : f) + B.base, ne);
    const BoxRes<R> Rr(r ? r + B.base : (R*)nullptr, r ? ne : 0);
    // a guess that is +0.0 everywhere (constant coefficient; one flag per
    // problem): the stencil sums are exactly +0.0, so the residual is f
    // itself and u need not be read -- the same values, norms and stores as
    // the full path
    const bool zero_guess = MODE == 0 && RES && nonzero && nonzero[B.pid] == 0;
    if (j <= B.hi[1]) {
        // z+ of one plane is z- of the next when walking planes 2 apart (see k_gs)
        const bool walk2 = th.dz == 2;
        T carry_u[2] = {T(0), T(0)}, carry_b[2] = {T(0), T(0)};
        bool carry[2] = {false, false};
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int k = B.lo[2] + th.z0 + z * th.dz;
            if (k > B.hi[2]) break;
            Nbr<T> nb[2];
            T fv[2];
            long long idx[2];
            bool ok[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int i = colour_i(B, th.x, j, k, c);
                ok[c] = i <= B.hi[0] && ((COLS >> c) & 1);
                if (!((COLS >> c) & 1)) continue;
                nb[c].zm = carry_u[c];
                nb[c].bzm = carry_b[c];
                if constexpr (RES) {
                    if (zero_guess) {
                        const int ic = ok[c] ? i : B.hi[0];
                        idx[c] = rb_off(B, ic, j, k);
                        fv[c] = F.ld((int)idx[c]);
                        nb[c].xm = nb[c].xp = nb[c].ym = nb[c].yp = nb[c].zm = nb[c].zp = nb[c].c = T(0);
                    } else {
                        // without a branch: a missing cell (odd row length)
                        // gathers the row's last cell, and its result is unused
                        idx[c] = gather_res<T, MODE, true>(U, Bt, fa, B, ok[c] ? i : B.hi[0], j, k, nb[c],
                                                           carry[c] && ok[c], &F, &fv[c]);
                    }
                } else if (ok[c]) {
                    idx[c] = gather<T, MODE, true>(u, beta, fa, B, i, j, k, nb[c], carry[c]);
                    fv[c] = f[idx[c]];
                }
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (!((COLS >> c) & 1)) continue;
                carry[c] = walk2 && ok[c];
                carry_u[c] = nb[c].zp;
                if constexpr (MODE == 1) carry_b[c] = nb[c].bzp;
                if (!ok[c]) continue;
                T su, sb;
                sums<T, MODE>(nb[c], su, sb);
                sb = sb + dg;
                const T rv = fv[c] - (su - sb * nb[c].c) * ih2;
                if (r) {
                    if constexpr (RES) Rr.st((int)idx[c], (R)rv);
                    else r[idx[c]] = (R)rv;
                }
                acc_norm((double)rv, mx, s2, bad);
            }
        }
    }
    block_reduce3(mx, s2, bad, sh);
    if (threadIdx.x == 0) {
        partials[3 * tix] = mx;
        partials[3 * tix + 1] = s2;
        partials[3 * tix + 2] = bad;
    }
}

// One workgroup of kNormThreads; each thread issues the loads of kNormUnroll
// partials before adding them (the reduction is latency-bound), in a fixed
// order, so the result does not depend on timing.
constexpr int kNormThreads = 1024, kNormUnroll = 4;
// The reduction of k_norm_final, for a workgroup of kNormThreads.
__device__ __forceinline__ void norm_reduce(const double* __restrict__ partials, int n, double* sh, double& mx,
                                            double& s2, double& bad) {
    mx = 0.0;
    s2 = 0.0;
    bad = 0.0;
    for (int q0 = threadIdx.x; q0 < n; q0 += kNormUnroll * kNormThreads) {
        double a[kNormUnroll][3];
#pragma unroll
        for (int v = 0; v < kNormUnroll; ++v) {
            const int q = q0 + v * kNormThreads;
            const bool in = q < n;
#pragma unroll
            for (int c = 0; c < 3; ++c) a[v][c] = in ? partials[3 * (long long)q + c] : 0.0;
        }
#pragma unroll
        for (int v = 0; v < kNormUnroll; ++v) {
            mx = fmax(mx, a[v][0]);
            s2 = s2 + a[v][1];
            bad = bad + a[v][2];
        }
    }
    block_reduce3(mx, s2, bad, sh);
}

__global__ void __launch_bounds__(kNormThreads) k_norm_final(const double* __restrict__ partials, int n,
                                                            double* __restrict__ out) {
    __shared__ double sh[3 * (kNormThreads / 64)];
    double mx, s2, bad;
    norm_reduce(partials, n, sh, mx, s2, bad);
    if (threadIdx.x == 0) { out[0] = mx; out[1] = s2; out[2] = bad; }
}

// Norms of a field's valid cells (the right-hand side's max norm).
__global__ void __launch_bounds__(kBlock) k_field_norm(Grid g, const double* __restrict__ x,
                                                      double* __restrict__ partials) {
    __shared__ double sh[3 * (kBlock / 64)];
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    const Tile tl = g.tiles[tile_index(g.rev)];
    const RBox B = g.boxes[tl.box];
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    if (j <= B.hi[1])
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int k = B.lo[2] + th.z0 + z * th.dz;
            if (k > B.hi[2]) break;
            for (int c = 0; c < 2; ++c) {
                const int i = colour_i(B, th.x, j, k, c);
                if (i <= B.hi[0]) acc_norm(x[rb_idx(B, i, j, k)], mx, s2, bad);
            }
        }
    block_reduce3(mx, s2, bad, sh);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x] = mx;
        partials[3 * blockIdx.x + 1] = s2;
        partials[3 * blockIdx.x + 2] = bad;
    }
}

// k_fab_to_rb<double> and k_field_norm of what it writes in one pass: the
// same tiles and cell order as k_field_norm, so the same partials.
__global__ void __launch_bounds__(kBlock) k_fab_to_rb_norm(Grid g, const double* __restrict__ fab,
                                                          const FBox* __restrict__ fb, double* __restrict__ rb,
                                                          double* __restrict__ partials) {
    __shared__ double sh[3 * (kBlock / 64)];
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    const Tile tl = g.tiles[tile_index(g.rev)];
    const RBox B = g.boxes[tl.box];
    const FBox F = fb[tl.box];
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    if (j <= B.hi[1])
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int k = B.lo[2] + th.z0 + z * th.dz;
            if (k > B.hi[2]) break;
            for (int c = 0; c < 2; ++c) {
                const int i = colour_i(B, th.x, j, k, c);
                if (i > B.hi[0]) continue;
                const double v = fab[fab_idx(F, i, j, k)];
                rb[rb_idx(B, i, j, k)] = v;
                acc_norm(v, mx, s2, bad);
            }
        }
    block_reduce3(mx, s2, bad, sh);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x] = mx;
        partials[3 * blockIdx.x + 1] = s2;
        partials[3 * blockIdx.x + 2] = bad;
    }
}

// Admission of many problems: the initial guess and the right-hand side of
// every box of the launch converted into level storage, the right-hand
// side's norms per tile (k_fab_to_rb and k_fab_to_rb_norm over boxes with
// their own source arrays).
__global__ void __launch_bounds__(kBlock) k_admit_convert(Grid g, const ConvSrc* __restrict__ src,
                                                         double* __restrict__ u, double* __restrict__ f,
                                                         double* __restrict__ partials, int* __restrict__ nonzero) {
    __shared__ double sh[3 * (kBlock / 64)];
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    bool nz = false;
    const int tix = tile_index(g.rev);
    const Tile tl = g.tiles[tix];
    const RBox B = g.boxes[tl.box];
    const ConvSrc S = src[tl.box];
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    if (j <= B.hi[1])
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int k = B.lo[2] + th.z0 + z * th.dz;
            if (k > B.hi[2]) break;
            for (int c = 0; c < 2; ++c) {
                const int i = colour_i(B, th.x, j, k, c);
                if (i > B.hi[0]) continue;
                const long long o = rb_idx(B, i, j, k);
                const double w = S.phi[fab_idx(S.fphi, i, j, k)];
                u[o] = w;
                nz = nz || __double_as_longlong(w) != 0;
                const double v = S.rhs[fab_idx(S.frhs, i, j, k)];
                f[o] = v;
                acc_norm(v, mx, s2, bad);
            }
        }
    if (__any(nz) && (threadIdx.x & 63) == 0) atomicOr(&nonzero[S.slot], 1);
    block_reduce3(mx, s2, bad, sh);
    if (threadIdx.x == 0) {
        partials[3 * tix] = mx;
        partials[3 * tix + 1] = s2;
        partials[3 * tix + 2] = bad;
    }
}

// Heat-step right-hand side: f = -((u * inv_dt) + s) at every valid cell,
// written into level storage, with its norms (as k_fab_to_rb_norm).
__global__ void __launch_bounds__(kBlock) k_heat_rhs(Grid g, const double* __restrict__ u,
                                                    const FBox* __restrict__ fu, const double* __restrict__ src,
                                                    const FBox* __restrict__ fs, double inv_dt,
                                                    double* __restrict__ rb, double* __restrict__ partials) {
    __shared__ double sh[3 * (kBlock / 64)];
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    const Tile tl = g.tiles[tile_index(g.rev)];
    const RBox B = g.boxes[tl.box];
    const FBox F = fu[tl.box];
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    if (j <= B.hi[1])
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int k = B.lo[2] + th.z0 + z * th.dz;
            if (k > B.hi[2]) break;
            for (int c = 0; c < 2; ++c) {
                const int i = colour_i(B, th.x, j, k, c);
                if (i > B.hi[0]) continue;
                double t = u[fab_idx(F, i, j, k)] * inv_dt;
                if (src) t = t + src[fab_idx(fs[tl.box], i, j, k)];
                const double v = -t;
                rb[rb_idx(B, i, j, k)] = v;
                acc_norm(v, mx, s2, bad);
            }
        }
    block_reduce3(mx, s2, bad, sh);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x] = mx;
        partials[3 * blockIdx.x + 1] = s2;
        partials[3 * blockIdx.x + 2] = bad;
    }
}

// ---------------------------------------------------------- fine <-> coarse
// Coarse cell (I, J, K) of the tile's fine box, or false past its end.
struct CoarseCell {
    int I, J, K;
};

// ------------------------------------------------------ restriction (fused)
// One thread per coarse cell: the residual at its 8 children, averaged
// as ((r000 + r100) + (r010 + r110)) + ((r001 + r101) + (r011 + r111)), * 1/8.
template <class T, int MODE>
__device__ __forceinline__ T resid_at(const T* __restrict__ u, const T* __restrict__ f, const T* __restrict__ beta,
                                      const FaceArrays<T>& fa, const RBox& B, int i, int j, int k, T ih2) {
    T su, sb, uc;
    long long idx;
    stencil<T, MODE>(u, beta, fa, B, i, j, k, su, sb, uc, idx);
    return f[idx] - (su - sb * uc) * ih2;
}

// uz != nullptr: also zero the coarse level's u (the coarse correction's
// first guess) at each coarse cell written, with the face ghosts mirroring
// it -- every value of it the first coarse sweep reads (levels that push).
template <class T, int MODE>
__global__ void __launch_bounds__(kBlock) k_resid_restrict(XGrid x, const T* __restrict__ u, const T* __restrict__ f,
                                                          const T* __restrict__ beta,
                                                          const FaceArrays<T>* __restrict__ fat, T* __restrict__ fc,
                                                          T* __restrict__ uz) {
    const Tile tl = x.tiles[tile_index(x.rev)];
    const RBox B = x.fboxes[tl.box];
    if (x.active && !x.active[B.pid]) return;
    FaceArrays<T> fa;
    if constexpr (MODE == 2) fa = fat[B.pid];
    const T ih2 = (T)(1.0 / (B.h * B.h));
    const T dg = diag_shift<T>(B);
    const RBox C = x.cboxes[x.cbox[tl.box]];
    const TileThread th = tile_thread(tl);
    const int I = (B.lo[0] >> 1) + th.x, J = (B.lo[1] >> 1) + th.y;
    if (I > (B.hi[0] >> 1) || J > (B.hi[1] >> 1)) return;
    if constexpr (MODE != 2) {
        // The 8 children's stencils touch 32 distinct cells of u (and of the
        // cell beta): the 2x2x2 block and the 4 cells beyond each of its 6
        // faces.  Load each once (v[x][y][z], offsets -1..2 around the
        // block's lower corner), then form the 8 residuals as resid_at does.
        const BoxRes<T> U(u + B.base, 2 * B.cstride), F(f + B.base, 2 * B.cstride);
        const BoxRes<T> Bt((MODE == 1 ? beta : f) + B.base, 2 * B.cstride);
        const BoxRes<T> Cw(fc + C.base, 2 * C.cstride);
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int K = (B.lo[2] >> 1) + th.z0 + z * th.dz;
            if (K > (B.hi[2] >> 1)) break;
            const int i = 2 * I, j = 2 * J, k = 2 * K;
            T v[4][4][4], bv[4][4][4], fv[2][2][2];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int outer = (a == 0 || a == 3) + (b == 0 || b == 3) + (c == 0 || c == 3);
                        if (outer > 1) continue;  // edges and corners of the 4x4x4 cube are not needed
                        const int o = rb_off(B, i - 1 + a, j - 1 + b, k - 1 + c);
                        if (x.res) v[a][b][c] = U.ld(o);
                        else v[a][b][c] = u[B.base + o];
                        if constexpr (MODE == 1) {
                            if (x.res) bv[a][b][c] = Bt.ld(o);
                            else bv[a][b][c] = beta[B.base + o];
                        }
                        if (outer == 0) {
                            if (x.res) fv[a - 1][b - 1][c - 1] = F.ld(o);
                            else fv[a - 1][b - 1][c - 1] = f[B.base + o];
                        }
                    }
            T r[2][2][2];
#pragma unroll
            for (int a = 1; a <= 2; ++a)
#pragma unroll
                for (int b = 1; b <= 2; ++b)
#pragma unroll
                    for (int c = 1; c <= 2; ++c) {
                        Nbr<T> n;
                        n.xm = v[a - 1][b][c];
                        n.xp = v[a + 1][b][c];
                        n.ym = v[a][b - 1][c];
                        n.yp = v[a][b + 1][c];
                        n.zm = v[a][b][c - 1];
                        n.zp = v[a][b][c + 1];
                        n.c = v[a][b][c];
                        if constexpr (MODE == 1) {
                            n.bxm = bv[a - 1][b][c];
                            n.bxp = bv[a + 1][b][c];
                            n.bym = bv[a][b - 1][c];
                            n.byp = bv[a][b + 1][c];
                            n.bzm = bv[a][b][c - 1];
                            n.bzp = bv[a][b][c + 1];
                            n.bc = bv[a][b][c];
                        }
                        T su, sb;
                        sums<T, MODE>(n, su, sb);
                        sb = sb + dg;
                        r[a - 1][b - 1][c - 1] = fv[a - 1][b - 1][c - 1] - (su - sb * n.c) * ih2;
                    }
            const T s = ((r[0][0][0] + r[1][0][0]) + (r[0][1][0] + r[1][1][0])) +
                        ((r[0][0][1] + r[1][0][1]) + (r[0][1][1] + r[1][1][1]));
            const int oc = rb_off(C, I, J, K);
            if (x.res) Cw.st(oc, s * T(0.125));
            else fc[C.base + oc] = s * T(0.125);
            if (uz) {
                uz[C.base + oc] = T(0);
                zero_ghosts(uz, x.cboxes, C, I, J, K);
            }
        }
        return;
    }
    for (int z = 0; z < (int)tl.zc; ++z) {
        const int K = (B.lo[2] >> 1) + th.z0 + z * th.dz;
        if (K > (B.hi[2] >> 1)) break;
        const int i = 2 * I, j = 2 * J, k = 2 * K;
        const T r000 = resid_at<T, MODE>(u, f, beta, fa, B, i, j, k, ih2);
        const T r100 = resid_at<T, MODE>(u, f, beta, fa, B, i + 1, j, k, ih2);
        const T r010 = resid_at<T, MODE>(u, f, beta, fa, B, i, j + 1, k, ih2);
        const T r110 = resid_at<T, MODE>(u, f, beta, fa, B, i + 1, j + 1, k, ih2);
        const T r001 = resid_at<T, MODE>(u, f, beta, fa, B, i, j, k + 1, ih2);
        const T r101 = resid_at<T, MODE>(u, f, beta, fa, B, i + 1, j, k + 1, ih2);
        const T r011 = resid_at<T, MODE>(u, f, beta, fa, B, i, j + 1, k + 1, ih2);
        const T r111 = resid_at<T, MODE>(u, f, beta, fa, B, i + 1, j + 1, k + 1, ih2);
        const T s = ((r000 + r100) + (r010 + r110)) + ((r001 + r101) + (r011 + r111));
        fc[rb_idx(C, I, J, K)] = s * T(0.125);
        if (uz) {
            uz[rb_idx(C, I, J, K)] = T(0);
            zero_ghosts(uz, x.cboxes, C, I, J, K);
        }
    }
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_restrict_plain(XGrid x, const T* __restrict__ rf, T* __restrict__ fc) {
    const Tile tl = x.tiles[tile_index(x.rev)];
    const RBox B = x.fboxes[tl.box];
    const RBox C = x.cboxes[x.cbox[tl.box]];
    const TileThread th = tile_thread(tl);
    const int I = (B.lo[0] >> 1) + th.x, J = (B.lo[1] >> 1) + th.y;
    if (I > (B.hi[0] >> 1) || J > (B.hi[1] >> 1)) return;
    for (int z = 0; z < (int)tl.zc; ++z) {
        const int K = (B.lo[2] >> 1) + th.z0 + z * th.dz;
        if (K > (B.hi[2] >> 1)) break;
        const int i = 2 * I, j = 2 * J, k = 2 * K;
        const T s = ((rf[rb_idx(B, i, j, k)] + rf[rb_idx(B, i + 1, j, k)]) +
                     (rf[rb_idx(B, i, j + 1, k)] + rf[rb_idx(B, i + 1, j + 1, k)])) +
                    ((rf[rb_idx(B, i, j, k + 1)] + rf[rb_idx(B, i + 1, j, k + 1)]) +
                     (rf[rb_idx(B, i, j + 1, k + 1)] + rf[rb_idx(B, i + 1, j + 1, k + 1)]));
        fc[rb_idx(C, I, J, K)] = s * T(0.125);
    }
}

// ---------------------------------------------------- prolongation + add
// Every fine cell gets e from its parent P = floor(i/2) per direction and the
// coarse neighbours on the child's side (P + s, s = +1 for an odd index, -1
// for an even one); with c_abc the coarse value at P shifted by a*sx, b*sy,
// c*sz,
//   e = (((27 c000 + 9 ((c100 + c010) + c001)) + 3 ((c110 + c101) + c011)) + c111) / 64
// (trilinear) or e = c000 (piecewise constant).  Coarse ghosts must be current.
//
// One thread per pair of fine cells (2I, 2I+1) of a row (fine boxes of a
// coarsened level are pair aligned): the pair shares its parent and its y/z
// neighbours, so 12 coarse values serve both cells (x = I-1, I, I+1 on the
// four rows (J, K), (J+sy, K), (J, K+sz), (J+sy, K+sz)).
template <class T, int ORDER>
__device__ __forceinline__ T prolong_e(const T (&p0)[2][3], const T (&p1)[2][3], int x) {
    if constexpr (ORDER == 1) return p0[0][1];
    const T c000 = p0[0][1], c100 = p0[0][x], c010 = p0[1][1], c001 = p1[0][1];
    const T c110 = p0[1][x], c101 = p1[0][x], c011 = p1[1][1], c111 = p1[1][x];
    return (((T(27) * c000 + T(9) * ((c100 + c010) + c001)) + T(3) * ((c110 + c101) + c011)) + c111) * T(0.015625);
}

// Planes whose fine values one thread loads before it computes any of them:
// fine u comes from HBM and there are only two such loads per plane, so they
// are issued as a group to keep enough of them in flight.
constexpr int kProlongGroup = 4;

template <class T, bool PUSH, int ORDER>
__global__ void __launch_bounds__(kBlock) k_prolong(Grid g, const RBox* __restrict__ cboxes, const int* __restrict__ cbox,
                                                   const T* __restrict__ ec, T* __restrict__ uf) {
    const Tile tl = g.tiles[tile_index(g.rev)];
    const RBox B = g.boxes[tl.box];
    if (g.active && !g.active[B.pid]) return;
    const RBox C = cboxes[cbox[tl.box]];
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    const int i0 = B.lo[0] + 2 * th.x;  // the even cell of the pair
    if (j > B.hi[1] || i0 > B.hi[0]) return;
    const int J = j >> 1, sj = (j & 1) ? 1 : -1, I = i0 >> 1;
    const T* __restrict__ cb = ec + C.base;
    T* __restrict__ fb = uf + B.base;
    // The two coarse planes (K and K+sz) a fine plane needs, each as rows J
    // and J+sy by x = I-1..I+1.  Planes the previous fine plane of this
    // thread used stay in registers: walking planes 2 apart, one of the two
    // carries over; walking consecutive planes, one or both do.  All lanes of
    // a wave walk the same planes, so the reuse tests are wave-uniform.
    T pa[2][3], pb[2][3];
    int ka = -0x7fffffff, kb = -0x7fffffff;  // no plane yet
    auto load_plane = [&](int Kq, T (&pl)[2][3]) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                if (ORDER == 1 && (r > 0 || x != 1)) continue;
                pl[r][x] = cb[rb_off(C, I - 1 + x, r ? J + sj : J, Kq)];
            }
    };
    auto take = [](T (&dst)[2][3], const T (&src)[2][3]) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int x = 0; x < 3; ++x) dst[r][x] = src[r][x];
    };
    const int zc = tl.zc;
    for (int z0 = 0; z0 < zc; z0 += kProlongGroup) {
        T fe[kProlongGroup], fo[kProlongGroup];
        int oe[kProlongGroup], oo[kProlongGroup];
#pragma unroll
        for (int q = 0; q < kProlongGroup; ++q) {
            const int k = min(B.lo[2] + th.z0 + (z0 + q) * th.dz, B.hi[2]);  // clamped: loads stay in the box
            oe[q] = rb_off(B, i0, j, k);
            oo[q] = rb_off(B, i0 + 1, j, k);
            fe[q] = fb[oe[q]];
            fo[q] = fb[oo[q]];
        }
        // one copy of the compute and push code: plane q's values are moved
        // to slot 0 (static register moves) instead of indexing by q
#pragma unroll 1
        for (int q = 0; q < kProlongGroup; ++q) {
            const int k = B.lo[2] + th.z0 + (z0 + q) * th.dz;
            if (z0 + q >= zc || k > B.hi[2]) break;
            const int K = k >> 1, K2 = K + ((k & 1) ? 1 : -1);
            T p0[2][3], p1[2][3];
            if (K == ka) take(p0, pa);
            else if (K == kb) take(p0, pb);
            else load_plane(K, p0);
            if constexpr (ORDER != 1) {
                if (K2 == ka) take(p1, pa);
                else if (K2 == kb) take(p1, pb);
                else load_plane(K2, p1);
                take(pb, p1);
                kb = K2;
            }
            take(pa, p0);
            ka = K;
            const T ve = fe[0] + prolong_e<T, ORDER>(p0, p1, 0);
            const T vo = fo[0] + prolong_e<T, ORDER>(p0, p1, 2);
            fb[oe[0]] = ve;
            fb[oo[0]] = vo;
            if constexpr (PUSH) {
                push_ghosts(uf, g.boxes, B, i0, j, k, ve);
                push_ghosts(uf, g.boxes, B, i0 + 1, j, k, vo);
            }
#pragma unroll
            for (int m = 0; m + 1 < kProlongGroup; ++m) {
                fe[m] = fe[m + 1];
                fo[m] = fo[m + 1];
                oe[m] = oe[m + 1];
                oo[m] = oo[m + 1];
            }
        }
    }
}

// Across a homogeneous-Dirichlet domain face only: -v into the box's own
// ghost beyond each such face the cell lies on (the rest of push_ghosts).
template <class T>
__device__ __forceinline__ void push_dirichlet(T* __restrict__ u, const RBox& B, int i, int j, int k, T v) {
    const int c[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            if (c[d] != (side ? B.hi[d] : B.lo[d]) || B.nb[2 * d + side] >= 0) continue;
            int t[3] = {i, j, k};
            t[d] += side ? 1 : -1;
            u[rb_idx(B, t[0], t[1], t[2])] = -v;
        }
}

// Prolongation that corrects only the colour-1 cells, for a V-cycle whose
// post-smoothing starts with a colour-0 sweep on a level that pushes its
// ghosts.  That sweep computes each colour-0 value from its neighbours only --
// except through the ghost beyond a Dirichlet face, which mirrors the cell
// itself (-u).  So: colour-1 cells are corrected and pushed as the two-colour
// kernel does; of the colour-0 cells only those on a Dirichlet face matter, and
// only through that mirrored ghost, which gets -(u + P e); correcting the
// other colour-0 values would be dead work (the sweep overwrites them before
// anything reads them, and their copies in neighbours' ghosts too).  One thread
// per colour-1 cell; the 8 coarse values are the parent and its neighbours
// towards the cell.
template <class T, int ORDER>
__global__ void __launch_bounds__(kBlock) k_prolong_c1(Grid g, const RBox* __restrict__ cboxes,
                                                      const int* __restrict__ cbox, const T* __restrict__ ec,
                                                      T* __restrict__ uf) {
    const Tile tl = g.tiles[tile_index(g.rev)];
    const RBox B = g.boxes[tl.box];
    if (g.active && !g.active[B.pid]) return;
    const RBox C = cboxes[cbox[tl.box]];
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    if (j > B.hi[1]) return;
    const int J = j >> 1, sj = (j & 1) ? 1 : -1;
    const T* __restrict__ cb = ec + C.base;
    T* __restrict__ fb = uf + B.base;
    // coarse rows J and J+sy at x = I and I+sx of the planes the previous fine
    // plane used stay in registers (see k_prolong)
    T pa[2][2], pb[2][2];
    int ka = -0x7fffffff, kb = -0x7fffffff;  // no plane yet
    auto load_plane = [&](int I, int si, int Kq, T (&pl)[2][2]) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                if (ORDER == 1 && (r > 0 || x > 0)) continue;
                pl[r][x] = cb[rb_off(C, I + x * si, r ? J + sj : J, Kq)];
            }
    };
    auto take = [](T (&dst)[2][2], const T (&src)[2][2]) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int x = 0; x < 2; ++x) dst[r][x] = src[r][x];
    };
    const int zc = tl.zc;
    for (int z0 = 0; z0 < zc; z0 += kProlongGroup) {
        T fv[kProlongGroup];
        int off[kProlongGroup];
#pragma unroll
        for (int q = 0; q < kProlongGroup; ++q) {
            const int k = min(B.lo[2] + th.z0 + (z0 + q) * th.dz, B.hi[2]);  // clamped: loads stay in the box
            const int i = min(colour_i(B, th.x, j, k, 1), B.hi[0]);
            off[q] = rb_off(B, i, j, k);  // the clamped cell may be colour 0: its value is never used
            fv[q] = fb[off[q]];
        }
        // one copy of the compute and push code (see k_prolong)
#pragma unroll 1
        for (int q = 0; q < kProlongGroup; ++q) {
            const int k = B.lo[2] + th.z0 + (z0 + q) * th.dz;
            if (z0 + q >= zc || k > B.hi[2]) break;
            const int i = colour_i(B, th.x, j, k, 1);
            const int I = i >> 1, si = (i & 1) ? 1 : -1;
            const int K = k >> 1, K2 = K + ((k & 1) ? 1 : -1);
            if (i <= B.hi[0]) {
                // the x side si is the same for every plane this thread walks
                // when the planes are 2 apart; otherwise the cached planes are
                // keyed by (plane, side)
                const int key = 2 * K + (si > 0), key2 = 2 * K2 + (si > 0);
                T p0[2][2], p1[2][2];
                if (key == ka) take(p0, pa);
                else if (key == kb) take(p0, pb);
                else load_plane(I, si, K, p0);
                if constexpr (ORDER != 1) {
                    if (key2 == ka) take(p1, pa);
                    else if (key2 == kb) take(p1, pb);
                    else load_plane(I, si, K2, p1);
                    take(pb, p1);
                    kb = key2;
                }
                take(pa, p0);
                ka = key;
                T e;
                if constexpr (ORDER == 1) {
                    e = p0[0][0];
                } else {
                    const T c000 = p0[0][0], c100 = p0[0][1], c010 = p0[1][0], c001 = p1[0][0];
                    const T c110 = p0[1][1], c101 = p1[0][1], c011 = p1[1][0], c111 = p1[1][1];
                    e = (((T(27) * c000 + T(9) * ((c100 + c010) + c001)) + T(3) * ((c110 + c101) + c011)) + c111) *
                        T(0.015625);
                }
                const T v = fv[0] + e;
                fb[off[0]] = v;
                push_ghosts(uf, g.boxes, B, i, j, k, v);
            }
            // the colour-0 cell of this row and plane, if it lies on a
            // Dirichlet face (few threads)
            const int i0 = colour_i(B, th.x, j, k, 0);
            const bool dir = i0 <= B.hi[0] &&
                             ((i0 == B.lo[0] && B.nb[0] < 0) || (i0 == B.hi[0] && B.nb[1] < 0) ||
                              (j == B.lo[1] && B.nb[2] < 0) || (j == B.hi[1] && B.nb[3] < 0) ||
                              (k == B.lo[2] && B.nb[4] < 0) || (k == B.hi[2] && B.nb[5] < 0));
            if (dir) {
                const int I = i0 >> 1, si = (i0 & 1) ? 1 : -1, K = k >> 1, sk = (k & 1) ? 1 : -1;
                T e;
                if constexpr (ORDER == 1) {
                    e = cb[rb_off(C, I, J, K)];
                } else {
                    const T c000 = cb[rb_off(C, I, J, K)], c100 = cb[rb_off(C, I + si, J, K)];
                    const T c010 = cb[rb_off(C, I, J + sj, K)], c001 = cb[rb_off(C, I, J, K + sk)];
                    const T c110 = cb[rb_off(C, I + si, J + sj, K)], c101 = cb[rb_off(C, I + si, J, K + sk)];
                    const T c011 = cb[rb_off(C, I, J + sj, K + sk)], c111 = cb[rb_off(C, I + si, J + sj, K + sk)];
                    e = (((T(27) * c000 + T(9) * ((c100 + c010) + c001)) + T(3) * ((c110 + c101) + c011)) + c111) *
                        T(0.015625);
                }
                push_dirichlet(uf, B, i0, j, k, fb[rb_off(B, i0, j, k)] + e);
            }
#pragma unroll
            for (int m = 0; m + 1 < kProlongGroup; ++m) {
                fv[m] = fv[m + 1];
                off[m] = off[m + 1];
            }
        }
    }
}

// k_prolong_c1 with the tile's coarse region staged in LDS: the workgroup
// loads every coarse value its tile reads (parents and the layer around
// them) once, then each cell takes its 8 values from LDS instead of from the
// vector memory path.  Same cells, values and arithmetic as k_prolong_c1.
// The host launches it where the region fits kProlongStage values.  SELF:
// the coarse level is one box, and the stage reads each ghost's mirror cell
// (see launch_prolong) instead of the ghost.

template <class T, int ORDER, bool SELF, bool FACES>
__global__ void __launch_bounds__(kBlock) k_prolong_c1s(Grid g, const RBox* __restrict__ cboxes,
                                                       const int* __restrict__ cbox, const T* __restrict__ ec,
                                                       T* __restrict__ uf) {
    __shared__ T cs[kProlongStage];
    const Tile tl = g.tiles[tile_index(g.rev)];
    const RBox B = g.boxes[tl.box];
    if (g.active && !g.active[B.pid]) return;  // the whole workgroup
    const RBox C = cboxes[cbox[tl.box]];
    // the tile's fine cells (clamped to the box) and the coarse cells around
    // their parents (inside the coarse box grown by its ghost layer)
    const int TX = 1 << tl.lx, TY = 1 << tl.ly, TZ = 1 << tl.lz;
    const int ilo = B.lo[0] + 2 * tl.x0, ihi = min(B.hi[0], B.lo[0] + 2 * (tl.x0 + TX) - 1);
    const int jlo = B.lo[1] + tl.y0, jhi = min(B.hi[1], jlo + TY - 1);
    const int klo = B.lo[2] + tl.z0, khi = min(B.hi[2], klo + TZ * tl.zc - 1);
    const int Ilo = (ilo >> 1) - 1, Jlo = (jlo >> 1) - 1, Klo = (klo >> 1) - 1;
    const int nI = (ihi >> 1) + 2 - Ilo, nJ = (jhi >> 1) + 2 - Jlo, nK = (khi >> 1) + 2 - Klo;
    const int n = nI * nJ * nK;
    const T* __restrict__ cb = ec + C.base;
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    T* __restrict__ fb = uf + B.base;
    // the fine values of a group of planes (clamped to the box: loads stay
    // in it; a clamped cell may be colour 0, and its value is never used)
    // The colour-0 cell of a row and plane that lies on a Dirichlet face
    // (few lanes, but in most waves) also needs its value: loaded with the
    // group, so no wave waits on a load inside the plane loop.
    auto dirichlet0 = [&](int i0, int k) {
        return i0 <= B.hi[0] && ((i0 == B.lo[0] && B.nb[0] < 0) || (i0 == B.hi[0] && B.nb[1] < 0) ||
                                 (j == B.lo[1] && B.nb[2] < 0) || (j == B.hi[1] && B.nb[3] < 0) ||
                                 (k == B.lo[2] && B.nb[4] < 0) || (k == B.hi[2] && B.nb[5] < 0));
    };
    T fv[kProlongGroup], f0[kProlongGroup];
    int off[kProlongGroup];
    auto load_group = [&](int z0) {
#pragma unroll
        for (int q = 0; q < kProlongGroup; ++q) {
            const int kk = B.lo[2] + th.z0 + (z0 + q) * th.dz;
            const int k = min(kk, B.hi[2]);
            const int i = min(colour_i(B, th.x, j, k, 1), B.hi[0]);
            off[q] = rb_off(B, i, j, k);
            fv[q] = fb[off[q]];
            const int i0 = colour_i(B, th.x, j, kk, 0);
            if constexpr (FACES) f0[q] = (kk <= B.hi[2] && dirichlet0(i0, kk)) ? fb[rb_off(B, i0, j, kk)] : T(0);
        }
    };
    // the first group is loaded before the stage barrier, so its latency
    // overlaps that of the coarse stage
    if (j <= B.hi[1]) load_group(0);
    {
        // stage index q = x + nI (y + nJ z), advanced by the block size
        // without divisions (the steps are uniform)
        const int bs = blockDim.x, qx = bs / nI, sx = bs - qx * nI, sz = qx / nJ, sy = qx - sz * nJ;
        const int t = threadIdx.x, ty = t / nI;
        int x = t - ty * nI, z = ty / nJ, y = ty - z * nJ;
        // a ghost of a one-box level: the cell it mirrors, negated once per
        // Dirichlet face crossed (the stage reaches one layer beyond the box)
        auto mirror = [&](int v, int d, bool& neg) {
            if (v < C.lo[d]) {
                if (C.nb[2 * d] >= 0) return v + (C.hi[d] - C.lo[d] + 1);
                neg = !neg;
                return 2 * C.lo[d] - 1 - v;
            }
            if (v > C.hi[d]) {
                if (C.nb[2 * d + 1] >= 0) return v - (C.hi[d] - C.lo[d] + 1);
                neg = !neg;
                return 2 * C.hi[d] + 1 - v;
            }
            return v;
        };
        // four values per step: their loads leave together
        for (int q0 = t; q0 < n; q0 += 4 * bs) {
            T v[4];
            bool ng[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int q = q0 + m * bs;
                ng[m] = false;
                int o = 0;
                if constexpr (SELF) {
                    const int I = mirror(Ilo + x, 0, ng[m]), Jq = mirror(Jlo + y, 1, ng[m]), K = mirror(Klo + z, 2, ng[m]);
                    o = rb_off(C, I, Jq, K);
                } else {
                    o = rb_off(C, Ilo + x, Jlo + y, Klo + z);
                }
                v[m] = q < n ? cb[o] : T(0);
                x += sx;
                y += sy;
                z += sz;
                if (x >= nI) { x -= nI; ++y; }
                if (y >= nJ) { y -= nJ; ++z; }
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int q = q0 + m * bs;
                if (q < n) cs[q] = ng[m] ? -v[m] : v[m];
            }
        }
    }
    __syncthreads();
    if (j > B.hi[1]) return;
    const int J = j >> 1, sj = (j & 1) ? 1 : -1;
    // LDS offsets: a cell's parent at (I - Ilo) + row + nIJ (K - Klo) with
    // this thread's coarse row (J - Jlo) nI; the other 7 values at fixed
    // offsets from it (24-bit products: the stage is at most 2048 values)
    const int nIJ = nI * nJ, row = __mul24(J - Jlo, nI), oy = sj * nI;
    auto interp = [&](int i, int k) -> T {
        const int I = i >> 1, si = (i & 1) ? 1 : -1, K = k >> 1;
        const int b = (I - Ilo) + row + __mul24(K - Klo, nIJ);
        if constexpr (ORDER == 1) return cs[b];
        const int oz = (k & 1) ? nIJ : -nIJ;
        const T c000 = cs[b], c100 = cs[b + si], c010 = cs[b + oy], c001 = cs[b + oz];
        const T c110 = cs[b + si + oy], c101 = cs[b + si + oz], c011 = cs[b + oy + oz];
        const T c111 = cs[b + si + oy + oz];
        return (((T(27) * c000 + T(9) * ((c100 + c010) + c001)) + T(3) * ((c110 + c101) + c011)) + c111) *
               T(0.015625);
    };
    const int zc = tl.zc;
    for (int z0 = 0; z0 < zc; z0 += kProlongGroup) {
        if (z0 > 0) load_group(z0);
#pragma unroll 1
        for (int q = 0; q < kProlongGroup; ++q) {
            const int k = B.lo[2] + th.z0 + (z0 + q) * th.dz;
            if (z0 + q >= zc || k > B.hi[2]) break;
            const int i = colour_i(B, th.x, j, k, 1);
            if (i <= B.hi[0]) {
                const T v = fv[0] + interp(i, k);
                fb[off[0]] = v;
                if constexpr (FACES) push_ghosts(uf, g.boxes, B, i, j, k, v);
            }
            // the colour-0 cell of this row and plane, if it lies on a
            // Dirichlet face: its mirrored ghost gets -(u + P e)
            const int i0 = colour_i(B, th.x, j, k, 0);
            if constexpr (FACES)
                if (dirichlet0(i0, k)) push_dirichlet(uf, B, i0, j, k, f0[0] + interp(i0, k));
#pragma unroll
            for (int m = 0; m + 1 < kProlongGroup; ++m) {
                fv[m] = fv[m + 1];
                f0[m] = f0[m + 1];
                off[m] = off[m + 1];
            }
        }
    }
}

// The face work k_prolong_c1s<..., FACES = false> leaves out, for a fine
// level that is one box: after it, every cell on a face of the box pushes
// its corrected colour-1 value into the ghosts that mirror it, and a
// colour-0 cell on a Dirichlet face writes -(u + P e) into its own ghosts
// there.  The same values, written by a second launch over the face cells
// only: in the main launch every wave holds a face lane and paid for this
// code on every plane.  A cell on an edge or corner is visited once per face
// and writes the same values each time.
template <class T, int ORDER>
__global__ void __launch_bounds__(kBlock) k_prolong_faces(Grid g, const RBox* __restrict__ cboxes,
                                                         const int* __restrict__ cbox, const T* __restrict__ ec,
                                                         T* __restrict__ uf) {
    const RBox B = g.boxes[0];
    if (g.active && !g.active[B.pid]) return;
    const RBox C = cboxes[cbox[0]];
    const int n0 = B.hi[0] - B.lo[0] + 1, n1 = B.hi[1] - B.lo[1] + 1, n2 = B.hi[2] - B.lo[2] + 1;
    const long long fx = (long long)n1 * n2, fy = (long long)n0 * n2, fz = (long long)n0 * n1;
    long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i, j, k;
    if (q < 2 * fx) {  // x faces: (j, k)
        const int side = q >= fx;
        q -= side * fx;
        i = side ? B.hi[0] : B.lo[0];
        j = B.lo[1] + (int)(q % n1);
        k = B.lo[2] + (int)(q / n1);
    } else if ((q -= 2 * fx) < 2 * fy) {  // y faces: (i, k)
        const int side = q >= fy;
        q -= side * fy;
        j = side ? B.hi[1] : B.lo[1];
        i = B.lo[0] + (int)(q % n0);
        k = B.lo[2] + (int)(q / n0);
    } else if ((q -= 2 * fy) < 2 * fz) {  // z faces: (i, j)
        const int side = q >= fz;
        q -= side * fz;
        k = side ? B.hi[2] : B.lo[2];
        i = B.lo[0] + (int)(q % n0);
        j = B.lo[1] + (int)(q / n0);
    } else {
        return;
    }
    const long long idx = rb_idx(B, i, j, k);
    if ((i + j + k) & 1) {
        push_ghosts(uf, g.boxes, B, i, j, k, uf[idx]);
        return;
    }
    const bool dir = (i == B.lo[0] && B.nb[0] < 0) || (i == B.hi[0] && B.nb[1] < 0) ||
                     (j == B.lo[1] && B.nb[2] < 0) || (j == B.hi[1] && B.nb[3] < 0) ||
                     (k == B.lo[2] && B.nb[4] < 0) || (k == B.hi[2] && B.nb[5] < 0);
    if (!dir) return;
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
    const T* __restrict__ cb = ec + C.base;
    T e;
    if constexpr (ORDER == 1) {
        e = cb[rb_off(C, I, J, K)];
    } else {
        const T c000 = cb[rb_off(C, I, J, K)], c100 = cb[rb_off(C, I + si, J, K)];
        const T c010 = cb[rb_off(C, I, J + sj, K)], c001 = cb[rb_off(C, I, J, K + sk)];
        const T c110 = cb[rb_off(C, I + si, J + sj, K)], c101 = cb[rb_off(C, I + si, J, K + sk)];
        const T c011 = cb[rb_off(C, I, J + sj, K + sk)], c111 = cb[rb_off(C, I + si, J + sj, K + sk)];
        e = (((T(27) * c000 + T(9) * ((c100 + c010) + c001)) + T(3) * ((c110 + c101) + c011)) + c111) *
            T(0.015625);
    }
    push_dirichlet(uf, B, i, j, k, uf[idx] + e);
}

// -------------------------------------------------------------- utilities
template <class T>
__global__ void __launch_bounds__(kBlock) k_zero(T* __restrict__ p, long long n, const int* __restrict__ active) {
    if (active && !active[0]) return;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) p[q] = T(0);
}

__global__ void __launch_bounds__(kBlock) k_cast_f32(const double* __restrict__ s, float* __restrict__ d, long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) d[q] = (float)s[q];
}

// Per-cell maps over both colours of the valid cells, tiled like the
// smoother; OP(B, i, j, k) does the work.
#define BXMG_FOR_VALID_CELLS(g, OP)                                          \
    const Tile tl = (g).tiles[tile_index((g).rev)];                                 \
    const RBox B = (g).boxes[tl.box];                                        \
    if ((g).active && !(g).active[B.pid]) return;                            \
    const TileThread th = tile_thread(tl);                           \
    const int j = B.lo[1] + th.y;                                            \
    if (j > B.hi[1]) return;                                                 \
    for (int z = 0; z < (int)tl.zc; ++z) {                                    \
        const int k = B.lo[2] + th.z0 + z * th.dz;                           \
        if (k > B.hi[2]) break;                                              \
        for (int c = 0; c < 2; ++c) {                                        \
            const int i = colour_i(B, th.x, j, k, c);                        \
            if (i > B.hi[0]) continue;                                       \
            OP;                                                              \
        }                                                                    \
    }

// F-order FP64 caller MultiFab (component 0) -> RB level, valid cells.
template <class T>
__global__ void __launch_bounds__(kBlock) k_fab_to_rb(Grid g, const double* __restrict__ fab, const FBox* __restrict__ fb,
                                                     T* __restrict__ rb) {
    BXMG_FOR_VALID_CELLS(g, rb[rb_idx(B, i, j, k)] = (T)fab[fab_idx(fb[tl.box], i, j, k)])
}

// k_fab_to_rb<double> that also sets *nonzero when any converted value is
// not +0.0 (bit pattern; one atomic per wave that saw one)
__global__ void __launch_bounds__(kBlock) k_fab_to_rb_nz(Grid g, const double* __restrict__ fab,
                                                        const FBox* __restrict__ fb, double* __restrict__ rb,
                                                        int* __restrict__ nonzero) {
    bool nz = false;
    const Tile tl = g.tiles[tile_index(g.rev)];
    const RBox B = g.boxes[tl.box];
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    if (j <= B.hi[1])
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int k = B.lo[2] + th.z0 + z * th.dz;
            if (k > B.hi[2]) break;
            for (int c = 0; c < 2; ++c) {
                const int i = colour_i(B, th.x, j, k, c);
                if (i > B.hi[0]) continue;
                const double v = fab[fab_idx(fb[tl.box], i, j, k)];
                rb[rb_idx(B, i, j, k)] = v;
                nz = nz || __double_as_longlong(v) != 0;
            }
        }
    if (__any(nz) && (threadIdx.x & 63) == 0) atomicOr(nonzero, 1);
}

__global__ void __launch_bounds__(kBlock) k_rb_to_fab(Grid g, const double* __restrict__ rb, double* __restrict__ fab,
                                                     const FBox* __restrict__ fb) {
    BXMG_FOR_VALID_CELLS(g, fab[fab_idx(fb[tl.box], i, j, k)] = rb[rb_idx(B, i, j, k)])
}

// ONE: a one-box, buffer-addressed level (Grid::push == 2, res): 32-bit
// offsets and the one-box push (a ghost is the box's own cell's mirror).
template <bool ONE>
__global__ void __launch_bounds__(kBlock) k_add_f32(Grid g, double* __restrict__ u, const float* __restrict__ e) {
    if constexpr (ONE) {
        const Tile tl = g.tiles[tile_index(g.rev)];
        const RBox B = g.boxes[tl.box];
        if (g.active && !g.active[B.pid]) return;
        const TileThread th = tile_thread(tl);
        const int j = B.lo[1] + th.y;
        if (j > B.hi[1]) return;
        const long long ne = 2 * B.cstride;
        const BoxRes<double> U(u + B.base, ne);
        const BoxRes<float> E(e + B.base, ne);
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int k = B.lo[2] + th.z0 + z * th.dz;
            if (k > B.hi[2]) break;
            for (int c = 0; c < 2; ++c) {
                const int i = colour_i(B, th.x, j, k, c);
                if (i > B.hi[0]) continue;
                const int idx = rb_off(B, i, j, k);
                const double v = U.ld(idx) + (double)E.ld(idx);
                U.st(idx, v);
                // the face ghosts mirroring the cell (push_self's targets)
                const int cc[3] = {i, j, k};
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                    for (int side = 0; side < 2; ++side) {
                        if (cc[d] != (side ? B.hi[d] : B.lo[d])) continue;
                        const int q = 2 * d + side;
                        int t[3] = {i, j, k};
                        t[d] += B.nb[q] >= 0 ? B.shift[q] : (side ? 1 : -1);
                        U.st(rb_off(B, t[0], t[1], t[2]), B.nb[q] >= 0 ? v : -v);
                    }
            }
        }
    } else {
        BXMG_FOR_VALID_CELLS(g, const long long idx = rb_idx(B, i, j, k); const double v = u[idx] + (double)e[idx];
                             u[idx] = v; if (g.push) push_ghosts(u, g.boxes, B, i, j, k, v))
    }
}

// Sum of valid cells (periodic mean projection), then subtraction.
__global__ void __launch_bounds__(kBlock) k_sum_valid(Grid g, const double* __restrict__ u,
                                                     double* __restrict__ partials) {
    __shared__ double sh[3 * (kBlock / 64)];
    double mx = 0.0, s = 0.0, cnt = 0.0;
    const Tile tl = g.tiles[tile_index(g.rev)];
    const RBox B = g.boxes[tl.box];
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    if (j <= B.hi[1])
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int k = B.lo[2] + th.z0 + z * th.dz;
            if (k > B.hi[2]) break;
            for (int c = 0; c < 2; ++c) {
                const int i = colour_i(B, th.x, j, k, c);
                if (i > B.hi[0]) continue;
                s = s + u[rb_idx(B, i, j, k)];
                cnt += 1.0;
            }
        }
    block_reduce3(mx, s, cnt, sh);
    if (threadIdx.x == 0) {
        partials[3 * blockIdx.x] = 0.0;
        partials[3 * blockIdx.x + 1] = s;
        partials[3 * blockIdx.x + 2] = cnt;
    }
}

__global__ void __launch_bounds__(kBlock) k_sub_mean(Grid g, double* __restrict__ u, const double* __restrict__ tot) {
    const double mean = tot[1] / tot[2];
    BXMG_FOR_VALID_CELLS(g, const long long idx = rb_idx(B, i, j, k); u[idx] = u[idx] - mean)
}

// Block of a launch over n tiles that tile_index sends to tile t (rev = 0):
// where a launch over one problem's tiles alone puts tile t's partial.
__device__ __forceinline__ int solo_block(int t, int n) {
    if ((n & 7) == 0) {
        const int per = n >> 3;
        return (t % per) * 8 + t / per;
    }
    return t;
}

// k_sum_valid over many problems' tiles, each tile's partial stored where a
// launch over its problem alone stores it.
__global__ void __launch_bounds__(kBlock) k_sum_valid_many(Grid g, const RetireBox* __restrict__ info,
                                                          const double* __restrict__ u,
                                                          double* __restrict__ partials) {
    __shared__ double sh[3 * (kBlock / 64)];
    double mx = 0.0, s = 0.0, cnt = 0.0;
    const int tix = tile_index(g.rev);
    const Tile tl = g.tiles[tix];
    const RBox B = g.boxes[tl.box];
    const RetireBox R = info[tl.box];
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    if (j <= B.hi[1])
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int k = B.lo[2] + th.z0 + z * th.dz;
            if (k > B.hi[2]) break;
            for (int c = 0; c < 2; ++c) {
                const int i = colour_i(B, th.x, j, k, c);
                if (i > B.hi[0]) continue;
                s = s + u[rb_idx(B, i, j, k)];
                cnt += 1.0;
            }
        }
    block_reduce3(mx, s, cnt, sh);
    if (threadIdx.x == 0) {
        const int q = R.tstart + solo_block(tix - R.tstart, R.nt);
        partials[3 * q] = 0.0;
        partials[3 * q + 1] = s;
        partials[3 * q + 2] = cnt;
    }
}

// k_norm_final per problem: block q reduces partials [seg[q], seg[q+1]).
__global__ void __launch_bounds__(kNormThreads) k_norm_final_seg(const double* __restrict__ partials,
                                                                const int* __restrict__ seg, double* __restrict__ out) {
    __shared__ double sh[3 * (kNormThreads / 64)];
    const int q = blockIdx.x;
    double mx, s2, bad;
    norm_reduce(partials + 3 * (long long)seg[q], seg[q + 1] - seg[q], sh, mx, s2, bad);
    if (threadIdx.x == 0) { out[3 * q] = mx; out[3 * q + 1] = s2; out[3 * q + 2] = bad; }
}

__global__ void __launch_bounds__(kBlock) k_sub_mean_many(Grid g, const RetireBox* __restrict__ info,
                                                         double* __restrict__ u, const double* __restrict__ tot) {
    BXMG_FOR_VALID_CELLS(g, const double* t3 = tot + 3 * (long long)info[tl.box].seg; const double mean = t3[1] / t3[2];
                         const long long idx = rb_idx(B, i, j, k); u[idx] = u[idx] - mean)
}

__global__ void __launch_bounds__(kBlock) k_rb_to_fab_many(Grid g, const double* __restrict__ rb,
                                                          const RetireBox* __restrict__ info) {
    BXMG_FOR_VALID_CELLS(g, const RetireBox& R = info[tl.box]; R.fab[fab_idx(R.f, i, j, k)] = rb[rb_idx(B, i, j, k)])
}

// ------------------------------------------------------ coefficient setup
// Level-1 faces from the level-0 cell beta (ghosts filled by the exchange
// and the even reflection): each fine face is the harmonic mean of its two
// cells, each coarse face the mean of its 4 fine faces,
//   ((a(t1,t2) + a(t1+1,t2)) + (a(t1,t2+1) + a(t1+1,t2+1))) * 1/4.
// Tiles cover the coarse faces of direction d anchored in each fine box:
// the low face of every coarse cell, plus the high face of the last cell
// when the box touches the domain's upper end in d (index range one larger).
template <class T>
__global__ void __launch_bounds__(kBlock) k_faces_from_cells(XGrid x, const T* __restrict__ beta, int d, int fdom_hi,
                                                            FaceArrays<T> out, T* __restrict__ dst) {
    const Tile tl = x.tiles[tile_index(x.rev)];
    const RBox B = x.fboxes[tl.box];
    const TileThread th = tile_thread(tl);
    int chi[3] = {B.hi[0] >> 1, B.hi[1] >> 1, B.hi[2] >> 1};
    if (B.hi[d] == fdom_hi) chi[d] += 1;
    const int I = (B.lo[0] >> 1) + th.x, J = (B.lo[1] >> 1) + th.y;
    if (I > chi[0] || J > chi[1]) return;
    const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    for (int z = 0; z < (int)tl.zc; ++z) {
        const int K = (B.lo[2] >> 1) + th.z0 + z * th.dz;
        if (K > chi[2]) break;
        const int f0[3] = {2 * I, 2 * J, 2 * K};
        T a[2][2];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                int cc[3] = {f0[0], f0[1], f0[2]};
                cc[t1] += p;
                cc[t2] += q;
                int lc[3] = {cc[0], cc[1], cc[2]};
                lc[d] -= 1;
                a[q][p] = harm(beta[rb_idx(B, lc[0], lc[1], lc[2])], beta[rb_idx(B, cc[0], cc[1], cc[2])]);
            }
        const T v = ((a[0][0] + a[0][1]) + (a[1][0] + a[1][1])) * T(0.25);
        const int xx = I - out.dlo[0], yy = J - out.dlo[1], zz = K - out.dlo[2];
        const int nx = out.n[0] + (d == 0), ny = out.n[1] + (d == 1);
        dst[(long long)xx + (long long)nx * ((long long)yy + (long long)ny * zz)] = v;
    }
}

// Level l+1 faces from level l faces (global arrays).
template <class T>
__global__ void __launch_bounds__(kBlock) k_faces_coarsen(FaceArrays<T> fine, FaceArrays<T> coarse, int d,
                                                         T* __restrict__ dst) {
    const int nxc = coarse.n[0] + (d == 0), nyc = coarse.n[1] + (d == 1), nzc = coarse.n[2] + (d == 2);
    const long long total = (long long)nxc * nyc * nzc;
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int x = (int)(g % nxc), y = (int)((g / nxc) % nyc), z = (int)(g / ((long long)nxc * nyc));
    const int nxf = fine.n[0] + (d == 0), nyf = fine.n[1] + (d == 1);
    const int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    const int f0[3] = {2 * x, 2 * y, 2 * z};
    T a[2][2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            int cc[3] = {f0[0], f0[1], f0[2]};
            cc[t1] += p;
            cc[t2] += q;
            a[q][p] = fine.c[d][(long long)cc[0] + (long long)nxf * ((long long)cc[1] + (long long)nyf * cc[2])];
        }
    dst[g] = ((a[0][0] + a[0][1]) + (a[1][0] + a[1][1])) * T(0.25);
}

// ---------------------------------------------------------------- bottom
// FP64 conjugate gradients on the coarsest level by one workgroup, vectors
// in LDS over the level domain (natural order, p with a ghost layer).
constexpr int kBotThreads = 1024;

// Dynamic LDS of the one-workgroup kernels (bottom CG, fused coarse cycle);
// the host sizes it per launch.
extern __shared__ __align__(16) unsigned char bxmg_lds[];

struct BottomGeom {
    int dlo[3], n[3];
    int per[3];
    int nboxes;
    double a;  // Helmholtz coefficient (0: Poisson; a fully periodic bottom is then singular)
};

__device__ __forceinline__ double bot_reduce(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = v + __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = sh[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) s = s + sh[w];
        sh[32] = s;
    }
    __syncthreads();
    return sh[32];
}

// Face ghost t of the CG's p grid (nx x ny x nz cells grown by one; the
// 7-point stencil reads face ghosts only): t runs over the 2(ny nz + nx nz +
// nx ny) face ghosts, x faces first, low side before high.  Returns the
// ghost's index in the grown grid, the index of the cell it copies and the
// sign (the periodic image, or odd reflection at a Dirichlet face).  Written
// without arrays indexed by the direction, which would live in scratch.
struct BottomGhost {
    int dst, src;
    double sgn;
};
__device__ __forceinline__ BottomGhost bottom_ghost(int t, int nx, int ny, int nz, bool px, bool py, bool pz) {
    const int gx = nx + 2, gy = ny + 2;
    const int nfx = ny * nz, nfy = nx * nz, nfz = nx * ny;
    int gi, gj, gk, si, sj, sk;
    bool per;
    if (t < 2 * nfx) {
        const int side = t / nfx, tt = t - side * nfx;
        gj = sj = tt % ny;
        gk = sk = tt / ny;
        gi = side ? nx : -1;
        si = px ? (side ? 0 : nx - 1) : (side ? nx - 1 : 0);
        per = px;
    } else if ((t -= 2 * nfx) < 2 * nfy) {
        const int side = t / nfy, tt = t - side * nfy;
        gi = si = tt % nx;
        gk = sk = tt / nx;
        gj = side ? ny : -1;
        sj = py ? (side ? 0 : ny - 1) : (side ? ny - 1 : 0);
        per = py;
    } else {
        t -= 2 * nfy;
        const int side = t / nfz, tt = t - side * nfz;
        gi = si = tt % nx;
        gj = sj = tt / nx;
        gk = side ? nz : -1;
        sk = pz ? (side ? 0 : nz - 1) : (side ? nz - 1 : 0);
        per = pz;
    }
    return {(gi + 1) + gx * ((gj + 1) + gy * (gk + 1)), (si + 1) + gx * ((sj + 1) + gy * (sk + 1)), per ? 1.0 : -1.0};
}

// The CG's vectors in LDS: p over the bottom grown by one cell, x, r, q over
// its N cells, 40 reduction slots (bottom_lds_bytes on the host side).
struct BottomLds {
    double *p, *x, *r, *q, *sh;
    __device__ BottomLds(unsigned char* base, int n, int ngrown) {
        p = (double*)base;
        x = p + ngrown;
        r = x + n;
        q = r + n;
        sh = q + n;
    }
};

// The whole CG, executed by one workgroup (any block size, multiple of 64).
template <class T, bool VAR>
__device__ void bottom_cg(T* __restrict__ u, const T* __restrict__ f, const FaceArrays<T>& fa,
                          const RBox* __restrict__ boxes, const BottomGeom& G, double h, double rtol,
                          int* __restrict__ iters_out, BottomLds& S) {
    double* p = S.p;
    double* x = S.x;
    double* r = S.r;
    double* q = S.q;
    double* sh = S.sh;
    const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
    const bool px = G.per[0] != 0, py = G.per[1] != 0, pz = G.per[2] != 0;
    const int N = nx * ny * nz;
    const int gx = nx + 2, gy = ny + 2;
    const double ih2 = 1.0 / (h * h);
    auto pidx = [&](int a, int b, int c) { return (a + 1) + gx * ((b + 1) + gy * (c + 1)); };
    // gather rhs
    for (int bi = 0; bi < G.nboxes; ++bi) {
        const RBox B = boxes[bi];
        const int bx = B.hi[0] - B.lo[0] + 1, by = B.hi[1] - B.lo[1] + 1, bz = B.hi[2] - B.lo[2] + 1;
        for (int qq = threadIdx.x; qq < bx * by * bz; qq += blockDim.x) {
            const int i = B.lo[0] + qq % bx, j = B.lo[1] + (qq / bx) % by, k = B.lo[2] + qq / (bx * by);
            const int n = (i - G.dlo[0]) + nx * ((j - G.dlo[1]) + ny * (k - G.dlo[2]));
            r[n] = (double)f[rb_idx(B, i, j, k)];
        }
    }
    __syncthreads();
    const bool sing = G.per[0] && G.per[1] && G.per[2] && G.a == 0.0;
    const double dg = G.a * (h * h);
    if (sing) {
        double s = 0.0;
        for (int n = threadIdx.x; n < N; n += blockDim.x) s = s + r[n];
        const double mean = bot_reduce(s, sh) / (double)N;
        for (int n = threadIdx.x; n < N; n += blockDim.x) r[n] = r[n] - mean;
        __syncthreads();
    }
    double rs = 0.0;
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
        x[n] = 0.0;
        const int a = n % nx, b = (n / nx) % ny, c = n / (nx * ny);
        p[pidx(a, b, c)] = r[n];
        rs = rs + r[n] * r[n];
    }
    rs = bot_reduce(rs, sh);
    const double rs0 = rs;
    int it = 0;
    if (rs0 != 0.0) {
        const int maxit = 4 * N;
        for (it = 0; it < maxit;) {
            // ghosts of p: face ghosts only (7-point stencil)
            const int nghost = 2 * (ny * nz + nx * nz + nx * ny);
            for (int t = threadIdx.x; t < nghost; t += blockDim.x) {
                const BottomGhost gh = bottom_ghost(t, nx, ny, nz, px, py, pz);
                p[gh.dst] = gh.sgn * p[gh.src];
            }
            __syncthreads();
            double pAp = 0.0;
            for (int n = threadIdx.x; n < N; n += blockDim.x) {
                const int a = n % nx, b = (n / nx) % ny, c = n / (nx * ny);
                const int pc = pidx(a, b, c);
                double su, sb;
                const double pxm = p[pc - 1], pxp = p[pc + 1], pym = p[pc - gx], pyp = p[pc + gx];
                const double pzm = p[pc - gx * gy], pzp = p[pc + gx * gy];
                if constexpr (!VAR) {
                    su = ((pxm + pxp) + (pym + pyp)) + (pzm + pzp);
                    sb = 6.0;
                } else {
                    const long long ix = (long long)a + (long long)(nx + 1) * ((long long)b + (long long)ny * c);
                    const long long iy = (long long)a + (long long)nx * ((long long)b + (long long)(ny + 1) * c);
                    const long long iz = (long long)a + (long long)nx * ((long long)b + (long long)ny * c);
                    const double bxm = (double)fa.c[0][ix], bxp = (double)fa.c[0][ix + 1];
                    const double bym = (double)fa.c[1][iy], byp = (double)fa.c[1][iy + nx];
                    const double bzm = (double)fa.c[2][iz], bzp = (double)fa.c[2][iz + (long long)nx * ny];
                    sb = ((bxm + bxp) + (bym + byp)) + (bzm + bzp);
                    su = ((bxm * pxm + bxp * pxp) + (bym * pym + byp * pyp)) + (bzm * pzm + bzp * pzp);
                }
                const double qv = (su - (sb + dg) * p[pc]) * ih2;
                q[n] = qv;
                pAp = pAp + p[pc] * qv;
            }
            pAp = bot_reduce(pAp, sh);
            const double alpha = rs / pAp;
            double rsn = 0.0;
            for (int n = threadIdx.x; n < N; n += blockDim.x) {
                const int a = n % nx, b = (n / nx) % ny, c = n / (nx * ny);
                x[n] = x[n] + alpha * p[pidx(a, b, c)];
                const double rn = r[n] - alpha * q[n];
                r[n] = rn;
                rsn = rsn + rn * rn;
            }
            rsn = bot_reduce(rsn, sh);
            ++it;
            if (sqrt(rsn) <= rtol * sqrt(rs0)) break;
            const double beta = rsn / rs;
            for (int n = threadIdx.x; n < N; n += blockDim.x) {
                const int a = n % nx, b = (n / nx) % ny, c = n / (nx * ny);
                const int pc = pidx(a, b, c);
                p[pc] = r[n] + beta * p[pc];
            }
            rs = rsn;
            __syncthreads();
        }
        if (sing) {
            double s = 0.0;
            for (int n = threadIdx.x; n < N; n += blockDim.x) s = s + x[n];
            const double mean = bot_reduce(s, sh) / (double)N;
            for (int n = threadIdx.x; n < N; n += blockDim.x) x[n] = x[n] - mean;
        }
    }
    __syncthreads();
    for (int bi = 0; bi < G.nboxes; ++bi) {
        const RBox B = boxes[bi];
        const int bx = B.hi[0] - B.lo[0] + 1, by = B.hi[1] - B.lo[1] + 1, bz = B.hi[2] - B.lo[2] + 1;
        for (int qq = threadIdx.x; qq < bx * by * bz; qq += blockDim.x) {
            const int i = B.lo[0] + qq % bx, j = B.lo[1] + (qq / bx) % by, k = B.lo[2] + qq / (bx * by);
            const int n = (i - G.dlo[0]) + nx * ((j - G.dlo[1]) + ny * (k - G.dlo[2]));
            u[rb_idx(B, i, j, k)] = (T)x[n];
        }
    }
    if (threadIdx.x == 0 && iters_out) *iters_out = it;
}

// Bottoms of at most 64 cells: the same CG run by one wave (lane n owns cell
// n), with wave-wide butterfly sums and no workgroup barriers -- a tiny
// bottom is all latency.  The butterfly leaves bitwise the same sum in every
// lane (IEEE addition commutes), so every lane takes the same decisions.
constexpr int kWaveBottomCells = 64;

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v = v + __shfl_xor(v, o);
    return v;
}

// orders this wave's LDS writes before its later LDS reads of other lanes' cells
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Executed by the 64 threads of wave 0 only; N = cells <= kWaveBottomCells.
template <class T, bool VAR>
__device__ void bottom_cg_wave(T* __restrict__ u, const T* __restrict__ f, const FaceArrays<T>& fa,
                               const RBox* __restrict__ boxes, const BottomGeom& G, double h, double rtol,
                               int* __restrict__ iters_out, BottomLds& S) {
    double* p = S.p;
    const int lane = threadIdx.x;
    const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
    const bool px = G.per[0] != 0, py = G.per[1] != 0, pz = G.per[2] != 0;
    const int N = nx * ny * nz;
    const int gx = nx + 2, gy = ny + 2;
    const int nghost = 2 * (ny * nz + nx * nz + nx * ny);
    const double ih2 = 1.0 / (h * h);
    const bool mine = lane < N;
    const int a = lane % nx, b = (lane / nx) % ny, c = lane / (nx * ny);
    const int pc = (a + 1) + gx * ((b + 1) + gy * (c + 1));
    // gather rhs into the owning lanes
    double r = 0.0;
    for (int bi = 0; bi < G.nboxes; ++bi) {
        const RBox B = boxes[bi];
        if (mine && G.dlo[0] + a >= B.lo[0] && G.dlo[0] + a <= B.hi[0] && G.dlo[1] + b >= B.lo[1] &&
            G.dlo[1] + b <= B.hi[1] && G.dlo[2] + c >= B.lo[2] && G.dlo[2] + c <= B.hi[2])
            r = (double)f[rb_idx(B, G.dlo[0] + a, G.dlo[1] + b, G.dlo[2] + c)];
    }
    const bool sing = G.per[0] && G.per[1] && G.per[2] && G.a == 0.0;
    const double dg = G.a * (h * h);
    if (sing) {
        const double mean = wave_sum(r) / (double)N;
        if (mine) r = r - mean;
    }
    double x = 0.0, pv = r;
    double rs = wave_sum(r * r);
    const double rs0 = rs;
    int it = 0;
    if (rs0 != 0.0) {
        const int maxit = 4 * N;
        for (it = 0; it < maxit;) {
            // p with its face ghosts in LDS (7-point stencil)
            if (mine) p[pc] = pv;
            wave_lds_sync();
            for (int t = lane; t < nghost; t += 64) {
                const BottomGhost gh = bottom_ghost(t, nx, ny, nz, px, py, pz);
                p[gh.dst] = gh.sgn * p[gh.src];
            }
            wave_lds_sync();
            double qv = 0.0;
            if (mine) {
                double su, sb;
                const double pxm = p[pc - 1], pxp = p[pc + 1], pym = p[pc - gx], pyp = p[pc + gx];
                const double pzm = p[pc - gx * gy], pzp = p[pc + gx * gy];
                if constexpr (!VAR) {
                    su = ((pxm + pxp) + (pym + pyp)) + (pzm + pzp);
                    sb = 6.0;
                } else {
                    const long long ix = (long long)a + (long long)(nx + 1) * ((long long)b + (long long)ny * c);
                    const long long iy = (long long)a + (long long)nx * ((long long)b + (long long)(ny + 1) * c);
                    const long long iz = (long long)a + (long long)nx * ((long long)b + (long long)ny * c);
                    const double bxm = (double)fa.c[0][ix], bxp = (double)fa.c[0][ix + 1];
                    const double bym = (double)fa.c[1][iy], byp = (double)fa.c[1][iy + nx];
                    const double bzm = (double)fa.c[2][iz], bzp = (double)fa.c[2][iz + (long long)nx * ny];
                    sb = ((bxm + bxp) + (bym + byp)) + (bzm + bzp);
                    su = ((bxm * pxm + bxp * pxp) + (bym * pym + byp * pyp)) + (bzm * pzm + bzp * pzp);
                }
                qv = (su - (sb + dg) * pv) * ih2;
            }
            const double pAp = wave_sum(pv * qv);
            const double alpha = rs / pAp;
            if (mine) {
                x = x + alpha * pv;
                r = r - alpha * qv;
            }
            const double rsn = wave_sum(r * r);
            ++it;
            if (sqrt(rsn) <= rtol * sqrt(rs0)) break;
            const double beta = rsn / rs;
            if (mine) pv = r + beta * pv;
            rs = rsn;
            wave_lds_sync();  // this iteration's reads of p come before the next writes
        }
        if (sing) {
            const double mean = wave_sum(x) / (double)N;
            if (mine) x = x - mean;
        }
    }
    for (int bi = 0; bi < G.nboxes; ++bi) {
        const RBox B = boxes[bi];
        if (mine && G.dlo[0] + a >= B.lo[0] && G.dlo[0] + a <= B.hi[0] && G.dlo[1] + b >= B.lo[1] &&
            G.dlo[1] + b <= B.hi[1] && G.dlo[2] + c >= B.lo[2] && G.dlo[2] + c <= B.hi[2])
            u[rb_idx(B, G.dlo[0] + a, G.dlo[1] + b, G.dlo[2] + c)] = (T)x;
    }
    if (lane == 0 && iters_out) *iters_out = it;
}

template <class T, bool VAR>
__global__ void __launch_bounds__(kBotThreads) k_bottom(T* __restrict__ u, const T* __restrict__ f, FaceArrays<T> fa,
                                                       const RBox* __restrict__ boxes, BottomGeom G, double h,
                                                       double rtol, int* __restrict__ iters_out) {
    const int N = G.n[0] * G.n[1] * G.n[2];
    BottomLds S(bxmg_lds, N, (G.n[0] + 2) * (G.n[1] + 2) * (G.n[2] + 2));
    if (N <= kWaveBottomCells) {
        if (threadIdx.x < 64) bottom_cg_wave<T, VAR>(u, f, fa, boxes, G, h, rtol, iters_out, S);
    } else {
        bottom_cg<T, VAR>(u, f, fa, boxes, G, h, rtol, iters_out, S);
    }
}

// --------------------------------------------------- fused coarse V-cycle
// The V-cycle below a level whose remaining levels are single boxes of at
// most kMaxBottomCells cells runs as one workgroup in one launch: the same
// stages in the same order as the level-by-level launches (pre-smoothing,
// residual + restriction, zero coarse guess, ..., CG bottom, ..., ghost fill
// of the coarse level, prolongation, post-smoothing), each a block-strided
// loop closed by a barrier.  Launch latency, not bandwidth, bounds these
// levels, so one launch replaces some 20 per level.
// Level storage of the fused coarse cycle, by 32-bit element offsets (the
// levels hold at most kMaxBottomCells cells): LDS through an address-space-3
// pointer, so the compiler emits LDS instructions rather than flat ones, or
// device memory.
template <class T, bool LDS>
struct LvMem;
template <class T>
struct LvMem<T, true> {
    __attribute__((address_space(3))) T* p;
    __device__ __forceinline__ T ld(int e) const { return p[e]; }
    __device__ __forceinline__ void st(int e, T v) const { p[e] = v; }
};
template <class T>
struct LvMem<T, false> {
    T* p;
    __device__ __forceinline__ T ld(int e) const { return p[e]; }
    __device__ __forceinline__ void st(int e, T v) const { p[e] = v; }
};

template <class T, bool LDS>
__device__ void blk_fill(const LvMem<T, LDS>& u, const GhostCopy* __restrict__ list, long long n) {
    for (int g = threadIdx.x; g < (int)n; g += blockDim.x) {
        const GhostCopy pc = list[g];
        const T v = u.ld((int)(pc.src & 0x7fffffffu));
        u.st((int)pc.dst, (pc.src >> 31) ? -v : v);
    }
    __syncthreads();
}

// q = a / d, r = a % d for 0 <= a < 2^20 and d >= 1: the float estimate with
// rd = 1/d is off by less than one, so one correction step makes it exact
__device__ __forceinline__ void small_divmod(int a, int d, float rd, int& q, int& r) {
    q = (int)((float)a * rd);
    r = a - q * d;
    if (r < 0) {
        --q;
        r += d;
    } else if (r >= d) {
        ++q;
        r -= d;
    }
}

// The colour cells of a single box, numbered g = t + tn (y + ny z).
struct BoxCells {
    int tn, ny, n;
    float rtn, rny;
};
__device__ __forceinline__ BoxCells box_cells(const RBox& B) {
    BoxCells c;
    const int nx = B.hi[0] - B.lo[0] + 1, nz = B.hi[2] - B.lo[2] + 1;
    c.ny = B.hi[1] - B.lo[1] + 1;
    c.tn = (nx + 1) >> 1;
    c.n = c.tn * c.ny * nz;
    c.rtn = 1.0f / (float)c.tn;
    c.rny = 1.0f / (float)c.ny;
    return c;
}
// colour cell g of colour c: (i, j, k), or false past the row's end
__device__ __forceinline__ bool box_colour_cell(const RBox& B, const BoxCells& bc, int g, int c, int& i, int& j,
                                                int& k) {
    int r, t, rz, y;
    small_divmod(g, bc.tn, bc.rtn, r, t);
    small_divmod(r, bc.ny, bc.rny, rz, y);
    j = B.lo[1] + y;
    k = B.lo[2] + rz;
    i = colour_i(B, t, j, k, c);
    return i <= B.hi[0];
}

// element of cell (i,j,k) in a coarse-cycle level's storage
__device__ __forceinline__ int blk_off(const RBox& B, int i, int j, int k) { return (int)B.base + rb_off(B, i, j, k); }

// gather() for the coarse-cycle levels: 32-bit offsets, level storage M
template <class T, int MODE, bool CENTRE, class M>
__device__ __forceinline__ int blk_gather(const M& U, const FaceArrays<T>& fa, const RBox& B, int i, int j, int k,
                                          Nbr<T>& n) {
    const int c = (i + j + k) & 1;
    const int row = (int)B.base + ((k - B.glo[2]) * B.G[1] + (j - B.glo[1])) * B.H;
    const int cs = (int)B.cstride;
    const int rc = c * cs + row, ro = (c ^ 1) * cs + row;
    const int Hy = B.H, Hz = B.H * B.G[1];
    const int m = (i - B.glo[0]) >> 1;
    const int mxm = (i - 1 - B.glo[0]) >> 1, mxp = (i + 1 - B.glo[0]) >> 1;
    n.xm = U.ld(ro + mxm);
    n.xp = U.ld(ro + mxp);
    n.ym = U.ld(ro - Hy + m);
    n.yp = U.ld(ro + Hy + m);
    n.zm = U.ld(ro - Hz + m);
    n.zp = U.ld(ro + Hz + m);
    if constexpr (CENTRE) n.c = U.ld(rc + m);
    if constexpr (MODE == 2) {
        const int x = i - fa.dlo[0], y = j - fa.dlo[1], z = k - fa.dlo[2];
        const int nx = fa.n[0], ny = fa.n[1];
        const int ix = x + (nx + 1) * (y + ny * z);
        const int iy = x + nx * (y + (ny + 1) * z);
        const int iz = x + nx * (y + ny * z);
        n.bxm = fa.c[0][ix];
        n.bxp = fa.c[0][ix + 1];
        n.bym = fa.c[1][iy];
        n.byp = fa.c[1][iy + nx];
        n.bzm = fa.c[2][iz];
        n.bzp = fa.c[2][iz + nx * ny];
    }
    return rc + m;
}

// push_ghosts() on a one-box coarse-cycle level: a face neighbour >= 0 is the
// box itself (periodic), else the face is a Dirichlet face
template <class T, class M>
__device__ __forceinline__ void blk_push(const M& U, const RBox& B, int i, int j, int k, T v) {
    const int c[3] = {i, j, k};
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            if (c[d] != (side ? B.hi[d] : B.lo[d])) continue;
            const int q = 2 * d + side;
            int t[3] = {i, j, k};
            if (B.nb[q] >= 0) {
                t[d] += B.shift[q];
                U.st(blk_off(B, t[0], t[1], t[2]), v);
            } else {
                t[d] += side ? 1 : -1;
                U.st(blk_off(B, t[0], t[1], t[2]), -v);
            }
        }
}

// A level of the coarse cycle: its descriptor and its u and f (LDS or device
// memory), with generic pointers for the bottom solver.
template <class T, bool LDS>
struct LevelData {
    const CoarseLevel<T>& L;
    LvMem<T, LDS> u, f;
    T* ug;
    T* fg;
};

template <class T, int MODE, bool LDS>
__device__ void blk_gs(const LevelData<T, LDS>& D, int colour) {
    const RBox& B = D.L.box;
    const BoxCells bc = box_cells(B);
    const T h2 = (T)(D.L.h * D.L.h);
    const T dg = diag_shift<T>(B);
    for (int g = threadIdx.x; g < bc.n; g += blockDim.x) {
        int i, j, k;
        if (!box_colour_cell(B, bc, g, colour, i, j, k)) continue;
        Nbr<T> nb;
        const int idx = blk_gather<T, MODE, false>(D.u, D.L.fa, B, i, j, k, nb);
        T su, sb;
        sums<T, MODE>(nb, su, sb);
        sb = sb + dg;
        const T v = (su - h2 * D.f.ld(idx)) / sb;
        D.u.st(idx, v);
        if (D.L.push) blk_push(D.u, B, i, j, k, v);
    }
    __syncthreads();
}

template <class T, int MODE, bool LDS>
__device__ void blk_smooth(const LevelData<T, LDS>& D, int nsweeps) {
    for (int s = 0; s < nsweeps; ++s)
        for (int c = 0; c < 2; ++c) {
            if (!D.L.push) blk_fill(D.u, D.L.face[c ^ 1], D.L.nface[c ^ 1]);
            blk_gs<T, MODE>(D, c);
        }
}

template <class T, int MODE, bool LDS>
__device__ void blk_resid_restrict(const LevelData<T, LDS>& F, const LevelData<T, LDS>& C) {
    const RBox& B = F.L.box;
    const int cnx = (B.hi[0] - B.lo[0] + 1) >> 1, cny = (B.hi[1] - B.lo[1] + 1) >> 1, cnz = (B.hi[2] - B.lo[2] + 1) >> 1;
    const int n = cnx * cny * cnz;
    const float rnx = 1.0f / (float)cnx, rny = 1.0f / (float)cny;
    const T ih2 = (T)(1.0 / (F.L.h * F.L.h));
    const T dg = diag_shift<T>(B);
    for (int g = threadIdx.x; g < n; g += blockDim.x) {
        int gy, gx, gz, gyy;
        small_divmod(g, cnx, rnx, gy, gx);
        small_divmod(gy, cny, rny, gz, gyy);
        const int I = (B.lo[0] >> 1) + gx, J = (B.lo[1] >> 1) + gyy, K = (B.lo[2] >> 1) + gz;
        const int i = 2 * I, j = 2 * J, k = 2 * K;
        auto ra = [&](int a, int b, int c) {
            Nbr<T> nb;
            const int idx = blk_gather<T, MODE, true>(F.u, F.L.fa, B, a, b, c, nb);
            T su, sb;
            sums<T, MODE>(nb, su, sb);
            sb = sb + dg;
            return F.f.ld(idx) - (su - sb * nb.c) * ih2;
        };
        const T r000 = ra(i, j, k), r100 = ra(i + 1, j, k), r010 = ra(i, j + 1, k), r110 = ra(i + 1, j + 1, k);
        const T r001 = ra(i, j, k + 1), r101 = ra(i + 1, j, k + 1), r011 = ra(i, j + 1, k + 1);
        const T r111 = ra(i + 1, j + 1, k + 1);
        const T s = ((r000 + r100) + (r010 + r110)) + ((r001 + r101) + (r011 + r111));
        C.f.st(blk_off(C.L.box, I, J, K), s * T(0.125));
    }
    __syncthreads();
}

template <class T, bool LDS>
__device__ void blk_zero(const LvMem<T, LDS>& u, long long n) {
    for (int g = threadIdx.x; g < (int)n; g += blockDim.x) u.st(g, T(0));
    __syncthreads();
}

// four elements per thread and step, loaded before any is stored (a copy
// from device memory waits for one load's latency per step, not per element)
template <class T, bool LD, bool LS>
__device__ void blk_copy(const LvMem<T, LD>& dst, const LvMem<T, LS>& src, long long n) {
    const int bs = blockDim.x, ni = (int)n;
    for (int g0 = threadIdx.x; g0 < ni; g0 += 4 * bs) {
        T v[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) v[m] = g0 + m * bs < ni ? src.ld(g0 + m * bs) : T(0);
#pragma unroll
        for (int m = 0; m < 4; ++m)
            if (g0 + m * bs < ni) dst.st(g0 + m * bs, v[m]);
    }
    __syncthreads();
}

template <class T, bool LDS>
__device__ void blk_prolong(const LevelData<T, LDS>& C, const LevelData<T, LDS>& F, int order) {
    const RBox& B = F.L.box;
    const RBox& Q = C.L.box;
    const BoxCells bc = box_cells(B);
    for (int g = threadIdx.x; g < bc.n; g += blockDim.x)
        for (int c = 0; c < 2; ++c) {
            int i, j, k;
            if (!box_colour_cell(B, bc, g, c, i, j, k)) continue;
            const int I = i >> 1, J = j >> 1, K = k >> 1;
            const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
            const T c000 = C.u.ld(blk_off(Q, I, J, K));
            T e;
            if (order == 1) {
                e = c000;
            } else {
                const T c100 = C.u.ld(blk_off(Q, I + si, J, K)), c010 = C.u.ld(blk_off(Q, I, J + sj, K));
                const T c001 = C.u.ld(blk_off(Q, I, J, K + sk));
                const T c110 = C.u.ld(blk_off(Q, I + si, J + sj, K)), c101 = C.u.ld(blk_off(Q, I + si, J, K + sk));
                const T c011 = C.u.ld(blk_off(Q, I, J + sj, K + sk));
                const T c111 = C.u.ld(blk_off(Q, I + si, J + sj, K + sk));
                e = (((T(27) * c000 + T(9) * ((c100 + c010) + c001)) + T(3) * ((c110 + c101) + c011)) + c111) *
                    T(0.015625);
            }
            const int idx = blk_off(B, i, j, k);
            const T v = F.u.ld(idx) + e;
            F.u.st(idx, v);
            if (F.L.push) blk_push(F.u, B, i, j, k, v);
        }
    __syncthreads();
}

// The fused coarse V-cycle of one problem per workgroup.  LDS: the levels'
// u and f live in LDS for the whole cycle (they are scratch below the top
// level); the top level's f is read at the start and its u, the correction,
// written back at the end.  Otherwise they stay in device memory.  Either
// way the cycle starts by zeroing the top level's u.
template <class T, int MODE, bool LDS>
__global__ void __launch_bounds__(kBotThreads) k_coarse_cycle(const CoarseCycle<T>* __restrict__ ccs,
                                                             const int* __restrict__ active) {
    typedef __attribute__((address_space(3))) T lds_T;
    const CoarseCycle<T>& cc = ccs[blockIdx.x];
    if (active && !active[cc.pid]) return;
    const int nl = cc.nlev;
    auto lev = [&](int m) {
        if constexpr (LDS) {
            T* ug = (T*)(bxmg_lds + cc.lds_u[m]);
            T* fg = (T*)(bxmg_lds + cc.lds_f[m]);
            return LevelData<T, true>{cc.L[m], {(lds_T*)ug}, {(lds_T*)fg}, ug, fg};
        } else {
            return LevelData<T, false>{cc.L[m], {cc.L[m].u}, {cc.L[m].f}, cc.L[m].u, cc.L[m].f};
        }
    };
    {
        const auto top = lev(0);
        blk_zero(top.u, cc.L[0].nelem);
        if constexpr (LDS) blk_copy(top.f, LvMem<T, false>{cc.L[0].f}, cc.L[0].nelem);
    }
    for (int l = 0; l + 1 < nl; ++l) {
        const auto F = lev(l), C = lev(l + 1);
        blk_smooth<T, MODE>(F, cc.nu1);
        if (!F.L.push) {
            blk_fill(F.u, F.L.face[0], F.L.nface[0]);
            blk_fill(F.u, F.L.face[1], F.L.nface[1]);
        }
        blk_resid_restrict<T, MODE>(F, C);
        blk_zero(C.u, C.L.nelem);
    }
    {
        const auto Db = lev(nl - 1);
        const CoarseLevel<T>& Lb = cc.L[nl - 1];
        BottomGeom G;
        for (int d = 0; d < 3; ++d) {
            G.dlo[d] = Lb.box.lo[d];
            G.n[d] = Lb.box.hi[d] - Lb.box.lo[d] + 1;
            G.per[d] = cc.per[d];
        }
        G.nboxes = 1;
        G.a = Lb.box.a;
        const int N = G.n[0] * G.n[1] * G.n[2];
        BottomLds S(bxmg_lds + cc.bot_off, N, (G.n[0] + 2) * (G.n[1] + 2) * (G.n[2] + 2));
        if (N <= kWaveBottomCells) {
            if (threadIdx.x < 64) bottom_cg_wave<T, MODE == 2>(Db.ug, Db.fg, Lb.fa, &Lb.box, G, Lb.h, cc.rtol, cc.iters, S);
        } else {
            bottom_cg<T, MODE == 2>(Db.ug, Db.fg, Lb.fa, &Lb.box, G, Lb.h, cc.rtol, cc.iters, S);
        }
        __syncthreads();
    }
    for (int l = nl - 2; l >= 0; --l) {
        const auto F = lev(l), C = lev(l + 1);
        blk_fill(C.u, C.L.full, C.L.nfull);
        blk_prolong(C, F, cc.prolong);
        blk_smooth<T, MODE>(F, cc.nu2);
    }
    if constexpr (LDS) blk_copy(LvMem<T, false>{cc.L[0].u}, lev(0).u, cc.L[0].nelem);
}

// ================================================================ launchers
static inline unsigned nblk(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

int lds_limit_bytes() {
    static int limit = 0;
    if (!limit) {
        int dev = 0, a = 0, b = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        (void)hipDeviceGetAttribute(&b, hipDeviceAttributeSharedMemPerBlockOptin, dev);
        limit = std::max(std::max(a, b), 65536);
    }
    return limit;
}

template <class T>
int coarse_lds_layout(CoarseCycle<T>& cc, bool allow_levels) {
    const RBox& B = cc.L[cc.nlev - 1].box;
    const int n0 = B.hi[0] - B.lo[0] + 1, n1 = B.hi[1] - B.lo[1] + 1, n2 = B.hi[2] - B.lo[2] + 1;
    const size_t bot = bottom_lds_bytes(n0 * n1 * n2, (n0 + 2) * (n1 + 2) * (n2 + 2));
    auto a16 = [](size_t x) { return (x + 15) / 16 * 16; };
    size_t off = 0;
    for (int m = 0; m < cc.nlev; ++m) {
        cc.lds_u[m] = (int)off;
        off += a16((size_t)cc.L[m].nelem * sizeof(T));
        cc.lds_f[m] = (int)off;
        off += a16((size_t)cc.L[m].nelem * sizeof(T));
    }
    if (allow_levels && off + bot <= (size_t)lds_limit_bytes()) {
        cc.lds = 1;
        cc.bot_off = (int)off;
        return (int)(off + bot);
    }
    cc.lds = 0;
    cc.bot_off = 0;
    return (int)bot;
}
template int coarse_lds_layout<double>(CoarseCycle<double>&, bool);
template int coarse_lds_layout<float>(CoarseCycle<float>&, bool);

// Lets a one-workgroup kernel take the device's whole LDS as dynamic LDS.
static bool allow_lds(const void* fn) {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_limit_bytes());
    return true;
}

hipError_t launch_fill_rb(hipStream_t s, void* data, bool f32, const GhostCopy* list, long long n, const int* active) {
    if (n <= 0) return hipSuccess;
    if (f32) hipLaunchKernelGGL(k_fill_rb<float>, dim3(nblk(n)), dim3(kBlock), 0, s, (float*)data, list, n, active);
    else hipLaunchKernelGGL(k_fill_rb<double>, dim3(nblk(n)), dim3(kBlock), 0, s, (double*)data, list, n, active);
    return hipGetLastError();
}

hipError_t launch_copy_fab(hipStream_t s, bool f32, void* dst, const FBox* dboxes, const void* src,
                           const FBox* sboxes, const Tag* tags, int ntags, long long ncells, int dcomp, int scomp,
                           int ncomp, const int* hints) {
    if (ncells <= 0) return hipSuccess;
    if (f32)
        hipLaunchKernelGGL(k_copy_fab<float>, dim3(nblk(ncells)), dim3(kBlock), 0, s, (float*)dst, dboxes,
                           (const float*)src, sboxes, tags, ntags, ncells, dcomp, scomp, ncomp, hints);
    else
        hipLaunchKernelGGL(k_copy_fab<double>, dim3(nblk(ncells)), dim3(kBlock), 0, s, (double*)dst, dboxes,
                           (const double*)src, sboxes, tags, ntags, ncells, dcomp, scomp, ncomp, hints);
    return hipGetLastError();
}

hipError_t launch_fill_fab(hipStream_t s, void* data, bool f32, const FBox* boxes, const Tag* tags, int ntags,
                           long long ncells, int comp0, int ncomp, const int* hints) {
    if (ncells <= 0) return hipSuccess;
    if (f32)
        hipLaunchKernelGGL(k_fill_fab<float>, dim3(nblk(ncells)), dim3(kBlock), 0, s, (float*)data, boxes, tags, ntags,
                           ncells, comp0, ncomp, hints);
    else
        hipLaunchKernelGGL(k_fill_fab<double>, dim3(nblk(ncells)), dim3(kBlock), 0, s, (double*)data, boxes, tags,
                           ntags, ncells, comp0, ncomp, hints);
    return hipGetLastError();
}

template <class T>
hipError_t launch_gs(hipStream_t s, const Grid& g, T* u, const T* f, const T* beta, const FaceArrays<T>* fat,
                     int colour, double* norm_partials) {
    if (g.ntiles <= 0) return hipSuccess;
    const dim3 G(g.ntiles), B(kBlock);
    if (norm_partials) {  // the fused residual: FP64, pushing, buffer-addressed levels
        if constexpr (std::is_same<T, double>::value) {
            if (!g.push || !g.res) return hipErrorInvalidValue;
#define BXMG_GSN(MODE, PUSH) \
    hipLaunchKernelGGL((k_gs<T, MODE, PUSH, true, true>), G, B, 0, s, g, u, f, beta, fat, colour, norm_partials)
            if (g.push == 2) {
                if (beta) BXMG_GSN(1, 2);
                else if (fat) BXMG_GSN(2, 2);
                else BXMG_GSN(0, 2);
            } else {
                if (beta) BXMG_GSN(1, 1);
                else if (fat) BXMG_GSN(2, 1);
                else BXMG_GSN(0, 1);
            }
#undef BXMG_GSN
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
#define BXMG_GS(MODE, PUSH, RES) \
    hipLaunchKernelGGL((k_gs<T, MODE, PUSH, RES, false>), G, B, 0, s, g, u, f, beta, fat, colour, (double*)nullptr)
#define BXMG_GS_MODES(PUSH, RES) \
    if (beta) BXMG_GS(1, PUSH, RES); else if (fat) BXMG_GS(2, PUSH, RES); else BXMG_GS(0, PUSH, RES)
    if (g.push == 2 && g.res) {
        BXMG_GS_MODES(2, true);
    } else if (g.push) {
        if (g.res) { BXMG_GS_MODES(1, true); } else { BXMG_GS_MODES(1, false); }
    } else {
        if (g.res) { BXMG_GS_MODES(0, true); } else { BXMG_GS_MODES(0, false); }
    }
#undef BXMG_GS_MODES
#undef BXMG_GS
    return hipGetLastError();
}
template hipError_t launch_gs<double>(hipStream_t, const Grid&, double*, const double*, const double*,
                                      const FaceArrays<double>*, int, double*);
template hipError_t launch_gs<float>(hipStream_t, const Grid&, float*, const float*, const float*,
                                     const FaceArrays<float>*, int, double*);

template <class T, class R>
hipError_t launch_resid(hipStream_t s, const Grid& g, const T* u, const T* f, const T* beta,
                        const FaceArrays<T>* fat, R* r, double* partials, bool colour0_only, const int* nonzero) {
    if (g.ntiles <= 0) return hipSuccess;
    const dim3 G(g.ntiles), B(kBlock);
    if (colour0_only) {  // after a fused colour-1 sweep: FP64, buffer-addressed, norms only
        if constexpr (std::is_same<T, double>::value && std::is_same<R, double>::value) {
            if (!g.res || r) return hipErrorInvalidValue;
#define BXMG_RS0(MODE) \
    hipLaunchKernelGGL((k_resid<T, MODE, R, true, 1>), G, B, 0, s, g, u, f, beta, fat, r, partials, nonzero)
            if (beta) BXMG_RS0(1);
            else if (fat) BXMG_RS0(2);
            else BXMG_RS0(0);
#undef BXMG_RS0
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    }
#define BXMG_RS(MODE, RES) \
    hipLaunchKernelGGL((k_resid<T, MODE, R, RES, 3>), G, B, 0, s, g, u, f, beta, fat, r, partials, nonzero)
    if (g.res) {
        if (beta) BXMG_RS(1, true); else if (fat) BXMG_RS(2, true); else BXMG_RS(0, true);
    } else {
        if (beta) BXMG_RS(1, false); else if (fat) BXMG_RS(2, false); else BXMG_RS(0, false);
    }
#undef BXMG_RS
    return hipGetLastError();
}
template hipError_t launch_resid<double, double>(hipStream_t, const Grid&, const double*, const double*, const double*,
                                                 const FaceArrays<double>*, double*, double*, bool, const int*);
template hipError_t launch_resid<double, float>(hipStream_t, const Grid&, const double*, const double*, const double*,
                                                const FaceArrays<double>*, float*, double*, bool, const int*);
template hipError_t launch_resid<float, float>(hipStream_t, const Grid&, const float*, const float*, const float*,
                                               const FaceArrays<float>*, float*, double*, bool, const int*);

hipError_t launch_norm_final(hipStream_t s, const double* partials, int n, double* out3) {
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kNormThreads), 0, s, partials, n, out3);
    return hipGetLastError();
}

hipError_t launch_field_norm(hipStream_t s, const Grid& g, const double* x, double* partials) {
    if (g.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_field_norm, dim3(g.ntiles), dim3(kBlock), 0, s, g, x, partials);
    return hipGetLastError();
}

template <class T>
hipError_t launch_resid_restrict(hipStream_t s, const XGrid& x, const T* u, const T* f, const T* beta,
                                 const FaceArrays<T>* fat, T* fc, T* uz) {
    if (x.ntiles <= 0) return hipSuccess;
    const dim3 G(x.ntiles), B(kBlock);
    if (beta) hipLaunchKernelGGL((k_resid_restrict<T, 1>), G, B, 0, s, x, u, f, beta, fat, fc, uz);
    else if (fat) hipLaunchKernelGGL((k_resid_restrict<T, 2>), G, B, 0, s, x, u, f, beta, fat, fc, uz);
    else hipLaunchKernelGGL((k_resid_restrict<T, 0>), G, B, 0, s, x, u, f, beta, fat, fc, uz);
    return hipGetLastError();
}
template hipError_t launch_resid_restrict<double>(hipStream_t, const XGrid&, const double*, const double*,
                                                  const double*, const FaceArrays<double>*, double*, double*);
template hipError_t launch_resid_restrict<float>(hipStream_t, const XGrid&, const float*, const float*, const float*,
                                                 const FaceArrays<float>*, float*, float*);

template <class T>
hipError_t launch_restrict_plain(hipStream_t s, const XGrid& x, const T* rf, T* fc) {
    if (x.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_restrict_plain<T>, dim3(x.ntiles), dim3(kBlock), 0, s, x, rf, fc);
    return hipGetLastError();
}
template hipError_t launch_restrict_plain<double>(hipStream_t, const XGrid&, const double*, double*);

template <class T>
hipError_t launch_prolong(hipStream_t s, const Grid& fine, const RBox* cboxes, const int* cbox, const T* ec, T* uf,
                          int order, bool only_c1, int stage_values, bool coarse_self, long long fine_face_cells) {
    if (fine.ntiles <= 0) return hipSuccess;
    // a one-box fine level: its face work goes to a second launch over the face cells
    const bool faces_apart = fine_face_cells > 0;
    const long long nface = fine_face_cells;
    const dim3 G(fine.ntiles), B(kBlock);
    // levels refreshed by fill lists copy ghosts from both colours' cells:
    // they keep the two-colour kernel
    const bool c1 = only_c1 && fine.push;
    const bool staged = prolong_staged(fine.push, only_c1, stage_values);
#define BXMG_PROLONG(PUSH, ORDER)                                                                    \
    do {                                                                                            \
        if (PUSH && c1 && staged && coarse_self)                                                    \
            hipLaunchKernelGGL((k_prolong_c1s<T, ORDER, true, true>), G, B, 0, s, fine, cboxes, cbox, ec, uf); \
        else if (PUSH && c1 && staged && faces_apart) {                                             \
            hipLaunchKernelGGL((k_prolong_c1s<T, ORDER, false, false>), G, B, 0, s, fine, cboxes, cbox, ec, uf); \
            hipLaunchKernelGGL((k_prolong_faces<T, ORDER>), dim3(nblk(nface)), B, 0, s, fine, cboxes, cbox, ec, uf); \
        } else if (PUSH && c1 && staged)                                                            \
            hipLaunchKernelGGL((k_prolong_c1s<T, ORDER, false, true>), G, B, 0, s, fine, cboxes, cbox, ec, uf); \
        else if (PUSH && c1) hipLaunchKernelGGL((k_prolong_c1<T, ORDER>), G, B, 0, s, fine, cboxes, cbox, ec, uf); \
        else hipLaunchKernelGGL((k_prolong<T, PUSH, ORDER>), G, B, 0, s, fine, cboxes, cbox, ec, uf); \
    } while (0)
    if (order == 1) {
        if (fine.push) BXMG_PROLONG(true, 1);
        else BXMG_PROLONG(false, 1);
    } else {
        if (fine.push) BXMG_PROLONG(true, 2);
        else BXMG_PROLONG(false, 2);
    }
#undef BXMG_PROLONG
    return hipGetLastError();
}
template hipError_t launch_prolong<double>(hipStream_t, const Grid&, const RBox*, const int*, const double*, double*,
                                           int, bool, int, bool, long long);
template hipError_t launch_prolong<float>(hipStream_t, const Grid&, const RBox*, const int*, const float*, float*, int,
                                          bool, int, bool, long long);

template <class T>
hipError_t launch_zero(hipStream_t s, T* p, long long n, const int* active) {
    if (n <= 0) return hipSuccess;
    const long long nb = std::min<long long>(nblk(n), 8192);
    hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)nb), dim3(kBlock), 0, s, p, n, active);
    return hipGetLastError();
}
template hipError_t launch_zero<double>(hipStream_t, double*, long long, const int*);
template hipError_t launch_zero<float>(hipStream_t, float*, long long, const int*);

hipError_t launch_cast_f32(hipStream_t s, const double* src, float* dst, long long n) {
    if (n <= 0) return hipSuccess;
    const long long nb = std::min<long long>(nblk(n), 8192);
    hipLaunchKernelGGL(k_cast_f32, dim3((unsigned)nb), dim3(kBlock), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_fab_to_rb_norm(hipStream_t s, const Grid& g, const double* fab, const FBox* fb, double* rb,
                                double* partials) {
    if (g.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fab_to_rb_norm, dim3(g.ntiles), dim3(kBlock), 0, s, g, fab, fb, rb, partials);
    return hipGetLastError();
}

hipError_t launch_heat_rhs(hipStream_t s, const Grid& g, const double* u, const FBox* fu, const double* src,
                           const FBox* fs, double inv_dt, double* f, double* partials) {
    if (g.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_heat_rhs, dim3(g.ntiles), dim3(kBlock), 0, s, g, u, fu, src, fs, inv_dt, f, partials);
    return hipGetLastError();
}

hipError_t launch_fab_to_rb(hipStream_t s, const Grid& g, const double* fab, const FBox* fb, void* rb, bool f32) {
    if (g.ntiles <= 0) return hipSuccess;
    if (f32) hipLaunchKernelGGL(k_fab_to_rb<float>, dim3(g.ntiles), dim3(kBlock), 0, s, g, fab, fb, (float*)rb);
    else hipLaunchKernelGGL(k_fab_to_rb<double>, dim3(g.ntiles), dim3(kBlock), 0, s, g, fab, fb, (double*)rb);
    return hipGetLastError();
}

hipError_t launch_fab_to_rb_nz(hipStream_t s, const Grid& g, const double* fab, const FBox* fb, double* rb,
                               int* nonzero) {
    if (g.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fab_to_rb_nz, dim3(g.ntiles), dim3(kBlock), 0, s, g, fab, fb, rb, nonzero);
    return hipGetLastError();
}

hipError_t launch_rb_to_fab(hipStream_t s, const Grid& g, const double* rb, double* fab, const FBox* fb) {
    if (g.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rb_to_fab, dim3(g.ntiles), dim3(kBlock), 0, s, g, rb, fab, fb);
    return hipGetLastError();
}

hipError_t launch_add_f32(hipStream_t s, const Grid& g, double* u, const float* e) {
    if (g.ntiles <= 0) return hipSuccess;
    if (g.push == 2 && g.res) hipLaunchKernelGGL(k_add_f32<true>, dim3(g.ntiles), dim3(kBlock), 0, s, g, u, e);
    else hipLaunchKernelGGL(k_add_f32<false>, dim3(g.ntiles), dim3(kBlock), 0, s, g, u, e);
    return hipGetLastError();
}

hipError_t launch_mean_sub_many(hipStream_t s, const Grid& g, const RetireBox* info, const int* seg_tiles, int nseg,
                                double* u, double* scratch) {
    if (g.ntiles <= 0 || nseg <= 0) return hipSuccess;
    double* tot = scratch + 3 * (long long)g.ntiles;
    hipLaunchKernelGGL(k_sum_valid_many, dim3(g.ntiles), dim3(kBlock), 0, s, g, info, u, scratch);
    hipLaunchKernelGGL(k_norm_final_seg, dim3(nseg), dim3(kNormThreads), 0, s, scratch, seg_tiles, tot);
    hipLaunchKernelGGL(k_sub_mean_many, dim3(g.ntiles), dim3(kBlock), 0, s, g, info, u, tot);
    return hipGetLastError();
}

hipError_t launch_rb_to_fab_many(hipStream_t s, const Grid& g, const double* rb, const RetireBox* info) {
    if (g.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rb_to_fab_many, dim3(g.ntiles), dim3(kBlock), 0, s, g, rb, info);
    return hipGetLastError();
}

hipError_t launch_mean_sub(hipStream_t s, const Grid& g, double* u, double* scratch) {
    if (g.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_valid, dim3(g.ntiles), dim3(kBlock), 0, s, g, u, scratch);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(kNormThreads), 0, s, scratch, g.ntiles,
                       scratch + 3 * (long long)g.ntiles);
    hipLaunchKernelGGL(k_sub_mean, dim3(g.ntiles), dim3(kBlock), 0, s, g, u, scratch + 3 * (long long)g.ntiles);
    return hipGetLastError();
}

template <class T>
hipError_t launch_faces_from_cells(hipStream_t s, const XGrid& x, const T* beta, int d, FaceArrays<T> out, T* dst) {
    if (x.ntiles <= 0) return hipSuccess;
    // fine domain upper end in d = 2 * (coarse upper end) + 1
    const int fdom_hi = 2 * (out.dlo[d] + out.n[d] - 1) + 1;
    hipLaunchKernelGGL(k_faces_from_cells<T>, dim3(x.ntiles), dim3(kBlock), 0, s, x, beta, d, fdom_hi, out, dst);
    return hipGetLastError();
}
template hipError_t launch_faces_from_cells<double>(hipStream_t, const XGrid&, const double*, int, FaceArrays<double>,
                                                    double*);
template hipError_t launch_faces_from_cells<float>(hipStream_t, const XGrid&, const float*, int, FaceArrays<float>,
                                                   float*);

template <class T>
hipError_t launch_faces_coarsen(hipStream_t s, FaceArrays<T> fine, FaceArrays<T> coarse, int d, T* dst) {
    const long long total = (long long)(coarse.n[0] + (d == 0)) * (coarse.n[1] + (d == 1)) * (coarse.n[2] + (d == 2));
    hipLaunchKernelGGL(k_faces_coarsen<T>, dim3(nblk(total)), dim3(kBlock), 0, s, fine, coarse, d, dst);
    return hipGetLastError();
}
template hipError_t launch_faces_coarsen<double>(hipStream_t, FaceArrays<double>, FaceArrays<double>, int, double*);
template hipError_t launch_faces_coarsen<float>(hipStream_t, FaceArrays<float>, FaceArrays<float>, int, float*);

template <class T>
hipError_t launch_bottom(hipStream_t s, T* u, const T* f, FaceArrays<T> fa, bool var, const RBox* boxes, int nboxes,
                         const int* dom_lo, const int* dom_hi, const int* periodic, double h, double alpha,
                         double rtol, int* iters_out) {
    BottomGeom G;
    G.a = alpha;
    for (int d = 0; d < 3; ++d) {
        G.dlo[d] = dom_lo[d];
        G.n[d] = dom_hi[d] - dom_lo[d] + 1;
        G.per[d] = periodic[d];
    }
    G.nboxes = nboxes;
    const int n = G.n[0] * G.n[1] * G.n[2], ng = (G.n[0] + 2) * (G.n[1] + 2) * (G.n[2] + 2);
    const size_t lds = bottom_lds_bytes(n, ng);
    if (var) {
        static const bool once = allow_lds((const void*)k_bottom<T, true>);
        (void)once;
        hipLaunchKernelGGL((k_bottom<T, true>), dim3(1), dim3(kBotThreads), lds, s, u, f, fa, boxes, G, h, rtol, iters_out);
    } else {
        static const bool once = allow_lds((const void*)k_bottom<T, false>);
        (void)once;
        hipLaunchKernelGGL((k_bottom<T, false>), dim3(1), dim3(kBotThreads), lds, s, u, f, fa, boxes, G, h, rtol, iters_out);
    }
    return hipGetLastError();
}
template hipError_t launch_bottom<double>(hipStream_t, double*, const double*, FaceArrays<double>, bool, const RBox*,
                                          int, const int*, const int*, const int*, double, double, double, int*);
template hipError_t launch_bottom<float>(hipStream_t, float*, const float*, FaceArrays<float>, bool, const RBox*, int,
                                         const int*, const int*, const int*, double, double, double, int*);

template <class T>
hipError_t launch_coarse_cycle(hipStream_t s, const CoarseCycle<T>* cc, int n, const int* active, bool var,
                               int lds_bytes, bool levels_lds) {
    if (n <= 0) return hipSuccess;
#define BXMG_CC(MODE, LDS)                                                                                 \
    do {                                                                                                   \
        static const bool once = allow_lds((const void*)k_coarse_cycle<T, MODE, LDS>);                     \
        (void)once;                                                                                        \
        hipLaunchKernelGGL((k_coarse_cycle<T, MODE, LDS>), dim3(n), dim3(kBotThreads), lds_bytes, s, cc, active); \
    } while (0)
    if (var) {
        if (levels_lds) BXMG_CC(2, true);
        else BXMG_CC(2, false);
    } else {
        if (levels_lds) BXMG_CC(0, true);
        else BXMG_CC(0, false);
    }
#undef BXMG_CC
    return hipGetLastError();
}
template hipError_t launch_coarse_cycle<double>(hipStream_t, const CoarseCycle<double>*, int, const int*, bool, int,
                                                bool);
template hipError_t launch_coarse_cycle<float>(hipStream_t, const CoarseCycle<float>*, int, const int*, bool, int,
                                               bool);

// ------------------------------------------------------------ batch kernels
// One block per segment: a fixed-tree reduction over the segment's tiles, in
// tile order (max norms are exact in any order; the L2 sums depend on the
// tree only in rounding).
__global__ void __launch_bounds__(kBlock) k_norm_seg(const double* __restrict__ partials, const int* __restrict__ tstart,
                                                    const int* __restrict__ seg_slot, const int* __restrict__ active,
                                                    double* __restrict__ norms) {
    __shared__ double sh[3 * (kBlock / 64)];
    const int q = blockIdx.x, p = seg_slot[q];
    if (active && !active[p]) return;
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    for (int t = tstart[q] + (int)threadIdx.x; t < tstart[q + 1]; t += blockDim.x) {
        mx = fmax(mx, partials[3 * t]);
        s2 = s2 + partials[3 * t + 1];
        bad = bad + partials[3 * t + 2];
    }
    block_reduce3(mx, s2, bad, sh);
    if (threadIdx.x == 0) { norms[3 * p] = mx; norms[3 * p + 1] = s2; norms[3 * p + 2] = bad; }
}

// One thread per member slot, one block: the same stop test as the
// single-problem driver (history entry, then stop or count one more cycle).
__global__ void __launch_bounds__(1024) k_batch_check(const int* __restrict__ slots, int n,
                                                     const double* __restrict__ norms, BatchSlot* __restrict__ st,
                                                     int* __restrict__ active, double* __restrict__ hist,
                                                     double* __restrict__ hist_l2, int* __restrict__ nactive,
                                                     int* __restrict__ seen) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int mine = 0;
    for (int q = threadIdx.x; q < n; q += blockDim.x) {
        const int p = slots[q];
        if (!active[p]) continue;
        if (seen) seen[p] = 1;  // the iterate after this check is no zero guess
        BatchSlot S = st[p];
        const double rinf = norms[3 * p + 2] > 0.0 ? (double)NAN : norms[3 * p];
        const int c = S.cycles;
        if (c < kHist) {
            hist[(long long)p * kHist + c] = rinf / S.fnorm;
            hist_l2[(long long)p * kHist + c] = sqrt(norms[3 * p + 1]);
            S.nhist = c + 1;
        }
        bool done = false;
        if (!(fabs(rinf) <= 1.7976931348623157e308)) {
            S.status = kStatusNonFinite;
            done = true;
        } else if (S.fixed_cycles > 0) {
            done = (c == S.fixed_cycles);
        } else if (rinf <= S.rel_tol * S.fnorm || rinf <= S.abs_tol) {
            done = true;
        } else if (c == S.max_cycles) {
            S.status = kStatusNoConv;
            done = true;
        }
        if (done) active[p] = 0;
        else { S.cycles = c + 1; ++mine; }
        st[p] = S;
    }
    if (mine) atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) *nactive = cnt;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_zero_ranges(T* __restrict__ p, const ZeroRange* __restrict__ r,
                                                       const int* __restrict__ active) {
    const ZeroRange R = r[blockIdx.y];
    if (active && !active[R.pid]) return;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < R.len; q += stride) p[R.start + q] = T(0);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_fill_sets(T* __restrict__ data, const GhostSet* __restrict__ sets,
                                                     const int* __restrict__ active) {
    const GhostSet S = sets[blockIdx.y];
    if (active && !active[S.pid]) return;
    T* d = data + S.off;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < S.n; g += stride) {
        const GhostCopy p = S.list[g];
        const T v = d[p.src & 0x7fffffffu];
        d[p.dst] = (p.src >> 31) ? -v : v;
    }
}

__global__ void k_batch_admit(const double* __restrict__ fn3, BatchSlot* __restrict__ st, int* __restrict__ active,
                              int slot) {
    if (threadIdx.x != 0) return;
    BatchSlot S = st[slot];
    S.fnorm = fn3[0];
    int act = 1;
    if (fn3[2] > 0.0) {
        S.status = kStatusNonFinite;
        act = 0;
    } else if (!(fn3[0] > 0.0)) {
        act = 0;  // f == 0: the solution is the initial guess
    }
    st[slot] = S;
    active[slot] = act;
}

hipError_t launch_fill_sets(hipStream_t s, void* data, bool f32, const GhostSet* sets, int nsets, long long max_n,
                            const int* active) {
    if (nsets <= 0 || max_n <= 0) return hipSuccess;
    const dim3 G((unsigned)std::min<long long>(nblk(max_n), 1024), (unsigned)nsets);
    if (f32) hipLaunchKernelGGL(k_fill_sets<float>, G, dim3(kBlock), 0, s, (float*)data, sets, active);
    else hipLaunchKernelGGL(k_fill_sets<double>, G, dim3(kBlock), 0, s, (double*)data, sets, active);
    return hipGetLastError();
}

// Admission in one launch: the norms of f reduced from the per-tile partials
// (as k_norm_final, into fn3), the slot state S written, then the decision
// of k_batch_admit.
__global__ void __launch_bounds__(kNormThreads) k_batch_admit_norms(const double* __restrict__ partials, int n,
                                                                   BatchSlot S, double* __restrict__ fn3,
                                                                   BatchSlot* __restrict__ st,
                                                                   int* __restrict__ active, int slot) {
    __shared__ double sh[3 * (kNormThreads / 64)];
    double mx, s2, bad;
    norm_reduce(partials, n, sh, mx, s2, bad);
    if (threadIdx.x != 0) return;
    fn3[0] = mx;
    fn3[1] = s2;
    fn3[2] = bad;
    S.fnorm = mx;
    int act = 1;
    if (bad > 0.0) {
        S.status = kStatusNonFinite;
        act = 0;
    } else if (!(mx > 0.0)) {
        act = 0;  // f == 0: the solution is the initial guess
    }
    st[slot] = S;
    active[slot] = act;
}

hipError_t launch_batch_admit_norms(hipStream_t s, const double* partials, int n, const BatchSlot& S, double* fn3,
                                    BatchSlot* st, int* active, int slot) {
    hipLaunchKernelGGL(k_batch_admit_norms, dim3(1), dim3(kNormThreads), 0, s, partials, n, S, fn3, st, active, slot);
    return hipGetLastError();
}

hipError_t launch_admit_convert(hipStream_t s, const Grid& g, const ConvSrc* src, double* u, double* f,
                                double* partials, int* nonzero) {
    if (g.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_admit_convert, dim3(g.ntiles), dim3(kBlock), 0, s, g, src, u, f, partials, nonzero);
    return hipGetLastError();
}

__global__ void k_batch_admit_many(const double* __restrict__ norms, const BatchSlot* __restrict__ states,
                                   const int* __restrict__ slots, int n, BatchSlot* __restrict__ st,
                                   int* __restrict__ active) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int slot = slots[q];
    const double* fn = norms + 3 * (long long)slot;
    BatchSlot S = states[q];
    S.fnorm = fn[0];
    int act = 1;
    if (fn[2] > 0.0) {
        S.status = kStatusNonFinite;
        act = 0;
    } else if (!(fn[0] > 0.0)) {
        act = 0;  // f == 0: the solution is the initial guess
    }
    st[slot] = S;
    active[slot] = act;
}

hipError_t launch_batch_admit_many(hipStream_t s, const double* norms, const BatchSlot* states, const int* slots,
                                   int n, BatchSlot* st, int* active) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_admit_many, dim3(nblk(n)), dim3(kBlock), 0, s, norms, states, slots, n, st, active);
    return hipGetLastError();
}

hipError_t launch_batch_admit(hipStream_t s, const double* fn3, BatchSlot* st, int* active, int slot) {
    hipLaunchKernelGGL(k_batch_admit, dim3(1), dim3(64), 0, s, fn3, st, active, slot);
    return hipGetLastError();
}

hipError_t launch_norm_seg(hipStream_t s, const double* partials, const int* tstart, const int* seg_slot, int nseg,
                           const int* active, double* norms) {
    if (nseg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_norm_seg, dim3(nseg), dim3(kBlock), 0, s, partials, tstart, seg_slot, active, norms);
    return hipGetLastError();
}

hipError_t launch_batch_check(hipStream_t s, const int* slots, int n, const double* norms, BatchSlot* st,
                              int* active, double* hist, double* hist_l2, int* nactive, int* seen) {
    hipLaunchKernelGGL(k_batch_check, dim3(1), dim3(1024), 0, s, slots, n, norms, st, active, hist, hist_l2, nactive,
                       seen);
    return hipGetLastError();
}

__global__ void k_set_slots(const int* __restrict__ slots, int n, int* __restrict__ a, int v) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) a[slots[q]] = v;
}

hipError_t launch_set_slots(hipStream_t s, const int* slots, int n, int* a, int v) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_slots, dim3((n + 255) / 256), dim3(256), 0, s, slots, n, a, v);
    return hipGetLastError();
}

template <class T>
hipError_t launch_zero_ranges(hipStream_t s, T* p, const ZeroRange* r, int n, long long max_len, const int* active) {
    if (n <= 0 || max_len <= 0) return hipSuccess;
    const long long nb = std::min<long long>(nblk(max_len), 1024);
    hipLaunchKernelGGL(k_zero_ranges<T>, dim3((unsigned)nb, (unsigned)n), dim3(kBlock), 0, s, p, r, active);
    return hipGetLastError();
}
template hipError_t launch_zero_ranges<double>(hipStream_t, double*, const ZeroRange*, int, long long, const int*);
template hipError_t launch_zero_ranges<float>(hipStream_t, float*, const ZeroRange*, int, long long, const int*);

// ------------------------------------ multigrid-preconditioned CG (level 0)
// Both colours of the valid cells of every tile, as k_resid walks them.

// p' = z + beta p, z = (double) e, over every element of the level (valid
// cells, ghosts and padding): the face ghosts of e and p hold reflections
// (-v) or periodic images of cells, and z + beta p of such values is exactly
// the same reflection or image of the cell's p', so p' needs no ghost
// refresh.  e is zeroed on the way: the next V-cycle starts from it.
template <class E>
__global__ void __launch_bounds__(kBlock) k_kr_axpy(E* __restrict__ e, const double* __restrict__ p,
                                                   double* __restrict__ pn, long long n,
                                                   const KrylovScalars* __restrict__ sc,
                                                   const int* __restrict__ active) {
    if (active && !active[0]) return;
    const double bs = sc->beta;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
        pn[q] = (double)e[q] + bs * p[q];
        e[q] = E(0);
    }
}

// q = L p = (su - sb p_c) / h^2 (k_resid's operation order) at every valid
// cell, partial sums of p.q per tile
template <int MODE, bool RES>
__global__ void __launch_bounds__(kBlock) k_kr_apply(Grid g, const double* __restrict__ p,
                                                    const double* __restrict__ beta, double* __restrict__ q,
                                                    double* __restrict__ partials) {
    __shared__ double sh[3 * (kBlock / 64)];
    double z0 = 0.0, pq = 0.0, z1 = 0.0;
    const int tix = tile_index(g.rev);
    const Tile tl = g.tiles[tix];
    const RBox B = g.boxes[tl.box];
    if (g.active && !g.active[B.pid]) return;
    const double ih2 = 1.0 / (B.h * B.h);
    const double dg = diag_shift<double>(B);
    const FaceArrays<double> fa{};
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    const long long ne = 2 * B.cstride;
    const BoxRes<double> P(p + B.base, ne), Bt((MODE == 1 ? beta : p) + B.base, ne), Q(q + B.base, ne);
    if (j <= B.hi[1])
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int k = B.lo[2] + th.z0 + z * th.dz;
            if (k > B.hi[2]) break;
            Nbr<double> nb[2];
            long long idx[2];
            bool ok[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {  // the loads of both cells first
                const int i = colour_i(B, th.x, j, k, c);
                ok[c] = i <= B.hi[0];
                if constexpr (RES) idx[c] = gather_res<double, MODE, true>(P, Bt, fa, B, ok[c] ? i : B.hi[0], j, k, nb[c]);
                else if (ok[c]) idx[c] = gather<double, MODE, true>(p, beta, fa, B, i, j, k, nb[c]);
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                if (!ok[c]) continue;
                double su, sb;
                sums<double, MODE>(nb[c], su, sb);
                sb = sb + dg;
                const double qv = (su - sb * nb[c].c) * ih2;
                if constexpr (RES) Q.st((int)idx[c], qv);
                else q[idx[c]] = qv;
                pq = pq + nb[c].c * qv;
            }
        }
    block_reduce3(z0, pq, z1, sh);
    if (threadIdx.x == 0) {
        partials[3 * tix] = 0.0;
        partials[3 * tix + 1] = pq;
        partials[3 * tix + 2] = 0.0;
    }
}

// x += alpha p, r -= alpha q, rhs = (E) r; norms of the new r
template <class E>
__global__ void __launch_bounds__(kBlock) k_kr_update(Grid g, double* __restrict__ x, const double* __restrict__ p,
                                                     double* __restrict__ r, const double* __restrict__ q,
                                                     E* __restrict__ rhs, const KrylovScalars* __restrict__ sc,
                                                     double* __restrict__ partials) {
    __shared__ double sh[3 * (kBlock / 64)];
    double mx = 0.0, s2 = 0.0, bad = 0.0;
    const int tix = tile_index(g.rev);
    const Tile tl = g.tiles[tix];
    const RBox B = g.boxes[tl.box];
    if (g.active && !g.active[B.pid]) return;
    const double a = sc->alpha;
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    if (j <= B.hi[1])
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int k = B.lo[2] + th.z0 + z * th.dz;
            if (k > B.hi[2]) break;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int i = colour_i(B, th.x, j, k, c);
                if (i > B.hi[0]) continue;
                const long long idx = rb_idx(B, i, j, k);
                const double pv = p[idx], qv = q[idx], xv = x[idx], rv0 = r[idx];
                x[idx] = xv + a * pv;
                const double rv = rv0 - a * qv;
                r[idx] = rv;
                rhs[idx] = (E)rv;
                acc_norm(rv, mx, s2, bad);
            }
        }
    block_reduce3(mx, s2, bad, sh);
    if (threadIdx.x == 0) {
        partials[3 * tix] = mx;
        partials[3 * tix + 1] = s2;
        partials[3 * tix + 2] = bad;
    }
}

// sums of z.q and z.r, z = (double) e
template <class E>
__global__ void __launch_bounds__(kBlock) k_kr_dots(Grid g, const E* __restrict__ e, const double* __restrict__ r,
                                                   const double* __restrict__ q, double* __restrict__ partials) {
    __shared__ double sh[3 * (kBlock / 64)];
    double z0 = 0.0, zq = 0.0, zr = 0.0;
    const int tix = tile_index(g.rev);
    const Tile tl = g.tiles[tix];
    const RBox B = g.boxes[tl.box];
    if (g.active && !g.active[B.pid]) return;
    const TileThread th = tile_thread(tl);
    const int j = B.lo[1] + th.y;
    if (j <= B.hi[1])
        for (int z = 0; z < (int)tl.zc; ++z) {
            const int k = B.lo[2] + th.z0 + z * th.dz;
            if (k > B.hi[2]) break;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int i = colour_i(B, th.x, j, k, c);
                if (i > B.hi[0]) continue;
                const long long idx = rb_idx(B, i, j, k);
                const double zv = (double)e[idx];
                zq = zq + zv * q[idx];
                zr = zr + zv * r[idx];
            }
        }
    block_reduce3(z0, zq, zr, sh);
    if (threadIdx.x == 0) {
        partials[3 * tix] = 0.0;
        partials[3 * tix + 1] = zq;
        partials[3 * tix + 2] = zr;
    }
}

__global__ void k_kr_step(const double* __restrict__ s3, KrylovScalars* __restrict__ sc, int step,
                          const int* __restrict__ active) {
    if (threadIdx.x != 0 || (active && !active[0])) return;
    KrylovScalars S = *sc;
    if (step == 0) {
        S.pq = s3[1];
        S.alpha = S.pq != 0.0 ? S.rz / S.pq : 0.0;
    } else if (step == 1) {
        S.beta = S.rz != 0.0 ? -S.alpha * s3[1] / S.rz : 0.0;
        S.rz = s3[2];
    } else {
        S.beta = 0.0;
        S.rz = s3[2];
    }
    *sc = S;
}

template <class E>
hipError_t launch_kr_axpy(hipStream_t s, E* e, const double* p, double* pn, long long n, const KrylovScalars* sc,
                          const int* active) {
    if (n <= 0) return hipSuccess;
    const long long nb = std::min<long long>(nblk(n), 8192);
    hipLaunchKernelGGL(k_kr_axpy<E>, dim3((unsigned)nb), dim3(kBlock), 0, s, e, p, pn, n, sc, active);
    return hipGetLastError();
}
hipError_t launch_kr_apply(hipStream_t s, const Grid& g, const double* p, const double* beta, double* q,
                           double* partials) {
    if (g.ntiles <= 0) return hipSuccess;
    const dim3 G(g.ntiles), B(kBlock);
    if (g.res) {
        if (beta) hipLaunchKernelGGL((k_kr_apply<1, true>), G, B, 0, s, g, p, beta, q, partials);
        else hipLaunchKernelGGL((k_kr_apply<0, true>), G, B, 0, s, g, p, beta, q, partials);
    } else {
        if (beta) hipLaunchKernelGGL((k_kr_apply<1, false>), G, B, 0, s, g, p, beta, q, partials);
        else hipLaunchKernelGGL((k_kr_apply<0, false>), G, B, 0, s, g, p, beta, q, partials);
    }
    return hipGetLastError();
}
template <class E>
hipError_t launch_kr_update(hipStream_t s, const Grid& g, double* x, const double* p, double* r, const double* q,
                            E* rhs, const KrylovScalars* sc, double* partials) {
    if (g.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kr_update<E>, dim3(g.ntiles), dim3(kBlock), 0, s, g, x, p, r, q, rhs, sc, partials);
    return hipGetLastError();
}
template <class E>
hipError_t launch_kr_dots(hipStream_t s, const Grid& g, const E* e, const double* r, const double* q,
                          double* partials) {
    if (g.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kr_dots<E>, dim3(g.ntiles), dim3(kBlock), 0, s, g, e, r, q, partials);
    return hipGetLastError();
}
hipError_t launch_kr_step(hipStream_t s, const double* sums3, KrylovScalars* sc, int step, const int* active) {
    hipLaunchKernelGGL(k_kr_step, dim3(1), dim3(64), 0, s, sums3, sc, step, active);
    return hipGetLastError();
}
#define BXMG_KR_INST(E)                                                                                          \
    template hipError_t launch_kr_axpy<E>(hipStream_t, E*, const double*, double*, long long,                    \
                                          const KrylovScalars*, const int*);                                     \
    template hipError_t launch_kr_update<E>(hipStream_t, const Grid&, double*, const double*, double*,           \
                                            const double*, E*, const KrylovScalars*, double*);                   \
    template hipError_t launch_kr_dots<E>(hipStream_t, const Grid&, const E*, const double*, const double*, double*);
BXMG_KR_INST(float)
BXMG_KR_INST(double)
#undef BXMG_KR_INST

// ------------------------------------------------ allocation-free staging
// One copy per GPU.  On the host this name stands for the array but is not
// its device address: host code uses only what scratch_address() returns.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void** out) {
    static std::mutex mu;
    static void* addr[kMaxScratchDevices] = {};
    if (device < 0 || device >= kMaxScratchDevices || !out) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

}  // namespace bxmg
