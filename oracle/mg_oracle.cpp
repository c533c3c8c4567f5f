// Oracle for the block-structured geometric-multigrid Poisson path.
//
// TEST INFRASTRUCTURE ONLY. Plain, slow, single-threaded, obviously-correct
// CPU implementation in FP64 (plus a float emulation of the FP32 inner
// V-cycle).  Only the test suite, the smoke check and the benchmark's
// CPU-baseline leg may load it.  It shares no code with the HIP library.
// Build: g++ -O2 -std=c++17 -ffp-contract=off (no FMA contraction, no
// -march=native), so every floating-point operation below is one IEEE RNE op.
//
// Data model (paper Section 2): a Box is an inclusive integer index range
// [lo, hi] in a global index space whose bounds may be negative; a FArrayBox
// holds the data of one box grown by ng ghost cells in Fortran order (x
// fastest); a MultiFab is the collection of FArrayBoxes over a BoxArray.
// Ghost cells covered by the valid region of some box (after a periodic shift)
// are filled by FillBoundary (Section 2: ghost cell exchange).
//
// The paper names the solver family only ("linear solvers for cell-centered
// data", Section 2).  The multigrid steps below are the textbook cell-centred
// V-cycle; every point the paper leaves open is a documented reading:
//   operator   : div(beta grad u) - alpha u = f (alpha >= 0; 0: Poisson),
//                7-point, cubic cells of width h; backward-Euler heat steps
//                are such solves with alpha = 1/dt
//   Dirichlet  : homogeneous, ghost = -(mirror cell), one sign per outside dim
//   smoother   : red-black Gauss-Seidel, red = (i+j+k) even (global indices),
//                ghosts refreshed before every colour
//   restriction: average of the 8 children
//   prolongation: trilinear cell-centred (27/9/3/1 over 64) or piecewise const
//   coarsening : by 2 while every domain edge is even and >= 4 and every box
//                holds whole cell pairs (even lower corner and edges); boxes
//                are coarsened one by one while every box edge is also >= 4,
//                else the coarse level is one box covering the domain.  Where boxes
//                are merged does not change any value (the iterates do not
//                depend on the decomposition), so the threshold is a
//                parameter: tests run both thresholds and compare bits
//   bottom     : FP64 conjugate gradients, rel. L2 residual 1e-12,
//                at most 4*cells iterations; periodic: mean-zero projection
//   stop test  : ||f - L u||_inf <= rel_tol * ||f||_inf (or <= abs_tol)
//   var coef   : fine faces = harmonic mean of the two cells (beta ghosts by
//                even reflection at Dirichlet faces, wrap at periodic ones);
//                coarse face = mean of the 4 fine faces it covers
//   mixed      : FP64 iterative refinement around one FP32 V(nu1,nu2) from zero
//                per outer step, FP64 bottom inside it.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

namespace orc {

struct Box {
    int lo[3], hi[3];
    int n(int d) const { return hi[d] - lo[d] + 1; }
    long cells() const { return (long)n(0) * n(1) * n(2); }
    bool has(int i, int j, int k) const {
        return i >= lo[0] && i <= hi[0] && j >= lo[1] && j <= hi[1] && k >= lo[2] && k <= hi[2];
    }
};

static int fdiv2(int a) { return (a >= 0) ? a / 2 : -((1 - a) / 2); }  // floor(a/2)
static int pmod(int a, int n) { int r = a % n; return r < 0 ? r + n : r; }
static int parity(int i, int j, int k) { return (i + j + k) & 1; }

struct Geom {
    Box dom;
    int per[3];
    double h;            // cell width (cubic cells)
    double alpha = 0.0;  // Helmholtz coefficient: the operator is div(beta grad u) - alpha u
    bool all_periodic() const { return per[0] && per[1] && per[2]; }
    // the operator annihilates the constants (fully periodic, no alpha term)
    bool singular() const { return all_periodic() && alpha == 0.0; }
    // alpha h^2, added to the stencil's diagonal weight sb
    template <class T>
    T shift() const { return (T)(alpha * (h * h)); }
};

// One FArrayBox: box grown by ng, F-order.
template <class T>
struct Fab {
    Box bx;
    int ng;
    int sy, sz;
    std::vector<T> v;
    void define(const Box& b, int g) {
        bx = b; ng = g;
        sy = b.n(0) + 2 * g;
        sz = sy * (b.n(1) + 2 * g);
        v.assign((size_t)sz * (b.n(2) + 2 * g), T(0));
    }
    size_t idx(int i, int j, int k) const {
        return (size_t)(i - bx.lo[0] + ng) + (size_t)(j - bx.lo[1] + ng) * sy + (size_t)(k - bx.lo[2] + ng) * sz;
    }
    T& operator()(int i, int j, int k) { return v[idx(i, j, k)]; }
    T operator()(int i, int j, int k) const { return v[idx(i, j, k)]; }
    bool in_grown(int i, int j, int k) const {
        return i >= bx.lo[0] - ng && i <= bx.hi[0] + ng && j >= bx.lo[1] - ng && j <= bx.hi[1] + ng &&
               k >= bx.lo[2] - ng && k <= bx.hi[2] + ng;
    }
};

template <class T>
struct MF {
    std::vector<Fab<T>> f;
    void define(const std::vector<Box>& bs, int ng) {
        f.resize(bs.size());
        for (size_t b = 0; b < bs.size(); ++b) f[b].define(bs[b], ng);
    }
    void zero() { for (auto& fb : f) std::fill(fb.v.begin(), fb.v.end(), T(0)); }
};

// Face coefficients of one level, global arrays: bx over faces i in [lo, hi+1]
// (face i sits between cells i-1 and i), likewise by, bz.
template <class T>
struct FacesT {
    Box dom;
    std::vector<T> c[3];
    size_t idx(int d, int i, int j, int k) const {
        int nx = dom.n(0) + (d == 0), ny = dom.n(1) + (d == 1);
        return (size_t)(i - dom.lo[0]) + (size_t)nx * ((size_t)(j - dom.lo[1]) + (size_t)ny * (k - dom.lo[2]));
    }
    T at(int d, int i, int j, int k) const { return c[d][idx(d, i, j, k)]; }
};
using Faces = FacesT<double>;

// ---------------------------------------------------------------- BoxArray
// Chop a domain edge of length n into pieces: blocking factor bf = largest
// power of two dividing n, capped at max_box; pieces of floor(max_box/bf)*bf
// and one remainder (a multiple of bf).
static std::vector<std::pair<int, int>> chop1(int lo, int n, int max_box) {
    int bf = 1;
    while (n % (bf * 2) == 0 && bf * 2 <= max_box) bf *= 2;
    int piece = (max_box / bf) * bf;
    std::vector<std::pair<int, int>> out;
    int s = 0;
    while (s < n) {
        int len = std::min(piece, n - s);
        out.push_back({lo + s, lo + s + len - 1});
        s += len;
    }
    return out;
}

static std::vector<Box> chop(const Box& dom, int max_box) {
    std::vector<std::pair<int, int>> p[3];
    for (int d = 0; d < 3; ++d) p[d] = chop1(dom.lo[d], dom.n(d), max_box);
    std::vector<Box> out;
    for (auto& z : p[2])
        for (auto& y : p[1])
            for (auto& x : p[0]) out.push_back(Box{{x.first, y.first, z.first}, {x.second, y.second, z.second}});
    return out;
}

static Box coarsen(const Box& b) {
    Box c;
    for (int d = 0; d < 3; ++d) { c.lo[d] = fdiv2(b.lo[d]); c.hi[d] = fdiv2(b.hi[d]); }
    return c;
}

static bool can_coarsen_domain(const Box& dom) {
    for (int d = 0; d < 3; ++d)
        if (dom.n(d) % 2 != 0 || dom.n(d) < 4 || (dom.lo[d] & 1)) return false;
    return true;
}

// Every box holds whole pairs of cells (even lower corner, even edges), so
// each coarse cell's 8 children lie in one box.
static bool pair_aligned(const std::vector<Box>& bs) {
    for (auto& b : bs)
        for (int d = 0; d < 3; ++d)
            if (b.n(d) % 2 != 0 || (b.lo[d] & 1)) return false;
    return true;
}

// Boxes are coarsened one by one while every box edge is at least min_edge
// (default 4) and they hold whole cell pairs; otherwise the coarser level is
// one box covering its domain.
constexpr int kDefaultMinBoxEdge = 4;

static bool can_coarsen_boxes(const std::vector<Box>& bs, int min_edge) {
    for (auto& b : bs)
        for (int d = 0; d < 3; ++d)
            if (b.n(d) % 2 != 0 || b.n(d) < min_edge || (b.lo[d] & 1)) return false;
    return true;
}

struct Level {
    Geom g;
    std::vector<Box> boxes;
};

static std::vector<Level> hierarchy(const Geom& g0, const std::vector<Box>& b0, int min_edge = kDefaultMinBoxEdge) {
    if (min_edge < 2) min_edge = kDefaultMinBoxEdge;
    std::vector<Level> L;
    L.push_back(Level{g0, b0});
    while (can_coarsen_domain(L.back().g.dom) && pair_aligned(L.back().boxes)) {
        Level c;
        c.g = L.back().g;
        c.g.dom = coarsen(L.back().g.dom);
        c.g.h = L.back().g.h * 2.0;
        if (can_coarsen_boxes(L.back().boxes, min_edge)) {
            for (auto& b : L.back().boxes) c.boxes.push_back(coarsen(b));
        } else {
            c.boxes.push_back(c.g.dom);
        }
        L.push_back(c);
    }
    return L;
}

// ----------------------------------------------------- ghost cell exchange
// Owner map: for every domain cell, the box whose valid region holds it.
static std::vector<int> owner_map(const Geom& g, const std::vector<Box>& bs) {
    const Box& D = g.dom;
    std::vector<int> own((size_t)D.cells(), -1);
    for (size_t b = 0; b < bs.size(); ++b)
        for (int k = bs[b].lo[2]; k <= bs[b].hi[2]; ++k)
            for (int j = bs[b].lo[1]; j <= bs[b].hi[1]; ++j)
                for (int i = bs[b].lo[0]; i <= bs[b].hi[0]; ++i) {
                    size_t q = (size_t)(i - D.lo[0]) + (size_t)D.n(0) * ((size_t)(j - D.lo[1]) + (size_t)D.n(1) * (k - D.lo[2]));
                    own[q] = (int)b;
                }
    return own;
}

// FillBoundary: every ghost cell that (after wrapping periodic directions) is
// a valid cell of some box takes that cell's value; all other ghosts are left
// untouched.  Faces, edges and corners.
template <class T>
static void fill_boundary(const Geom& g, MF<T>& mf, int ncomp_stride_unused = 0) {
    (void)ncomp_stride_unused;
    std::vector<Box> bs;
    for (auto& fb : mf.f) bs.push_back(fb.bx);
    std::vector<int> own = owner_map(g, bs);
    const Box& D = g.dom;
    for (size_t b = 0; b < mf.f.size(); ++b) {
        Fab<T>& F = mf.f[b];
        const Box& B = F.bx;
        for (int k = B.lo[2] - F.ng; k <= B.hi[2] + F.ng; ++k)
            for (int j = B.lo[1] - F.ng; j <= B.hi[1] + F.ng; ++j)
                for (int i = B.lo[0] - F.ng; i <= B.hi[0] + F.ng; ++i) {
                    if (B.has(i, j, k)) continue;
                    int c[3] = {i, j, k};
                    bool inside = true;
                    for (int d = 0; d < 3; ++d) {
                        if (c[d] < D.lo[d] || c[d] > D.hi[d]) {
                            if (g.per[d]) c[d] = D.lo[d] + pmod(c[d] - D.lo[d], D.n(d));
                            else inside = false;
                        }
                    }
                    if (!inside) continue;
                    size_t q = (size_t)(c[0] - D.lo[0]) + (size_t)D.n(0) * ((size_t)(c[1] - D.lo[1]) + (size_t)D.n(1) * (c[2] - D.lo[2]));
                    int o = own[q];
                    if (o < 0) continue;
                    F(i, j, k) = mf.f[o](c[0], c[1], c[2]);
                }
    }
}

// Physical boundary: ghost cells outside a non-periodic domain face take
// sign * (mirror cell), mirror reflected across every such face; sign = -1
// per reflected direction for the homogeneous Dirichlet condition (odd), +1
// for the even reflection used for cell coefficients.  Call after
// fill_boundary (the mirror may be a ghost that fill_boundary set).
template <class T>
static void apply_bc(const Geom& g, MF<T>& mf, bool odd) {
    const Box& D = g.dom;
    for (auto& F : mf.f) {
        const Box& B = F.bx;
        for (int k = B.lo[2] - F.ng; k <= B.hi[2] + F.ng; ++k)
            for (int j = B.lo[1] - F.ng; j <= B.hi[1] + F.ng; ++j)
                for (int i = B.lo[0] - F.ng; i <= B.hi[0] + F.ng; ++i) {
                    int m[3] = {i, j, k};
                    int flips = 0;
                    for (int d = 0; d < 3; ++d) {
                        if (g.per[d]) continue;
                        if (m[d] < D.lo[d]) { m[d] = 2 * D.lo[d] - 1 - m[d]; ++flips; }
                        else if (m[d] > D.hi[d]) { m[d] = 2 * D.hi[d] + 1 - m[d]; ++flips; }
                    }
                    if (flips == 0) continue;
                    T v = F(m[0], m[1], m[2]);
                    F(i, j, k) = (odd && (flips & 1)) ? -v : v;
                }
    }
}

template <class T>
static void fill_and_bc(const Geom& g, MF<T>& mf) {
    fill_boundary(g, mf);
    apply_bc(g, mf, true);
}

// ------------------------------------------------------- coefficients
// Level-0 faces from a global cell-centred beta (F-order over the domain),
// computed in T from beta rounded to T.
template <class T>
static FacesT<T> faces_from_beta(const Geom& g, const double* beta) {
    const Box& D = g.dom;
    FacesT<T> F;
    F.dom = D;
    auto B = [&](int i, int j, int k) -> T {
        int c[3] = {i, j, k};
        for (int d = 0; d < 3; ++d) {
            if (c[d] < D.lo[d] || c[d] > D.hi[d]) {
                if (g.per[d]) c[d] = D.lo[d] + pmod(c[d] - D.lo[d], D.n(d));
                else c[d] = (c[d] < D.lo[d]) ? 2 * D.lo[d] - 1 - c[d] : 2 * D.hi[d] + 1 - c[d];  // even reflection
            }
        }
        return (T)beta[(size_t)(c[0] - D.lo[0]) + (size_t)D.n(0) * ((size_t)(c[1] - D.lo[1]) + (size_t)D.n(1) * (c[2] - D.lo[2]))];
    };
    for (int d = 0; d < 3; ++d) {
        int nx = D.n(0) + (d == 0), ny = D.n(1) + (d == 1), nz = D.n(2) + (d == 2);
        F.c[d].assign((size_t)nx * ny * nz, T(0));
        for (int k = D.lo[2]; k < D.lo[2] + nz; ++k)
            for (int j = D.lo[1]; j < D.lo[1] + ny; ++j)
                for (int i = D.lo[0]; i < D.lo[0] + nx; ++i) {
                    int e[3] = {0, 0, 0};
                    e[d] = 1;
                    T bl = B(i - e[0], j - e[1], k - e[2]);
                    T br = B(i, j, k);
                    F.c[d][F.idx(d, i, j, k)] = (bl * br) * T(2) / (bl + br);  // harmonic mean
                }
    }
    return F;
}

// Coarse faces: mean of the four fine faces that make up each coarse face.
template <class T>
static FacesT<T> coarsen_faces(const FacesT<T>& Ff, const Box& cdom) {
    FacesT<T> C;
    C.dom = cdom;
    for (int d = 0; d < 3; ++d) {
        int nx = cdom.n(0) + (d == 0), ny = cdom.n(1) + (d == 1), nz = cdom.n(2) + (d == 2);
        C.c[d].assign((size_t)nx * ny * nz, T(0));
        int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;  // the two tangential directions
        for (int K = cdom.lo[2]; K < cdom.lo[2] + nz; ++K)
            for (int J = cdom.lo[1]; J < cdom.lo[1] + ny; ++J)
                for (int I = cdom.lo[0]; I < cdom.lo[0] + nx; ++I) {
                    int f0[3] = {2 * I, 2 * J, 2 * K};
                    T a[2][2];
                    for (int q = 0; q < 2; ++q)
                        for (int p = 0; p < 2; ++p) {
                            int c[3] = {f0[0], f0[1], f0[2]};
                            c[t1] += p;
                            c[t2] += q;
                            a[q][p] = Ff.at(d, c[0], c[1], c[2]);
                        }
                    C.c[d][C.idx(d, I, J, K)] = ((a[0][0] + a[0][1]) + (a[1][0] + a[1][1])) * T(0.25);
                }
    }
    return C;
}

// ------------------------------------------------------------ operators
// 7-point operator, constant coefficient:
//   s = ((u[i-1]+u[i+1]) + (u[j-1]+u[j+1])) + (u[k-1]+u[k+1])
//   (L u) = (s - 6 u) / h^2,   GS: u = (s - h^2 f) / 6
// variable coefficient (face coefficients b):
//   sb = ((bxm+bxp) + (bym+byp)) + (bzm+bzp)
//   su = ((bxm u[i-1] + bxp u[i+1]) + (bym u[j-1] + byp u[j+1])) + (bzm u[k-1] + bzp u[k+1])
//   (L u) = (su - sb u) / h^2, GS: u = (su - h^2 f) / sb
template <class T>
static inline void stencil(const Fab<T>& U, const FacesT<T>* fc, int i, int j, int k, T& su, T& sb) {
    if (!fc) {
        su = ((U(i - 1, j, k) + U(i + 1, j, k)) + (U(i, j - 1, k) + U(i, j + 1, k))) + (U(i, j, k - 1) + U(i, j, k + 1));
        sb = T(6);
        return;
    }
    // periodic: the face at hi+1 and the face at lo hold the same value
    auto F = [&](int d, int a, int b, int c) -> T { return fc->at(d, a, b, c); };
    T bxm = F(0, i, j, k), bxp = F(0, i + 1, j, k);
    T bym = F(1, i, j, k), byp = F(1, i, j + 1, k);
    T bzm = F(2, i, j, k), bzp = F(2, i, j, k + 1);
    sb = ((bxm + bxp) + (bym + byp)) + (bzm + bzp);
    su = ((bxm * U(i - 1, j, k) + bxp * U(i + 1, j, k)) + (bym * U(i, j - 1, k) + byp * U(i, j + 1, k))) +
         (bzm * U(i, j, k - 1) + bzp * U(i, j, k + 1));
}

// One colour of red-black Gauss-Seidel (ghosts of u must be current).
// With the Helmholtz term: u = (su - h^2 f) / (sb + alpha h^2).
template <class T>
static void gs_colour(const Geom& g, MF<T>& u, const MF<T>& f, const FacesT<T>* fc, int colour) {
    const T h2 = (T)(g.h * g.h);
    const T dg = g.shift<T>();
    for (size_t b = 0; b < u.f.size(); ++b) {
        Fab<T>& U = u.f[b];
        const Fab<T>& Fb = f.f[b];
        const Box& B = U.bx;
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) {
                    if (parity(i, j, k) != colour) continue;
                    T su, sb;
                    stencil(U, fc, i, j, k, su, sb);
                    U(i, j, k) = (su - h2 * Fb(i, j, k)) / (sb + dg);
                }
    }
}

// r = f - L u on valid cells (ghosts of u must be current).  Returns the
// max-norm and the sum of squares (in box, k, j, i order).
template <class T>
static void residual(const Geom& g, const MF<T>& u, const MF<T>& f, const FacesT<T>* fc, MF<T>& r, double* rinf,
                     double* rl2sq) {
    const T ih2 = (T)(1.0 / (g.h * g.h));
    const T dg = g.shift<T>();
    double mx = 0.0, s2 = 0.0;
    bool bad = false;
    for (size_t b = 0; b < u.f.size(); ++b) {
        const Fab<T>& U = u.f[b];
        const Box& B = U.bx;
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) {
                    T su, sb;
                    stencil(U, fc, i, j, k, su, sb);
                    T Lu = (su - (sb + dg) * U(i, j, k)) * ih2;
                    T rv = f.f[b](i, j, k) - Lu;
                    r.f[b](i, j, k) = rv;
                    double a = std::fabs((double)rv);
                    if (std::isnan(a)) bad = true;
                    else if (a > mx) mx = a;
                    s2 += (double)rv * (double)rv;
                }
    }
    if (bad) mx = std::nan("");
    if (rinf) *rinf = mx;
    if (rl2sq) *rl2sq = s2;
}

// Index of the coarse box that contains the coarsened fine box.
static int coarse_owner(const std::vector<Box>& cb, const Box& fine) {
    Box c = coarsen(fine);
    for (size_t q = 0; q < cb.size(); ++q)
        if (cb[q].has(c.lo[0], c.lo[1], c.lo[2]) && cb[q].has(c.hi[0], c.hi[1], c.hi[2])) return (int)q;
    return -1;
}

// f_c(I) = (1/8) * sum of the 8 children of I.
template <class T>
static void restrict_avg(const MF<T>& rf, MF<T>& fc) {
    std::vector<Box> cbs;
    for (auto& F : fc.f) cbs.push_back(F.bx);
    for (size_t b = 0; b < rf.f.size(); ++b) {
        const Fab<T>& R = rf.f[b];
        Box c = coarsen(R.bx);
        Fab<T>& C = fc.f[coarse_owner(cbs, R.bx)];
        for (int K = c.lo[2]; K <= c.hi[2]; ++K)
            for (int J = c.lo[1]; J <= c.hi[1]; ++J)
                for (int I = c.lo[0]; I <= c.hi[0]; ++I) {
                    int i = 2 * I, j = 2 * J, k = 2 * K;
                    T s = ((R(i, j, k) + R(i + 1, j, k)) + (R(i, j + 1, k) + R(i + 1, j + 1, k))) +
                          ((R(i, j, k + 1) + R(i + 1, j, k + 1)) + (R(i, j + 1, k + 1) + R(i + 1, j + 1, k + 1)));
                    C(I, J, K) = s * T(0.125);
                }
    }
}

// u_f += P e_c.  Trilinear (order 2): per direction the parent P = floor(i/2)
// weighs 3/4 and its neighbour P+s (s = +1 for odd i, -1 for even i) 1/4, so
//   e = (((27 c000 + 9 ((c100 + c010) + c001)) + 3 ((c110 + c101) + c011)) + c111) / 64.
// Piecewise constant (order 1): e = c000.  Ghosts of e_c must be current.
template <class T>
static void prolong_add(const MF<T>& ec, MF<T>& uf, int order) {
    std::vector<Box> cbs;
    for (auto& F : ec.f) cbs.push_back(F.bx);
    for (size_t b = 0; b < uf.f.size(); ++b) {
        Fab<T>& U = uf.f[b];
        const Fab<T>& E = ec.f[coarse_owner(cbs, U.bx)];
        const Box& B = U.bx;
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) {
                    int I = fdiv2(i), J = fdiv2(j), K = fdiv2(k);
                    T e;
                    if (order == 1) {
                        e = E(I, J, K);
                    } else {
                        int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
                        T c000 = E(I, J, K);
                        T c100 = E(I + si, J, K), c010 = E(I, J + sj, K), c001 = E(I, J, K + sk);
                        T c110 = E(I + si, J + sj, K), c101 = E(I + si, J, K + sk), c011 = E(I, J + sj, K + sk);
                        T c111 = E(I + si, J + sj, K + sk);
                        e = (((T(27) * c000 + T(9) * ((c100 + c010) + c001)) + T(3) * ((c110 + c101) + c011)) + c111) *
                            T(0.015625);
                    }
                    U(i, j, k) = U(i, j, k) + e;
                }
    }
}

// ------------------------------------------------------------- bottom
// FP64 conjugate gradients for L x = rhs on one level (any box layout).
// The operator is negative definite (Dirichlet) or negative semidefinite
// with the constants as null space (fully periodic); CG applies unchanged.
struct CGStats { int iters = 0; double rel = 0.0; };

static double dot(const MF<double>& a, const MF<double>& b) {
    double s = 0.0;
    for (size_t q = 0; q < a.f.size(); ++q) {
        const Box& B = a.f[q].bx;
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) s += a.f[q](i, j, k) * b.f[q](i, j, k);
    }
    return s;
}

static double mean_valid(const MF<double>& a) {
    double s = 0.0;
    long n = 0;
    for (auto& F : a.f) {
        const Box& B = F.bx;
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) { s += F(i, j, k); ++n; }
    }
    return s / (double)n;
}

static void add_const_valid(MF<double>& a, double c) {
    for (auto& F : a.f) {
        const Box& B = F.bx;
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) F(i, j, k) -= c;
    }
}

static void apply_op(const Geom& g, MF<double>& p, const Faces* fc, MF<double>& Ap) {
    fill_and_bc(g, p);
    const double ih2 = 1.0 / (g.h * g.h);
    const double dg = g.shift<double>();
    for (size_t b = 0; b < p.f.size(); ++b) {
        const Box& B = p.f[b].bx;
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) {
                    double su, sb;
                    stencil(p.f[b], fc, i, j, k, su, sb);
                    Ap.f[b](i, j, k) = (su - (sb + dg) * p.f[b](i, j, k)) * ih2;
                }
    }
}

static CGStats bottom_cg(const Geom& g, const std::vector<Box>& bs, const MF<double>& rhs_in, const Faces* fc,
                         MF<double>& x, double rtol) {
    CGStats st;
    MF<double> r, p, Ap;
    r.define(bs, 0);
    p.define(bs, 1);
    Ap.define(bs, 0);
    x.zero();
    for (size_t b = 0; b < bs.size(); ++b) {
        const Box& B = bs[b];
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) r.f[b](i, j, k) = rhs_in.f[b](i, j, k);
    }
    const bool sing = g.singular();
    if (sing) add_const_valid(r, mean_valid(r));
    for (size_t b = 0; b < bs.size(); ++b) {
        const Box& B = bs[b];
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) p.f[b](i, j, k) = r.f[b](i, j, k);
    }
    double rs = dot(r, r);
    const double rs0 = rs;
    if (rs0 == 0.0) return st;
    long ncell = 0;
    for (auto& B : bs) ncell += B.cells();
    const long maxit = 4 * ncell;
    for (long it = 0; it < maxit; ++it) {
        apply_op(g, p, fc, Ap);
        double pAp = dot(p, Ap);
        double alpha = rs / pAp;
        for (size_t b = 0; b < bs.size(); ++b) {
            const Box& B = bs[b];
            for (int k = B.lo[2]; k <= B.hi[2]; ++k)
                for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                    for (int i = B.lo[0]; i <= B.hi[0]; ++i) {
                        x.f[b](i, j, k) += alpha * p.f[b](i, j, k);
                        r.f[b](i, j, k) -= alpha * Ap.f[b](i, j, k);
                    }
        }
        double rsn = dot(r, r);
        st.iters = (int)(it + 1);
        st.rel = std::sqrt(rsn / rs0);
        if (std::sqrt(rsn) <= rtol * std::sqrt(rs0)) break;
        double beta = rsn / rs;
        for (size_t b = 0; b < bs.size(); ++b) {
            const Box& B = bs[b];
            for (int k = B.lo[2]; k <= B.hi[2]; ++k)
                for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                    for (int i = B.lo[0]; i <= B.hi[0]; ++i)
                        p.f[b](i, j, k) = r.f[b](i, j, k) + beta * p.f[b](i, j, k);
        }
        rs = rsn;
    }
    if (sing) add_const_valid(x, mean_valid(x));
    return st;
}

// ------------------------------------------------------------ V-cycle
struct Params {
    int nu1 = 2, nu2 = 2, max_cycles = 200, precision = 0, prolong = 2, fixed_cycles = 0;
    double rel_tol = 1e-10, abs_tol = 0.0, h = 0.0, bottom_rtol = 1e-12;
    int min_box_edge = kDefaultMinBoxEdge;
    int krylov = 0;      // 1: conjugate gradients preconditioned by one V-cycle
    int use_guess = 0;   // 1: start from the caller's u (else from zero)
};

// Multigrid hierarchy of storage type T: per level u, f, r and (variable
// coefficient) the face coefficients in T, plus the bottom level's faces in
// FP64 for the FP64 bottom solve.
template <class T>
struct Hier {
    std::vector<Level> L;
    std::vector<FacesT<T>> faces;  // empty: constant coefficient
    Faces bottom_faces;
    std::vector<MF<T>> u, f, r;
    const FacesT<T>* fc(size_t l) const { return faces.empty() ? nullptr : &faces[l]; }
    const Faces* bfc() const { return faces.empty() ? nullptr : &bottom_faces; }
    void define(const std::vector<Level>& lv, const double* beta);
};

template <class T>
static std::vector<FacesT<T>> build_faces(const std::vector<Level>& L, const double* beta) {
    std::vector<FacesT<T>> out;
    if (!beta) return out;
    out.push_back(faces_from_beta<T>(L[0].g, beta));
    for (size_t l = 1; l < L.size(); ++l) out.push_back(coarsen_faces(out[l - 1], L[l].g.dom));
    return out;
}

template <class T>
void Hier<T>::define(const std::vector<Level>& lv, const double* beta) {
    L = lv;
    u.resize(L.size()); f.resize(L.size()); r.resize(L.size());
    for (size_t l = 0; l < L.size(); ++l) {
        u[l].define(L[l].boxes, 1);
        f[l].define(L[l].boxes, 1);
        r[l].define(L[l].boxes, 1);
    }
    faces = build_faces<T>(L, beta);
    if (!faces.empty()) {
        const FacesT<T>& fb = faces.back();
        bottom_faces.dom = fb.dom;
        for (int d = 0; d < 3; ++d) bottom_faces.c[d].assign(fb.c[d].begin(), fb.c[d].end());
    }
}

template <class T>
static void copy_valid(const MF<T>& a, MF<double>& b) {
    for (size_t q = 0; q < a.f.size(); ++q) {
        const Box& B = a.f[q].bx;
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) b.f[q](i, j, k) = (double)a.f[q](i, j, k);
    }
}

template <class T>
static void copy_valid_back(const MF<double>& a, MF<T>& b) {
    for (size_t q = 0; q < a.f.size(); ++q) {
        const Box& B = a.f[q].bx;
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) b.f[q](i, j, k) = (T)a.f[q](i, j, k);
    }
}

template <class T>
static void smooth(Hier<T>& H, size_t l, int nsweeps) {
    const Geom& g = H.L[l].g;
    for (int s = 0; s < nsweeps; ++s)
        for (int c = 0; c < 2; ++c) {
            fill_and_bc(g, H.u[l]);
            gs_colour(g, H.u[l], H.f[l], H.fc(l), c);
        }
}

// V(nu1, nu2) from level l down: pre-smooth, residual, restrict, zero the
// coarse guess, recurse, prolong-correct, post-smooth; FP64 CG at the bottom.
template <class T>
static void vcycle(Hier<T>& H, const Params& P, size_t l, std::vector<CGStats>* cgs) {
    const size_t last = H.L.size() - 1;
    if (l == last) {
        MF<double> rhs, x;
        rhs.define(H.L[l].boxes, 0);
        x.define(H.L[l].boxes, 1);
        copy_valid(H.f[l], rhs);
        CGStats st = bottom_cg(H.L[l].g, H.L[l].boxes, rhs, H.bfc(), x, P.bottom_rtol);
        if (cgs) cgs->push_back(st);
        copy_valid_back(x, H.u[l]);
        return;
    }
    smooth(H, l, P.nu1);
    fill_and_bc(H.L[l].g, H.u[l]);
    residual(H.L[l].g, H.u[l], H.f[l], H.fc(l), H.r[l], nullptr, nullptr);
    restrict_avg(H.r[l], H.f[l + 1]);
    H.u[l + 1].zero();
    vcycle(H, P, l + 1, cgs);
    fill_and_bc(H.L[l + 1].g, H.u[l + 1]);
    prolong_add(H.u[l + 1], H.u[l], P.prolong);
    smooth(H, l, P.nu2);
}

struct Info {
    int status, cycles, nhist, levels;
    double rel_inf, rel_l2, f_inf;
    double hist[256];
    double hist_l2[256];
    int cg_iters_max;
};

static void scatter_global(const Box& D, const double* glob, MF<double>& mf) {
    for (auto& F : mf.f) {
        const Box& B = F.bx;
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i)
                    F(i, j, k) = glob[(size_t)(i - D.lo[0]) + (size_t)D.n(0) * ((size_t)(j - D.lo[1]) + (size_t)D.n(1) * (k - D.lo[2]))];
    }
}

static void gather_global(const Box& D, const MF<double>& mf, double* glob) {
    for (auto& F : mf.f) {
        const Box& B = F.bx;
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i)
                    glob[(size_t)(i - D.lo[0]) + (size_t)D.n(0) * ((size_t)(j - D.lo[1]) + (size_t)D.n(1) * (k - D.lo[2]))] = F(i, j, k);
    }
}

static double max_abs_valid(const MF<double>& a) {
    double m = 0.0;
    bool bad = false;
    for (auto& F : a.f) {
        const Box& B = F.bx;
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) {
                    double v = std::fabs(F(i, j, k));
                    if (std::isnan(v)) bad = true;
                    else if (v > m) m = v;
                }
    }
    return bad ? std::nan("") : m;
}

template <class F>
static void for_valid(const MF<double>& a, F fn) {
    for (size_t q = 0; q < a.f.size(); ++q) {
        const Box& B = a.f[q].bx;
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) fn(q, i, j, k);
    }
}

// z = M r: one V(nu1, nu2) from a zero guess with r as its right-hand side,
// in FP64 (precision 0) or in float storage and arithmetic with an FP64
// bottom (precision 1).
static void precondition(const Params& P, Hier<double>& H64, Hier<float>& H32, const MF<double>& r, MF<double>& z,
                         std::vector<CGStats>* cgs) {
    if (P.precision == 0) {
        for_valid(r, [&](size_t q, int i, int j, int k) { H64.f[0].f[q](i, j, k) = r.f[q](i, j, k); });
        H64.u[0].zero();
        vcycle(H64, P, 0, cgs);
        for_valid(r, [&](size_t q, int i, int j, int k) { z.f[q](i, j, k) = H64.u[0].f[q](i, j, k); });
    } else {
        for_valid(r, [&](size_t q, int i, int j, int k) { H32.f[0].f[q](i, j, k) = (float)r.f[q](i, j, k); });
        H32.u[0].zero();
        vcycle(H32, P, 0, cgs);
        for_valid(r, [&](size_t q, int i, int j, int k) { z.f[q](i, j, k) = (double)H32.u[0].f[q](i, j, k); });
    }
}

// Multigrid-preconditioned conjugate gradients for L u = f (the Krylov use
// of the multigrid cycle among the framework's linear solvers, Section 2).
// L is negative definite (semidefinite when fully periodic); in the SPD form
// A = -L, b = -f the residual is -r and the preconditioned residual is
// z = M r itself, so the signs cancel in alpha = (r.z) / (p.Lp).  The
// V-cycle preconditioner is not exactly symmetric (both smoothing passes
// sweep red then black, the Dirichlet ghosts lag) and in FP32 it is not
// exactly linear, so the update of p takes the flexible (Polak-Ribiere)
// form beta = z'.(r' - r) / (z.r) of Notay's flexible CG, which equals the
// Fletcher-Reeves value when the preconditioner is fixed and symmetric.
// With r' - r = -alpha q it reads beta = -alpha (z'.q) / (z.r).
// Each iteration records the max-norm of the updated residual; when it
// meets the tolerance the residual f - L u is computed afresh and the solve
// stops only if that meets it too (else the iteration restarts from it).
static int pcg(const Params& P, const Geom& g0, const std::vector<Box>& b0, Hier<double>& H64, Hier<float>& H32,
               MF<double>& u, MF<double>& f, MF<double>& r, const Faces* fc0, double fnorm, Info* info,
               std::vector<CGStats>* cgs, int* cycles) {
    MF<double> z, p, q, rt;
    z.define(b0, 0);
    p.define(b0, 1);
    q.define(b0, 0);
    rt.define(b0, 1);
    auto norms = [&](const MF<double>& a, double* rinf, double* rl2) {
        double mx = 0.0, s2 = 0.0;
        bool bad = false;
        for_valid(a, [&](size_t c, int i, int j, int k) {
            const double v = a.f[c](i, j, k);
            const double av = std::fabs(v);
            if (std::isnan(av)) bad = true;
            else if (av > mx) mx = av;
            s2 += v * v;
        });
        *rinf = bad ? std::nan("") : mx;
        *rl2 = s2;
    };
    auto record = [&](int cyc, double rinf, double rl2) {
        if (cyc < 256) { info->hist[cyc] = rinf / fnorm; info->hist_l2[cyc] = std::sqrt(rl2); info->nhist = cyc + 1; }
    };
    auto converged = [&](double rinf) { return rinf <= P.rel_tol * fnorm || rinf <= P.abs_tol; };
    auto true_residual = [&](double* rinf, double* rl2) {
        fill_and_bc(g0, u);
        residual(g0, u, f, fc0, rt, nullptr, nullptr);
        norms(rt, rinf, rl2);
    };
    double rinf, rl2;
    true_residual(&rinf, &rl2);
    for_valid(rt, [&](size_t c, int i, int j, int k) { r.f[c](i, j, k) = rt.f[c](i, j, k); });
    record(0, rinf, rl2);
    info->rel_inf = rinf / fnorm;
    info->rel_l2 = std::sqrt(rl2);
    int cyc = 0, status = 0;
    bool restart = true;
    double rz = 0.0;
    for (;;) {
        if (!std::isfinite(rinf)) { status = -5; break; }
        if (P.fixed_cycles > 0) {
            if (cyc == P.fixed_cycles) break;
        } else if (converged(rinf)) {
            break;
        } else if (cyc == P.max_cycles) {
            status = -4;
            break;
        }
        if (restart) {  // p = z = M r
            precondition(P, H64, H32, r, z, cgs);
            for_valid(z, [&](size_t c, int i, int j, int k) { p.f[c](i, j, k) = z.f[c](i, j, k); });
            rz = dot(r, z);
            restart = false;
        }
        apply_op(g0, p, fc0, q);  // q = L p (fills p's ghosts)
        const double alpha = rz / dot(p, q);
        for_valid(r, [&](size_t c, int i, int j, int k) {
            u.f[c](i, j, k) += alpha * p.f[c](i, j, k);
            r.f[c](i, j, k) -= alpha * q.f[c](i, j, k);
        });
        ++cyc;
        norms(r, &rinf, &rl2);
        record(cyc, rinf, rl2);
        info->rel_inf = rinf / fnorm;
        info->rel_l2 = std::sqrt(rl2);
        const bool stop = (P.fixed_cycles > 0) ? cyc == P.fixed_cycles : converged(rinf);
        if (stop && std::isfinite(rinf)) {
            // the updated residual says stop: check f - L u itself
            double tinf, tl2;
            true_residual(&tinf, &tl2);
            info->rel_inf = tinf / fnorm;
            info->rel_l2 = std::sqrt(tl2);
            if (P.fixed_cycles > 0 || converged(tinf) || !std::isfinite(tinf)) {
                rinf = tinf;
                if (!std::isfinite(tinf)) status = -5;
                break;
            }
            for_valid(rt, [&](size_t c, int i, int j, int k) { r.f[c](i, j, k) = rt.f[c](i, j, k); });
            rinf = tinf;
            restart = true;
            continue;
        }
        if (!std::isfinite(rinf) || cyc == P.max_cycles) continue;  // decided at the top of the loop
        precondition(P, H64, H32, r, z, cgs);
        const double zq = dot(z, q);
        const double rz_new = dot(r, z);
        const double beta = -alpha * zq / rz;
        for_valid(z, [&](size_t c, int i, int j, int k) { p.f[c](i, j, k) = z.f[c](i, j, k) + beta * p.f[c](i, j, k); });
        rz = rz_new;
    }
    *cycles = cyc;
    return status;
}

// Driver.  u starts at zero; each cycle: ghosts, residual and its norms, stop
// test, then one V-cycle (FP64) or one refinement step around an FP32
// V-cycle.  Status codes: 0 ok, -4 not converged, -5 non-finite.
static int solve(const Params& P, const Geom& g0, const std::vector<Box>& b0, const double* fglob, const double* beta,
                 double* uglob, Info* info) {
    std::vector<Level> L = hierarchy(g0, b0, P.min_box_edge);
    std::memset(info, 0, sizeof(Info));
    info->levels = (int)L.size();

    Hier<double> H64;
    Hier<float> H32;
    MF<double> u_ir, f_ir, r_ir;
    std::vector<Faces> faces64;
    MF<double>* u;
    MF<double>* f;
    MF<double>* r;
    const Faces* fc0;
    if (P.precision == 0 && !P.krylov) {
        H64.define(L, beta);
        u = &H64.u[0]; f = &H64.f[0]; r = &H64.r[0];
        fc0 = H64.fc(0);
    } else {
        // the iterate lives outside the hierarchy, whose level 0 holds the
        // correction of the inner V-cycle
        if (P.precision == 0) H64.define(L, beta);
        else H32.define(L, beta);
        u_ir.define(b0, 1); f_ir.define(b0, 1); r_ir.define(b0, 1);
        u = &u_ir; f = &f_ir; r = &r_ir;
        if (beta) faces64.push_back(faces_from_beta<double>(g0, beta));
        fc0 = beta ? &faces64[0] : nullptr;
    }
    scatter_global(g0.dom, fglob, *f);
    const double fnorm = max_abs_valid(*f);
    info->f_inf = fnorm;
    std::vector<CGStats> cgs;

    int status = 0;
    if (!(fnorm > 0.0)) {  // f == 0: u = 0; non-finite f: u left as it was
        if (std::isnan(fnorm)) status = -5;
        if (status == 0 || !P.use_guess) u->zero();
        else scatter_global(g0.dom, uglob, *u);
        gather_global(g0.dom, *u, uglob);
        info->status = status;
        return status;
    }
    if (P.use_guess) scatter_global(g0.dom, uglob, *u);
    int cyc = 0;
    if (P.krylov) {
        status = pcg(P, g0, b0, H64, H32, *u, *f, *r, fc0, fnorm, info, &cgs, &cyc);
    } else for (;; ++cyc) {
        fill_and_bc(g0, *u);
        double rinf, rl2;
        residual(g0, *u, *f, fc0, *r, &rinf, &rl2);
        if (cyc < 256) { info->hist[cyc] = rinf / fnorm; info->hist_l2[cyc] = std::sqrt(rl2); info->nhist = cyc + 1; }
        info->rel_inf = rinf / fnorm;
        info->rel_l2 = std::sqrt(rl2);
        if (!std::isfinite(rinf)) { status = -5; break; }
        if (P.fixed_cycles > 0) {
            if (cyc == P.fixed_cycles) break;
        } else {
            if (rinf <= P.rel_tol * fnorm || rinf <= P.abs_tol) break;
            if (cyc == P.max_cycles) { status = -4; break; }
        }
        if (P.precision == 0) {
            vcycle(H64, P, 0, &cgs);
        } else {
            for (size_t q = 0; q < u->f.size(); ++q) {
                const Box& B = u->f[q].bx;
                for (int k = B.lo[2]; k <= B.hi[2]; ++k)
                    for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                        for (int i = B.lo[0]; i <= B.hi[0]; ++i) H32.f[0].f[q](i, j, k) = (float)r->f[q](i, j, k);
            }
            H32.u[0].zero();
            vcycle(H32, P, 0, &cgs);
            for (size_t q = 0; q < u->f.size(); ++q) {
                const Box& B = u->f[q].bx;
                for (int k = B.lo[2]; k <= B.hi[2]; ++k)
                    for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                        for (int i = B.lo[0]; i <= B.hi[0]; ++i) u->f[q](i, j, k) += (double)H32.u[0].f[q](i, j, k);
            }
        }
    }
    info->cycles = cyc;
    for (auto& s : cgs) info->cg_iters_max = std::max(info->cg_iters_max, s.iters);
    gather_global(g0.dom, *u, uglob);
    if (g0.singular()) {
        // mean-zero representative; the mean is summed in global F-order so
        // that it does not depend on the box decomposition
        const size_t N = (size_t)g0.dom.cells();
        double s = 0.0;
        for (size_t q = 0; q < N; ++q) s += uglob[q];
        const double m = s / (double)N;
        for (size_t q = 0; q < N; ++q) uglob[q] -= m;
    }
    info->status = status;
    return status;
}



// ====================================================== nodal Poisson
// Node-centred data (the framework's other solver family, Section 2): on a
// domain of n_d cells of width h per direction the nodes sit at x = i h,
// i = 0 .. n_d.  A homogeneous-Dirichlet direction keeps its boundary nodes
// (i = 0, n_d) at 0; they are not unknowns.  In a periodic direction node
// n_d is node 0 (its value is kept equal to node 0's).  Arrays hold every
// node of the domain, (n_0+1)(n_1+1)(n_2+1) values in F-order.
//   operator    : (L u)_i = (sum of the 6 neighbours - 6 u_i) / h^2, summed as
//                 ((x- + x+) + (y- + y+)) + (z- + z+)
//   smoother    : red-black Gauss-Seidel over the unknown nodes, red =
//                 (i+j+k) even first, u = (s - h^2 f) / 6
//   coarsening  : coarse node I is fine node 2I, while every n_d is even and
//                 > 2 (a Dirichlet n_d = 2 leaves one unknown node)
//   restriction : full weighting, weights w(0) = 1/2, w(+-1) = 1/4 per
//                 direction (their product over the 27 fine neighbours of 2I)
//   prolongation: trilinear: fine node 2I + o (o in {0,1}^3) takes the mean
//                 of the 2^|o| coarse nodes I + o' with o' <= o componentwise
//   bottom      : FP64 CG on the unknowns, rel. L2 1e-12, at most 4 N
//                 iterations; fully periodic: right-hand side projected to
//                 mean 0, solution mean 0 (over the n_0 n_1 n_2 distinct nodes)
namespace nodal {

struct NGrid {
    int n[3];     // cells per direction
    int per[3];
    double h;
    long nx() const { return n[0] + 1; }
    long size() const { return (long)(n[0] + 1) * (n[1] + 1) * (n[2] + 1); }
    long idx(int i, int j, int k) const { return i + (long)(n[0] + 1) * (j + (long)(n[1] + 1) * k); }
    // an unknown: not a Dirichlet boundary node, not the periodic copy n_d
    bool unknown(int i, int j, int k) const {
        const int c[3] = {i, j, k};
        for (int d = 0; d < 3; ++d) {
            if (per[d] ? c[d] == n[d] : (c[d] == 0 || c[d] == n[d])) return false;
        }
        return true;
    }
    // neighbour index along d by +-1, wrapped in periodic directions
    int wrap(int d, int c) const {
        if (!per[d]) return c;
        if (c < 0) return c + n[d];
        if (c >= n[d]) return c - n[d];
        return c;
    }
    bool singular() const { return per[0] && per[1] && per[2]; }
    NGrid coarse() const {
        NGrid c = *this;
        for (int d = 0; d < 3; ++d) c.n[d] = n[d] / 2;
        c.h = h * 2.0;
        return c;
    }
    bool coarsenable() const {
        for (int d = 0; d < 3; ++d)
            if (n[d] % 2 || n[d] <= 2) return false;
        return true;
    }
};

template <class F>
static void for_unknowns(const NGrid& g, F fn) {
    for (int k = 0; k <= g.n[2]; ++k)
        for (int j = 0; j <= g.n[1]; ++j)
            for (int i = 0; i <= g.n[0]; ++i)
                if (g.unknown(i, j, k)) fn(i, j, k);
}

// sum of the six neighbours of an unknown node
static double nsum(const NGrid& g, const std::vector<double>& u, int i, int j, int k) {
    const double xm = u[g.idx(g.wrap(0, i - 1), j, k)], xp = u[g.idx(g.wrap(0, i + 1), j, k)];
    const double ym = u[g.idx(i, g.wrap(1, j - 1), k)], yp = u[g.idx(i, g.wrap(1, j + 1), k)];
    const double zm = u[g.idx(i, j, g.wrap(2, k - 1))], zp = u[g.idx(i, j, g.wrap(2, k + 1))];
    return ((xm + xp) + (ym + yp)) + (zm + zp);
}

// the periodic copies n_d take the values of nodes 0 (after any update)
static void sync_copies(const NGrid& g, std::vector<double>& u) {
    for (int k = 0; k <= g.n[2]; ++k)
        for (int j = 0; j <= g.n[1]; ++j)
            for (int i = 0; i <= g.n[0]; ++i) {
                int c[3] = {i, j, k};
                bool copy = false;
                for (int d = 0; d < 3; ++d)
                    if (g.per[d] && c[d] == g.n[d]) { c[d] = 0; copy = true; }
                if (copy) u[g.idx(i, j, k)] = u[g.idx(c[0], c[1], c[2])];
            }
}

static void gs(const NGrid& g, std::vector<double>& u, const std::vector<double>& f, int colour) {
    const double h2 = g.h * g.h;
    for_unknowns(g, [&](int i, int j, int k) {
        if (((i + j + k) & 1) != colour) return;
        u[g.idx(i, j, k)] = (nsum(g, u, i, j, k) - h2 * f[g.idx(i, j, k)]) / 6.0;
    });
    sync_copies(g, u);
}

// r = f - L u at the unknowns (0 elsewhere); returns max |r| and sum r^2
static void residual(const NGrid& g, const std::vector<double>& u, const std::vector<double>& f,
                     std::vector<double>& r, double* rinf, double* rl2) {
    const double ih2 = 1.0 / (g.h * g.h);
    std::fill(r.begin(), r.end(), 0.0);
    double mx = 0.0, s2 = 0.0;
    bool bad = false;
    for_unknowns(g, [&](int i, int j, int k) {
        const long q = g.idx(i, j, k);
        const double rv = f[q] - (nsum(g, u, i, j, k) - 6.0 * u[q]) * ih2;
        r[q] = rv;
        const double a = std::fabs(rv);
        if (std::isnan(a)) bad = true;
        else if (a > mx) mx = a;
        s2 += rv * rv;
    });
    if (rinf) *rinf = bad ? std::nan("") : mx;
    if (rl2) *rl2 = s2;
}

// full weighting of r onto the coarse unknowns
static void restrict_fw(const NGrid& gf, const std::vector<double>& r, const NGrid& gc, std::vector<double>& fc) {
    std::fill(fc.begin(), fc.end(), 0.0);
    const double w[3] = {0.25, 0.5, 0.25};
    for_unknowns(gc, [&](int I, int J, int K) {
        double s = 0.0;
        for (int c = -1; c <= 1; ++c)
            for (int b = -1; b <= 1; ++b)
                for (int a = -1; a <= 1; ++a) {
                    const int i = gf.wrap(0, 2 * I + a), j = gf.wrap(1, 2 * J + b), k = gf.wrap(2, 2 * K + c);
                    s += ((w[a + 1] * w[b + 1]) * w[c + 1]) * r[gf.idx(i, j, k)];
                }
        fc[gc.idx(I, J, K)] = s;
    });
    sync_copies(gc, fc);
}

// u_f += P e_c (trilinear) at the fine unknowns
static void prolong_add(const NGrid& gc, const std::vector<double>& e, const NGrid& gf, std::vector<double>& u) {
    for_unknowns(gf, [&](int i, int j, int k) {
        const int c[3] = {i, j, k};
        int I[3], o[3];
        for (int d = 0; d < 3; ++d) { I[d] = c[d] >> 1; o[d] = c[d] & 1; }
        double s = 0.0;
        int cnt = 0;
        for (int cz = 0; cz <= o[2]; ++cz)
            for (int cy = 0; cy <= o[1]; ++cy)
                for (int cx = 0; cx <= o[0]; ++cx) {
                    s += e[gc.idx(I[0] + cx, I[1] + cy, I[2] + cz)];
                    ++cnt;
                }
        u[gf.idx(i, j, k)] += s / (double)cnt;
    });
    sync_copies(gf, u);
}

static double dotu(const NGrid& g, const std::vector<double>& a, const std::vector<double>& b) {
    double s = 0.0;
    for_unknowns(g, [&](int i, int j, int k) { s += a[g.idx(i, j, k)] * b[g.idx(i, j, k)]; });
    return s;
}

static long nunknowns(const NGrid& g) {
    long n = 0;
    for_unknowns(g, [&](int, int, int) { ++n; });
    return n;
}

static double mean_unknowns(const NGrid& g, const std::vector<double>& a) {
    double s = 0.0;
    for_unknowns(g, [&](int i, int j, int k) { s += a[g.idx(i, j, k)]; });
    return s / (double)nunknowns(g);
}

static void add_unknowns(const NGrid& g, std::vector<double>& a, double c) {
    for_unknowns(g, [&](int i, int j, int k) { a[g.idx(i, j, k)] += c; });
    sync_copies(g, a);
}

// L u at the unknowns (0 elsewhere)
static void apply(const NGrid& g, const std::vector<double>& u, std::vector<double>& Lu) {
    const double ih2 = 1.0 / (g.h * g.h);
    std::fill(Lu.begin(), Lu.end(), 0.0);
    for_unknowns(g, [&](int i, int j, int k) {
        const long q = g.idx(i, j, k);
        Lu[q] = (nsum(g, u, i, j, k) - 6.0 * u[q]) * ih2;
    });
}

static int bottom_cg(const NGrid& g, const std::vector<double>& f, std::vector<double>& x, double rtol) {
    const long N = g.size();
    std::vector<double> r(N, 0.0), p(N, 0.0), Ap(N, 0.0);
    for_unknowns(g, [&](int i, int j, int k) { r[g.idx(i, j, k)] = f[g.idx(i, j, k)]; });
    std::fill(x.begin(), x.end(), 0.0);
    if (g.singular()) add_unknowns(g, r, -mean_unknowns(g, r));
    p = r;
    sync_copies(g, p);
    double rs = dotu(g, r, r);
    const double rs0 = rs;
    int it = 0;
    if (rs0 == 0.0) return 0;
    const long maxit = 4 * nunknowns(g);
    for (; it < maxit;) {
        apply(g, p, Ap);
        const double alpha = rs / dotu(g, p, Ap);
        for_unknowns(g, [&](int i, int j, int k) {
            const long q = g.idx(i, j, k);
            x[q] += alpha * p[q];
            r[q] -= alpha * Ap[q];
        });
        const double rsn = dotu(g, r, r);
        ++it;
        if (std::sqrt(rsn) <= rtol * std::sqrt(rs0)) break;
        const double beta = rsn / rs;
        for_unknowns(g, [&](int i, int j, int k) {
            const long q = g.idx(i, j, k);
            p[q] = r[q] + beta * p[q];
        });
        sync_copies(g, p);
        rs = rsn;
    }
    if (g.singular()) add_unknowns(g, x, -mean_unknowns(g, x));
    sync_copies(g, x);
    return it;
}

struct NLevel {
    NGrid g;
    std::vector<double> u, f, r;
};

static void vcycle(std::vector<NLevel>& L, size_t l, int nu1, int nu2, double brtol) {
    NLevel& F = L[l];
    if (l + 1 == L.size()) {
        bottom_cg(F.g, F.f, F.u, brtol);
        return;
    }
    for (int s = 0; s < nu1; ++s) { gs(F.g, F.u, F.f, 0); gs(F.g, F.u, F.f, 1); }
    residual(F.g, F.u, F.f, F.r, nullptr, nullptr);
    NLevel& C = L[l + 1];
    restrict_fw(F.g, F.r, C.g, C.f);
    std::fill(C.u.begin(), C.u.end(), 0.0);
    vcycle(L, l + 1, nu1, nu2, brtol);
    prolong_add(C.g, C.u, F.g, F.u);
    for (int s = 0; s < nu2; ++s) { gs(F.g, F.u, F.f, 0); gs(F.g, F.u, F.f, 1); }
}

static std::vector<NLevel> hierarchy(const NGrid& g0) {
    std::vector<NLevel> L;
    NGrid g = g0;
    for (;;) {
        NLevel lv;
        lv.g = g;
        lv.u.assign(g.size(), 0.0);
        lv.f.assign(g.size(), 0.0);
        lv.r.assign(g.size(), 0.0);
        L.push_back(std::move(lv));
        if (!g.coarsenable()) break;
        g = g.coarse();
    }
    return L;
}

// Driver as for the cell-centred solve: residual, stop test on the max-norm
// relative to |f|_inf over the unknowns, one V(nu1, nu2) per cycle.
static int solve(const NGrid& g0, int nu1, int nu2, int max_cycles, int fixed_cycles, double rel_tol,
                 double brtol, const double* f_in, double* u_out, Info* info) {
    std::memset(info, 0, sizeof(Info));
    std::vector<NLevel> L = hierarchy(g0);
    info->levels = (int)L.size();
    NLevel& T = L[0];
    for (long q = 0; q < g0.size(); ++q) T.f[q] = f_in[q];
    double fnorm = 0.0;
    bool bad = false;
    for_unknowns(g0, [&](int i, int j, int k) {
        const double a = std::fabs(T.f[g0.idx(i, j, k)]);
        if (std::isnan(a)) bad = true;
        else if (a > fnorm) fnorm = a;
    });
    info->f_inf = bad ? std::nan("") : fnorm;
    int status = 0, cyc = 0;
    if (bad) status = -5;
    else if (fnorm > 0.0)
        for (;; ++cyc) {
            double rinf, rl2;
            residual(g0, T.u, T.f, T.r, &rinf, &rl2);
            if (cyc < 256) { info->hist[cyc] = rinf / fnorm; info->hist_l2[cyc] = std::sqrt(rl2); info->nhist = cyc + 1; }
            info->rel_inf = rinf / fnorm;
            info->rel_l2 = std::sqrt(rl2);
            if (!std::isfinite(rinf)) { status = -5; break; }
            if (fixed_cycles > 0) {
                if (cyc == fixed_cycles) break;
            } else {
                if (rinf <= rel_tol * fnorm) break;
                if (cyc == max_cycles) { status = -4; break; }
            }
            vcycle(L, 0, nu1, nu2, brtol);
        }
    info->cycles = cyc;
    if (status == 0 && g0.singular()) add_unknowns(g0, T.u, -mean_unknowns(g0, T.u));
    for (long q = 0; q < g0.size(); ++q) u_out[q] = T.u[q];
    info->status = status;
    return status;
}

}  // namespace nodal

// =========================================== two-level composite solve
// A coarse level over the domain and a fine level (refinement ratio 2) over
// a union of fine boxes, the paper's block-structured AMR pattern (Sections
// 1 and 2: levels of boxes, inter-level interpolation and copies).  The
// unknowns are the fine cells and the coarse cells not covered by the fine
// boxes; a covered coarse cell holds the mean of its 8 children.
//   fine ghosts   : from other fine boxes where they are fine cells; across
//                   the coarse-fine boundary, from the coarse cell C beyond
//                   it and the two fine cells inward: g = (8/15) U_t +
//                   (2/3) u_1 - (1/5) u_2 (the quadratic through the three
//                   centres along the normal); U_t is the quadratic through
//                   the 3x3 coarse cells around C in the face plane (with
//                   the mixed term) at the ghost's offset (s_a, s_b) h0/4,
//                   s = +1 for the upper half of C, -1 for the lower:
//                   U_C + sum_t [s_t (U_{+t} - U_{-t}) / 8 + (U_{+t} - 2 U_C
//                   + U_{-t}) / 32] + s_a s_b (U_{++} - U_{+-} - U_{-+} +
//                   U_{--}) / 64
//   fine operator : the 7-point operator with those ghosts
//   coarse        : at an uncovered cell, (sum over faces of the outward
//                   gradient) / h0; a face against a covered cell takes the
//                   mean of the 4 fine gradients (u_i - g_i) / h1 across it
//                   (flux matching), other faces (U_J - U_I) / h0, a
//                   Dirichlet face (-U_I - U_I) / h0
//   cycle         : nu1 fine GS sweeps (ghosts refreshed before each
//                   colour), fine residual, composite coarse residual at the
//                   uncovered cells and the mean of the fine residuals at the
//                   covered ones, one coarse V-cycle from zero on it (over
//                   the coarse domain as one box, whatever the coarse boxes),
//                   coarse update at the uncovered cells, fine update by
//                   trilinear interpolation of the coarse correction, nu2
//                   fine sweeps, covered cells := mean of their children
// The fine boxes must lie 2 coarse cells inside the domain (so a ghost's
// coarse cell and its tangential neighbours are domain cells).
namespace composite {

constexpr double kW8_15 = 8.0 / 15.0, kW2_3 = 2.0 / 3.0, kW1_5 = 1.0 / 5.0;

struct CFGhost {
    int box;         // fine box
    int g[3];        // the ghost cell (fine index)
    int i1[3], i2[3];  // the two fine cells inward
    int C[3];        // coarse cell of the ghost
    int ta, tb;      // tangential directions
    int sa, sb;      // +-1: the ghost's half of C along ta, tb
};

struct Comp {
    Geom gc, gf;
    std::vector<Box> cboxes, fboxes;
    std::vector<char> covered;  // coarse domain cells, F-order
    std::vector<int> fown;      // fine domain cells: owning fine box or -1
    std::vector<CFGhost> ghosts;
    size_t cq(int I, int J, int K) const {
        const Box& D = gc.dom;
        return (size_t)(I - D.lo[0]) + (size_t)D.n(0) * ((size_t)(J - D.lo[1]) + (size_t)D.n(1) * (K - D.lo[2]));
    }
    size_t fq(int i, int j, int k) const {
        const Box& D = gf.dom;
        return (size_t)(i - D.lo[0]) + (size_t)D.n(0) * ((size_t)(j - D.lo[1]) + (size_t)D.n(1) * (k - D.lo[2]));
    }
    bool in_fine(int i, int j, int k) const {
        const Box& D = gf.dom;
        if (!D.has(i, j, k)) return false;
        return fown[fq(i, j, k)] >= 0;
    }
};

// The layout this solve supports: fine boxes with even corners and odd
// upper corners (unions of whole coarse cells), pairwise disjoint, and 2
// coarse cells away from every domain face.
static bool layout_ok(const Geom& gc, const std::vector<Box>& fboxes) {
    for (size_t b = 0; b < fboxes.size(); ++b) {
        const Box& B = fboxes[b];
        for (int d = 0; d < 3; ++d) {
            if ((B.lo[d] & 1) || !(B.hi[d] & 1) || B.hi[d] < B.lo[d]) return false;
            if (B.lo[d] < 2 * gc.dom.lo[d] + 4 || B.hi[d] > 2 * gc.dom.hi[d] + 1 - 4) return false;
        }
        for (size_t q = 0; q < b; ++q) {
            const Box& Q = fboxes[q];
            bool sep = false;
            for (int d = 0; d < 3; ++d) sep = sep || Q.hi[d] < B.lo[d] || B.hi[d] < Q.lo[d];
            if (!sep) return false;
        }
    }
    return true;
}

static Comp setup(const Geom& gc, const std::vector<Box>& cboxes, const std::vector<Box>& fboxes) {
    Comp c;
    c.gc = gc;
    c.gf = gc;
    for (int d = 0; d < 3; ++d) { c.gf.dom.lo[d] = 2 * gc.dom.lo[d]; c.gf.dom.hi[d] = 2 * gc.dom.hi[d] + 1; }
    c.gf.h = gc.h * 0.5;
    c.cboxes = cboxes;
    c.fboxes = fboxes;
    c.fown = owner_map(c.gf, fboxes);
    c.covered.assign((size_t)gc.dom.cells(), 0);
    for (auto& b : fboxes)
        for (int k = b.lo[2] / 2; k <= b.hi[2] / 2; ++k)
            for (int j = b.lo[1] / 2; j <= b.hi[1] / 2; ++j)
                for (int i = b.lo[0] / 2; i <= b.hi[0] / 2; ++i) c.covered[c.cq(i, j, k)] = 1;
    for (size_t b = 0; b < fboxes.size(); ++b) {
        const Box& B = fboxes[b];
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i)
                    for (int d = 0; d < 3; ++d)
                        for (int side = 0; side < 2; ++side) {
                            int g[3] = {i, j, k};
                            g[d] += side ? 1 : -1;
                            if (B.has(g[0], g[1], g[2]) || c.in_fine(g[0], g[1], g[2])) continue;
                            CFGhost h;
                            h.box = (int)b;
                            for (int e = 0; e < 3; ++e) { h.g[e] = g[e]; h.i1[e] = (e == d) ? g[e] + (side ? -1 : 1) : g[e];
                                                          h.i2[e] = (e == d) ? g[e] + (side ? -2 : 2) : g[e];
                                                          h.C[e] = g[e] >> 1; }
                            h.ta = (d + 1) % 3;
                            h.tb = (d + 2) % 3;
                            h.sa = (g[h.ta] & 1) ? 1 : -1;
                            h.sb = (g[h.tb] & 1) ? 1 : -1;
                            c.ghosts.push_back(h);
                        }
    }
    return c;
}

// coarse values at any domain cell (covered cells hold the mean of the fine)
static double ghost_value(const Comp& c, const std::vector<double>& ug, const Fab<double>& F, const CFGhost& h) {
    // coarse values on the 3x3 cells around C in the face plane
    auto U = [&](int p, int q) {
        int x[3] = {h.C[0], h.C[1], h.C[2]};
        x[h.ta] += p;
        x[h.tb] += q;
        return ug[c.cq(x[0], x[1], x[2])];
    };
    const double UC = U(0, 0);
    const double da = (U(1, 0) - U(-1, 0)) * 0.125 * (double)h.sa, db = (U(0, 1) - U(0, -1)) * 0.125 * (double)h.sb;
    const double qa = ((U(1, 0) + U(-1, 0)) - 2.0 * UC) * (1.0 / 32.0);
    const double qb = ((U(0, 1) + U(0, -1)) - 2.0 * UC) * (1.0 / 32.0);
    const double xab = ((U(1, 1) - U(1, -1)) - (U(-1, 1) - U(-1, -1))) * (1.0 / 64.0) * (double)(h.sa * h.sb);
    const double Ut = UC + ((da + db) + (qa + qb)) + xab;
    const double u1 = F(h.i1[0], h.i1[1], h.i1[2]), u2 = F(h.i2[0], h.i2[1], h.i2[2]);
    return (kW8_15 * Ut + kW2_3 * u1) - kW1_5 * u2;
}

// fine ghosts: from other fine boxes, then the coarse-fine ones
static void fill_fine(const Comp& c, const std::vector<double>& ug, MF<double>& uf) {
    fill_boundary(c.gf, uf);
    for (const CFGhost& h : c.ghosts) {
        Fab<double>& F = uf.f[h.box];
        F(h.g[0], h.g[1], h.g[2]) = ghost_value(c, ug, F, h);
    }
}

// covered coarse cells := mean of their 8 children
static void sync_covered(const Comp& c, const MF<double>& uf, std::vector<double>& ug) {
    for (size_t b = 0; b < c.fboxes.size(); ++b) {
        const Box& B = c.fboxes[b];
        const Fab<double>& F = uf.f[b];
        for (int K = B.lo[2] / 2; K <= B.hi[2] / 2; ++K)
            for (int J = B.lo[1] / 2; J <= B.hi[1] / 2; ++J)
                for (int I = B.lo[0] / 2; I <= B.hi[0] / 2; ++I) {
                    const int i = 2 * I, j = 2 * J, k = 2 * K;
                    ug[c.cq(I, J, K)] = (((F(i, j, k) + F(i + 1, j, k)) + (F(i, j + 1, k) + F(i + 1, j + 1, k))) +
                                         ((F(i, j, k + 1) + F(i + 1, j, k + 1)) + (F(i, j + 1, k + 1) + F(i + 1, j + 1, k + 1)))) * 0.125;
                }
    }
}

// outward gradient across face (d, side) of uncovered coarse cell I
static double coarse_grad(const Comp& c, const std::vector<double>& ug, const MF<double>& uf, int I, int J, int K,
                          int d, int side) {
    const Geom& g = c.gc;
    const double h0 = g.h, h1 = c.gf.h;
    int n[3] = {I, J, K};
    n[d] += side ? 1 : -1;
    const double UI = ug[c.cq(I, J, K)];
    if (n[d] < g.dom.lo[d] || n[d] > g.dom.hi[d]) {
        if (!g.per[d]) return (-UI - UI) / h0;
        n[d] = g.dom.lo[d] + pmod(n[d] - g.dom.lo[d], g.dom.n(d));
    }
    if (!c.covered[c.cq(n[0], n[1], n[2])]) return (ug[c.cq(n[0], n[1], n[2])] - UI) / h0;
    // flux matching: the 4 fine cells of the neighbour against the face
    const int ta = (d + 1) % 3, tb = (d + 2) % 3;
    double a[2][2];
    for (int q = 0; q < 2; ++q)
        for (int p = 0; p < 2; ++p) {
            int fi[3];
            fi[d] = 2 * n[d] + (side ? 0 : 1);
            fi[ta] = 2 * n[ta] + p;
            fi[tb] = 2 * n[tb] + q;
            const int b = c.fown[c.fq(fi[0], fi[1], fi[2])];
            const Fab<double>& F = uf.f[b];
            int gcell[3] = {fi[0], fi[1], fi[2]};
            gcell[d] += side ? -1 : 1;
            // the ghost of fine cell fi toward I, as fill_fine computes it
            CFGhost h;
            h.box = b;
            for (int e = 0; e < 3; ++e) { h.g[e] = gcell[e]; h.i1[e] = fi[e]; h.i2[e] = fi[e]; h.C[e] = gcell[e] >> 1; }
            h.i2[d] += side ? 1 : -1;
            h.ta = ta;
            h.tb = tb;
            h.sa = (gcell[ta] & 1) ? 1 : -1;
            h.sb = (gcell[tb] & 1) ? 1 : -1;
            const double gv = ghost_value(c, ug, F, h);
            a[q][p] = (F(fi[0], fi[1], fi[2]) - gv) / h1;
        }
    return ((a[0][0] + a[0][1]) + (a[1][0] + a[1][1])) * 0.25;
}

static double coarse_op(const Comp& c, const std::vector<double>& ug, const MF<double>& uf, int I, int J, int K) {
    double gr[6];
    for (int d = 0; d < 3; ++d)
        for (int side = 0; side < 2; ++side) gr[2 * d + side] = coarse_grad(c, ug, uf, I, J, K, d, side);
    return (((gr[0] + gr[1]) + (gr[2] + gr[3])) + (gr[4] + gr[5])) / c.gc.h;
}

template <class F>
static void for_uncovered(const Comp& c, F fn) {
    const Box& D = c.gc.dom;
    for (int K = D.lo[2]; K <= D.hi[2]; ++K)
        for (int J = D.lo[1]; J <= D.hi[1]; ++J)
            for (int I = D.lo[0]; I <= D.hi[0]; ++I)
                if (!c.covered[c.cq(I, J, K)]) fn(I, J, K);
}

struct State {
    std::vector<double> uc, fc;  // global coarse arrays
    MF<double> uf, ff, rf;
};

// composite residual: rc at uncovered cells (0 at covered), rf at fine cells;
// returns max |r| over both and sum r^2
static void comp_residual(const Comp& c, State& S, std::vector<double>& rc, double* rinf, double* rl2) {
    fill_fine(c, S.uc, S.uf);
    double fi, fl;
    residual(c.gf, S.uf, S.ff, (const Faces*)nullptr, S.rf, &fi, &fl);
    double mx = fi, s2 = fl;
    bool bad = std::isnan(fi);
    std::fill(rc.begin(), rc.end(), 0.0);
    for_uncovered(c, [&](int I, int J, int K) {
        const double r = S.fc[c.cq(I, J, K)] - coarse_op(c, S.uc, S.uf, I, J, K);
        rc[c.cq(I, J, K)] = r;
        const double a = std::fabs(r);
        if (std::isnan(a)) bad = true;
        else if (a > mx) mx = a;
        s2 += r * r;
    });
    *rinf = bad ? std::nan("") : mx;
    *rl2 = s2;
}

static void cycle(const Comp& c, State& S, Hier<double>& H, const Params& P, std::vector<double>& rc) {
    auto sweeps = [&](int n) {
        for (int s = 0; s < n; ++s)
            for (int col = 0; col < 2; ++col) {
                fill_fine(c, S.uc, S.uf);
                gs_colour(c.gf, S.uf, S.ff, (const Faces*)nullptr, col);
            }
    };
    sweeps(P.nu1);
    double ri, rl;
    comp_residual(c, S, rc, &ri, &rl);
    // covered cells: the mean of the fine residuals below them
    for (size_t b = 0; b < c.fboxes.size(); ++b) {
        const Box& B = c.fboxes[b];
        const Fab<double>& R = S.rf.f[b];
        for (int K = B.lo[2] / 2; K <= B.hi[2] / 2; ++K)
            for (int J = B.lo[1] / 2; J <= B.hi[1] / 2; ++J)
                for (int I = B.lo[0] / 2; I <= B.hi[0] / 2; ++I) {
                    const int i = 2 * I, j = 2 * J, k = 2 * K;
                    rc[c.cq(I, J, K)] = (((R(i, j, k) + R(i + 1, j, k)) + (R(i, j + 1, k) + R(i + 1, j + 1, k))) +
                                         ((R(i, j, k + 1) + R(i + 1, j, k + 1)) + (R(i, j + 1, k + 1) + R(i + 1, j + 1, k + 1)))) * 0.125;
                }
    }
    // coarse correction: one V-cycle from zero
    scatter_global(c.gc.dom, rc.data(), H.f[0]);
    H.u[0].zero();
    vcycle(H, P, 0, nullptr);
    std::vector<double> e((size_t)c.gc.dom.cells());
    gather_global(c.gc.dom, H.u[0], e.data());
    for_uncovered(c, [&](int I, int J, int K) { S.uc[c.cq(I, J, K)] += e[c.cq(I, J, K)]; });
    // fine update: trilinear interpolation of e (parent and its neighbours on
    // the child's side, weights 27, 9, 3, 1 over 64)
    for (size_t b = 0; b < c.fboxes.size(); ++b) {
        const Box& B = c.fboxes[b];
        Fab<double>& F = S.uf.f[b];
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) {
                    const int I = i >> 1, J = j >> 1, K = k >> 1;
                    const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
                    auto E = [&](int a, int bb, int cc) { return e[c.cq(a, bb, cc)]; };
                    const double c000 = E(I, J, K), c100 = E(I + si, J, K), c010 = E(I, J + sj, K), c001 = E(I, J, K + sk);
                    const double c110 = E(I + si, J + sj, K), c101 = E(I + si, J, K + sk), c011 = E(I, J + sj, K + sk);
                    const double c111 = E(I + si, J + sj, K + sk);
                    const double v = (((27.0 * c000 + 9.0 * ((c100 + c010) + c001)) + 3.0 * ((c110 + c101) + c011)) + c111) * (1.0 / 64.0);
                    F(i, j, k) += v;
                }
    }
    sweeps(P.nu2);
    sync_covered(c, S.uf, S.uc);
}

static int solve(const Geom& gc, const std::vector<Box>& cboxes, const std::vector<Box>& fboxes, const Params& P,
                 const double* fc_glob, const double* ff_glob, double* uc_glob, double* uf_glob, Info* info) {
    std::memset(info, 0, sizeof(Info));
    Comp c = setup(gc, cboxes, fboxes);
    // the coarse correction's V-cycle runs over the coarse domain as one box,
    // whatever the caller's coarse boxes (the same correction for every
    // decomposition of the coarse level)
    (void)cboxes;
    std::vector<Level> L = hierarchy(gc, std::vector<Box>{gc.dom}, P.min_box_edge);
    info->levels = (int)L.size() + 1;
    Hier<double> H;
    H.define(L, nullptr);
    State S;
    const size_t Nc = (size_t)gc.dom.cells();
    S.uc.assign(Nc, 0.0);
    S.fc.assign(fc_glob, fc_glob + Nc);
    S.uf.define(fboxes, 1);
    S.ff.define(fboxes, 1);
    S.rf.define(fboxes, 1);
    scatter_global(c.gf.dom, ff_glob, S.ff);
    double fnorm = 0.0;
    bool bad = false;
    for_uncovered(c, [&](int I, int J, int K) {
        const double a = std::fabs(S.fc[c.cq(I, J, K)]);
        if (std::isnan(a)) bad = true; else if (a > fnorm) fnorm = a;
    });
    const double ffn = max_abs_valid(S.ff);
    if (std::isnan(ffn)) bad = true; else if (ffn > fnorm) fnorm = ffn;
    info->f_inf = bad ? std::nan("") : fnorm;
    std::vector<double> rc(Nc, 0.0);
    int status = 0, cyc = 0;
    if (bad) status = -5;
    else if (fnorm > 0.0)
        for (;; ++cyc) {
            double rinf, rl2;
            comp_residual(c, S, rc, &rinf, &rl2);
            if (cyc < 256) { info->hist[cyc] = rinf / fnorm; info->hist_l2[cyc] = std::sqrt(rl2); info->nhist = cyc + 1; }
            info->rel_inf = rinf / fnorm;
            info->rel_l2 = std::sqrt(rl2);
            if (!std::isfinite(rinf)) { status = -5; break; }
            if (P.fixed_cycles > 0) {
                if (cyc == P.fixed_cycles) break;
            } else {
                if (rinf <= P.rel_tol * fnorm) break;
                if (cyc == P.max_cycles) { status = -4; break; }
            }
            cycle(c, S, H, P, rc);
        }
    info->cycles = cyc;
    std::memcpy(uc_glob, S.uc.data(), Nc * sizeof(double));
    const size_t Nf = (size_t)c.gf.dom.cells();
    for (size_t q = 0; q < Nf; ++q) uf_glob[q] = 0.0;
    gather_global(c.gf.dom, S.uf, uf_glob);
    info->status = status;
    return status;
}

// The composite operator on given fields (covered coarse cells are taken
// as the mean of uf): Lc at uncovered cells (0 at covered), Lf at fine cells.
static void apply(const Geom& gc, const std::vector<Box>& cboxes, const std::vector<Box>& fboxes, const double* uc_glob,
                  const double* uf_glob, double* Lc_glob, double* Lf_glob) {
    Comp c = setup(gc, cboxes, fboxes);
    const size_t Nc = (size_t)gc.dom.cells(), Nf = (size_t)c.gf.dom.cells();
    std::vector<double> ug(uc_glob, uc_glob + Nc);
    MF<double> uf, lf;
    uf.define(fboxes, 1);
    lf.define(fboxes, 0);
    scatter_global(c.gf.dom, uf_glob, uf);
    sync_covered(c, uf, ug);
    fill_fine(c, ug, uf);
    const double ih2 = 1.0 / (c.gf.h * c.gf.h);
    for (size_t b = 0; b < fboxes.size(); ++b) {
        const Box& B = fboxes[b];
        for (int k = B.lo[2]; k <= B.hi[2]; ++k)
            for (int j = B.lo[1]; j <= B.hi[1]; ++j)
                for (int i = B.lo[0]; i <= B.hi[0]; ++i) {
                    double su, sb;
                    stencil(uf.f[b], (const Faces*)nullptr, i, j, k, su, sb);
                    lf.f[b](i, j, k) = (su - sb * uf.f[b](i, j, k)) * ih2;
                }
    }
    for (size_t q = 0; q < Nc; ++q) Lc_glob[q] = 0.0;
    for_uncovered(c, [&](int I, int J, int K) { Lc_glob[c.cq(I, J, K)] = coarse_op(c, ug, uf, I, J, K); });
    for (size_t q = 0; q < Nf; ++q) Lf_glob[q] = 0.0;
    gather_global(c.gf.dom, lf, Lf_glob);
}

}  // namespace composite
}  // namespace orc

// ====================================================================== C API
// Multi-box arrays cross this interface "packed": the grown boxes (ng ghost
// cells) of a level, one after another in box order, each in F-order with
// the component index slowest.  Global arrays are domain-sized, F-order.
using namespace orc;

static Box box6(const int* p) { return Box{{p[0], p[1], p[2]}, {p[3], p[4], p[5]}}; }
static std::vector<Box> boxes_of(int nb, const int* lohi) {
    std::vector<Box> v;
    for (int b = 0; b < nb; ++b) v.push_back(box6(lohi + 6 * b));
    return v;
}
static Geom geom_of(const int* dom6, const int* per, double h) {
    Geom g;
    g.dom = box6(dom6);
    for (int d = 0; d < 3; ++d) g.per[d] = per[d] ? 1 : 0;
    g.h = h;
    return g;
}
template <class T>
static void unpack(MF<T>& mf, const T* data, int comp, int ncomp) {
    size_t off = 0;
    for (auto& F : mf.f) {
        size_t n = F.v.size();
        std::memcpy(F.v.data(), data + off + (size_t)comp * n, n * sizeof(T));
        off += n * ncomp;
    }
}
template <class T>
static void pack(const MF<T>& mf, T* data, int comp, int ncomp) {
    size_t off = 0;
    for (auto& F : mf.f) {
        size_t n = F.v.size();
        std::memcpy(data + off + (size_t)comp * n, F.v.data(), n * sizeof(T));
        off += n * ncomp;
    }
}

extern "C" {

int orc_chop(const int* dom6, int max_box, int cap, int* out_lohi) {
    std::vector<Box> bs = chop(box6(dom6), max_box);
    if ((int)bs.size() > cap) return -(int)bs.size();
    for (size_t b = 0; b < bs.size(); ++b)
        for (int d = 0; d < 3; ++d) { out_lohi[6 * b + d] = bs[b].lo[d]; out_lohi[6 * b + 3 + d] = bs[b].hi[d]; }
    return (int)bs.size();
}

// Hierarchy of levels: per level the domain and the boxes (min_edge < 2:
// the default threshold).  Returns the number of levels, or a negative count
// if the caps are too small.
int orc_hierarchy(const int* dom6, int nb, const int* lohi, int min_edge, int cap_levels, int cap_boxes,
                  int* lev_nb, int* lev_dom6, int* lev_lohi) {
    const int noper[3] = {0, 0, 0};
    Geom g = geom_of(dom6, noper, 1.0);
    std::vector<Level> L = hierarchy(g, boxes_of(nb, lohi), min_edge);
    int tot = 0;
    for (auto& l : L) tot += (int)l.boxes.size();
    if ((int)L.size() > cap_levels || tot > cap_boxes) return -1;
    int o = 0;
    for (size_t l = 0; l < L.size(); ++l) {
        lev_nb[l] = (int)L[l].boxes.size();
        for (int d = 0; d < 3; ++d) { lev_dom6[6 * l + d] = L[l].g.dom.lo[d]; lev_dom6[6 * l + 3 + d] = L[l].g.dom.hi[d]; }
        for (auto& b : L[l].boxes) {
            for (int d = 0; d < 3; ++d) { lev_lohi[6 * o + d] = b.lo[d]; lev_lohi[6 * o + 3 + d] = b.hi[d]; }
            ++o;
        }
    }
    return (int)L.size();
}

void orc_fill_boundary(const int* dom6, const int* per, int nb, const int* lohi, int ng, int ncomp, double* data) {
    MF<double> mf;
    mf.define(boxes_of(nb, lohi), ng);
    Geom g = geom_of(dom6, per, 1.0);
    for (int c = 0; c < ncomp; ++c) {
        unpack(mf, data, c, ncomp);
        fill_boundary(g, mf);
        pack(mf, data, c, ncomp);
    }
}

// ParallelCopy between two decompositions of one domain (paper, Section 2:
// copies from one distribution to another): every cell of a destination box
// grown by ngc (<= ngd) that, wrapped into the domain through its periodic
// directions, lies in the valid region of a source box takes that cell's
// value, components [scomp, scomp+ncomp) into [dcomp, dcomp+ncomp); other
// cells keep theirs.  Brute force: the owner of every domain cell.
void orc_parallel_copy(const int* dom6, const int* per, int nbd, const int* lohid, int ngd, int ncd, int ngc,
                       int nbs, const int* lohis, int ngs, int ncs, int dcomp, int scomp, int ncomp, double* dst,
                       const double* src) {
    Geom g = geom_of(dom6, per, 1.0);
    const std::vector<Box> bd = boxes_of(nbd, lohid), bs = boxes_of(nbs, lohis);
    const std::vector<int> own = owner_map(g, bs);
    const Box& D = g.dom;
    for (int c = 0; c < ncomp; ++c) {
        MF<double> S, T;
        S.define(bs, ngs);
        T.define(bd, ngd);
        unpack(S, src, scomp + c, ncs);
        unpack(T, dst, dcomp + c, ncd);
        for (size_t b = 0; b < bd.size(); ++b) {
            Fab<double>& F = T.f[b];
            const Box& B = bd[b];
            for (int k = B.lo[2] - ngc; k <= B.hi[2] + ngc; ++k)
                for (int j = B.lo[1] - ngc; j <= B.hi[1] + ngc; ++j)
                    for (int i = B.lo[0] - ngc; i <= B.hi[0] + ngc; ++i) {
                        int w[3] = {i, j, k};
                        bool inside = true;
                        for (int d = 0; d < 3; ++d)
                            if (w[d] < D.lo[d] || w[d] > D.hi[d]) {
                                if (g.per[d]) w[d] = D.lo[d] + pmod(w[d] - D.lo[d], D.n(d));
                                else inside = false;
                            }
                        if (!inside) continue;
                        const size_t q = (size_t)(w[0] - D.lo[0]) +
                                         (size_t)D.n(0) * ((size_t)(w[1] - D.lo[1]) + (size_t)D.n(1) * (w[2] - D.lo[2]));
                        const int o = own[q];
                        if (o < 0) continue;
                        F(i, j, k) = S.f[o](w[0], w[1], w[2]);
                    }
        }
        pack(T, dst, dcomp + c, ncd);
    }
}

void orc_apply_bc(const int* dom6, const int* per, int nb, const int* lohi, int ng, int ncomp, int odd, double* data) {
    MF<double> mf;
    mf.define(boxes_of(nb, lohi), ng);
    Geom g = geom_of(dom6, per, 1.0);
    for (int c = 0; c < ncomp; ++c) {
        unpack(mf, data, c, ncomp);
        apply_bc(g, mf, odd != 0);
        pack(mf, data, c, ncomp);
    }
}

void orc_fill_boundary_f32(const int* dom6, const int* per, int nb, const int* lohi, int ng, int ncomp, float* data) {
    MF<float> mf;
    mf.define(boxes_of(nb, lohi), ng);
    Geom g = geom_of(dom6, per, 1.0);
    for (int c = 0; c < ncomp; ++c) {
        unpack(mf, data, c, ncomp);
        fill_boundary(g, mf);
        pack(mf, data, c, ncomp);
    }
}

// One red-black colour on a level (ng = 1, ghosts must be current).
// beta_glob: NULL for constant coefficient, else the level's cell beta as a
// global array (only valid for a level-0 call: faces from the cell field).
static void gs_impl(const int* dom6, const int* per, int nb, const int* lohi, double h, int colour, double* u,
                    const double* f, const double* beta_glob, double alpha) {
    Geom g = geom_of(dom6, per, h);
    g.alpha = alpha;
    MF<double> U, F;
    U.define(boxes_of(nb, lohi), 1);
    F.define(boxes_of(nb, lohi), 1);
    unpack(U, u, 0, 1);
    unpack(F, f, 0, 1);
    Faces fc;
    if (beta_glob) fc = faces_from_beta<double>(g, beta_glob);
    gs_colour(g, U, F, beta_glob ? &fc : nullptr, colour);
    pack(U, u, 0, 1);
}

void orc_gs(const int* dom6, const int* per, int nb, const int* lohi, double h, int colour, double* u,
            const double* f, const double* beta_glob, double alpha) {
    gs_impl(dom6, per, nb, lohi, h, colour, u, f, beta_glob, alpha);
}

void orc_gs_f32(const int* dom6, const int* per, int nb, const int* lohi, double h, int colour, float* u,
                const float* f) {
    Geom g = geom_of(dom6, per, h);
    MF<float> U, F;
    U.define(boxes_of(nb, lohi), 1);
    F.define(boxes_of(nb, lohi), 1);
    unpack(U, u, 0, 1);
    unpack(F, f, 0, 1);
    gs_colour<float>(g, U, F, nullptr, colour);
    pack(U, u, 0, 1);
}

void orc_residual(const int* dom6, const int* per, int nb, const int* lohi, double h, const double* u,
                  const double* f, const double* beta_glob, double alpha, double* r, double* norms) {
    Geom g = geom_of(dom6, per, h);
    g.alpha = alpha;
    MF<double> U, F, R;
    U.define(boxes_of(nb, lohi), 1);
    F.define(boxes_of(nb, lohi), 1);
    R.define(boxes_of(nb, lohi), 1);
    unpack(U, u, 0, 1);
    unpack(F, f, 0, 1);
    unpack(R, r, 0, 1);
    Faces fc;
    if (beta_glob) fc = faces_from_beta<double>(g, beta_glob);
    residual(g, U, F, beta_glob ? &fc : nullptr, R, &norms[0], &norms[1]);
    pack(R, r, 0, 1);
}

// Restriction from a fine level (ng_f) to a coarse level (ng_c).
void orc_restrict(int nbf, const int* lohif, int ngf, int nbc, const int* lohic, int ngc, const double* rf,
                  double* fc) {
    MF<double> R, C;
    R.define(boxes_of(nbf, lohif), ngf);
    C.define(boxes_of(nbc, lohic), ngc);
    unpack(R, rf, 0, 1);
    unpack(C, fc, 0, 1);
    restrict_avg(R, C);
    pack(C, fc, 0, 1);
}

void orc_prolong(int nbf, const int* lohif, int ngf, int nbc, const int* lohic, int ngc, int order, const double* ec,
                 double* uf) {
    MF<double> U, E;
    U.define(boxes_of(nbf, lohif), ngf);
    E.define(boxes_of(nbc, lohic), ngc);
    unpack(U, uf, 0, 1);
    unpack(E, ec, 0, 1);
    prolong_add(E, U, order);
    pack(U, uf, 0, 1);
}

// Face coefficients of every level from a global cell beta.  out receives,
// level by level, the x, y and z face arrays (global, F-order, sized
// (nx+1)*ny*nz, nx*(ny+1)*nz, nx*ny*(nz+1)).  Returns the number of doubles.
long orc_faces(const int* dom6, const int* per, int nb, const int* lohi, const double* beta, double* out, long cap) {
    Geom g = geom_of(dom6, per, 1.0);
    std::vector<Level> L = hierarchy(g, boxes_of(nb, lohi));
    std::vector<Faces> F = build_faces<double>(L, beta);
    long n = 0;
    for (auto& fl : F)
        for (int d = 0; d < 3; ++d) n += (long)fl.c[d].size();
    if (n > cap) return -n;
    long o = 0;
    for (auto& fl : F)
        for (int d = 0; d < 3; ++d) { std::memcpy(out + o, fl.c[d].data(), fl.c[d].size() * sizeof(double)); o += (long)fl.c[d].size(); }
    return n;
}

// L u for a global array u (one box covering the domain), FP64.
void orc_apply_op(const int* dom6, const int* per, double h, const double* u_glob, const double* beta_glob,
                  double alpha, double* Lu_glob) {
    Geom g = geom_of(dom6, per, h);
    g.alpha = alpha;
    std::vector<Box> one{g.dom};
    MF<double> U, A;
    U.define(one, 1);
    A.define(one, 0);
    scatter_global(g.dom, u_glob, U);
    Faces fc;
    if (beta_glob) fc = faces_from_beta<double>(g, beta_glob);
    apply_op(g, U, beta_glob ? &fc : nullptr, A);
    gather_global(g.dom, A, Lu_glob);
}

typedef struct {
    int nu1, nu2, max_cycles, precision, prolong, fixed_cycles;
    double rel_tol, abs_tol, h, bottom_rtol;
    int min_box_edge;  // < 2: the default hierarchy threshold
    int krylov;        // 1: multigrid-preconditioned conjugate gradients
    int use_guess;     // 1: u_glob holds the initial guess on entry
    int pad;
    double alpha;      // Helmholtz coefficient: solves div(beta grad u) - alpha u = f
} orc_params;

int orc_solve(const orc_params* p, const int* dom6, const int* per, int nb, const int* lohi, const double* f_glob,
              const double* beta_glob, double* u_glob, Info* info) {
    Params P;
    P.nu1 = p->nu1; P.nu2 = p->nu2; P.max_cycles = p->max_cycles; P.precision = p->precision;
    P.prolong = p->prolong; P.fixed_cycles = p->fixed_cycles;
    P.rel_tol = p->rel_tol; P.abs_tol = p->abs_tol; P.h = p->h; P.bottom_rtol = p->bottom_rtol;
    P.min_box_edge = p->min_box_edge >= 2 ? p->min_box_edge : kDefaultMinBoxEdge;
    P.krylov = p->krylov;
    P.use_guess = p->use_guess;
    Geom g = geom_of(dom6, per, p->h);
    g.alpha = p->alpha;
    return solve(P, g, boxes_of(nb, lohi), f_glob, beta_glob, u_glob, info);
}

// One backward-Euler step of the heat equation u_t = div(beta grad u) + s:
// (u' - u) / dt = div(beta grad u') + s, i.e. div(beta grad u') - u'/dt = f
// with f = -(u/dt + s): a Helmholtz solve with alpha = 1/dt, started from u.
// u_glob: u on entry, u' on return; s_glob may be NULL.  p->alpha and
// p->use_guess are ignored (alpha = 1/dt, guess = u).
int orc_heat_step(const orc_params* p, const int* dom6, const int* per, int nb, const int* lohi, double dt,
                  const double* s_glob, const double* beta_glob, double* u_glob, Info* info) {
    const Box D = box6(dom6);
    const size_t N = (size_t)D.cells();
    const double inv = 1.0 / dt;
    std::vector<double> f(N);
    for (size_t q = 0; q < N; ++q) {
        double t = u_glob[q] * inv;
        if (s_glob) t = t + s_glob[q];
        f[q] = -t;
    }
    orc_params q = *p;
    q.alpha = inv;
    q.use_guess = 1;
    return orc_solve(&q, dom6, per, nb, lohi, f.data(), beta_glob, u_glob, info);
}

// Bottom solve on its own (global arrays, one box): for tests of the CG stage.
int orc_bottom(const int* dom6, const int* per, double h, const double* f_glob, const double* beta_glob,
               double alpha, double rtol, double* u_glob, int* iters) {
    Geom g = geom_of(dom6, per, h);
    g.alpha = alpha;
    std::vector<Box> one{g.dom};
    std::vector<Level> L{Level{g, one}};
    std::vector<Faces> F = build_faces<double>(L, beta_glob);
    MF<double> rhs, x;
    rhs.define(one, 0);
    x.define(one, 1);
    scatter_global(g.dom, f_glob, rhs);
    CGStats st = bottom_cg(g, one, rhs, F.empty() ? nullptr : &F[0], x, rtol);
    gather_global(g.dom, x, u_glob);
    if (iters) *iters = st.iters;
    return 0;
}

// ---------------------------------------------------------------- nodal
static nodal::NGrid ngrid(const int* n, const int* per, double h) {
    nodal::NGrid g;
    for (int d = 0; d < 3; ++d) { g.n[d] = n[d]; g.per[d] = per[d] ? 1 : 0; }
    g.h = h;
    return g;
}

// Node arrays are (n0+1)(n1+1)(n2+1) values in F-order.
int orc_nodal_solve(const int* n, const int* per, double h, int nu1, int nu2, int max_cycles, int fixed_cycles,
                    double rel_tol, double bottom_rtol, const double* f, double* u, Info* info) {
    return nodal::solve(ngrid(n, per, h), nu1, nu2, max_cycles, fixed_cycles, rel_tol, bottom_rtol, f, u, info);
}

void orc_nodal_apply(const int* n, const int* per, double h, const double* u, double* Lu) {
    nodal::NGrid g = ngrid(n, per, h);
    std::vector<double> U(u, u + g.size()), A(g.size());
    nodal::apply(g, U, A);
    std::memcpy(Lu, A.data(), A.size() * sizeof(double));
}

void orc_nodal_gs(const int* n, const int* per, double h, int colour, double* u, const double* f) {
    nodal::NGrid g = ngrid(n, per, h);
    std::vector<double> U(u, u + g.size()), F(f, f + g.size());
    nodal::gs(g, U, F, colour);
    std::memcpy(u, U.data(), U.size() * sizeof(double));
}

void orc_nodal_residual(const int* n, const int* per, double h, const double* u, const double* f, double* r,
                        double* norms) {
    nodal::NGrid g = ngrid(n, per, h);
    std::vector<double> U(u, u + g.size()), F(f, f + g.size()), R(g.size());
    nodal::residual(g, U, F, R, &norms[0], &norms[1]);
    std::memcpy(r, R.data(), R.size() * sizeof(double));
}

// fine grid n (even edges); the coarse grid has n/2 cells per direction
void orc_nodal_restrict(const int* n, const int* per, const double* rf, double* fc) {
    nodal::NGrid g = ngrid(n, per, 1.0), c = g.coarse();
    std::vector<double> R(rf, rf + g.size()), F(c.size());
    nodal::restrict_fw(g, R, c, F);
    std::memcpy(fc, F.data(), F.size() * sizeof(double));
}

void orc_nodal_prolong_add(const int* n, const int* per, const double* ec, double* uf) {
    nodal::NGrid g = ngrid(n, per, 1.0), c = g.coarse();
    std::vector<double> E(ec, ec + c.size()), U(uf, uf + g.size());
    nodal::prolong_add(c, E, g, U);
    std::memcpy(uf, U.data(), U.size() * sizeof(double));
}

int orc_nodal_bottom(const int* n, const int* per, double h, const double* f, double* u, double rtol) {
    nodal::NGrid g = ngrid(n, per, h);
    std::vector<double> F(f, f + g.size()), X(g.size());
    const int it = nodal::bottom_cg(g, F, X, rtol);
    std::memcpy(u, X.data(), X.size() * sizeof(double));
    return it;
}

// ------------------------------------------------------------ composite
// Coarse arrays over the domain (n cells per direction), fine arrays over
// the refined domain (2n), both F-order; fine boxes in fine indices.
int orc_composite_solve(const int* dom6, const int* per, int nbc, const int* lohic, int nbf, const int* lohif,
                        double h, int nu1, int nu2, int max_cycles, int fixed_cycles, double rel_tol,
                        const double* fc, const double* ff, double* uc, double* uf, Info* info) {
    Geom g = geom_of(dom6, per, h);
    Params P;
    P.nu1 = nu1; P.nu2 = nu2; P.max_cycles = max_cycles; P.fixed_cycles = fixed_cycles; P.rel_tol = rel_tol;
    std::vector<Box> fb = boxes_of(nbf, lohif);
    if (!composite::layout_ok(g, fb)) { std::memset(info, 0, sizeof(Info)); info->status = -2; return -2; }
    return composite::solve(g, boxes_of(nbc, lohic), fb, P, fc, ff, uc, uf, info);
}

int orc_composite_apply(const int* dom6, const int* per, int nbc, const int* lohic, int nbf, const int* lohif,
                        double h, const double* uc, const double* uf, double* Lc, double* Lf) {
    Geom g = geom_of(dom6, per, h);
    std::vector<Box> fb = boxes_of(nbf, lohif);
    if (!composite::layout_ok(g, fb)) return -2;
    composite::apply(g, boxes_of(nbc, lohic), fb, uc, uf, Lc, Lf);
    return 0;
}

}  // extern "C"
