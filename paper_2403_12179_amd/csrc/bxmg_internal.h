// Internal declarations shared by the host driver (bxmg_host.cpp) and the
// HIP kernels (bxmg_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace bxmg {

constexpr int kMaxBottomCells = 4096;  // bottom level: one workgroup, vectors in LDS
constexpr int kBlock = 256;            // threads per block of the cell kernels

// Box of a level in the multigrid hierarchy, colour-split storage ("RB").
// Cells of colour c = (i+j+k)&1 of the box grown by ng are stored as half
// rows: element (i,j,k) sits at
//   base + c*cstride + ((k-glo.z)*G.y + (j-glo.y))*H + ((i-glo.x)>>1).
// Both colours of a row share the half-row index m = (i-glo.x)>>1.
struct RBox {
    int lo[3], hi[3];  // valid cells, global
    int glo[3];        // lo - ng
    int G[3];          // grown extents
    int H;             // half-row pitch = (G.x + 1) / 2
    int pid;           // problem id (batches); 0 for a single problem
    long long base;    // element offset of colour 0
    long long cstride; // elements between colour 0 and colour 1
};

// Box of a caller MultiFab (F-order): element (i,j,k,n) at
//   base + n*cs + (i-glo.x) + G.x*((j-glo.y) + G.y*(k-glo.z)).
struct FBox {
    int lo[3], hi[3];
    int glo[3];
    int G[3];
    long long base;
    long long cs;  // component stride
};

// One rectangular ghost-copy region: destination cells dlo + (x,y,z),
// 0 <= x < n[0] ..., of box dbox take neg ? -v : v, v = the cell
// s_d = sgn_d * dst_d + soff_d of box sbox.  prefix = cells before it.
struct Tag {
    int dbox, sbox;
    int dlo[3];
    int n[3];
    int soff[3];
    int sgn[3];
    int neg;
    int pad;
    long long prefix;
};

// Work decomposition of a level's valid cells of one colour (or of the
// coarse cells of every fine box) flattened over boxes: cell g of the
// launch belongs to box b with cstart[b] <= g < cstart[b+1]; within the box
// it is (t, j, k) with t fastest, t < tn[b] (= half-row cells or coarse x).
struct WorkBox {
    long long cstart;
    int tn, ny, nz;
    int box;  // box index in the level
    int cbox; // coarse box owning coarsen(box) (transfer kernels), else -1
    int pad;
};

// Face coefficients of a level >= 1: global arrays over the level domain,
// x faces (nx+1)*ny*nz, y faces nx*(ny+1)*nz, z faces nx*ny*(nz+1), F-order.
template <class T>
struct FaceArrays {
    const T* c[3];
    int dlo[3];
    int n[3];  // domain extents
};

// ------------------------------------------------------------ launchers
// All launchers enqueue on `s` and return hipSuccess or the launch error.
hipError_t launch_fill_rb(hipStream_t s, void* data, bool f32, const RBox* boxes, const Tag* tags, int ntags,
                          long long ncells, int cmask);
hipError_t launch_fill_fab(hipStream_t s, void* data, bool f32, const FBox* boxes, const Tag* tags, int ntags,
                           long long ncells, int comp0, int ncomp);

template <class T>
hipError_t launch_gs(hipStream_t s, T* u, const T* f, const T* beta, FaceArrays<T> fa, const RBox* boxes,
                     const WorkBox* work, int nwork, long long ncells, T h2, int colour);

template <class T>
hipError_t launch_resid_norm(hipStream_t s, const T* u, const T* f, const T* beta, FaceArrays<T> fa,
                             const RBox* boxes, const WorkBox* work, int nwork, long long ncells, T ih2, T* r,
                             double* partials, int nblocks);
hipError_t launch_norm_final(hipStream_t s, const double* partials, int nblocks, double* out3);

template <class T>
hipError_t launch_resid_restrict(hipStream_t s, const T* u, const T* f, const T* beta, FaceArrays<T> fa,
                                 const RBox* fboxes, const RBox* cboxes, const WorkBox* work, int nwork,
                                 long long ncells, T ih2, T* fc);
template <class T>
hipError_t launch_prolong(hipStream_t s, const T* ec, T* uf, const RBox* fboxes, const RBox* cboxes,
                          const WorkBox* work, int nwork, long long ncells, int order);
template <class T>
hipError_t launch_restrict_plain(hipStream_t s, const T* rf, T* fc, const RBox* fboxes, const RBox* cboxes,
                                 const WorkBox* work, int nwork, long long ncells);

template <class T>
hipError_t launch_zero(hipStream_t s, T* p, long long n);

// layout conversions: F-order caller MultiFab (FP64, comp 0) <-> RB level
hipError_t launch_fab_to_rb(hipStream_t s, const double* fab, const FBox* fb, void* rb, bool f32, const RBox* rbx,
                            const WorkBox* work, int nwork, long long ncells);
hipError_t launch_rb_to_fab(hipStream_t s, const double* rb, const RBox* rbx, double* fab, const FBox* fb,
                            const WorkBox* work, int nwork, long long ncells);

// mixed precision: r32 = float(f - L u) with fused norms; u64 += e32
hipError_t launch_resid_cast(hipStream_t s, const double* u, const double* f, const double* beta,
                             FaceArrays<double> fa, const RBox* boxes, const WorkBox* work, int nwork,
                             long long ncells, double ih2, float* r32, double* partials, int nblocks);
hipError_t launch_add_f32(hipStream_t s, double* u, const float* e, const RBox* boxes, const WorkBox* work,
                          int nwork, long long ncells);
hipError_t launch_cast_f32(hipStream_t s, const double* src, float* dst, long long n);

// variable coefficient setup
template <class T>
hipError_t launch_faces_from_cells(hipStream_t s, const T* beta, const RBox* fboxes, const WorkBox* work, int nwork,
                                   long long ncells, int d, FaceArrays<T> out, T* dst);
template <class T>
hipError_t launch_faces_coarsen(hipStream_t s, FaceArrays<T> fine, FaceArrays<T> coarse, int d, T* dst);

// bottom: one workgroup, FP64 CG in LDS
template <class T>
hipError_t launch_bottom(hipStream_t s, T* u, const T* f, FaceArrays<T> fa, bool var, const RBox* boxes, int nboxes,
                         const int* dom_lo, const int* dom_hi, const int* periodic, double h, double rtol,
                         int* iters_out);

// max |x|, sum x^2, non-finite count of an RB field's valid cells -> partials
hipError_t launch_field_norm(hipStream_t s, const double* x, const RBox* boxes, const WorkBox* work, int nwork,
                             long long ncells, double* partials, int nblocks);

// periodic projection of a level-0 RB field: subtract the mean of valid cells
hipError_t launch_mean_sub(hipStream_t s, double* u, const RBox* boxes, const WorkBox* work, int nwork,
                           long long ncells, double* scratch, int nblocks);

}  // namespace bxmg
