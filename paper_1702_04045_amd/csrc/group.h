// Grouped launches: one kernel launch that runs the work of many cells.
//
// A grouped launch covers up to kGroupMax entries (a cell, or one 64-band
// chunk of a cell).  Entry e owns the virtual blocks start[e] .. start[e+1]-1
// of a one-dimensional grid, laid out as a gx[e]-wide two-dimensional grid
// (or, for the matrix-core products, as a range of work units); args[e]
// points at the entry's kernel arguments in device memory.  The table is
// passed by value, so a launch needs no copy to the device.  Each entry's
// blocks compute exactly what the cell's own launch computes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace paro {

constexpr int kGroupMax = 64;

struct GroupTab {
    const void *args[kGroupMax];
    int32_t start[kGroupMax + 1];
    int32_t gx[kGroupMax];
    int32_t n;
};

// entry and two-dimensional block coordinates of virtual block b
__device__ __forceinline__ int group_entry(const GroupTab &t, int64_t b)
{
    int lo = 0, hi = t.n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (t.start[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}
__device__ __forceinline__ void group_block(const GroupTab &t, int &e, int &bx, int &by)
{
    e = group_entry(t, blockIdx.x);
    const int l = (int)blockIdx.x - t.start[e];
    bx = l % t.gx[e];
    by = l / t.gx[e];
}

// Host side: entries are appended with their block (or unit) counts.
struct GroupBuilder {
    GroupTab t{};
    int64_t total = 0;
    GroupBuilder() { t.start[0] = 0; }
    bool full() const { return t.n == kGroupMax; }
    void add(const void *dev_args, int64_t blocks, int gx)
    {
        t.args[t.n] = dev_args;
        t.gx[t.n] = gx;
        total += blocks;
        t.start[t.n + 1] = (int32_t)total;
        ++t.n;
    }
};

// Kernel arguments of the grouped source solve, one set per cell (the
// stick and plane kernels one per 64-band chunk).
template <class C2> struct GReal;
template <> struct GReal<double2> { using T = double; };
template <> struct GReal<float2> { using T = float; };

template <class C2> struct StickInvArgs {
    const C2 *src;
    int64_t ld;
    C2 *pbuf;
    const double *beta;
    C2 *sticks;
    const int32_t *st_start, *pt_sz;
    const C2 *tw;
    int nst;
};
template <class C2> struct PlaneArgs {
    C2 *sticks;
    const int32_t *cols;
    const typename GReal<C2>::T *vperm;
    const C2 *tw;
    int nst, N3, nb, nmax1, bpb;  // bpb: bands per work-group
};
template <class C2> struct StickFwdArgs {
    const C2 *sticks;
    const int32_t *st_start, *pt_sz;
    const C2 *tw, *xin;
    int64_t ld;
    C2 *out;
    const double *kin, *shift;
    double scale;
    double *dot_part;
    int nst, part_stride;
};
struct PcgInitPartsArgs {
    const double2 *psi;
    int64_t ld;
    const double *kin;
    double *dots;
    int64_t ng;
    int nb;
};
template <class CV, class CU> struct PcgInitArgs {
    const double2 *psi, *hpsi;
    int64_t ld;
    const double *eps, *kin;
    CU *u;
    int64_t ldu;
    CV *r, *z;
    int64_t ldv;
    double *dots, *sc;
    int64_t ng;
    int nparts, nb, correction;
};
struct PcgScalarsArgs {
    const double *dots_pq, *dots_rz;
    double *sc;
    int32_t *active, *bflags, *band_flags_out, *status;
    int nb, nparts_rz, npq;
};
template <class CV, class CU> struct PcgUpdateArgs {
    const CV *p, *q;
    int64_t ldv;
    CU *u;
    int64_t ldu;
    CV *r, *z;
    const double *kin, *dots_pq;
    double *dots_rz;
    const double *sc;
    const int32_t *active;
    int64_t ng;
    int npq, nb;
};
template <class C2> struct GemmHnArgs {
    const C2 *A;
    int64_t lda;
    const C2 *B;
    int64_t ldb;
    double2 *part;
    int64_t K, kchunk, units;
    int M, N, bm, bn;
};
template <class CO> struct GemmHnRedArgs {
    const double2 *part;
    CO *C;
    int64_t ldc;
    const double *dscale;
    double *quad;
    int M, N, nsplit;
};
template <class C2> struct GemmNnArgs {
    const C2 *A;
    int64_t lda;
    const C2 *B;
    int64_t ldb;
    C2 *C;
    int64_t ldc, M, units;
    int N, K, bn, accumulate;
};

constexpr int kGroupChunks = 16;  // band chunks of up to 1024 bands (FP64: 64 bands each; FP32: 160)

// The kernels of one cell's source solve in one precision of its vectors
// (FP64, or FP32 for the mixed-precision solve of the correction).
template <class C2> struct GroupSolveArgs {
    StickInvArgs<C2> sinv[kGroupChunks];
    PlaneArgs<C2> plane[kGroupChunks];
    StickFwdArgs<C2> sfwd[kGroupChunks];
    GemmHnArgs<C2> hn;
    GemmHnRedArgs<C2> hred;
    GemmNnArgs<C2> nn;
    PcgInitArgs<C2, C2> init;
    PcgUpdateArgs<C2, C2> upd;
};

// Rayleigh-Ritz, residuals and shift of Algorithm 1 (steps 4-5)
struct CholArgs {
    const double2 *gram;
    double2 *L, *X;
    int32_t *fail, *status;
    int m, hs;
};
struct TrsmArgs {
    const double2 *L, *src;
    double2 *out;
    int m, transb, mode;
};
struct TridiagArgs {
    double2 *A;
    double *d, *e;
    double2 *tau;
    int m;
};
struct EigvalsArgs {
    const double *d, *e;
    double *lam, *lam2;
    int m, nout;
};
struct EigvecsArgs {
    const double *d, *e, *lam;
    double *Z;
    int m;
};
struct BacktArgs {
    const double2 *A, *tau;
    const double *Z;
    double2 *Y;
    int m;
};
struct ResPartsArgs {
    const double2 *psi, *hpsi;
    int64_t ld;
    const double *eps;
    double *dots;
    int64_t ng;
};
struct ResFinalArgs {
    const double *dots;
    double *res;
    int nb, nparts;
};
struct BookArgs {
    const double *eps, *res;
    double *sig_all, *sig_out, *stats;  // stats: the statistics table (row it + 1 is written)
    int32_t *conv;
    double sigma_lb, tol_res;
    int nb, n_conv, shift_mode, row;
};
struct GroupFinishArgs {
    // W = H U
    StickInvArgs<double2> sinv[kGroupChunks];
    PlaneArgs<double2> plane[kGroupChunks];
    StickFwdArgs<double2> sfwd[kGroupChunks];
    GemmHnArgs<double2> nl_hn;
    GemmHnRedArgs<double2> nl_red;
    GemmNnArgs<double2> nl_nn;
    // S = U^H U, H_s = U^H W, the dense eigenproblem, psi = U C, H psi = W C
    GemmHnArgs<double2> s_hn, h_hn;
    GemmHnRedArgs<double2> s_red, h_red;
    CholArgs chol;
    TrsmArgs trsm[3];
    TridiagArgs tri;
    EigvalsArgs evals;
    EigvecsArgs evecs;
    BacktArgs back;
    GemmNnArgs<double2> rot_psi, rot_hpsi;
    ResPartsArgs rparts;
    ResFinalArgs rfinal;
    BookArgs book;
};

// Everything one cell's source solve and Rayleigh-Ritz need, in the
// cell's workspace.
struct GroupCellDesc {
    GroupSolveArgs<double2> f64;
    GroupSolveArgs<float2> f32;
    PcgInitPartsArgs iparts;
    PcgScalarsArgs sc0, sc1;
    GroupFinishArgs fin;
};
// device address of a cell descriptor's arguments for vectors of type C2
template <class C2> inline const GroupSolveArgs<C2> *group_solve_args(const GroupCellDesc *d)
{
    const char *b = reinterpret_cast<const char *>(d);
    if constexpr (sizeof(C2) == 16) return reinterpret_cast<const GroupSolveArgs<C2> *>(b + offsetof(GroupCellDesc, f64));
    else return reinterpret_cast<const GroupSolveArgs<C2> *>(b + offsetof(GroupCellDesc, f32));
}

}  // namespace paro
