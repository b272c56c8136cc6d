// Internal declarations of libparo (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "group.h"
#include "paro.h"

namespace paro {

constexpr int kMaxBandsPerChunk = 64;     // FP64 bands per sphere->stick->plane pass
constexpr int kMaxBandsPerChunk32 = 160;  // FP32 bands per pass (the same stick buffer holds either)
template <class C2> constexpr int chunk_bands() { return sizeof(C2) == 16 ? kMaxBandsPerChunk : kMaxBandsPerChunk32; }
static_assert(kGroupChunks * kMaxBandsPerChunk >= 1024 && kGroupChunks * kMaxBandsPerChunk32 >= 1024,
              "grouped descriptors cover every chunk of a 1024-band cell");
constexpr int kPartSplits = 64;        // split-K partials the workspaces hold per output element
constexpr int kMaxParts = 512;         // partial sums per band per reduction
constexpr int kDensityBandsPerGroup = 8;  // bands one work-group of the density kernel sums
constexpr int kPlaneBandsDefault = 4;     // bands per work-group of the plane kernel unless tuned
// Plane-stage launch choice a new plan takes for grid n and precision slot
// pi (0: FP64, 1: FP32): schedule 0 with kPlaneBandsDefault bands per
// work-group, except FP64 at 96 points: the compressed-column schedule 2
// with 2 bands per work-group, the fastest choice measured at that grid.
// A plan builds its potential in schedule 0's order, which schedule 2
// shares, so the default needs no re-layout.
inline void plane_default(int n, int pi, int32_t *sched, int32_t *bands)
{
    const bool cc = n == 96 && pi == 0;
    *sched = cc ? 2 : 0;
    *bands = cc ? 2 : kPlaneBandsDefault;
}
constexpr int kPlaneBandsMax = 64;

// per-band scalar slots (Workspace::sc, each nb long)
enum { SC_GAMMA = 0, SC_GAMMA0, SC_TAU, SC_BETA, SC_NLQ, kScalars };
// partial-sum slots (Workspace::dots, each nb x kMaxParts)
enum { DOT_PQ = 0, DOT_RZ, DOT_TKIN, DOT_NRM, DOT_RES, DOT_PJR, DOT_PJI, DOT_PJN, kDotSlots };

struct Plan {
    hipStream_t stream = nullptr;
    double cell[9], bvec[9], omega, ecut, vmin;
    int32_t grid[3], nmax[3];
    int64_t ng = 0, ldv = 0;  // sphere size; padded length of workspace vectors
    int32_t nst = 0, nproj = 0, ncol = 0;
    // device arrays inside the caller's plan buffer
    double *kin = nullptr;        // (1/2)|G|^2, ng
    int32_t *pt_sz = nullptr;     // per sphere point: (stick << 8) | (n3 mod N3)
    int32_t *st_start = nullptr;  // per stick: first sphere point, nst + 1
    int32_t *cols = nullptr;      // per n1 column (n1 = -nmax1 ..): first stick, lowest n2, stick count
    double *vplane = nullptr;     // local potential in the plane kernel's row-thread order
    double2 *tw[3] = {nullptr, nullptr, nullptr};  // exp(-2 pi i m / N_d)
    double2 *beta = nullptr;      // KB projectors, nproj x ldv (projector-major)
    // single-precision copies for the mixed-precision source solves
    float *vplane32 = nullptr;
    float2 *tw32[3] = {nullptr, nullptr, nullptr};
    float2 *beta32 = nullptr;
    // the projectors as BF16 hi / lo pairs for the split-BF16 products:
    // nproj x bf_ldk (projector-major) and ng x bf_ldp (transposed), zero padded
    uint32_t *bs_hi = nullptr, *bs_lo = nullptr, *bt_hi = nullptr, *bt_lo = nullptr;
    int64_t bf_ldk = 0;
    int32_t bf_ldp = 0;
    double *dkb = nullptr;        // KB energies
    int32_t *status = nullptr;    // sticky status bits
    int32_t *miller = nullptr;    // Miller indices of the sphere, ng x 3
    // plane-stage launch choices per precision (0: FP64, 1: FP32): the line
    // schedule (PlaneSched variant; vplane / vplane32 are laid out for it)
    // and the bands one work-group takes through its z-plane
    int32_t plane_sched[2] = {0, 0};
    int32_t plane_bands[2] = {kPlaneBandsDefault, kPlaneBandsDefault};
};

// Workspace carve-up for calls on up to nb bands (m <= 2 nb for Rayleigh-Ritz).
struct Workspace {
    double2 *sticks;          // min(64, 2 nb) x N3 x nst
    double2 *sticks2;         // grids above 96 points: a second stick buffer (else null)
    double2 *r, *z, *p, *q;   // PCG vectors, nb x ldv each
    double2 *U, *W;           // 2 nb x ldv each: Rayleigh-Ritz basis and its H image
    double2 *gram;            // [S Hs], m x 2m
    double2 *part;            // split-K partial tiles
    size_t part_elems;
    double2 *P;               // projector coefficients, nproj x 2 nb
    double2 *dense[5];        // max(2 nb, nproj)^2 each: L, X, Hhat, Y, C
    double *dreal;            // real scratch of the tridiagonal eigensolver
    size_t dreal_elems;
    double *sc;               // per-band scalars, kScalars x nb
    double *dots;             // per-band partial sums, kDotSlots x nb x kMaxParts
    int32_t *iflags;          // per band: active (nb) and status bits (nb)
    double *sig_all, *res, *eps_all;  // 2 nb each
    double *scal;             // 8 doubles of device scalars
    // single-precision PCG vectors of the mixed-precision source solve,
    // aliased onto r, z, p, q and W (unused while it runs): nb x ldv each
    float2 *r32, *z32, *p32, *q32, *d32;
    // kernel arguments of this cell's grouped source-solve launches
    GroupCellDesc *desc;
};

size_t workspace_bytes(const Plan &pl, int nb);
Workspace carve_workspace(const Plan &pl, int nb, void *ws);
// bytes of the paro_density workspace; *part_off: offset of the partial grids
size_t density_workspace_bytes(const Plan &pl, int nb, size_t *part_off);
// carve-up of the paro_projector_gradient workspace (ws may be null to size it)
struct ProjGradWs {
    double2 *gbeta;           // G_a beta_p, (3 n_proj) x ldv, component-major
    double2 *P, *S;           // beta^H psi (n_proj x nb), (G beta)^H psi (3 n_proj x nb), column-major
    double2 *part;            // split-K partials
    size_t part_elems;
};
ProjGradWs proj_grad_workspace(const Plan &pl, int nb, void *ws, size_t *bytes);
size_t dense_real_elems(int mmax);

void set_error(const std::string &msg);
// HIP event pair around launches of the kernel class being profiled (no-op otherwise)
void prof_mark(int kernel, hipStream_t s, bool begin);
#define PARO_HIP_TRY(expr)                                                      \
    do {                                                                        \
        hipError_t _e = (expr);                                                 \
        if (_e != hipSuccess) {                                                 \
            ::paro::set_error(std::string(#expr ": ") + hipGetErrorString(_e)); \
            return PARO_EHIP;                                                   \
        }                                                                       \
    } while (0)

// ---- launchers (return the hipError_t of the launches) ----
// apply.hip
bool fft_supported(int n);
// grids above 96 points: the plane stage keeps only the populated columns
// in LDS and writes the forward sticks to a second stick buffer
bool big_grid(int n);
// the local potential re-laid in the order the plane kernel's row threads use it
void build_plane_potential(int n, const int32_t *grid, const double *vloc, double *out);
void build_plane_potential(int n, const int32_t *grid, const double *vloc, float *out);
// selectable line schedules of the plane stage at n points
int plane_schedules(int n);
// map[p'] = p: row position p of line schedule `from` that holds the entry
// row position p' of schedule `to` holds (n entries; Stockham grids only)
bool plane_row_map(int n, bool fp32, int from, int to, int32_t *map);
// only the plane kernel of a local apply (the sticks as they are), for the autotuner
hipError_t launch_plane_only(const Plan &pl, const Workspace &w, int nb, bool fp32);
// Local part on nb bands: out_b = FFT^-1 (V FFT(x_b)) / N + (kin - shift_b) x_b,
// x = src, or in PCG mode (pbuf != null) x = p with p <- z + beta_b p first
// (first: p <- z) and src = z; dot_part then gets partial Re(x^H out).
hipError_t launch_local_apply(const Plan &pl, const Workspace &w, int nb, const double2 *src, int64_t ld,
                              double2 *out, const double *shift, double2 *pbuf, const double *beta, bool first,
                              double *dot_part, int *nparts_out);
// the same in single precision (FP32 tables of the plan, FP32 sticks)
hipError_t launch_local_apply(const Plan &pl, const Workspace &w, int nb, const float2 *src, int64_t ld, float2 *out,
                              const double *shift, float2 *pbuf, const double *beta, bool first, double *dot_part,
                              int *nparts_out);
// rho (C order [i1][i2][i3]) = sum_b w_b |psi_b(r)|^2 on the FFT grid, weights
// null = 1; sticks: min(64, nb) x N3 x nst, part: ceil(min(64, nb) / 8) grids
hipError_t launch_density(const Plan &pl, double2 *sticks, double *part, int nb, const double2 *psi, int64_t ld,
                          const double *weights, double *rho, bool accumulate = false);
// gemm.hip
hipError_t gemm_hn(hipStream_t s, int M, int N, int64_t K, const double2 *A, int64_t lda, const double2 *B,
                   int64_t ldb, double2 *C, int64_t ldc, double2 *part, size_t part_elems, const double *dscale,
                   double *quad);
hipError_t gemm_nn(hipStream_t s, int64_t M, int N, int K, const double2 *A, int64_t lda, const double2 *B,
                   int64_t ldb, double2 *C, int64_t ldc, bool accumulate);
// single-precision operands on the FP32 matrix cores; split partials are
// summed in FP64
hipError_t gemm_hn(hipStream_t s, int M, int N, int64_t K, const float2 *A, int64_t lda, const float2 *B,
                   int64_t ldb, float2 *C, int64_t ldc, double2 *part, size_t part_elems, const double *dscale,
                   double *quad);
hipError_t gemm_nn(hipStream_t s, int64_t M, int N, int K, const float2 *A, int64_t lda, const float2 *B,
                   int64_t ldb, float2 *C, int64_t ldc, bool accumulate);
hipError_t launch_to_single(hipStream_t s, int64_t n, const double2 *src, float2 *dst);
// split-BF16 projector products (gemm_bf16.hip)
int64_t bf16_ldk(int64_t ng);
int bf16_ldp(int nproj);
hipError_t launch_split_beta(const Plan &pl);
size_t bf16_apply_scratch_bytes(const Plan &pl, int nb);
hipError_t apply_nl_bf16(const Plan &pl, const Workspace &w, int nb, const float2 *x, int64_t ld, float2 *out,
                         int64_t ldo, void *scratch, double *quad);
// dd[p] = sum_b w_b |P_pb|^2, dR[3p + a] = sum_b w_b d_p 2 Re(conj(P_pb) Q_pb^a)
// with P = beta^H psi and Q^a = (-i G_a beta)^H psi (weights null = 1)
hipError_t launch_projector_gradient(const Plan &pl, const ProjGradWs &w, int nb, const double2 *psi, int64_t ld,
                                     const double *weights, double *dd, double *dR);
hipError_t launch_build_projectors(const Plan &pl, const int32_t *miller_dev, const double *centers,
                                   const int32_t *lm, const double *widths);
// vec.hip
// proj_psi != null: the projected correction equation of Algorithm 3 (r0
// and every z projected onto the complement of psi; implies correction)
hipError_t launch_pcg_init(const Plan &pl, const Workspace &w, int nb, const double2 *psi, const double2 *hpsi,
                           int64_t ld, const double *eps, double2 *u, int64_t ldu, int32_t *band_flags,
                           bool correction, const double2 *proj_psi = nullptr);
hipError_t launch_pcg_update(const Plan &pl, const Workspace &w, int nb, double2 *u, int64_t ldu, int npq,
                             int32_t *band_flags, const double2 *proj_psi = nullptr, int64_t ldpsi = 0);
// x_b <- x_b - psi_b (psi_b^H x_b) / |psi_b|^2 (PCG vectors, leading dimension ldv)
hipError_t launch_project_out(const Plan &pl, const Workspace &w, int nb, const double2 *psi, int64_t ld,
                              double2 *x);
// Mixed precision: the correction d = u - psi from d = 0 with FP32 vectors
// (r32, z32, p32, q32, d32); r = eps psi - H psi is formed in FP64.
hipError_t launch_pcg_init_mixed(const Plan &pl, const Workspace &w, int nb, const double2 *psi,
                                 const double2 *hpsi, int64_t ld, const double *eps, int32_t *band_flags);
hipError_t launch_pcg_update_mixed(const Plan &pl, const Workspace &w, int nb, int npq, int32_t *band_flags);
// u_b = base_b + d32_b (base = psi), or u_b = d32_b (base = null), in FP64
hipError_t launch_finish_correction(const Plan &pl, const Workspace &w, int nb, const double2 *base, int64_t ld,
                                    double2 *u, int64_t ldu);
hipError_t launch_residuals(const Plan &pl, const Workspace &w, int nb, const double2 *psi, const double2 *hpsi,
                            int64_t ld, const double *eps, double *res);
hipError_t launch_normalize_bands(const Plan &pl, const Workspace &w, int nb, double2 *e, int64_t lde);
hipError_t launch_copy_bands(hipStream_t s, int nb, int64_t ng, const double2 *src, int64_t lds, double2 *dst,
                             int64_t ldd);
// solver.hip
// out_b = (H - shift_b) x_b (shift null: H), local and nonlocal parts
hipError_t apply_full(const Plan &pl, const Workspace &w, int nb, const double2 *x, int64_t ld, double2 *out,
                      const double *shift);
// n_cg PCG steps of the source problems (mode 0: Algorithm 1, from u = psi;
// 1: the correction equation of Algorithm 2; 2: the projected one of Algorithm 3)
hipError_t source_solve(const Plan &pl, const Workspace &w, int nb, const double2 *psi, const double2 *hpsi,
                        int64_t ld, const double *eps, const double *shift, int ncg, double2 *u, int64_t ldu,
                        int32_t *band_flags, int mode = 0);
// Rayleigh-Ritz on span{U} with W = H U (m vectors, ld); the eigenvector
// coefficients C (m x n_keep, column-major) are left in w.dense[4]
hipError_t rayleigh_ritz(const Plan &pl, const Workspace &w, int m, int nkeep, const double2 *U, const double2 *W,
                         int64_t ld, double *eps, double2 *psi, double2 *hpsi, int64_t ldo);
// dense.hip
hipError_t launch_rr_dense(const Plan &pl, const Workspace &w, int m, int n_keep, double *eps_out, double2 *C);
hipError_t launch_heev(hipStream_t st, const Workspace &w, int m, const double2 *A, double *wout, double2 *V);
hipError_t launch_shift_bound(const Plan &pl, const Workspace &w, double *sigma);
hipError_t launch_bookkeeping(const Plan &pl, int nb, const paro_iter_opts &o, const double *eps, const double *res,
                              double *sig_all, double *sig_out, double *stats_row, int32_t *conv);

// Grouped source solve over many cells (one launch per kernel and FFT
// length): the cells, each with its descriptor in device memory.
struct GroupCell {
    const Plan *pl;
    const Workspace *w;
    int nb;
    const GroupCellDesc *dev;   // in the cell's workspace
    const GroupCellDesc *host;  // the host copy it was written from
};
void describe_pcg(const Plan &pl, const Workspace &w, int nb, const double2 *psi, const double2 *hpsi, int64_t ld,
                  const double *eps, double2 *u, int64_t ldu, int32_t *band_flags, bool correction, int npq,
                  GroupCellDesc &d);
// the mixed-precision solve's PCG (launch_pcg_init_mixed, launch_pcg_update_mixed)
void describe_pcg_mixed(const Plan &pl, const Workspace &w, int nb, const double2 *psi, const double2 *hpsi,
                        int64_t ld, const double *eps, int32_t *band_flags, int npq, GroupCellDesc &d);
// C2 = double2: the FP64 solve; float2: the mixed-precision solve
template <class C2> hipError_t launch_pcg_init_grouped(hipStream_t s, const GroupCell *cells, int n);
template <class C2> hipError_t launch_pcg_update_grouped(hipStream_t s, const GroupCell *cells, int n);
// the stick and plane launches of (H - sigma) p with the PCG prologue, as
// launch_local_apply(z, q, shift, p, beta = w.sc + SC_BETA nb) with the FP64
// vectors (and the FP32 ones of the mixed solve); returns the number of
// partial sums of p^H q per band
int describe_local_apply(const Plan &pl, const Workspace &w, int nb, const double *shift, GroupCellDesc &d);
bool grouped_grid(int n);  // FFT lengths with grouped kernels
template <class C2> hipError_t launch_local_apply_grouped(hipStream_t s, const GroupCell *cells, int n, bool first);
// the projector products of the solve (FP64, and FP32 matrix cores)
void describe_nonlocal(const Plan &pl, const Workspace &w, int nb, GroupCellDesc &d);
template <class C2> hipError_t launch_nonlocal_grouped(hipStream_t s, const GroupCell *cells, int n);
// matrix-core products of many cells (device arguments, and the host copy for the work counts)
template <class C2> struct HnRef {
    const GemmHnArgs<C2> *dev, *host;
    const GemmHnRedArgs<C2> *dred;
};
template <class C2> struct NnRef {
    const GemmNnArgs<C2> *dev, *host;
};
template <class C2> hipError_t launch_hn_grouped(hipStream_t s, const HnRef<C2> *v, int n);
template <class C2> hipError_t launch_nn_grouped(hipStream_t s, const NnRef<C2> *v, int n);
// host bytes to device memory through kernel arguments (capturable)
hipError_t upload_bytes(hipStream_t s, void *dst, const void *src, size_t bytes);
// The grouped end of an outer iteration of Algorithm 1 (W = H U,
// Rayleigh-Ritz at m = nb <= 92, residuals, next shift)
void describe_finish_local(const Plan &pl, const Workspace &w, int nb, const double2 *U, double2 *W, int64_t ld,
                           GroupFinishArgs &f);
hipError_t launch_finish_local_grouped(hipStream_t s, const GroupCell *cells, int n);
void describe_finish_products(const Plan &pl, const Workspace &w, int m, int nkeep, const double2 *U,
                              const double2 *W, int64_t ld, double2 *psi, double2 *hpsi, int64_t ldo,
                              GroupFinishArgs &f);
bool rr_dense_groupable(int m);
void describe_rr_dense(const Plan &pl, const Workspace &w, int m, int n_keep, double *eps_out, double2 *C,
                       GroupFinishArgs &f);
hipError_t launch_rr_dense_grouped(hipStream_t s, const GroupCell *cells, int n);
void describe_residuals(const Plan &pl, const Workspace &w, int nb, const double2 *psi, const double2 *hpsi,
                        int64_t ld, const double *eps, double *res, GroupFinishArgs &f);
hipError_t launch_residuals_grouped(hipStream_t s, const GroupCell *cells, int n);
void describe_bookkeeping(const Plan &pl, int nb, const paro_iter_opts &o, const double *eps, const double *res,
                          double *sig_all, double *sig_out, double *stats, int32_t *conv, GroupFinishArgs &f);
hipError_t launch_bookkeeping_grouped(hipStream_t s, const GroupCell *cells, int n, int it);

}  // namespace paro

struct paro_plan_s {
    paro::Plan pl;
};
