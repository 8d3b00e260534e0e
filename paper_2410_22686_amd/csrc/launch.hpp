// Host-side launch wrappers shared between the kernel files and the API.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "fft_lds.hpp"

namespace pcop {

// blocks of `kernel` that stay resident on one CU (at least 1): the size of
// a persistent grid is this times the number of CUs
template <class K>
inline int resident_blocks(K kernel, int threads, size_t dyn_lds) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, dyn_lds) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  return nb;
}

// Optional per-kernel timing: when set, launch wrappers bracket every kernel
// with begin/end (HIP events on the launch stream) and report the kernel
// family and its algorithmic HBM bytes.
enum KFamily {
  KF_KKT = 0, KF_TIME_FWD, KF_DST_ROWS, KF_DST_AX2, KF_DST_LAST, KF_TIME_INV, KF_MG_SMOOTH,
  KF_MG_RESTRICT, KF_MG_PROLONG, KF_MDOT, KF_UPDATE, KF_COMBINE, KF_SMALL, KF_IDEAL_STEP, KF_COUNT
};
struct KTimer {
  void (*begin)(void* self, int family, double bytes);
  void (*end)(void* self);
  void* self;
};
inline void tbeg(const KTimer* t, int fam, double bytes) {
  if (t && t->begin) t->begin(t->self, fam, bytes);
}
inline void tend(const KTimer* t) {
  if (t && t->end) t->end(t->self);
}

// Tables used by the preconditioner kernels (all device pointers into the
// workspace, filled at setup).
struct MgLevel {
  int nx;              // points per dimension on this level
  long long m;         // nx^dim
  double h2inv;        // 1/h_l^2
  const float* coef;   // [1 + 2 dim][m] tau-scaled stencil of K_a on this level (FP32), or null (a = 1)
  const double* coef64;  // same in FP64
  void* z;             // [B][2K][m] complex correction on this level (levels >= 1)
  void* r;             // [B][2K][m] complex right-hand side on this level (levels >= 1)
};

// multigrid levels a hierarchy can hold: vertex-centred coarsening of
// nx = 2^p - 1 reaches one point after p levels, and the largest accepted
// grid (m <= 2^28, so nx <= 16383 in 2-D) needs 14
constexpr int kMaxMgLevels = 16;

struct PrecondTables {
  const double* dpow;    // [n]  eps^{j/n}
  const double* twn64;   // [n]  exp(-2 pi i t/n) as (re, im)
  const float* twn32;
  const double* twM64;   // [M]  exp(-2 pi i t/M)      (Bluestein)
  const float* twM32;
  const double* chirp64; // [n]  exp(-i pi (t^2 mod 2n)/n)
  const float* chirp32;
  const double* bhat64;  // [M]  FFT_M of the chirp filter
  const float* bhat32;
  const double* pr64;    // prime-factor plans (n = N1 PR): [RC] exp(-2 pi i t/RC), then [RC]
  const float* pr32;     //   the Rader filter DFT_RC(b)/RC, RC = PR - 1; null for other n
  const double* twL64;   // [L]  exp(-2 pi i t/L), L = 2(nx+1)
  const float* twL32;
  const double* mu1;     // [nx] 1-D eigenvalue of K per sine mode k = 1..nx: (4/h^2) sin^2(pi k h/2)
                         // (finite differences) or k_k / m_k (Q1 elements, see im1)
  const double* im1;     // [nx] 1 / m_k, m_k = (h/3)(2 + cos(pi k h)) the 1-D Q1 mass eigenvalue; null when M = I
  const double* lam;     // [K] lambda_k as (re, im)
  const double* alpha;   // [B]
  const int* active;     // [B] or null
  int nact;              // members with active != 0 (for byte accounting)
  int ncu;               // compute units of the device (persistent grids)
  int dst_variant;       // 0: register kernels, 1: LDS-staged kernels, 2: register, 8-line column tiles
  int time_cols;         // time-kernel request, as pcop_options::time_cols
  const KTimer* timer;   // or null
  FftPlan plan;          // radices of n
  int mg_levels;
  int mg_smoother;       // 0 red-black, 1 lexicographic, 2 symmetric lexicographic Gauss-Seidel
  MgLevel mg[kMaxMgLevels];
  const void* mg_res;    // finest-level residual scratch [B][2K][m] complex
};

void launch_kkt_apply(const Geo& g, const double* x, double* y, const double* c, const double* alpha,
                      const double* xscale, int xs_stride, const int* active, bool transpose,
                      const double* ecoef, double ediag, double eoff, int jchunk, hipStream_t st);
// Q1 finite elements (fem.hip): the KKT matvec with M != I (same arguments
// as launch_kkt_apply, which forwards to it when g.fem), and y = M x on
// ngroups groups of spg consecutive spatial slices (group k of x at
// k * sgs doubles, of y at k * dgs)
void launch_kkt_fem(const Geo& g, const double* x, double* y, const double* c, const double* alpha,
                    const double* xscale, int xs_stride, const int* active, bool transpose, hipStream_t st);
void launch_mass_apply(const Geo& g, const double* x, long long sgs, double* y, long long dgs, int spg,
                       int ngroups, hipStream_t st);
// dst = src or J src (flip), members at b * dvs / b * svs
void launch_restride(const Geo& g, const double* src, long long svs, double* dst, long long dvs, bool flip,
                     hipStream_t st);
void launch_rhs(const Geo& g, const double* gg, const double* ff, const double* y0, const double* sg,
                double* b, hipStream_t st);
void launch_unpack(const Geo& g, const double* x, const double* sg, double* y, double* p, hipStream_t st);
void launch_pack_cotangent(const Geo& g, const double* yb, const double* pb, const double* sg, double* r,
                           hipStream_t st);
void launch_data_grad(const Geo& g, const double* lam, const double* sg, double* dg, double* df,
                      double* dy0, hipStream_t st);

bool time_lds_fits(int n, bool fp32);
// time-pass kernels that launch_precond runs for tb.time_cols: 0 chirp-z,
// -P two LDS buffers, +P in place, with P points per block
int time_choice(const Geo& g, const PrecondTables& tb, bool fp32);
FftPlan make_time_plan(int n, bool fp32);
// lengths with a prime-factor plan (time_pr.hip): the prime PR of the Rader
// transform and the generator g of the group mod PR used by its filter table
bool pr_params(int n, int* pr, int* gen);
bool launch_precond(const Geo& g, const double* v, double* w, void* spec, bool fp32, int spatial,
                    const PrecondTables& tb, const double* vscale, int vs_stride, int accum,
                    hipStream_t st);
// shifted spatial solves on spm complex slices per member, slice q of member
// b shifted by lam_{q/2} + alpha_b (q even) or its conjugate (q odd)
bool launch_mg_solve(const Geo& g, void* spec, bool fp32, const PrecondTables& tb, int spm, const double* lam,
                     hipStream_t st);
bool launch_dst_solve(const Geo& g, void* spec, bool fp32, const PrecondTables& tb, int spm, const double* lam,
                      hipStream_t st);
// ideal RBD preconditioner (sequential in time); unit = device (1.0, 0.0);
// uses ideal_spec_bytes(g, fp32) bytes of spec
bool launch_ideal_precond(const Geo& g, const double* v, double* w, void* spec, bool fp32, int spatial,
                          const PrecondTables& tb, const double* unit, const double* vscale, int vs_stride,
                          int accum, hipStream_t st);
size_t ideal_spec_bytes(const Geo& g, bool fp32);

// post-solve of the end levels (post.hip): buffers of the refinement
struct PostArgs {
  double* rhs;          // [B][2][m] right-hand sides (real, imaginary planes)
  double* z;            // [B][2][m] iterate
  double* part;         // [B][ceil(m/256)] block partial sums
  double* norm2;        // [B] squared residual norms
  const double* ecoef;  // variable-coefficient stencil of E, or null
  double ediag, eoff;   // constant-coefficient stencil of E
};
void launch_post_rhs(const Geo& g, const double* x, const double* fN, const double* g0, const double* y0,
                     const double* sg, const PostArgs& a, hipStream_t st);
// residual into the slice (norm2 = its squared norms), one spatial solve, z += slice
bool launch_post_step(const Geo& g, const PostArgs& a, void* slice, bool fp32, int spatial,
                      const PrecondTables& tb, const double* unit, hipStream_t st);
// residual norms only
void launch_post_residual(const Geo& g, const PostArgs& a, void* slice, hipStream_t st);
void launch_post_store(const Geo& g, const PostArgs& a, double* yN, double* p0, hipStream_t st);
// e_h per member into eh[B]; sq: [B][N][2] scratch
void launch_error_eh(const Geo& g, const double* x, const double* yN, const double* p0, const double* sg,
                     const double* yex, const double* pex, double* sq, double* eh, hipStream_t st);

// Krylov kernels (krylov.hip).  Basis slot i of member b starts at
// basis + i * slot_stride + b * vl.
struct KrylovArgs {
  const double* basis;
  long long slot_stride;  // doubles between consecutive basis slots
  long long vl;           // doubles per member vector
  long long ms;           // doubles between members' vectors
  int B;
  const int* active;      // [B] or null
  int pairs;              // Gram-Schmidt update on double2 pairs (1) or doubles (0)
};
constexpr int kMaxBasis = 41;   // restart <= 40
constexpr int kRedStride = 48;  // doubles per (member, block) partial record

int krylov_blocks(long long vl);
// partial[b][blk][0..nv-1] = <basis_i, w>, partial[b][blk][nv] = <w, w>
void launch_mdot(const KrylovArgs& ka, int nv, const double* w, double* partial, int nblk, hipStream_t st);
// w <- w - sum_i coef[b][i] basis_i; then partial dots of the updated w as in mdot.
// skip[b] != 0 leaves member b untouched (and its partials unwritten).
void launch_update(const KrylovArgs& ka, int nv, double* w, const double* coef, int coef_ld,
                   double* partial, int nblk, const int* skip, hipStream_t st);
// out = (accum ? out : 0) + sum_i coef[b][i] basis_i   (zero coefficients skip their load)
void launch_combine(const KrylovArgs& ka, int nv, const double* coef, int coef_ld, double* out,
                    int accum, hipStream_t st);
// fixed-order sum of partial records: out[b][c] = sum_blk partial[b][blk][c], c < ncols
void launch_reduce_partials(const double* partial, int nblk, int ncols, int B, double* out,
                            hipStream_t st);
// Gram-Schmidt bookkeeping on the device (one thread per member), see krylov.hip
void launch_gs_step1(const double* red, int j, int B, const double* sc, double* H, int H_ld,
                     double* coef, int coef_ld, double* wnorm2, const int* active, hipStream_t st);
void launch_gs_step2(const double* red, int j, int B, const double* sc, double* H, int H_ld,
                     double* coef, int coef_ld, const double* wnorm2, double reorth_tol, int* skip,
                     double* sc_out, const int* active, int final_pass, hipStream_t st);
void launch_pack_hcol(const double* H, int H_ld, int j, int B, const int* skip, double* out, hipStream_t st);
void launch_set_scale(const double* red, int col, int B, double* sc, double* norm, const int* active,
                      hipStream_t st);

}  // namespace pcop
