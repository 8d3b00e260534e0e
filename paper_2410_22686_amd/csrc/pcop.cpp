// Host side of the C ABI declared in include/pcop.h: argument validation,
// workspace layout, FP64 host tables, and the host-side GMRES loop that
// sequences the HIP kernels.  The loop keeps only O(restart^2) scalars per
// member on the host (Givens rotations of the Hessenberg columns it reads
// back).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/pcop.h"
#include "launch.hpp"

using namespace pcop;

// Spectrum scratch of pcop_precond_apply_noalloc: one copy per device, held
// from the library's first use on that device until the process ends.  In
// host code `scratch` is only a stand-in for the symbol: its device address
// is taken per device with hipGetSymbolAddress (in pcop_setup) and only that
// address is ever handed to kernels.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

thread_local std::string g_last_error;

// device -> address of that device's copy of `scratch` (filled once per
// device, with the device current)
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;

hipError_t static_scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_addr[dev] = p;
  *out = p;
  return hipSuccess;
}

pcop_status fail(pcop_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define PCOP_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(PCOP_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

bool is_pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }

// ---------------------------------------------------------------------------
// validation (host only)
// ---------------------------------------------------------------------------
pcop_status validate(const pcop_problem* p, const pcop_options* o) {
  if (!p || !o) return fail(PCOP_ERR_INVALID_ARG, "null problem or options");
  if (p->dim != 2 && p->dim != 3) return fail(PCOP_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (p->nx < 1) return fail(PCOP_ERR_INVALID_ARG, "nx must be >= 1");
  if (p->nt < 2) return fail(PCOP_ERR_INVALID_ARG, "nt must be >= 2");
  if (!(p->T > 0.0) || !std::isfinite(p->T)) return fail(PCOP_ERR_INVALID_ARG, "T must be finite and > 0");
  if (p->batch < 1) return fail(PCOP_ERR_INVALID_ARG, "batch must be >= 1");
  if (!p->gamma) return fail(PCOP_ERR_INVALID_ARG, "gamma is null");
  for (int b = 0; b < p->batch; ++b)
    if (!(p->gamma[b] > 0.0) || !std::isfinite(p->gamma[b]))
      return fail(PCOP_ERR_INVALID_ARG, "gamma must be finite and > 0");
  if (!std::isfinite(p->eps) || p->eps > 1.0)
    return fail(PCOP_ERR_INVALID_ARG, "eps must lie in (0, 1] (or <= 0 for sqrt(tau))");
  // sizes first, in floating point, so that no integer arithmetic below
  // (here, in the workspace layout or in the kernel plans) can overflow
  const double md = std::pow((double)p->nx, p->dim);
  if (p->nx > (1 << 20) || md > (double)((1LL << 31) / 8)) return fail(PCOP_ERR_UNSUPPORTED, "spatial grid too large");
  if (p->nt > (1 << 24) || 2.0 * (p->nt - 1) * md > (double)(1LL << 40))
    return fail(PCOP_ERR_UNSUPPORTED, "problem too large");
  if (p->coeff_kind == PCOP_COEFF_ONE) {
    if (p->coeff) return fail(PCOP_ERR_INVALID_ARG, "coeff must be null for PCOP_COEFF_ONE");
  } else if (p->coeff_kind == PCOP_COEFF_HALFGRID) {
    if (!p->coeff) return fail(PCOP_ERR_INVALID_ARG, "coeff is null");
    const long long hn = (long long)std::pow(2.0 * p->nx + 1.0, p->dim) + 0.5;
    for (long long k = 0; k < hn; ++k)
      if (!(p->coeff[k] > 0.0) || !std::isfinite(p->coeff[k]))
        return fail(PCOP_ERR_INVALID_ARG, "coefficient samples must be finite and > 0");
  } else {
    return fail(PCOP_ERR_INVALID_ARG, "unknown coeff_kind");
  }
  if (p->mass != PCOP_MASS_IDENTITY && p->mass != PCOP_MASS_Q1) return fail(PCOP_ERR_INVALID_ARG, "unknown mass");
  if (p->mass == PCOP_MASS_Q1) {
    if (p->coeff_kind != PCOP_COEFF_ONE)
      return fail(PCOP_ERR_UNSUPPORTED, "finite elements are built for a = 1 (PCOP_COEFF_ONE)");
    if (o->spatial != PCOP_DST) return fail(PCOP_ERR_UNSUPPORTED, "finite elements need PCOP_DST");
    if (o->precond != PCOP_PRECOND_EPS) return fail(PCOP_ERR_UNSUPPORTED, "finite elements need PCOP_PRECOND_EPS");
  }
  if (o->precision != PCOP_FP64 && o->precision != PCOP_MIXED)
    return fail(PCOP_ERR_INVALID_ARG, "unknown precision");
  if (o->spatial != PCOP_DST && o->spatial != PCOP_MG) return fail(PCOP_ERR_INVALID_ARG, "unknown spatial");
  if (o->side != PCOP_RIGHT && o->side != PCOP_LEFT && o->side != PCOP_FLEXIBLE)
    return fail(PCOP_ERR_INVALID_ARG, "unknown side");
  if (o->restart < 1 || o->restart > kMaxBasis - 1) return fail(PCOP_ERR_INVALID_ARG, "restart must be in 1..40");
  if (o->maxit < 1) return fail(PCOP_ERR_INVALID_ARG, "maxit must be >= 1");
  if (!(o->rtol > 0.0) || !std::isfinite(o->rtol)) return fail(PCOP_ERR_INVALID_ARG, "rtol must be > 0");
  if (!std::isfinite(o->reorth_tol)) return fail(PCOP_ERR_INVALID_ARG, "reorth_tol must be finite");
  if (o->graph != 0 && o->graph != 1) return fail(PCOP_ERR_INVALID_ARG, "graph must be 0 or 1");
  if (o->graph && o->graph_chunk < 1) return fail(PCOP_ERR_INVALID_ARG, "graph_chunk must be >= 1");
  {
    const int tc = o->time_cols < 0 ? -o->time_cols : o->time_cols;
    if (tc != 0 && tc != 1 && tc != 4 && tc != 8 && tc != 16 && tc != 32 && tc != 64)
      return fail(PCOP_ERR_INVALID_ARG, "time_cols must be 0, -1, +-4, +-8, +-16, +-32 or +-64");
  }
  if (o->dst_kernel < 0 || o->dst_kernel > 5) return fail(PCOP_ERR_INVALID_ARG, "dst_kernel must be in 0..5");
  if (o->tune != 0 && o->tune != 1) return fail(PCOP_ERR_INVALID_ARG, "tune must be 0 or 1");
  if (o->precond != PCOP_PRECOND_EPS && o->precond != PCOP_PRECOND_IDEAL)
    return fail(PCOP_ERR_INVALID_ARG, "unknown precond");
  if (o->kkt_jchunk < -64 || o->kkt_jchunk > 64) return fail(PCOP_ERR_INVALID_ARG, "kkt_jchunk must be in -64..64");
  if (o->krylov_blocks < 0 || o->krylov_blocks > 4096)
    return fail(PCOP_ERR_INVALID_ARG, "krylov_blocks must be in 0..4096");
  if (o->gs_update < 0 || o->gs_update > 2) return fail(PCOP_ERR_INVALID_ARG, "gs_update must be 0, 1 or 2");
  if (o->mg_smoother < 0 || o->mg_smoother > 2) return fail(PCOP_ERR_INVALID_ARG, "mg_smoother must be 0, 1 or 2");
  if (o->precision == PCOP_MIXED && o->side != PCOP_FLEXIBLE)
    return fail(PCOP_ERR_INVALID_ARG, "the mixed-precision preconditioner needs side = PCOP_FLEXIBLE");
  if (o->spatial == PCOP_DST) {
    if (p->coeff_kind != PCOP_COEFF_ONE)
      return fail(PCOP_ERR_INVALID_ARG, "sine transforms need a constant coefficient (use PCOP_MG)");
    if (!is_pow2(p->nx + 1) || p->nx + 1 < 4 || p->nx + 1 > 512)
      return fail(PCOP_ERR_UNSUPPORTED, "sine transforms need nx + 1 a power of two in 4..512");
  } else {
    if (!is_pow2(p->nx + 1)) return fail(PCOP_ERR_INVALID_ARG, "multigrid needs nx = 2^p - 1");
    int levels = 0;
    for (long long v = p->nx + 1; v > 1; v >>= 1) ++levels;
    if (levels > kMaxMgLevels) return fail(PCOP_ERR_UNSUPPORTED, "multigrid hierarchy deeper than 16 levels");
  }
  const int n = p->nt - 1;
  if (o->precond == PCOP_PRECOND_EPS && !time_lds_fits(n, o->precision == PCOP_MIXED))
    return fail(PCOP_ERR_UNSUPPORTED, "nt too large for the LDS time FFT");
  return PCOP_OK;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
struct Layout {
  size_t total = 0;
  size_t dpow, twn64, twn32, twL64, twL32, mu1, im1, lam, alpha, sg, ecoef, unit, zero, post;
  size_t twM64, twM32, chirp64, chirp32, bhat64, bhat32;
  size_t pr64 = 0, pr32 = 0;
  int M = 1;
  int RC = 0;  // Rader convolution length of a prime-factor plan, or 0
  size_t sc, H, coef, red, partial, wnorm2, norm, skip, active, finish, hcol;
  size_t basis, zbasis, tmp1, tmp2, xpad, spec;
  size_t mgcoef[kMaxMgLevels], mgz[kMaxMgLevels], mgr[kMaxMgLevels];
  int mg_levels = 0;
  int mg_nx[kMaxMgLevels];
  int nblk = 1;      // default blocks per member of the Krylov reductions
  int nblk_max = 1;  // the most the partial-sum buffer holds (tuner candidates)
  long long vl = 0;
  long long vs = 0;  // member stride of the solver's vectors: vl padded to 256 bytes
};

size_t take(Layout& L, size_t bytes) {
  size_t off = (L.total + 255) & ~(size_t)255;
  L.total = off + bytes;
  return off;
}

void plan_layout(const pcop_problem* p, const pcop_options* o, Layout& L) {
  const int d = p->dim, nx = p->nx, n = p->nt - 1, B = p->batch;
  const long long m = (long long)std::llround(std::pow((double)nx, d));
  const int K = n / 2 + 1;
  const int Lf = 2 * (nx + 1);
  const bool fp32 = o->precision == PCOP_MIXED;
  const size_t csz = fp32 ? 8 : 16;
  L.vl = 2LL * n * m;
  L.nblk = krylov_blocks(L.vl);
  L.nblk_max = std::max(std::min(4 * L.nblk, 4096), o->krylov_blocks);
  L.dpow = take(L, sizeof(double) * n);
  L.unit = take(L, 2 * sizeof(double));
  L.zero = take(L, sizeof(double) * B);
  // post-solve partial sums [B][ceil(m/256)], norms [B], e_h level sums [B][n+1][2], e_h [B]
  L.post = take(L, sizeof(double) * ((size_t)B * ((m + 255) / 256) + B + 2 * (size_t)B * (n + 1) + B));
  L.twn64 = take(L, 16 * (size_t)n);
  L.twn32 = take(L, 8 * (size_t)n);
  const FftPlan tp = make_time_plan(n, o->precision == PCOP_MIXED);
  L.M = tp.bluestein ? tp.M : 1;
  L.twM64 = take(L, 16 * (size_t)L.M);
  L.twM32 = take(L, 8 * (size_t)L.M);
  L.chirp64 = take(L, 16 * (size_t)n);
  L.chirp32 = take(L, 8 * (size_t)n);
  L.bhat64 = take(L, 16 * (size_t)L.M);
  L.bhat32 = take(L, 8 * (size_t)L.M);
  {
    int pr = 0, gen = 0;
    L.RC = pr_params(n, &pr, &gen) ? pr - 1 : 0;
    if (L.RC > 0) {
      L.pr64 = take(L, 16 * 2 * (size_t)L.RC);
      L.pr32 = take(L, 8 * 2 * (size_t)L.RC);
    }
  }
  L.twL64 = take(L, 16 * (size_t)Lf);
  L.twL32 = take(L, 8 * (size_t)Lf);
  L.mu1 = take(L, sizeof(double) * nx);
  L.im1 = take(L, sizeof(double) * nx);
  L.lam = take(L, 16 * (size_t)K);
  L.alpha = take(L, sizeof(double) * B);
  L.sg = take(L, sizeof(double) * B);
  L.ecoef = (p->coeff_kind == PCOP_COEFF_HALFGRID) ? take(L, sizeof(double) * (1 + 2 * d) * m) : 0;
  L.sc = take(L, sizeof(double) * B * kMaxBasis);
  L.H = take(L, sizeof(double) * B * (kMaxBasis - 1) * kMaxBasis);
  L.coef = take(L, sizeof(double) * B * kMaxBasis);
  L.red = take(L, sizeof(double) * B * kRedStride);
  L.partial = take(L, sizeof(double) * B * (size_t)L.nblk_max * kRedStride);
  L.wnorm2 = take(L, sizeof(double) * B);
  L.norm = take(L, sizeof(double) * B);
  L.skip = take(L, sizeof(int) * B);
  L.active = take(L, sizeof(int) * B);
  L.finish = take(L, sizeof(int) * B);
  L.hcol = take(L, sizeof(double) * B * (kMaxBasis + 1));
  L.vs = (L.vl + 31) / 32 * 32;
  const size_t vec = sizeof(double) * (size_t)L.vs * B;
  L.basis = take(L, vec * (o->restart + 1));
  L.zbasis = (o->side == PCOP_FLEXIBLE) ? take(L, vec * o->restart) : 0;
  L.tmp1 = take(L, vec);
  L.tmp2 = take(L, vec);
  L.xpad = take(L, vec);  // the iterate x in the padded layout
  {
    // epsilon-circulant spectrum [B][2K][m], or the ideal preconditioner's
    // z[B][2][n][m] plus one slice [B][m] (real/complex of the same precision)
    const size_t t = fp32 ? 4 : 8;
    const size_t ideal = ((t * (size_t)B * 2 * n * m + 255) & ~(size_t)255) + 2 * t * (size_t)B * m;
    L.spec = take(L, std::max<size_t>(csz * (size_t)B * 2 * K * m, o->precond == PCOP_PRECOND_IDEAL ? ideal : 0));
  }
  L.mg_levels = 0;
  if (o->spatial == PCOP_MG) {
    int lnx = nx;
    int l = 0;
    while (true) {
      const long long lm = (long long)std::llround(std::pow((double)lnx, d));
      L.mg_nx[l] = lnx;
      L.mgcoef[l] = take(L, (fp32 ? 4 : 8) * (size_t)(1 + 2 * d) * lm);
      // level 0 needs a residual buffer; coarser levels a correction and a rhs
      L.mgr[l] = take(L, csz * (size_t)B * 2 * K * lm);
      L.mgz[l] = (l > 0) ? take(L, csz * (size_t)B * 2 * K * lm) : 0;
      ++l;
      if (lnx == 1) break;  // validate() bounds the depth by kMaxMgLevels
      lnx = (lnx - 1) / 2;
    }
    L.mg_levels = l;
  }
  L.total = (L.total + 255) & ~(size_t)255;
}

}  // namespace

// ---------------------------------------------------------------------------
// per-kernel event timing
// ---------------------------------------------------------------------------
const char* kFamilyName[KF_COUNT] = {"kkt_apply", "time_fwd", "dst_rows", "dst_ax2", "dst_last_solve",
                                     "time_inv", "mg_smooth", "mg_restrict", "mg_prolong", "mdot",
                                     "gs_update", "combine", "small", "ideal_step"};

struct EventTimer {
  hipStream_t st = nullptr;
  bool enabled = false;
  std::vector<hipEvent_t> ev;   // start/stop pairs
  std::vector<int> fam;
  std::vector<double> bytes;
  size_t used = 0;
  long long launches[KF_COUNT] = {0};
  double ms[KF_COUNT] = {0};
  double tbytes[KF_COUNT] = {0};
  hipError_t err = hipSuccess;

  void flush() {
    if (used == 0) return;
    hipError_t e = hipEventSynchronize(ev[2 * used - 1]);
    if (e != hipSuccess) err = e;
    for (size_t i = 0; i < used; ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]) == hipSuccess) {
        ms[fam[i]] += t;
        launches[fam[i]] += 1;
        tbytes[fam[i]] += bytes[i];
      }
    }
    used = 0;
  }
  void reset() {
    flush();
    for (int f = 0; f < KF_COUNT; ++f) {
      launches[f] = 0;
      ms[f] = 0;
      tbytes[f] = 0;
    }
  }
  ~EventTimer() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  static void on_begin(void* self, int family, double nbytes) {
    EventTimer* t = static_cast<EventTimer*>(self);
    if (!t->enabled) return;
    if (t->used >= 16384) t->flush();
    if (2 * t->used + 2 > t->ev.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        t->enabled = false;
        return;
      }
      t->ev.push_back(a);
      t->ev.push_back(b);
      t->fam.push_back(0);
      t->bytes.push_back(0);
    }
    t->fam[t->used] = family;
    t->bytes[t->used] = nbytes;
    (void)hipEventRecord(t->ev[2 * t->used], t->st);
  }
  static void on_end(void* self) {
    EventTimer* t = static_cast<EventTimer*>(self);
    if (!t->enabled) return;
    (void)hipEventRecord(t->ev[2 * t->used + 1], t->st);
    t->used += 1;
  }
};

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct pcop_ctx_s {
  Geo g{};
  pcop_options opt{};
  int coeff_kind = PCOP_COEFF_ONE;
  int mass = PCOP_MASS_IDENTITY;
  double eps = 0, T = 0;
  std::vector<double> gamma, alpha, sgam;
  hipStream_t st = nullptr;
  char* ws = nullptr;
  Layout L;
  PrecondTables tb{};
  double ediag = 0, eoff = 0;
  const double* ecoef = nullptr;
  bool fp32 = false;
  double tuned_ms = 0;
  int kkt_jchunk = -8;  // matvec kernel: > 0 levels per thread, < 0 LDS tiles of -kkt_jchunk levels
  // per basis size nv: blocks per member of the multi-dot and of the
  // Gram-Schmidt update, and the update kernel (double2 pairs or doubles);
  // the best block count depends on how many vectors a kernel streams
  std::array<int, kMaxBasis> nb_mdot{}, nb_upd{}, pairs_upd{};
  EventTimer timer;
  int device = 0;                  // the device current at pcop_setup
  void* static_scratch = nullptr;  // this device's copy of `scratch`
  KTimer ktimer{&EventTimer::on_begin, &EventTimer::on_end, nullptr};
  // pinned host staging for every scalar transfer of the solver
  double* pin = nullptr;
  double* pin_col = nullptr;    // [B][kMaxBasis]  Hessenberg column
  double* pin_sc = nullptr;     // [B][kMaxBasis]  basis scales
  double* pin_coef = nullptr;   // [B][kMaxBasis]  combination coefficients
  double* pin_red = nullptr;    // [B][kRedStride] reductions
  double* pin_H = nullptr;      // [B][kMaxBasis - 1][kMaxBasis] Hessenberg (graph mode)
  double* pin_norm = nullptr;   // [B]
  int* pin_active = nullptr;    // [B]
  int* pin_finish = nullptr;    // [B]
  // HIP graphs of Arnoldi chunks (graph = 1): captured on a private stream
  hipStream_t gst = nullptr;
  std::vector<std::pair<int, hipGraphExec_t>> graphs;  // key j0 * 64 + count
  ~pcop_ctx_s() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    if (gst) (void)hipStreamDestroy(gst);
    if (pin) (void)hipHostFree(pin);
  }
  const KTimer* kt() const { return timer.enabled ? &ktimer : nullptr; }

  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  double* basis(int slot) const { return at<double>(L.basis) + (size_t)slot * (size_t)g.vs * g.B; }
  double* zbasis(int slot) const { return at<double>(L.zbasis) + (size_t)slot * (size_t)g.vs * g.B; }
  KrylovArgs kargs(const double* base, const int* mask) const {
    return KrylovArgs{base, (long long)g.vs * g.B, g.vl, g.vs, g.B, mask, 0};
  }
  // the geometry of the caller's unpadded vectors
  Geo user_geo() const {
    Geo u = g;
    u.vs = u.vl;
    return u;
  }
};

namespace {

// the configured preconditioner with tables tb (epsilon-circulant or ideal)
bool run_precond(pcop_ctx c, const Geo& g, const PrecondTables& tb, const double* v, double* w,
                 const double* vscale, int vs_stride, int accum, void* spec_override = nullptr) {
  void* spec = spec_override ? spec_override : c->at<void>(c->L.spec);
  if (c->opt.precond == PCOP_PRECOND_IDEAL)
    return launch_ideal_precond(g, v, w, spec, c->fp32, c->opt.spatial, tb, c->at<double>(c->L.unit), vscale,
                                vs_stride, accum, c->st);
  return launch_precond(g, v, w, spec, c->fp32, c->opt.spatial, tb, vscale, vs_stride, accum, c->st);
}

// preconditioner on the solver's padded vectors, or (geo = the caller's
// geometry) on unpadded ones
pcop_status do_precond(pcop_ctx c, const double* v, double* w, const double* vscale, int vs_stride, int accum,
                       const int* mask, int nact, const Geo* geo = nullptr) {
  PrecondTables tb = c->tb;
  tb.active = mask;
  tb.nact = nact;
  tb.timer = c->kt();
  if (!run_precond(c, geo ? *geo : c->g, tb, v, w, vscale, vs_stride, accum))
    return fail(PCOP_ERR_UNSUPPORTED, "preconditioner variant not available for this shape");
  return PCOP_OK;
}

void do_kkt(pcop_ctx c, const double* x, double* y, const double* cvec, const double* xscale, int xs_stride,
            const int* mask, int nact) {
  tbeg(c->kt(), KF_KKT, (cvec ? 24.0 : 16.0) * c->g.vl * nact);
  launch_kkt_apply(c->g, x, y, cvec, c->at<double>(c->L.alpha), xscale, xs_stride, mask, false, c->ecoef,
                   c->ediag, c->eoff, c->kkt_jchunk, c->st);
  tend(c->kt());
}

void do_mdot(pcop_ctx c, const KrylovArgs& ka, int nv, const double* w, int nact) {
  tbeg(c->kt(), KF_MDOT, 8.0 * (nv + 1) * c->g.vl * nact);
  launch_mdot(ka, nv, w, c->at<double>(c->L.partial), c->nb_mdot[nv], c->st);
  tend(c->kt());
}

// the Gram-Schmidt update over nv basis vectors with the kernel and block
// count chosen for that size (partials as launch_update writes them)
void launch_update_nv(pcop_ctx c, const KrylovArgs& ka, int nv, double* w, const int* skip, hipStream_t st) {
  KrylovArgs k2 = ka;
  k2.pairs = c->pairs_upd[nv];
  launch_update(k2, nv, w, c->at<double>(c->L.coef), kMaxBasis, c->at<double>(c->L.partial), c->nb_upd[nv], skip,
                st);
}

void do_update(pcop_ctx c, const KrylovArgs& ka, int nv, double* w, const int* skip, int nact) {
  tbeg(c->kt(), KF_UPDATE, 8.0 * (nv + 2) * c->g.vl * nact);
  launch_update_nv(c, ka, nv, w, skip, c->st);
  tend(c->kt());
}

// squared norms of member vectors (into red[b][0])
void do_norm2(pcop_ctx c, const double* w, const int* mask, int nact) {
  KrylovArgs ka = c->kargs(c->basis(0), mask);
  do_mdot(c, ka, 0, w, nact);
  launch_reduce_partials(c->at<double>(c->L.partial), c->nb_mdot[0], 1, c->g.B, c->at<double>(c->L.red), c->st);
}

// ---------------------------------------------------------------------------
// kernel autotuner: times every candidate pair (time-pass kernels, sine-
// transform kernels) of the preconditioner on the context's stream and keeps
// the fastest.  Candidates compute the same transforms with the same
// arithmetic per element; only blocking and LDS use differ.
// ---------------------------------------------------------------------------
struct TuneResult {
  int time_cols, dst_variant;
  double ms;  // fastest preconditioner apply
  int jchunk;
  std::array<int, kMaxBasis> nb_mdot, nb_upd, pairs_upd;
};
// The choice is cached per device model (architecture and compute-unit
// count) and shape for the process, and, when the environment variable
// PCOP_TUNE_CACHE names a file, in that file: one text line per tuned shape
//   pcop-tune <version> <device> <14 key ints> <time_cols> <dst_variant>
//             <jchunk> <ms> <nb_mdot x 41> <nb_upd x 41> <pairs_upd x 41>
// read once per process before the first tuning and appended after each
// new one, so separate processes (a benchmark and a profiler run) run the
// same kernels.  Lines of another version, malformed lines and entries that
// do not fit the context are ignored (the shape is then tuned afresh).
constexpr int kTuneVersion = 2;  // bump when the meaning of a kernel choice changes
using TuneKey = std::pair<std::string, std::array<int, 14>>;
std::mutex g_tune_mu;
std::map<TuneKey, TuneResult> g_tune_cache;
std::set<std::string> g_tune_files_read;

std::string device_id(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string arch(prop.gcnArchName);
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  return arch + ":" + std::to_string(prop.multiProcessorCount);
}

// caller holds g_tune_mu
void read_tune_file(const std::string& path) {
  if (!g_tune_files_read.insert(path).second) return;
  std::ifstream in(path);
  std::string line;
  while (in && std::getline(in, line)) {
    std::istringstream ss(line);
    std::string tag, dev;
    int ver = 0;
    if (!(ss >> tag >> ver >> dev) || tag != "pcop-tune" || ver != kTuneVersion) continue;
    std::array<int, 14> k{};
    TuneResult r{};
    bool ok = true;
    for (int& v : k) ok = ok && static_cast<bool>(ss >> v);
    ok = ok && static_cast<bool>(ss >> r.time_cols >> r.dst_variant >> r.jchunk >> r.ms);
    for (auto* arr : {&r.nb_mdot, &r.nb_upd, &r.pairs_upd})
      for (int& v : *arr) ok = ok && static_cast<bool>(ss >> v);
    if (ok) g_tune_cache[{dev, k}] = r;  // a later line for the same key wins
  }
}

void append_tune_file(const std::string& path, const TuneKey& key, const TuneResult& r) {
  std::ostringstream ss;
  ss << "pcop-tune " << kTuneVersion << " " << key.first;
  for (int v : key.second) ss << " " << v;
  char ms[32];
  std::snprintf(ms, sizeof(ms), "%.6g", r.ms);
  ss << " " << r.time_cols << " " << r.dst_variant << " " << r.jchunk << " " << ms;
  for (const auto* arr : {&r.nb_mdot, &r.nb_upd, &r.pairs_upd})
    for (int v : *arr) ss << " " << v;
  ss << "\n";
  const std::string text = ss.str();
  // one append of the whole line
  if (FILE* fh = std::fopen(path.c_str(), "a")) {
    (void)std::fwrite(text.data(), 1, text.size(), fh);
    (void)std::fclose(fh);
  }
}

// a cached choice this context can run (the partial-sum buffer holds
// nblk_max blocks per member; a file may hold anything)
bool tune_entry_fits(pcop_ctx c, const TuneResult& r) {
  if (r.dst_variant < 0 || r.dst_variant > 4) return false;
  if (r.jchunk == 0 || r.jchunk < -64 || r.jchunk > 64) return false;
  for (int nv = 0; nv < kMaxBasis; ++nv) {
    if (r.nb_mdot[nv] < 1 || r.nb_mdot[nv] > c->L.nblk_max) return false;
    if (r.nb_upd[nv] < 1 || r.nb_upd[nv] > c->L.nblk_max) return false;
    if (r.pairs_upd[nv] != 0 && r.pairs_upd[nv] != 1) return false;
  }
  if (c->opt.precond == PCOP_PRECOND_EPS) {
    const int tc = r.time_cols < 0 ? -r.time_cols : r.time_cols;
    if (tc != 0 && tc != 1 && tc != 4 && tc != 8 && tc != 16 && tc != 32 && tc != 64) return false;
    PrecondTables t = c->tb;
    t.time_cols = r.time_cols;
    if (time_choice(c->g, t, c->fp32) == 0) return false;
  }
  return true;
}

void apply_tune_result(pcop_ctx c, const TuneResult& r) {
  c->tb.time_cols = r.time_cols;
  c->tb.dst_variant = r.dst_variant;
  c->tuned_ms = r.ms;
  c->kkt_jchunk = r.jchunk;
  c->nb_mdot = r.nb_mdot;
  c->nb_upd = r.nb_upd;
  c->pairs_upd = r.pairs_upd;
}

pcop_status tune_kernels(pcop_ctx c) {
  const Geo& g = c->g;
  int dev = 0;
  PCOP_HIP(hipGetDevice(&dev));
  const TuneKey key{device_id(dev),
                    {g.dim, g.nx, g.n, g.B, (int)c->fp32, c->opt.spatial, c->opt.time_cols, c->opt.dst_kernel,
                     c->coeff_kind + 2 * c->mass, c->opt.precond, c->opt.kkt_jchunk, c->opt.krylov_blocks,
                     c->opt.gs_update, c->opt.restart}};
  const char* env = std::getenv("PCOP_TUNE_CACHE");
  const std::string cache_file = (env && *env) ? env : "";
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!cache_file.empty()) read_tune_file(cache_file);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end() && tune_entry_fits(c, it->second)) {
      apply_tune_result(c, it->second);
      return PCOP_OK;
    }
  }
  std::vector<int> tcs;
  if (c->opt.time_cols != 0 || c->opt.precond == PCOP_PRECOND_IDEAL) {
    tcs.push_back(c->tb.time_cols);
  } else {
    std::vector<int> seen;
    // chirp-z: the automatic choice first, then the prime-factor kernels,
    // the three-stage kernels with 256 and 512 threads and the two-FFT
    // kernels with every width; Stockham: two buffers and in place with 16,
    // 8, 4 points
    const std::vector<int> wants = c->tb.plan.bluestein ? std::vector<int>{0, 64, -64, 32, -32, 16, 8, 4, -16, -8, -4}
                                                        : std::vector<int>{-8, -16, -4, 16, 8, 4, 64, -64};
    for (int want : wants) {
      PrecondTables t = c->tb;
      t.time_cols = want;
      const int eff = time_choice(g, t, c->fp32);
      if (eff == 0) continue;
      // a Stockham request of one kind that falls back to the other
      if (!c->tb.plan.bluestein && (eff < 0) != (want < 0)) continue;
      if (std::find(seen.begin(), seen.end(), eff) != seen.end()) continue;
      seen.push_back(eff);
      tcs.push_back(want);
    }
  }
  std::vector<int> dvs;
  if (c->opt.spatial == PCOP_DST && c->opt.dst_kernel == 0) dvs = {0, 1, 2, 3, 4};
  else dvs = {c->tb.dst_variant};
  double* v = c->basis(0);
  double* w = c->basis(1);
  hipStream_t st = c->st;
  PCOP_HIP(hipMemsetAsync(v, 0, sizeof(double) * (size_t)g.vs * g.B, st));
  hipEvent_t e0, e1;
  PCOP_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(PCOP_ERR_DEVICE, "tuner: event creation failed");
  }
  constexpr int kReps = 5;
  hipError_t err = hipSuccess;
  // fastest of kReps individually timed runs of f, after one warm-up run
  auto time_it = [&](auto&& f, double& ms_out) -> bool {
    f();
    ms_out = 1e300;
    for (int r = 0; r < kReps; ++r) {
      if ((err = hipEventRecord(e0, st)) != hipSuccess) return false;
      f();
      if ((err = hipEventRecord(e1, st)) != hipSuccess) return false;
      if ((err = hipEventSynchronize(e1)) != hipSuccess) return false;
      float ms = 0.f;
      if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return false;
      ms_out = std::min(ms_out, (double)ms);
    }
    return true;
  };
  // a later candidate must beat the current best by 1% (the candidate lists
  // start with the built-in choices), so timing noise does not flip choices
  auto better = [](double ms, double best_ms) { return ms < 0.99 * best_ms; };
  TuneResult best{c->tb.time_cols, c->tb.dst_variant, 1e300, c->kkt_jchunk, c->nb_mdot, c->nb_upd, c->pairs_upd};
  // preconditioner kernels
  for (int tc : tcs) {
    for (int dv : dvs) {
      PrecondTables t = c->tb;
      t.time_cols = tc;
      t.dst_variant = dv;
      t.active = nullptr;
      t.nact = g.B;
      t.timer = nullptr;
      if (!run_precond(c, g, t, v, w, nullptr, 0, 0)) continue;
      double ms = 0;
      if (!time_it([&] { run_precond(c, g, t, v, w, nullptr, 0, 0); }, ms)) break;
      if (better(ms, best.ms)) {
        best.time_cols = tc;
        best.dst_variant = dv;
        best.ms = ms;
      }
    }
    if (err != hipSuccess) break;
  }
  // matvec: time levels per thread
  double best_kkt = 1e300;
  // levels per block of the LDS-tiled kernel (the built-in -8 first), then
  // levels per thread of the one-thread-per-point kernel
  for (int jc : {-8, -16, -32, 16, 1, 2, 4, 8, 32}) {
    if (err != hipSuccess || c->opt.kkt_jchunk != 0) break;
    double ms = 0;
    if (!time_it([&] {
          launch_kkt_apply(g, v, w, nullptr, c->at<double>(c->L.alpha), nullptr, 0, nullptr, false, c->ecoef,
                           c->ediag, c->eoff, jc, st);
        }, ms))
      break;
    if (better(ms, best_kkt)) {
      best_kkt = ms;
      best.jchunk = jc;
    }
  }
  // Krylov reductions: blocks per member for the multi-dot and the update,
  // and the update kernel, timed at sample basis sizes; every size takes the
  // choice of the nearest sample.  A restart cycle runs every size from 1 to
  // the restart length, and the best block count moves with the number of
  // vectors streamed (more blocks hide more latency once the kernels hold
  // many vectors in registers, fewer finish short sweeps sooner).  The
  // samples are dense where the compiled multi-dot changes shape: from 19
  // vectors on it keeps fewer loads in flight per thread, and with 512
  // blocks it was measured at 4.3 TB/s against 6.7 with 1024 (at 18 vectors
  // 512 blocks are the fastest), so 18 and 20 are both sampled.  The
  // vectors are zeroed first, the coefficients and skip flags too.
  std::vector<int> nvs;
  for (int nv : {1, 2, 4, 8, 12, 16, 18, 20, 24, 28, 32, 36, 40})
    if (nv < c->opt.restart) nvs.push_back(nv);
  nvs.push_back(c->opt.restart);
  if (err == hipSuccess)
    err = hipMemsetAsync(c->basis(0), 0, sizeof(double) * (size_t)g.vs * g.B * (nvs.back() + 1), st);
  if (err == hipSuccess) err = hipMemsetAsync(c->at<double>(c->L.coef), 0, sizeof(double) * g.B * kMaxBasis, st);
  if (err == hipSuccess) err = hipMemsetAsync(c->at<int>(c->L.skip), 0, sizeof(int) * g.B, st);
  // half .. four times the default block count (the default first), unless fixed by the caller
  std::vector<int> nbs;
  for (int f : {2, 1, 4, 8}) {
    const int nb = c->opt.krylov_blocks != 0 ? c->nb_mdot[0] : std::max(1, c->L.nblk * f / 2);
    if (nb <= c->L.nblk_max && std::find(nbs.begin(), nbs.end(), nb) == nbs.end()) nbs.push_back(nb);
  }
  std::vector<int> prs;
  for (int pr : {0, 1})
    if (c->opt.gs_update == 0 || pr == c->pairs_upd[0]) prs.push_back(pr);
  std::vector<int> s_mdot(nvs.size(), c->nb_mdot[0]), s_upd(nvs.size(), c->nb_upd[0]),
      s_pairs(nvs.size(), c->pairs_upd[0]);
  KrylovArgs ka = c->kargs(c->basis(0), nullptr);
  double* part = c->at<double>(c->L.partial);
  for (size_t si = 0; si < nvs.size() && err == hipSuccess; ++si) {
    const int nv = nvs[si];
    double* wv = c->basis(nv);
    double best_m = 1e300, best_u = 1e300;
    for (int nb : nbs) {
      double ms = 0;
      if (!time_it([&] { launch_mdot(ka, nv, wv, part, nb, st); }, ms)) break;
      if (better(ms, best_m)) {
        best_m = ms;
        s_mdot[si] = nb;
      }
      for (int pr : prs) {
        KrylovArgs k2 = ka;
        k2.pairs = pr;
        if (!time_it([&] {
              launch_update(k2, nv, wv, c->at<double>(c->L.coef), kMaxBasis, part, nb, c->at<int>(c->L.skip), st);
            }, ms))
          break;
        if (better(ms, best_u)) {
          best_u = ms;
          s_upd[si] = nb;
          s_pairs[si] = pr;
        }
      }
      if (err != hipSuccess) break;
    }
  }
  for (int nv = 0; nv < kMaxBasis; ++nv) {
    size_t k = 0;  // nearest sample (the larger one on a tie)
    for (size_t si = 1; si < nvs.size(); ++si)
      if (std::abs(nvs[si] - nv) <= std::abs(nvs[k] - nv)) k = si;
    best.nb_mdot[nv] = s_mdot[k];
    best.nb_upd[nv] = s_upd[k];
    best.pairs_upd[nv] = s_pairs[k];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err == hipSuccess) err = hipGetLastError();
  if (err != hipSuccess) return fail(PCOP_ERR_DEVICE, std::string("tuner: ") + hipGetErrorString(err));
  if (best.ms >= 1e300) return fail(PCOP_ERR_UNSUPPORTED, "tuner: no preconditioner variant runs for this shape");
  apply_tune_result(c, best);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = best;
  if (!cache_file.empty()) append_tune_file(cache_file, key, best);
  return PCOP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void pcop_default_options(pcop_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = PCOP_FP64;
  o->spatial = PCOP_DST;
  o->side = PCOP_RIGHT;
  o->restart = 30;
  o->maxit = 300;
  o->rtol = 1e-8;
  o->graph = 0;
  o->graph_chunk = 4;
  o->reorth_tol = 1e-8;
  o->stream = nullptr;
}

pcop_status pcop_validate(const pcop_problem* prob, const pcop_options* opts) { return validate(prob, opts); }

pcop_status pcop_workspace_size(const pcop_problem* prob, const pcop_options* opts, size_t* bytes) {
  pcop_status s = validate(prob, opts);
  if (s != PCOP_OK) return s;
  if (!bytes) return fail(PCOP_ERR_INVALID_ARG, "bytes is null");
  Layout L;
  plan_layout(prob, opts, L);
  *bytes = L.total;
  return PCOP_OK;
}

pcop_status pcop_setup(pcop_ctx* out, const pcop_problem* prob, const pcop_options* opts, void* workspace,
                       size_t bytes) {
  if (!out) return fail(PCOP_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  pcop_status s = validate(prob, opts);
  if (s != PCOP_OK) return s;
  Layout L;
  plan_layout(prob, opts, L);
  if (!workspace || bytes < L.total) return fail(PCOP_ERR_WORKSPACE, "workspace too small");
  if (((uintptr_t)workspace & 255) != 0) return fail(PCOP_ERR_WORKSPACE, "workspace must be 256-byte aligned");

  pcop_ctx c = new pcop_ctx_s();
  c->L = L;
  c->opt = *opts;
  c->st = reinterpret_cast<hipStream_t>(opts->stream);
  c->ws = reinterpret_cast<char*>(workspace);
  c->fp32 = opts->precision == PCOP_MIXED;
  c->coeff_kind = prob->coeff_kind;
  c->mass = prob->mass;
  const int d = prob->dim, nx = prob->nx, n = prob->nt - 1, B = prob->batch;
  const long long m = (long long)std::llround(std::pow((double)nx, d));
  Geo& g = c->g;
  g.dim = d;
  g.nx = nx;
  g.n = n;
  g.m = (int)m;
  g.B = B;
  g.K = n / 2 + 1;
  g.vl = L.vl;
  g.vs = L.vs;
  c->T = prob->T;
  g.tau = prob->T / prob->nt;
  const double h = 1.0 / (nx + 1);
  g.h2inv = 1.0 / (h * h);
  g.fem = prob->mass == PCOP_MASS_Q1 ? 1 : 0;
  c->eps = prob->eps > 0.0 ? prob->eps : std::sqrt(g.tau);
  c->gamma.assign(prob->gamma, prob->gamma + B);
  c->alpha.resize(B);
  c->sgam.resize(B);
  for (int b = 0; b < B; ++b) {
    c->sgam[b] = std::sqrt(c->gamma[b]);
    c->alpha[b] = g.tau / c->sgam[b];
  }

  // host tables in long double, rounded once
  const long double PI = 3.141592653589793238462643383279502884L;
  std::vector<double> dpow(n), twn64(2 * n), mu1(nx), im1(nx, 1.0), lam(2 * g.K), twL64(2 * (2 * (nx + 1)));
  std::vector<float> twn32(2 * n), twL32(2 * (2 * (nx + 1)));
  const long double le = std::log((long double)c->eps);
  for (int j = 0; j < n; ++j) dpow[j] = (double)std::exp(le * j / n);
  for (int t = 0; t < n; ++t) {
    long double a = -2.0L * PI * t / n;
    twn64[2 * t] = (double)std::cos(a);
    twn64[2 * t + 1] = (double)std::sin(a);
    twn32[2 * t] = (float)std::cos(a);
    twn32[2 * t + 1] = (float)std::sin(a);
  }
  // Bluestein tables: chirp w_t = exp(-i pi (t^2 mod 2n)/n), filter
  // bb[m] = conj(w_m) for |m| < n wrapped cyclically into length M, bhat = FFT_M(bb)
  const int M = L.M;
  std::vector<double> twM64(2 * M), chirp64(2 * n), bhat64(2 * M);
  std::vector<float> twM32(2 * M), chirp32(2 * n), bhat32(2 * M);
  {
    std::vector<long double> cM(M), sM(M);
    for (int t = 0; t < M; ++t) {
      long double a = -2.0L * PI * t / M;
      cM[t] = std::cos(a);
      sM[t] = std::sin(a);
      twM64[2 * t] = (double)cM[t];
      twM64[2 * t + 1] = (double)sM[t];
      twM32[2 * t] = (float)cM[t];
      twM32[2 * t + 1] = (float)sM[t];
    }
    std::vector<long double> cw(n), sw(n);
    for (int t = 0; t < n; ++t) {
      const long long q = ((long long)t * t) % (2LL * n);
      long double a = -PI * (long double)q / n;
      cw[t] = std::cos(a);
      sw[t] = std::sin(a);
      chirp64[2 * t] = (double)cw[t];
      chirp64[2 * t + 1] = (double)sw[t];
      chirp32[2 * t] = (float)cw[t];
      chirp32[2 * t + 1] = (float)sw[t];
    }
    if (M > 1) {
      std::vector<long double> br(M, 0.0L), bi(M, 0.0L);
      for (int t = 0; t < n; ++t) {
        br[t] = cw[t];
        bi[t] = -sw[t];
        if (t > 0) {
          br[M - t] = cw[t];
          bi[M - t] = -sw[t];
        }
      }
      for (int k = 0; k < M; ++k) {
        long double re = 0.0L, im = 0.0L;
        for (int t = 0; t < M; ++t) {
          const int e = (int)(((long long)k * t) % M);
          re += br[t] * cM[e] - bi[t] * sM[e];
          im += br[t] * sM[e] + bi[t] * cM[e];
        }
        bhat64[2 * k] = (double)re;
        bhat64[2 * k + 1] = (double)im;
        bhat32[2 * k] = (float)re;
        bhat32[2 * k + 1] = (float)im;
      }
    }
  }
  // prime-factor plans: W_RC^t and the Rader filter B[k] = DFT_RC(b)[k] / RC,
  // b_m = exp(-2 pi i (g^m mod PR)/PR)
  const int RC = L.RC;
  std::vector<double> pr64(4 * (size_t)RC);
  std::vector<float> pr32(4 * (size_t)RC);
  if (RC > 0) {
    int pr = 0, gen = 0;
    (void)pr_params(n, &pr, &gen);
    std::vector<long double> cR(RC), sR(RC), br(RC), bi(RC);
    for (int t = 0; t < RC; ++t) {
      const long double a = -2.0L * PI * t / RC;
      cR[t] = std::cos(a);
      sR[t] = std::sin(a);
    }
    long long gm = 1;
    for (int t = 0; t < RC; ++t) {
      const long double a = -2.0L * PI * (long double)gm / pr;
      br[t] = std::cos(a);
      bi[t] = std::sin(a);
      gm = gm * gen % pr;
    }
    for (int k = 0; k < RC; ++k) {
      long double re = 0.0L, im = 0.0L;
      for (int t = 0; t < RC; ++t) {
        const int e = (int)(((long long)k * t) % RC);
        re += br[t] * cR[e] - bi[t] * sR[e];
        im += br[t] * sR[e] + bi[t] * cR[e];
      }
      re /= RC;
      im /= RC;
      pr64[2 * k] = (double)cR[k];
      pr64[2 * k + 1] = (double)sR[k];
      pr64[2 * (RC + k)] = (double)re;
      pr64[2 * (RC + k) + 1] = (double)im;
      pr32[2 * k] = (float)cR[k];
      pr32[2 * k + 1] = (float)sR[k];
      pr32[2 * (RC + k)] = (float)re;
      pr32[2 * (RC + k) + 1] = (float)im;
    }
  }
  const int Lf = 2 * (nx + 1);
  for (int t = 0; t < Lf; ++t) {
    long double a = -2.0L * PI * t / Lf;
    twL64[2 * t] = (double)std::cos(a);
    twL64[2 * t + 1] = (double)std::sin(a);
    twL32[2 * t] = (float)std::cos(a);
    twL32[2 * t + 1] = (float)std::sin(a);
  }
  for (int k = 1; k <= nx; ++k) {
    long double sv = std::sin(PI * k * (long double)h / 2.0L);
    if (g.fem) {
      // Q1 elements: sine-mode eigenvalues m_k = (h/3)(2 + cos(pi k h)) of
      // M1 and k_k = (4/h) sin^2(pi k h/2) of K1; the divide uses k_k/m_k and 1/m_k
      const long double mk = (long double)h / 3.0L * (2.0L + std::cos(PI * k * (long double)h));
      const long double kk = 4.0L / (long double)h * sv * sv;
      mu1[k - 1] = (double)(kk / mk);
      im1[k - 1] = (double)(1.0L / mk);
    } else {
      mu1[k - 1] = (double)(4.0L / ((long double)h * h) * sv * sv);
    }
  }
  const long double e1n = std::exp(le / n);
  for (int k = 0; k < g.K; ++k) {
    long double a = -2.0L * PI * k / n;  // theta^{-k}
    lam[2 * k] = (double)(1.0L - e1n * std::cos(a));
    lam[2 * k + 1] = (double)(-e1n * std::sin(a));
  }
  hipStream_t st = c->st;
  auto up = [&](size_t off, const void* src, size_t nb) -> hipError_t {
    return hipMemcpyAsync(c->ws + off, src, nb, hipMemcpyHostToDevice, st);
  };
  hipError_t e = hipSuccess;
  std::vector<int> ones(B, 1);
  if (e == hipSuccess) e = up(L.dpow, dpow.data(), sizeof(double) * n);
  if (e == hipSuccess) e = up(L.twn64, twn64.data(), sizeof(double) * 2 * n);
  if (e == hipSuccess) e = up(L.twn32, twn32.data(), sizeof(float) * 2 * n);
  if (e == hipSuccess) e = up(L.twM64, twM64.data(), sizeof(double) * 2 * M);
  if (e == hipSuccess) e = up(L.twM32, twM32.data(), sizeof(float) * 2 * M);
  if (e == hipSuccess) e = up(L.chirp64, chirp64.data(), sizeof(double) * 2 * n);
  if (e == hipSuccess) e = up(L.chirp32, chirp32.data(), sizeof(float) * 2 * n);
  if (e == hipSuccess) e = up(L.bhat64, bhat64.data(), sizeof(double) * 2 * M);
  if (e == hipSuccess) e = up(L.bhat32, bhat32.data(), sizeof(float) * 2 * M);
  if (e == hipSuccess && RC > 0) e = up(L.pr64, pr64.data(), sizeof(double) * 4 * RC);
  if (e == hipSuccess && RC > 0) e = up(L.pr32, pr32.data(), sizeof(float) * 4 * RC);
  if (e == hipSuccess) e = up(L.twL64, twL64.data(), sizeof(double) * 2 * Lf);
  if (e == hipSuccess) e = up(L.twL32, twL32.data(), sizeof(float) * 2 * Lf);
  if (e == hipSuccess) e = up(L.mu1, mu1.data(), sizeof(double) * nx);
  if (e == hipSuccess) e = up(L.im1, im1.data(), sizeof(double) * nx);
  if (e == hipSuccess) e = up(L.lam, lam.data(), sizeof(double) * 2 * g.K);
  if (e == hipSuccess) e = up(L.alpha, c->alpha.data(), sizeof(double) * B);
  if (e == hipSuccess) e = up(L.sg, c->sgam.data(), sizeof(double) * B);
  if (e == hipSuccess) e = up(L.active, ones.data(), sizeof(int) * B);
  static const double kUnit[2] = {1.0, 0.0};
  if (e == hipSuccess) e = up(L.unit, kUnit, sizeof(kUnit));
  std::vector<double> zeros(B, 0.0);
  if (e == hipSuccess) e = up(L.zero, zeros.data(), sizeof(double) * B);

  // stencil E = I + tau K
  std::vector<double> ecoef;
  std::vector<std::vector<double>> mgc64;
  std::vector<std::vector<float>> mgc32;
  const double tau = g.tau;
  if (prob->coeff_kind == PCOP_COEFF_ONE) {
    c->ediag = 1.0 + tau * 2.0 * d * g.h2inv;
    c->eoff = -tau * g.h2inv;
  }
  // coefficient on level l at half-grid offsets; the fine half grid has
  // 2nx+1 points per dimension, node c (0-based) of level l sits at half index
  // (c+1) 2^{l+1} - 1 and its faces at +/- 2^l
  const int hn = 2 * nx + 1;
  auto a_at = [&](const int* hk) -> double {
    long long idx = 0, stride = 1;
    for (int ax = 0; ax < d; ++ax) {
      idx += (long long)hk[ax] * stride;
      stride *= hn;
    }
    return prob->coeff[idx];
  };
  auto build_stencil = [&](int level, int lnx, double scale_diag_one, std::vector<double>& outc) {
    const long long lm = (long long)std::llround(std::pow((double)lnx, d));
    const double hl = 1.0 / (lnx + 1);
    const double s = tau / (hl * hl);
    outc.assign((size_t)(1 + 2 * d) * lm, 0.0);
    const int step = 1 << (level + 1), half = 1 << level;
    for (long long i = 0; i < lm; ++i) {
      int cc[3] = {0, 0, 0};
      long long r = i;
      for (int ax = 0; ax < d; ++ax) {
        cc[ax] = (int)(r % lnx);
        r /= lnx;
      }
      int hk[3];
      for (int ax = 0; ax < d; ++ax) hk[ax] = (cc[ax] + 1) * step - 1;
      double diag = 0.0;
      for (int ax = 0; ax < d; ++ax) {
        int hm[3] = {hk[0], hk[1], hk[2]}, hp[3] = {hk[0], hk[1], hk[2]};
        hm[ax] -= half;
        hp[ax] += half;
        const double am = a_at(hm), ap = a_at(hp);
        diag += am + ap;
        if (cc[ax] > 0) outc[(size_t)(1 + 2 * ax) * lm + i] = -s * am;
        if (cc[ax] < lnx - 1) outc[(size_t)(2 + 2 * ax) * lm + i] = -s * ap;
      }
      outc[i] = scale_diag_one + s * diag;
    }
  };
  if (prob->coeff_kind == PCOP_COEFF_HALFGRID) {
    build_stencil(0, nx, 1.0, ecoef);
    if (e == hipSuccess) e = up(L.ecoef, ecoef.data(), sizeof(double) * ecoef.size());
    c->ecoef = c->at<double>(L.ecoef);
  }
  // multigrid tables: tau K_a on every level (sigma is added per slice)
  if (opts->spatial == PCOP_MG) {
    const double* use = (prob->coeff_kind == PCOP_COEFF_ONE) ? nullptr : prob->coeff;
    mgc64.resize(L.mg_levels);
    mgc32.resize(L.mg_levels);
    for (int l = 0; l < L.mg_levels; ++l) {
      const int lnx = L.mg_nx[l];
      if (use) {
        build_stencil(l, lnx, 0.0, mgc64[l]);
      } else {
        // constant coefficient on this level
        const long long lm = (long long)std::llround(std::pow((double)lnx, d));
        const double hl = 1.0 / (lnx + 1);
        const double s = tau / (hl * hl);
        mgc64[l].assign((size_t)(1 + 2 * d) * lm, 0.0);
        for (long long i = 0; i < lm; ++i) {
          long long r = i;
          mgc64[l][i] = s * 2.0 * d;
          for (int ax = 0; ax < d; ++ax) {
            const int cc = (int)(r % lnx);
            r /= lnx;
            if (cc > 0) mgc64[l][(size_t)(1 + 2 * ax) * lm + i] = -s;
            if (cc < lnx - 1) mgc64[l][(size_t)(2 + 2 * ax) * lm + i] = -s;
          }
        }
      }
      mgc32[l].assign(mgc64[l].begin(), mgc64[l].end());
      if (e == hipSuccess) {
        if (c->fp32)
          e = up(L.mgcoef[l], mgc32[l].data(), sizeof(float) * mgc32[l].size());
        else
          e = up(L.mgcoef[l], mgc64[l].data(), sizeof(double) * mgc64[l].size());
      }
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    delete c;
    return fail(PCOP_ERR_DEVICE, std::string("setup upload: ") + hipGetErrorString(e));
  }

  {
    const size_t nd = (size_t)B * (3 * kMaxBasis + 1 + kRedStride + 1 + (kMaxBasis - 1) * kMaxBasis) +
                      2 * (size_t)B + 8;
    hipError_t pe = hipHostMalloc(reinterpret_cast<void**>(&c->pin), nd * sizeof(double), hipHostMallocDefault);
    if (pe != hipSuccess) {
      delete c;
      return fail(PCOP_ERR_DEVICE, std::string("pinned staging: ") + hipGetErrorString(pe));
    }
    double* q = c->pin;
    c->pin_col = q;
    q += (size_t)B * (kMaxBasis + 1);
    c->pin_sc = q;
    q += (size_t)B * kMaxBasis;
    c->pin_coef = q;
    q += (size_t)B * kMaxBasis;
    c->pin_red = q;
    q += (size_t)B * kRedStride;
    c->pin_H = q;
    q += (size_t)B * (kMaxBasis - 1) * kMaxBasis;
    c->pin_norm = q;
    q += B;
    c->pin_active = reinterpret_cast<int*>(q);
    q += B;
    c->pin_finish = reinterpret_cast<int*>(q);
  }
  PrecondTables& tb = c->tb;
  tb.dpow = c->at<double>(L.dpow);
  tb.twn64 = c->at<double>(L.twn64);
  tb.twn32 = c->at<float>(L.twn32);
  tb.twL64 = c->at<double>(L.twL64);
  tb.twL32 = c->at<float>(L.twL32);
  tb.mu1 = c->at<double>(L.mu1);
  tb.im1 = g.fem ? c->at<double>(L.im1) : nullptr;
  tb.lam = c->at<double>(L.lam);
  tb.alpha = c->at<double>(L.alpha);
  tb.active = nullptr;
  tb.plan = make_time_plan(n, opts->precision == PCOP_MIXED);
  tb.twM64 = c->at<double>(L.twM64);
  tb.twM32 = c->at<float>(L.twM32);
  tb.chirp64 = c->at<double>(L.chirp64);
  tb.chirp32 = c->at<float>(L.chirp32);
  tb.bhat64 = c->at<double>(L.bhat64);
  tb.bhat32 = c->at<float>(L.bhat32);
  tb.pr64 = L.RC > 0 ? c->at<double>(L.pr64) : nullptr;
  tb.pr32 = L.RC > 0 ? c->at<float>(L.pr32) : nullptr;
  tb.time_cols = opts->time_cols;
  tb.mg_smoother = opts->mg_smoother;
  tb.dst_variant = (opts->dst_kernel >= 2) ? opts->dst_kernel - 1 : 0;
  c->nb_mdot.fill(opts->krylov_blocks > 0 ? opts->krylov_blocks : L.nblk);
  c->nb_upd = c->nb_mdot;
  c->kkt_jchunk = opts->kkt_jchunk != 0 ? opts->kkt_jchunk : -8;
  c->pairs_upd.fill(opts->gs_update == 2 ? 1 : 0);
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) {
      delete c;
      return fail(PCOP_ERR_DEVICE, "cannot query the number of compute units");
    }
    tb.ncu = ncu;
    c->device = dev;
    const hipError_t se = static_scratch_address(dev, &c->static_scratch);
    if (se != hipSuccess) {
      delete c;
      return fail(PCOP_ERR_DEVICE, std::string("static scratch address: ") + hipGetErrorString(se));
    }
  }
  tb.mg_levels = L.mg_levels;
  for (int l = 0; l < L.mg_levels; ++l) {
    MgLevel& lv = tb.mg[l];
    lv.nx = L.mg_nx[l];
    lv.m = (long long)std::llround(std::pow((double)lv.nx, d));
    const double hl = 1.0 / (lv.nx + 1);
    lv.h2inv = 1.0 / (hl * hl);
    lv.coef = c->fp32 ? c->at<float>(L.mgcoef[l]) : nullptr;
    lv.coef64 = c->fp32 ? nullptr : c->at<double>(L.mgcoef[l]);
    lv.r = c->at<void>(L.mgr[l]);
    lv.z = (l > 0) ? c->at<void>(L.mgz[l]) : nullptr;
  }
  if (opts->tune) {
    pcop_status ts = tune_kernels(c);
    if (ts != PCOP_OK) {
      delete c;
      return ts;
    }
  }
  if (opts->graph) {
    hipError_t ge = hipStreamCreateWithFlags(&c->gst, hipStreamNonBlocking);
    if (ge != hipSuccess) {
      delete c;
      return fail(PCOP_ERR_DEVICE, std::string("graph stream: ") + hipGetErrorString(ge));
    }
  }
  *out = c;
  return PCOP_OK;
}

void pcop_destroy(pcop_ctx c) { delete c; }

pcop_status pcop_get_params(pcop_ctx c, double* tau, double* alpha, double* eps) {
  if (!c) return fail(PCOP_ERR_INVALID_ARG, "null context");
  if (tau) *tau = c->g.tau;
  if (alpha)
    for (int b = 0; b < c->g.B; ++b) alpha[b] = c->alpha[b];
  if (eps) *eps = c->eps;
  return PCOP_OK;
}

pcop_status pcop_get_kernels(pcop_ctx c, pcop_kernel_choice* out) {
  if (!c || !out) return fail(PCOP_ERR_INVALID_ARG, "null argument");
  out->time_cols = (c->opt.precond == PCOP_PRECOND_EPS) ? time_choice(c->g, c->tb, c->fp32) : 0;
  out->dst_kernel = (c->opt.spatial == PCOP_DST) ? c->tb.dst_variant + 1 : 0;
  out->kkt_jchunk = c->kkt_jchunk;
  out->krylov_blocks = c->nb_mdot[c->opt.restart];
  out->gs_update = c->pairs_upd[c->opt.restart] ? 2 : 1;
  out->tuned_precond_ms = c->tuned_ms;
  return PCOP_OK;
}

pcop_status pcop_post_solve(pcop_ctx c, const double* x, const double* fN, const double* g0, const double* y0,
                            double* yN, double* p0, double* relres) {
  if (!c || !x || !fN || !g0 || !y0 || !yN || !p0) return fail(PCOP_ERR_INVALID_ARG, "null argument");
  const Geo& g = c->g;
  const int B = g.B;
  hipStream_t st = c->st;
  double* post = c->at<double>(c->L.post);
  PostArgs a{c->at<double>(c->L.tmp1), c->at<double>(c->L.tmp2), post, post + (size_t)B * ((g.m + 255) / 256),
             c->ecoef, c->ediag, c->eoff};
  void* slice = c->at<void>(c->L.spec);
  PrecondTables tb = c->tb;
  tb.alpha = c->at<double>(c->L.zero);  // shift 1: E = I + tau K
  tb.active = nullptr;
  tb.nact = B;
  tb.timer = nullptr;
  const double* unit = c->at<double>(c->L.unit);
  if (g.fem) {
    // Q1 elements: the right-hand sides without M into the (still unused)
    // correction slice, then M on both planes of every member
    PostArgs a0 = a;
    a0.rhs = c->at<double>(c->L.spec);
    launch_post_rhs(c->user_geo(), x, fN, g0, y0, c->at<double>(c->L.sg), a0, st);
    launch_mass_apply(g, a0.rhs, 0, a.rhs, 0, 2 * B, 1, st);
  } else {
    launch_post_rhs(c->user_geo(), x, fN, g0, y0, c->at<double>(c->L.sg), a, st);
  }
  PCOP_HIP(hipGetLastError());
  auto read_norms = [&](std::vector<double>& out) -> hipError_t {
    hipError_t e = hipMemcpyAsync(c->pin_norm, a.norm2, sizeof(double) * B, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    for (int b = 0; b < B; ++b) out[b] = std::sqrt(c->pin_norm[b]);
    return e;
  };
  // refinement: sine transforms solve E exactly (a second step removes the
  // last rounding); the V-cycle contracts the error by a constant factor
  const int max_steps = (c->opt.spatial == PCOP_DST) ? 3 : 200;
  std::vector<double> r0(B), r(B), prev(B, 1e300);
  for (int it = 0; it < max_steps; ++it) {
    if (!launch_post_step(g, a, slice, c->fp32, c->opt.spatial, tb, unit, st))
      return fail(PCOP_ERR_UNSUPPORTED, "post-solve: spatial solver not available for this shape");
    PCOP_HIP(hipGetLastError());
    PCOP_HIP(read_norms(it == 0 ? r0 : r));
    if (it == 0) continue;
    // stop at 1e-14 of the initial residual, or once it stalls at rounding level
    bool done = true;
    for (int b = 0; b < B; ++b)
      if (r[b] > 1e-14 * r0[b] && r[b] < 0.9 * prev[b]) done = false;
    prev = r;
    if (done) break;
  }
  launch_post_residual(g, a, slice, st);
  PCOP_HIP(hipGetLastError());
  PCOP_HIP(read_norms(r));
  launch_post_store(g, a, yN, p0, st);
  PCOP_HIP(hipGetLastError());
  double worst = 0.0;
  for (int b = 0; b < B; ++b) {
    const double rel = r0[b] > 0 ? r[b] / r0[b] : 0.0;
    if (relres) relres[b] = rel;
    worst = std::max(worst, rel);
  }
  if (worst > 1e-10) return fail(PCOP_NOT_CONVERGED, "post-solve residual above 1e-10");
  return PCOP_OK;
}

pcop_status pcop_error_eh(pcop_ctx c, const double* x, const double* yN, const double* p0, const double* y_exact,
                          const double* p_exact, double* eh) {
  if (!c || !x || !yN || !p0 || !y_exact || !p_exact || !eh) return fail(PCOP_ERR_INVALID_ARG, "null argument");
  const Geo& g = c->g;
  const int B = g.B;
  hipStream_t st = c->st;
  double* post = c->at<double>(c->L.post);
  double* sq = post + (size_t)B * ((g.m + 255) / 256) + B;
  double* dev_eh = sq + 2 * (size_t)B * (g.n + 1);
  launch_error_eh(c->user_geo(), x, yN, p0, c->at<double>(c->L.sg), y_exact, p_exact, sq, dev_eh, st);
  PCOP_HIP(hipGetLastError());
  PCOP_HIP(hipMemcpyAsync(c->pin_norm, dev_eh, sizeof(double) * B, hipMemcpyDeviceToHost, st));
  PCOP_HIP(hipStreamSynchronize(st));
  for (int b = 0; b < B; ++b) eh[b] = c->pin_norm[b];
  return PCOP_OK;
}

pcop_status pcop_rhs(pcop_ctx c, const double* g, const double* f, const double* y0, double* b) {
  if (!c || !g || !f || !y0 || !b) return fail(PCOP_ERR_INVALID_ARG, "null argument");
  if (c->g.fem) {
    // b = (I (x) M) b_fd: the finite-difference right-hand side into scratch,
    // then the mass matrix on every spatial slice
    const Geo gu = c->user_geo();
    double* t = c->at<double>(c->L.tmp1);
    launch_rhs(gu, g, f, y0, c->at<double>(c->L.sg), t, c->st);
    launch_mass_apply(gu, t, 0, b, 0, 2 * gu.n * gu.B, 1, c->st);
    PCOP_HIP(hipGetLastError());
    return PCOP_OK;
  }
  launch_rhs(c->user_geo(), g, f, y0, c->at<double>(c->L.sg), b, c->st);
  PCOP_HIP(hipGetLastError());
  return PCOP_OK;
}

pcop_status pcop_kkt_apply(pcop_ctx c, const double* x, double* y, int transpose) {
  if (!c || !x || !y) return fail(PCOP_ERR_INVALID_ARG, "null argument");
  if (x == y) return fail(PCOP_ERR_INVALID_ARG, "x and y must not overlap");
  tbeg(c->kt(), KF_KKT, 16.0 * c->g.vl * c->g.B);
  launch_kkt_apply(c->user_geo(), x, y, nullptr, c->at<double>(c->L.alpha), nullptr, 0, nullptr, transpose != 0,
                   c->ecoef, c->ediag, c->eoff, c->kkt_jchunk, c->st);
  tend(c->kt());
  PCOP_HIP(hipGetLastError());
  return PCOP_OK;
}

pcop_status pcop_precond_apply(pcop_ctx c, const double* v, double* w) {
  if (!c || !v || !w) return fail(PCOP_ERR_INVALID_ARG, "null argument");
  const Geo gu = c->user_geo();
  pcop_status s = do_precond(c, v, w, nullptr, 0, 0, nullptr, c->g.B, &gu);
  if (s != PCOP_OK) return s;
  PCOP_HIP(hipGetLastError());
  return PCOP_OK;
}

pcop_status pcop_precond_apply_noalloc(pcop_ctx c, const double* v, double* w) {
  if (!c || !v || !w) return fail(PCOP_ERR_INVALID_ARG, "null argument");
  if (c->opt.precond != PCOP_PRECOND_EPS || c->opt.spatial != PCOP_DST)
    return fail(PCOP_ERR_UNSUPPORTED,
                "pcop_precond_apply_noalloc needs the epsilon-circulant preconditioner with sine transforms");
  const Geo gu = c->user_geo();
  const size_t need = (c->fp32 ? 8 : 16) * (size_t)gu.B * 2 * gu.K * (size_t)gu.m;
  if (need > kStaticScratchBytes)
    return fail(PCOP_ERR_UNSUPPORTED, "pcop_precond_apply_noalloc: the spectrum needs " + std::to_string(need) +
                                          " bytes, more than the " + std::to_string(kStaticScratchBytes) +
                                          "-byte static scratch");
  if (!c->static_scratch) return fail(PCOP_ERR_DEVICE, "static scratch address unavailable");
  int dev = 0;
  PCOP_HIP(hipGetDevice(&dev));
  if (dev != c->device) return fail(PCOP_ERR_INVALID_ARG, "the current device is not the context's device");
  // the forward time pass writes every spectrum value before any is read,
  // so the scratch needs no clearing; no per-kernel timing (its events
  // would be created on demand)
  PrecondTables tb = c->tb;
  tb.active = nullptr;
  tb.nact = gu.B;
  tb.timer = nullptr;
  if (!run_precond(c, gu, tb, v, w, nullptr, 0, 0, c->static_scratch))
    return fail(PCOP_ERR_UNSUPPORTED, "preconditioner variant not available for this shape");
  PCOP_HIP(hipGetLastError());
  return PCOP_OK;
}

pcop_status pcop_unpack(pcop_ctx c, const double* x, double* y, double* p) {
  if (!c || !x || !y || !p) return fail(PCOP_ERR_INVALID_ARG, "null argument");
  launch_unpack(c->user_geo(), x, c->at<double>(c->L.sg), y, p, c->st);
  PCOP_HIP(hipGetLastError());
  return PCOP_OK;
}

pcop_status pcop_pack_cotangent(pcop_ctx c, const double* ybar, const double* pbar, double* r) {
  if (!c || !r) return fail(PCOP_ERR_INVALID_ARG, "null argument");
  launch_pack_cotangent(c->user_geo(), ybar, pbar, c->at<double>(c->L.sg), r, c->st);
  PCOP_HIP(hipGetLastError());
  return PCOP_OK;
}

pcop_status pcop_data_grad(pcop_ctx c, const double* lam, double* dg, double* df, double* dy0) {
  if (!c || !lam) return fail(PCOP_ERR_INVALID_ARG, "null argument");
  if (c->g.fem) {
    // the finite-difference maps into scratch, then M on every slice
    // (b depends on the data through I (x) M, and M is symmetric)
    const Geo gu = c->user_geo();
    const long long nm = (long long)gu.n * gu.m * gu.B;
    double* t1 = c->at<double>(c->L.tmp1);
    double* t2 = c->at<double>(c->L.tmp2);
    launch_data_grad(gu, lam, c->at<double>(c->L.sg), dg ? t1 : nullptr, df ? t1 + nm : nullptr, dy0 ? t2 : nullptr,
                     c->st);
    if (dg) launch_mass_apply(gu, t1, 0, dg, 0, gu.n * gu.B, 1, c->st);
    if (df) launch_mass_apply(gu, t1 + nm, 0, df, 0, gu.n * gu.B, 1, c->st);
    if (dy0) launch_mass_apply(gu, t2, 0, dy0, 0, gu.B, 1, c->st);
    PCOP_HIP(hipGetLastError());
    return PCOP_OK;
  }
  launch_data_grad(c->user_geo(), lam, c->at<double>(c->L.sg), dg, df, dy0, c->st);
  PCOP_HIP(hipGetLastError());
  return PCOP_OK;
}

const char* pcop_status_string(pcop_status s) {
  // a C caller may pass any int: read the bits as one, not as the enum
  int v = 0;
  std::memcpy(&v, &s, sizeof(v));
  switch (v) {
    case PCOP_OK: return "ok";
    case PCOP_ERR_INVALID_ARG: return "invalid argument";
    case PCOP_ERR_UNSUPPORTED: return "unsupported";
    case PCOP_ERR_WORKSPACE: return "workspace";
    case PCOP_ERR_DEVICE: return "device error";
    case PCOP_NOT_CONVERGED: return "not converged";
  }
  return "unknown status";
}

const char* pcop_last_error(void) { return g_last_error.c_str(); }

pcop_status pcop_timing_enable(pcop_ctx c, int enable) {
  if (!c) return fail(PCOP_ERR_INVALID_ARG, "null context");
  c->timer.st = c->st;
  c->ktimer.self = &c->timer;
  c->timer.reset();
  c->timer.enabled = enable != 0;
  if (c->timer.err != hipSuccess) return fail(PCOP_ERR_DEVICE, hipGetErrorString(c->timer.err));
  return PCOP_OK;
}

pcop_status pcop_timing_read(pcop_ctx c, pcop_kernel_stat* out, int cap, int* count, int reset) {
  if (!c || (!out && cap > 0)) return fail(PCOP_ERR_INVALID_ARG, "null argument");
  c->timer.flush();
  if (c->timer.err != hipSuccess) return fail(PCOP_ERR_DEVICE, hipGetErrorString(c->timer.err));
  int k = 0;
  for (int f = 0; f < KF_COUNT; ++f) {
    if (c->timer.launches[f] == 0) continue;
    if (k < cap) {
      out[k].name = kFamilyName[f];
      out[k].launches = c->timer.launches[f];
      out[k].ms = c->timer.ms[f];
      out[k].bytes = c->timer.tbytes[f];
    }
    ++k;
  }
  if (count) *count = k;
  if (reset) c->timer.reset();
  return PCOP_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// GMRES driver
// ---------------------------------------------------------------------------
namespace {

// Enqueue Arnoldi step j on stream st: operator, first Gram-Schmidt pass,
// measured orthogonality, and (full = true) the member-masked second pass.
pcop_status enqueue_iteration(pcop_ctx c, int j, bool full, int n_active, hipStream_t st) {
  const Layout& L = c->L;
  const int B = c->g.B;
  double* tmp1 = c->at<double>(L.tmp1);
  double* sc = c->at<double>(L.sc);
  double* H = c->at<double>(L.H);
  double* coef = c->at<double>(L.coef);
  double* red = c->at<double>(L.red);
  double* partial = c->at<double>(L.partial);
  double* wnorm2 = c->at<double>(L.wnorm2);
  int* skip = c->at<int>(L.skip);
  int* active = c->at<int>(L.active);
  const int H_ld = kMaxBasis;
  double* vj = c->basis(j);
  double* w = c->basis(j + 1);
  const double* scj = sc + j;  // member stride kMaxBasis
  pcop_status s = PCOP_OK;
  const int side = c->opt.side;
  if (side == PCOP_RIGHT) {
    s = do_precond(c, vj, tmp1, scj, kMaxBasis, 0, active, n_active);
    do_kkt(c, tmp1, w, nullptr, nullptr, 0, active, n_active);
  } else if (side == PCOP_FLEXIBLE) {
    s = do_precond(c, vj, c->zbasis(j), scj, kMaxBasis, 0, active, n_active);
    do_kkt(c, c->zbasis(j), w, nullptr, nullptr, 0, active, n_active);
  } else {
    do_kkt(c, vj, tmp1, nullptr, scj, kMaxBasis, active, n_active);
    s = do_precond(c, tmp1, w, nullptr, 0, 0, active, n_active);
  }
  if (s != PCOP_OK) return s;
  // classical Gram-Schmidt; the update pass also measures the new vector
  KrylovArgs ka = c->kargs(c->basis(0), active);
  do_mdot(c, ka, j + 1, w, n_active);
  launch_reduce_partials(partial, c->nb_mdot[j + 1], j + 2, B, red, st);
  launch_gs_step1(red, j, B, sc, H, H_ld, coef, kMaxBasis, wnorm2, active, st);
  do_update(c, ka, j + 1, w, nullptr, n_active);
  launch_reduce_partials(partial, c->nb_upd[j + 1], j + 2, B, red, st);
  launch_gs_step2(red, j, B, sc, H, H_ld, coef, kMaxBasis, wnorm2, c->opt.reorth_tol, skip, sc, active, 0, st);
  if (full) {
    launch_update_nv(c, ka, j + 1, w, skip, st);
    launch_reduce_partials(partial, c->nb_upd[j + 1], j + 2, B, red, st);
    launch_gs_step2(red, j, B, sc, H, H_ld, coef, kMaxBasis, wnorm2, c->opt.reorth_tol, skip, sc, active, 1, st);
  }
  return PCOP_OK;
}

// The graph for Arnoldi steps j0 .. j0 + cnt - 1 (captured on first use).
pcop_status chunk_graph(pcop_ctx c, int j0, int cnt, hipGraphExec_t* out) {
  const int key = j0 * 64 + cnt;
  for (auto& g : c->graphs)
    if (g.first == key) {
      *out = g.second;
      return PCOP_OK;
    }
  const bool timing = c->timer.enabled;
  c->timer.enabled = false;  // events are not recorded inside captured graphs
  hipStream_t saved = c->st;
  c->st = c->gst;
  PCOP_HIP(hipStreamBeginCapture(c->gst, hipStreamCaptureModeThreadLocal));
  pcop_status s = PCOP_OK;
  for (int j = j0; j < j0 + cnt && s == PCOP_OK; ++j) s = enqueue_iteration(c, j, true, c->g.B, c->gst);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(c->gst, &graph);
  c->st = saved;
  c->timer.enabled = timing;
  if (s != PCOP_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return fail(PCOP_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(PCOP_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  c->graphs.push_back({key, exec});
  *out = exec;
  return PCOP_OK;
}

struct MemberState {
  bool active = true;      // still iterating
  bool converged = false;
  int iters = 0;
  double beta0 = 0.0;      // initial residual norm of the solve
  double est = 1.0;        // last relative residual estimate
  // Givens data of the current cycle
  double cs[kMaxBasis], sn[kMaxBasis], gv[kMaxBasis + 1];
  double R[kMaxBasis - 1][kMaxBasis];  // rotated columns
};

// solve the upper-triangular k x k system of the rotated Hessenberg
void back_substitute(const MemberState& s, int k, double* y) {
  for (int i = k - 1; i >= 0; --i) {
    double acc = s.gv[i];
    for (int j = i + 1; j < k; ++j) acc -= s.R[j][i] * y[j];
    y[i] = acc / s.R[i][i];
  }
}

}  // namespace

extern "C" pcop_status pcop_solve(pcop_ctx c, const double* b, double* x, int transpose, pcop_member_info* info,
                                  double* res_hist) {
  if (!c || !b || !x) return fail(PCOP_ERR_INVALID_ARG, "null argument");
  if (((uintptr_t)b | (uintptr_t)x) & 15) return fail(PCOP_ERR_INVALID_ARG, "b and x must be 16-byte aligned");
  // graph mode runs the whole solve on the context's private stream, after
  // the caller's stream has delivered b and x
  const bool use_graph = c->opt.graph && c->gst && !c->timer.enabled;
  struct StreamSwap {
    pcop_ctx c;
    hipStream_t saved;
    bool on;
    ~StreamSwap() {
      if (on) c->st = saved;
    }
  } swap{c, c->st, false};
  if (use_graph) {
    PCOP_HIP(hipStreamSynchronize(c->st));
    c->st = c->gst;
    swap.on = true;
  }
  const Geo& g = c->g;
  const int B = g.B;
  const int side = c->opt.side;
  const int restart = c->opt.restart;
  const int maxit = c->opt.maxit;
  const double rtol = c->opt.rtol;
  hipStream_t st = c->st;
  const Layout& L = c->L;
  double* tmp1 = c->at<double>(L.tmp1);
  double* tmp2 = c->at<double>(L.tmp2);
  double* sc = c->at<double>(L.sc);
  double* H = c->at<double>(L.H);
  double* coef = c->at<double>(L.coef);
  double* red = c->at<double>(L.red);
  double* partial = c->at<double>(L.partial);
  double* wnorm2 = c->at<double>(L.wnorm2);
  double* norm = c->at<double>(L.norm);
  int* skip = c->at<int>(L.skip);
  int* active = c->at<int>(L.active);
  int* finish = c->at<int>(L.finish);
  const int H_ld = kMaxBasis;

  // the solve runs on padded copies of b and x (member stride g.vs);
  // A^T = J A J: solve A z = J b and return x = J z
  const double* bb = tmp2;
  double* const xu = x;
  x = c->at<double>(L.xpad);
  launch_restride(g, b, g.vl, tmp2, g.vs, transpose != 0, st);
  launch_restride(g, xu, g.vl, x, g.vs, transpose != 0, st);
  std::vector<MemberState> ms(B);
  std::vector<int> h_active(B, 1), h_finish(B, 0);
  std::vector<double> h_norm(B), h_col((size_t)B * (kMaxBasis + 1)), h_coef((size_t)B * kMaxBasis);
  std::vector<double> bnorm(B), h_sc((size_t)B * kMaxBasis);
  const size_t H_member = (size_t)(kMaxBasis - 1) * kMaxBasis;
  std::vector<double> h_H(use_graph ? (size_t)B * H_member : 0);
  double* hcol = c->at<double>(L.hcol);
  // Every host<->device transfer goes through pinned staging; an upload
  // buffer is only rewritten after a stream synchronisation.
  bool pending = false;
  auto sync = [&]() -> hipError_t {
    pending = false;
    return hipStreamSynchronize(st);
  };
  auto upload_ints = [&](int* dev, const std::vector<int>& src, int* pinbuf) -> hipError_t {
    if (pending) {
      hipError_t e = sync();
      if (e != hipSuccess) return e;
    }
    std::memcpy(pinbuf, src.data(), sizeof(int) * B);
    pending = true;
    return hipMemcpyAsync(dev, pinbuf, sizeof(int) * B, hipMemcpyHostToDevice, st);
  };
  auto download = [&](double* host, const double* dev, double* pinbuf, size_t count) -> hipError_t {
    hipError_t e = hipMemcpyAsync(pinbuf, dev, sizeof(double) * count, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = sync();
    if (e == hipSuccess) std::memcpy(host, pinbuf, sizeof(double) * count);
    return e;
  };
  std::vector<double> h_red((size_t)B * kRedStride);

  // ||b|| for the final true residual
  PCOP_HIP(upload_ints(active, h_active, c->pin_active));
  do_norm2(c, bb, nullptr, B);
  PCOP_HIP(download(h_red.data(), red, c->pin_red, (size_t)B * kRedStride));
  for (int m = 0; m < B; ++m) bnorm[m] = std::sqrt(h_red[(size_t)m * kRedStride]);

  bool first_cycle = true;
  pcop_status result = PCOP_OK;
  while (true) {
    int n_active = 0;
    for (int m = 0; m < B; ++m) n_active += ms[m].active ? 1 : 0;
    if (n_active == 0) break;
    for (int m = 0; m < B; ++m) h_active[m] = ms[m].active ? 1 : 0;
    PCOP_HIP(upload_ints(active, h_active, c->pin_active));
    // r0 = b - A x (right/flexible) or P^{-1}(b - A x) (left) into slot 0
    if (side == PCOP_LEFT) {
      do_kkt(c, x, tmp1, bb, nullptr, 0, active, n_active);
      pcop_status s = do_precond(c, tmp1, c->basis(0), nullptr, 0, 0, active, n_active);
      if (s != PCOP_OK) return s;
    } else {
      do_kkt(c, x, c->basis(0), bb, nullptr, 0, active, n_active);
    }
    KrylovArgs kv = c->kargs(c->basis(0), active);
    do_mdot(c, kv, 0, c->basis(0), n_active);
    launch_reduce_partials(partial, c->nb_mdot[0], 1, B, red, st);
    launch_set_scale(red, 0, B, sc, norm, active, st);
    PCOP_HIP(download(h_norm.data(), norm, c->pin_norm, (size_t)B));
    for (int m = 0; m < B; ++m) {
      MemberState& s = ms[m];
      if (!s.active) continue;
      const double beta = h_norm[m];
      if (!std::isfinite(beta)) {
        return fail(PCOP_ERR_INVALID_ARG, "non-finite residual (right-hand side or initial guess)");
      }
      if (first_cycle) {
        s.beta0 = beta;
        if (res_hist) res_hist[(size_t)m * (maxit + 1)] = 1.0;
      }
      if (beta == 0.0 || (!first_cycle && beta <= rtol * s.beta0)) {
        s.active = false;
        s.converged = true;
        s.est = (s.beta0 > 0.0) ? beta / s.beta0 : 0.0;
        continue;
      }
      s.gv[0] = beta;
      for (int i = 1; i <= kMaxBasis; ++i) s.gv[i] = 0.0;
    }
    first_cycle = false;
    n_active = 0;
    for (int m = 0; m < B; ++m) {
      h_active[m] = ms[m].active ? 1 : 0;
      n_active += h_active[m];
    }
    if (n_active == 0) break;
    PCOP_HIP(upload_ints(active, h_active, c->pin_active));

    int j = 0;
    while (j < restart) {
      n_active = 0;
      for (int m = 0; m < B; ++m) n_active += h_active[m];
      int cnt = 1;
      if (use_graph) {
        // a chunk of Arnoldi steps as one graph; members that converge inside
        // the chunk run to its end and their extra steps are ignored
        cnt = std::min(c->opt.graph_chunk, restart - j);
        hipGraphExec_t ge = nullptr;
        pcop_status gs = chunk_graph(c, j, cnt, &ge);
        if (gs != PCOP_OK) return gs;
        PCOP_HIP(hipGraphLaunch(ge, st));
        PCOP_HIP(download(h_H.data(), H, c->pin_H, (size_t)B * H_member));
      } else {
        pcop_status s = enqueue_iteration(c, j, false, n_active, st);
        if (s != PCOP_OK) return s;
        // column j of H for every member, with the flag for a second pass
        launch_pack_hcol(H, H_ld, j, B, skip, hcol, st);
        PCOP_HIP(download(h_col.data(), hcol, c->pin_col, (size_t)B * (kMaxBasis + 1)));
        int n_again = 0;
        for (int m = 0; m < B; ++m)
          if (h_active[m] && h_col[(size_t)m * (kMaxBasis + 1) + kMaxBasis] == 0.0) ++n_again;
        if (n_again > 0) {
          // second classical Gram-Schmidt pass for the members that need it
          KrylovArgs ka = c->kargs(c->basis(0), active);
          do_update(c, ka, j + 1, c->basis(j + 1), skip, n_again);
          launch_reduce_partials(partial, c->nb_upd[j + 1], j + 2, B, red, st);
          launch_gs_step2(red, j, B, sc, H, H_ld, coef, kMaxBasis, wnorm2, c->opt.reorth_tol, skip, sc, active, 1,
                          st);
          launch_pack_hcol(H, H_ld, j, B, skip, hcol, st);
          PCOP_HIP(download(h_col.data(), hcol, c->pin_col, (size_t)B * (kMaxBasis + 1)));
        }
      }
      // Givens rotations of the new columns; a member ends its cycle at the
      // first step that converges, exhausts maxit or reaches the restart
      bool any_finish = false;
      int n_fin = 0;
      int kmax = 0;
      std::fill(h_finish.begin(), h_finish.end(), 0);
      std::vector<int> kfin(B, 0);
      for (int m = 0; m < B; ++m) {
        MemberState& ms_ = ms[m];
        if (!h_active[m]) continue;
        for (int jj = j; jj < j + cnt; ++jj) {
          double colbuf[kMaxBasis + 1];
          double* col = colbuf;
          if (use_graph) {
            const double* src = &h_H[(size_t)m * H_member + (size_t)jj * H_ld];
            for (int i = 0; i <= jj + 1; ++i) col[i] = src[i];
          } else {
            col = &h_col[(size_t)m * (kMaxBasis + 1)];
          }
          for (int i = 0; i < jj; ++i) {
            const double t = ms_.cs[i] * col[i] + ms_.sn[i] * col[i + 1];
            col[i + 1] = -ms_.sn[i] * col[i] + ms_.cs[i] * col[i + 1];
            col[i] = t;
          }
          const double a = col[jj], bsub = col[jj + 1];
          double cth = 1.0, sth = 0.0;
          if (bsub != 0.0) {
            const double r = std::hypot(a, bsub);
            cth = a / r;
            sth = bsub / r;
          }
          ms_.cs[jj] = cth;
          ms_.sn[jj] = sth;
          col[jj] = cth * a + sth * bsub;
          col[jj + 1] = 0.0;
          for (int i = 0; i <= jj; ++i) ms_.R[jj][i] = col[i];
          ms_.gv[jj + 1] = -sth * ms_.gv[jj];
          ms_.gv[jj] = cth * ms_.gv[jj];
          ms_.iters += 1;
          ms_.est = std::fabs(ms_.gv[jj + 1]) / ms_.beta0;
          if (res_hist && ms_.iters <= maxit) res_hist[(size_t)m * (maxit + 1) + ms_.iters] = ms_.est;
          const bool conv = ms_.est <= rtol || bsub == 0.0;
          if (conv || ms_.iters >= maxit || jj == restart - 1) {
            h_finish[m] = 1;
            kfin[m] = jj + 1;
            kmax = std::max(kmax, jj + 1);
            any_finish = true;
            ++n_fin;
            if (conv) ms_.converged = true;
            break;
          }
        }
      }
      j += cnt;
      if (!any_finish) continue;
      // form the correction for the members that end their cycle here
      std::fill(h_coef.begin(), h_coef.end(), 0.0);
      PCOP_HIP(download(h_sc.data(), sc, c->pin_sc, (size_t)B * kMaxBasis));
      for (int m = 0; m < B; ++m) {
        if (!h_finish[m]) continue;
        const int k = kfin[m];
        double y[kMaxBasis];
        back_substitute(ms[m], k, y);
        for (int i = 0; i < k; ++i)
          h_coef[(size_t)m * kMaxBasis + i] = (side == PCOP_FLEXIBLE) ? y[i] : y[i] * h_sc[(size_t)m * kMaxBasis + i];
      }
      std::memcpy(c->pin_coef, h_coef.data(), sizeof(double) * B * kMaxBasis);
      PCOP_HIP(hipMemcpyAsync(coef, c->pin_coef, sizeof(double) * B * kMaxBasis, hipMemcpyHostToDevice, st));
      PCOP_HIP(upload_ints(finish, h_finish, c->pin_finish));
      const int k = kmax;
      if (side == PCOP_LEFT) {
        tbeg(c->kt(), KF_COMBINE, 8.0 * (k + 2) * g.vl * n_fin);
        launch_combine(c->kargs(c->basis(0), finish), k, coef, kMaxBasis, x, 1, st);
        tend(c->kt());
      } else if (side == PCOP_FLEXIBLE) {
        tbeg(c->kt(), KF_COMBINE, 8.0 * (k + 2) * g.vl * n_fin);
        launch_combine(c->kargs(c->zbasis(0), finish), k, coef, kMaxBasis, x, 1, st);
        tend(c->kt());
      } else {
        tbeg(c->kt(), KF_COMBINE, 8.0 * (k + 1) * g.vl * n_fin);
        launch_combine(c->kargs(c->basis(0), finish), k, coef, kMaxBasis, tmp1, 0, st);
        tend(c->kt());
        pcop_status s2 = do_precond(c, tmp1, x, nullptr, 0, 1, finish, n_fin);
        if (s2 != PCOP_OK) return s2;
      }
      bool any_left = false;
      for (int m = 0; m < B; ++m) {
        if (!h_finish[m]) {
          any_left = any_left || ms[m].active;
          continue;
        }
        // a member ends: converged or out of iterations; otherwise it restarts
        if (ms[m].converged || ms[m].iters >= maxit) ms[m].active = false;
      }
      for (int m = 0; m < B; ++m) h_active[m] = (ms[m].active && !h_finish[m] && h_active[m]) ? 1 : 0;
      PCOP_HIP(upload_ints(active, h_active, c->pin_active));
      if (!any_left) break;
    }
  }

  // true residual ||b - A x|| / ||b||
  std::fill(h_active.begin(), h_active.end(), 1);
  PCOP_HIP(upload_ints(active, h_active, c->pin_active));
  do_kkt(c, x, tmp1, bb, nullptr, 0, nullptr, B);
  do_norm2(c, tmp1, nullptr, B);
  launch_restride(g, x, g.vs, xu, g.vl, transpose != 0, st);
  PCOP_HIP(download(h_red.data(), red, c->pin_red, (size_t)B * kRedStride));
  PCOP_HIP(hipGetLastError());
  for (int m = 0; m < B; ++m) {
    const double rt = std::sqrt(h_red[(size_t)m * kRedStride]);
    if (info) {
      info[m].iters = ms[m].iters;
      info[m].converged = ms[m].converged ? 1 : 0;
      info[m].relres_est = ms[m].est;
      info[m].relres_true = bnorm[m] > 0.0 ? rt / bnorm[m] : rt;
    }
    if (!ms[m].converged) result = PCOP_NOT_CONVERGED;
  }
  if (result == PCOP_NOT_CONVERGED) g_last_error = "tolerance not met within maxit";
  return result;
}
