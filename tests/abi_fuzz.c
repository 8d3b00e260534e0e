/* Randomised checks of the host-only part of the C ABI: option defaults,
 * problem/option validation, workspace sizing, and the argument checks that
 * pcop_setup makes before it touches a device.  Built with the host
 * sanitizers (address, undefined behaviour) by test_host_sanitizers.py and
 * run on the CPU; every call here returns before any device work.
 *
 * Exit status 0 when every invariant held; otherwise a message on stderr
 * and status 1 (a sanitizer report aborts the process by itself). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pcop.h"

static uint64_t g_state = 0x9e3779b97f4a7c15ull;

/* splitmix64: a counter-based generator used only to pick test inputs */
static uint64_t next_u64(void) {
  uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
static int pick(int k) { return (int)(next_u64() % (uint64_t)k); }
static double unif(void) { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); }

static int g_fail = 0;
#define CHECK(cond, ...)                         \
  do {                                           \
    if (!(cond)) {                               \
      fprintf(stderr, "check failed: " #cond " "); \
      fprintf(stderr, __VA_ARGS__);              \
      fprintf(stderr, "\n");                     \
      g_fail = 1;                                \
    }                                            \
  } while (0)

static const int kNx[] = {-5, 0, 1, 2, 3, 6, 7, 15, 30, 31, 63, 127, 255, 511, 1023, 2047, 1 << 20, 2147483647};
static const int kNt[] = {-3, 0, 1, 2, 3, 8, 32, 33, 65, 128, 256, 512, 1000, 1024, 1153, 2049, 2050, 4096,
                          1 << 20, 1 << 30, 2147483647};
static const double kReal[] = {1.0, 0.5, 1e-8, 0.0, -1.0, 1e300, INFINITY, NAN};

static double pick_real(void) { return pick(3) ? unif() * 4.0 + 1e-3 : kReal[pick(8)]; }

static void random_options(pcop_options* o) {
  pcop_default_options(o);
  if (pick(2)) o->precision = pick(4) ? pick(2) : pick(7) - 3;
  if (pick(3) == 0) o->spatial = pick(4) ? pick(2) : 9;
  if (pick(2)) o->side = pick(5) ? pick(3) : -1;
  if (o->precision == PCOP_MIXED && pick(4)) o->side = PCOP_FLEXIBLE;
  if (pick(4) == 0) o->restart = pick(50) - 3;
  if (pick(6) == 0) o->maxit = pick(4) - 1;
  if (pick(6) == 0) o->rtol = kReal[pick(8)];
  if (pick(8) == 0) o->reorth_tol = kReal[pick(8)];
  if (pick(4) == 0) o->graph = pick(3);
  if (pick(4) == 0) o->graph_chunk = pick(6) - 1;
  if (pick(3) == 0) o->time_cols = pick(70) - 35;
  if (pick(4) == 0) o->dst_kernel = pick(8) - 1;
  if (pick(6) == 0) o->tune = pick(3);
  if (pick(4) == 0) o->precond = pick(4) - 1;
  if (pick(4) == 0) o->kkt_jchunk = pick(140) - 70;
  if (pick(4) == 0) o->krylov_blocks = pick(5000) - 2;
  if (pick(4) == 0) o->gs_update = pick(5) - 1;
  if (pick(6) == 0) o->mg_smoother = pick(5) - 1;
}

int main(int argc, char** argv) {
  const int iters = argc > 1 ? atoi(argv[1]) : 20000;
  if (argc > 2) g_state = strtoull(argv[2], NULL, 10);

  /* defaults validate on a small problem */
  {
    double gam = 1e-4;
    pcop_problem p;
    memset(&p, 0, sizeof(p));
    p.dim = 2, p.nx = 31, p.nt = 32, p.T = 1.0, p.batch = 1, p.gamma = &gam, p.eps = -1.0;
    pcop_options o;
    pcop_default_options(&o);
    CHECK(pcop_validate(&p, &o) == PCOP_OK, "defaults: %s", pcop_last_error());
    pcop_default_options(NULL);
    CHECK(pcop_validate(NULL, &o) == PCOP_ERR_INVALID_ARG, "null problem");
    CHECK(pcop_validate(&p, NULL) == PCOP_ERR_INVALID_ARG, "null options");
    CHECK(pcop_workspace_size(&p, &o, NULL) == PCOP_ERR_INVALID_ARG, "null bytes");
    CHECK(pcop_setup(NULL, &p, &o, NULL, 0) == PCOP_ERR_INVALID_ARG, "null out");
  }
  for (int s = -2; s < 12; ++s) CHECK(pcop_status_string(s) != NULL && pcop_status_string(s)[0], "status %d", s);

  int n_ok = 0;
  for (int it = 0; it < iters; ++it) {
    pcop_problem p;
    memset(&p, 0, sizeof(p));
    p.dim = pick(8) ? 2 + pick(2) : pick(6) - 1;
    p.nx = pick(3) ? kNx[3 + pick(11)] : kNx[pick(sizeof(kNx) / sizeof(kNx[0]))];
    p.nt = pick(3) ? kNt[3 + pick(10)] : (pick(2) ? kNt[pick(sizeof(kNt) / sizeof(kNt[0]))] : pick(3000));
    p.T = pick(6) ? 1.0 + unif() : kReal[pick(8)];
    p.batch = pick(8) ? 1 + pick(4) : pick(3) - 1;
    const int nb = p.batch > 0 ? p.batch : 1;
    double* gam = (double*)malloc(sizeof(double) * (size_t)nb);
    for (int b = 0; b < nb; ++b) gam[b] = pick(10) ? pow(10.0, -8.0 * unif()) : pick_real();
    p.gamma = pick(30) ? gam : NULL;
    p.eps = pick(3) ? -1.0 : pick_real();
    p.mass = pick(6) ? PCOP_MASS_IDENTITY : pick(4) - 1;
    p.coeff_kind = pick(4) ? PCOP_COEFF_ONE : (pick(8) ? PCOP_COEFF_HALFGRID : 7);
    double* coeff = NULL; /* owned */
    if (p.coeff_kind == PCOP_COEFF_HALFGRID) {
      /* exactly (2 nx + 1)^dim samples, so that any read past them is reported */
      const double side = 2.0 * p.nx + 1.0;
      const double hn = (p.dim >= 1 && p.dim <= 3 && p.nx >= 1) ? pow(side, p.dim) : 0.0;
      if (hn >= 1.0 && hn <= (double)(1 << 22)) {
        coeff = (double*)malloc(sizeof(double) * (size_t)hn);
        for (size_t k = 0; k < (size_t)hn; ++k) coeff[k] = 0.5 + unif();
        if (pick(5) == 0) coeff[pick((int)hn)] = kReal[3 + pick(5)];
      } else {
        p.coeff_kind = PCOP_COEFF_ONE;
      }
    } else if (p.coeff_kind == PCOP_COEFF_ONE && pick(40) == 0) {
      static double junk = 1.0;
      p.coeff = &junk; /* refused: coeff must be null for PCOP_COEFF_ONE */
    }
    if (coeff) p.coeff = coeff;
    pcop_options o;
    random_options(&o);

    const pcop_status sv = pcop_validate(&p, &o);
    CHECK(sv >= PCOP_OK && sv <= PCOP_ERR_UNSUPPORTED, "status %d", (int)sv);
    if (sv != PCOP_OK) CHECK(pcop_last_error()[0] != 0, "empty error after status %d", (int)sv);
    size_t bytes = 0;
    const pcop_status sw = pcop_workspace_size(&p, &o, &bytes);
    CHECK(sw == sv, "workspace_size %d vs validate %d", (int)sw, (int)sv);
    pcop_ctx ctx = (pcop_ctx)0x1;
    const pcop_status ss = pcop_setup(&ctx, &p, &o, NULL, 0);
    CHECK(ctx == NULL, "setup left *out set");
    if (sv != PCOP_OK) {
      CHECK(ss == sv, "setup %d vs validate %d", (int)ss, (int)sv);
    } else {
      ++n_ok;
      /* a valid problem: the workspace holds at least the Krylov basis */
      const double m = pow((double)p.nx, p.dim);
      const double vec = 8.0 * 2.0 * (p.nt - 1) * m * p.batch;
      CHECK(bytes % 256 == 0, "bytes %zu not 256-aligned", bytes);
      CHECK((double)bytes >= vec * (o.restart + 3), "bytes %zu below %g", bytes, vec * (o.restart + 3));
      CHECK(ss == PCOP_ERR_WORKSPACE, "setup without workspace: %d", (int)ss);
      /* too small, then misaligned: both refused before any device call */
      CHECK(pcop_setup(&ctx, &p, &o, (void*)(uintptr_t)4096, bytes - 256) == PCOP_ERR_WORKSPACE, "small");
      CHECK(pcop_setup(&ctx, &p, &o, (void*)(uintptr_t)4100, bytes) == PCOP_ERR_WORKSPACE, "misaligned");
      CHECK(ctx == NULL, "setup left *out set");
      /* one more member never needs less workspace */
      if (p.gamma) {
        double* g2 = (double*)malloc(sizeof(double) * (size_t)(p.batch + 1));
        memcpy(g2, p.gamma, sizeof(double) * (size_t)p.batch);
        g2[p.batch] = 1e-3;
        pcop_problem p2 = p;
        p2.gamma = g2;
        p2.batch += 1;
        size_t b2 = 0;
        if (pcop_workspace_size(&p2, &o, &b2) == PCOP_OK) CHECK(b2 > bytes, "batch+1: %zu <= %zu", b2, bytes);
        free(g2);
      }
    }
    free(coeff);
    free(gam);
    if (g_fail) {
      fprintf(stderr, "iteration %d: dim %d nx %d nt %d batch %d coeff_kind %d mass %d\n", it, p.dim, p.nx,
              p.nt, p.batch, p.coeff_kind, p.mass);
      return 1;
    }
  }
  printf("abi_fuzz: %d cases, %d valid\n", iters, n_ok);
  return n_ok > 0 ? 0 : 1;
}
