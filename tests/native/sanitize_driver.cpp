// Host-code sanitizer driver for libmudiff: every entry point of the C ABI is
// called through its host logic (argument validation, workspace layout, the
// operator schedules, tile timing, graph capture, the no-allocation path) in a
// build whose host code carries AddressSanitizer and UndefinedBehaviorSanitizer
// (device code is unchanged).  Any sanitizer report aborts the process.
//
//   sanitize_driver cpu   validation paths only: no device call is reached
//   sanitize_driver gpu   small problems through every entry point on device 0
//
// The numerical checks here are self-consistency only (finite outputs,
// converged flags, the circulant and direct forms of one apply agreeing); the
// parity with the oracle is the business of the Python tests.
#include <hip/hip_runtime_api.h>
#include <sanitizer/lsan_interface.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "mudiff.h"

using cd = std::complex<double>;

static int g_fail = 0;

#define EXPECT(cond, ...)                                    \
  do {                                                       \
    if (!(cond)) {                                           \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                     \
      std::fprintf(stderr, "\n");                            \
      ++g_fail;                                              \
    }                                                        \
  } while (0)

#define STATUS(call, want)                                                              \
  do {                                                                                \
    const int st_ = (call);                                                           \
    if (st_ != (want)) {                                                              \
      std::fprintf(stderr, "FAIL %s:%d: %s -> %d (want %d): %s\n", __FILE__, __LINE__, \
                   #call, st_, (want), mudiff_last_error());                          \
      ++g_fail;                                                                       \
    }                                                                                 \
  } while (0)

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      std::fprintf(stderr, "HIP %s at %s:%d: %s\n", #call, __FILE__, __LINE__,          \
                   hipGetErrorString(e_));                                              \
      std::exit(3);                                                                    \
    }                                                                                  \
  } while (0)

static void step(const char* what) {
  std::printf("== %s\n", what);
  std::fflush(stdout);
}

// ------------------------------------------------------------------ geometry

struct Batch {
  std::vector<int64_t> off{0};
  std::vector<double> xy, a, k;
  std::vector<int32_t> N;
  int B() const { return (int)off.size() - 1; }
  int64_t M() const { return off.back(); }
};

// Instance of n disks on a jittered square grid of spacing h (radii in
// [a0, a1], a1 < h/2 - 0.1 so that no two disks touch), N_p = ceil(k a) + extra,
// or n_fixed for every disk when n_fixed >= 0.
static void add_instance(Batch& b, std::mt19937_64& g, int n, double h, double a0, double a1,
                         double k, int extra, int n_fixed) {
  std::uniform_real_distribution<double> u(0.0, 1.0);
  const int side = (int)std::ceil(std::sqrt((double)n));
  const double jit = 0.5 * (h - 2.0 * a1) - 0.05;
  for (int i = 0; i < n; ++i) {
    const double x = h * (i % side) + jit * (2 * u(g) - 1);
    const double y = h * (i / side) + jit * (2 * u(g) - 1);
    const double r = a0 + (a1 - a0) * u(g);
    b.xy.push_back(x);
    b.xy.push_back(y);
    b.a.push_back(r);
    b.N.push_back(n_fixed >= 0 ? n_fixed : (int)std::ceil(k * r) + extra);
  }
  b.off.push_back(b.off.back() + n);
  b.k.push_back(k);
}

static std::vector<int64_t> unknowns(const Batch& b) {
  std::vector<int64_t> n(b.B(), 0);
  for (int i = 0; i < b.B(); ++i)
    for (int64_t p = b.off[i]; p < b.off[i + 1]; ++p) n[i] += 2 * b.N[p] + 1;
  return n;
}

// --------------------------------------------------------------- device memory

struct Dev {
  std::vector<void*> ptrs;
  void* get(size_t bytes) {
    void* p = nullptr;
    HIPCHK(hipMalloc(&p, bytes < 256 ? 256 : bytes));
    HIPCHK(hipMemset(p, 0, bytes < 256 ? 256 : bytes));
    ptrs.push_back(p);
    return p;
  }
  template <class T>
  T* put(const std::vector<T>& v) {
    T* p = (T*)get(v.size() * sizeof(T));
    HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
  }
  ~Dev() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

template <class T>
static std::vector<T> fetch(const void* p, size_t n) {
  std::vector<T> v(n);
  HIPCHK(hipMemcpy(v.data(), p, n * sizeof(T), hipMemcpyDeviceToHost));
  return v;
}

static bool all_finite(const std::vector<cd>& v) {
  for (const cd& z : v)
    if (!std::isfinite(z.real()) || !std::isfinite(z.imag())) return false;
  return true;
}

static double rel_diff(const std::vector<cd>& a, const std::vector<cd>& b) {
  double num = 0, den = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    num += std::norm(a[i] - b[i]);
    den += std::norm(b[i]);
  }
  return std::sqrt(num / (den > 0 ? den : 1));
}

static std::vector<cd> random_vec(std::mt19937_64& g, size_t n) {
  std::normal_distribution<double> nd;
  std::vector<cd> v(n);
  for (auto& z : v) z = cd(nd(g), nd(g));
  return v;
}

struct Handle {
  mudiff_t h = nullptr;
  void* ws = nullptr;
  int64_t total = 0;  // sum_b R-independent unknowns
  std::vector<int64_t> n;
  ~Handle() {
    if (h) mudiff_destroy(h);
  }
};

static void make(Handle& H, Dev& dev, const Batch& b, int flags) {
  const size_t ws = mudiff_tables_workspace_size(b.B(), b.off.data(), b.N.data(), flags);
  EXPECT(ws > 0, "workspace size");
  H.ws = dev.get(ws);
  STATUS(mudiff_tables(b.B(), b.off.data(), b.xy.data(), b.a.data(), b.N.data(), b.k.data(), H.ws,
                       ws, flags, nullptr, &H.h),
         MUDIFF_OK);
  H.n = unknowns(b);
  std::vector<int64_t> n2(b.B());
  STATUS(mudiff_sizes(H.h, n2.data()), MUDIFF_OK);
  EXPECT(n2 == H.n, "sizes");
  H.total = 0;
  for (int64_t x : H.n) H.total += x;
}

// y = op(x) on R columns with a fresh zeroed workspace
static std::vector<cd> apply(Handle& H, Dev& dev, int R, const std::vector<cd>& x, int op) {
  const size_t ws = mudiff_matvec_workspace_size(H.h, R);
  EXPECT(ws > 0, "matvec workspace");
  void* w = dev.get(ws);
  cd* xd = dev.put(x);
  void* y = dev.get(x.size() * sizeof(cd));
  STATUS(mudiff_matvec(H.h, R, xd, y, op, w, ws, nullptr), MUDIFF_OK);
  HIPCHK(hipDeviceSynchronize());
  return fetch<cd>(y, x.size());
}

// ------------------------------------------------------------------ cpu mode

static void cpu_mode() {
  step("workspace size queries");
  const int64_t off4[] = {0, 4}, off_bad0[] = {1, 4}, off_empty[] = {0, 2, 2};
  const int32_t n4[] = {15, 15, 15, 15}, n_neg[] = {15, 15, -1, 15}, n_big[] = {15, 15, 201, 15};
  const int32_t n40[] = {40, 3, 3, 3};
  EXPECT(mudiff_tables_workspace_size(1, off4, n4, 0) > 0, "size");
  EXPECT(mudiff_tables_workspace_size(1, off4, n4, MUDIFF_TABLES_CIRCULANT) >
             mudiff_tables_workspace_size(1, off4, n4, 0),
         "circulant size");
  EXPECT(mudiff_tables_workspace_size(1, off4, n_neg, 0) == 0, "N<0");
  EXPECT(mudiff_tables_workspace_size(1, off4, n_big, 0) == 0, "N>max");
  EXPECT(mudiff_tables_workspace_size(1, off_bad0, n4, 0) == 0, "off[0]");
  EXPECT(mudiff_tables_workspace_size(2, off_empty, n4, 0) == 0, "empty instance");
  EXPECT(mudiff_tables_workspace_size(0, off4, n4, 0) == 0, "B=0");
  EXPECT(mudiff_tables_workspace_size(1, nullptr, n4, 0) == 0, "NULL offsets");
  EXPECT(mudiff_tables_workspace_size(1, off4, n4, 2) == 0, "unknown flag");
  EXPECT(mudiff_tables_workspace_size(1, off4, n40, MUDIFF_TABLES_CIRCULANT) == 0,
         "circulant with N_p > 31");
  const size_t big = mudiff_tables_workspace_size(1, off4, n4, 0);

  step("tables validation");
  const double xy[] = {0, 0, 3, 0, 0, 3, 3, 3}, a[] = {1, 1, 1, 1}, k[] = {6.28};
  const double xy_ov[] = {0, 0, 1.5, 0, 0, 3, 3, 3}, a_bad[] = {1, -1, 1, 1};
  const double k_bad[] = {-1.0}, xy_nan[] = {0, NAN, 3, 0, 0, 3, 3, 3};
  mudiff_t h = nullptr;
  char dummy[512];
  void* ws = dummy;  // never dereferenced: every call below fails validation first
  STATUS(mudiff_tables(1, off4, xy_ov, a, n4, k, ws, big, 0, nullptr, &h), MUDIFF_ERR_OVERLAP);
  STATUS(mudiff_tables(1, off4, xy, a_bad, n4, k, ws, big, 0, nullptr, &h), MUDIFF_ERR_INVALID);
  STATUS(mudiff_tables(1, off4, xy, a, n4, k_bad, ws, big, 0, nullptr, &h), MUDIFF_ERR_INVALID);
  STATUS(mudiff_tables(1, off4, xy_nan, a, n4, k, ws, big, 0, nullptr, &h), MUDIFF_ERR_INVALID);
  STATUS(mudiff_tables(1, off4, xy, a, n_neg, k, ws, big, 0, nullptr, &h), MUDIFF_ERR_INVALID);
  STATUS(mudiff_tables(1, off4, xy, a, n4, k, ws, big - 1, 0, nullptr, &h), MUDIFF_ERR_NOMEM);
  STATUS(mudiff_tables(1, off4, xy, a, n4, k, nullptr, big, 0, nullptr, &h), MUDIFF_ERR_INVALID);
  STATUS(mudiff_tables(1, off4, xy, a, n4, k, ws, big, 0, nullptr, nullptr), MUDIFF_ERR_INVALID);
  STATUS(mudiff_tables(1, off4, xy, a, n40, k, ws, big, MUDIFF_TABLES_CIRCULANT, nullptr, &h),
         MUDIFF_ERR_INVALID);
  STATUS(mudiff_tables(1, off4, xy, a, n4, k, ws, big, 4, nullptr, &h), MUDIFF_ERR_INVALID);
  EXPECT(h == nullptr, "no handle on failure");
  EXPECT(std::strlen(mudiff_last_error()) > 0, "error text");

  step("NULL handle on every handle call");
  int64_t i64 = 0;
  int i32 = 0;
  double ms[MUDIFF_N_PHASES];
  STATUS(mudiff_destroy(nullptr), MUDIFF_OK);  // like free(NULL)
  STATUS(mudiff_sizes(nullptr, &i64), MUDIFF_ERR_INVALID);
  STATUS(mudiff_circulant_info(nullptr, &i64, &i64, &i32), MUDIFF_ERR_INVALID);
  STATUS(mudiff_set_circulant(nullptr, 8, 1), MUDIFF_ERR_INVALID);
  STATUS(mudiff_circulant_tile(nullptr, 8, &i32, &i32, &i32, &i32, &i32, &i32), MUDIFF_ERR_INVALID);
  STATUS(mudiff_set_circulant_tile(nullptr, 8, 64, 32, 16, 2, 256, 4), MUDIFF_ERR_INVALID);
  STATUS(mudiff_disk_tables(nullptr, nullptr, nullptr, nullptr), MUDIFF_ERR_INVALID);
  STATUS(mudiff_pair_tables(nullptr, nullptr, &i64, nullptr), MUDIFF_ERR_INVALID);
  STATUS(mudiff_apply_config(nullptr, 1, &i32, &i32, &i32, &i32, &i32, nullptr),
         MUDIFF_ERR_INVALID);
  STATUS(mudiff_set_apply_config(nullptr, 8, 1, 4, 0, 256), MUDIFF_ERR_INVALID);
  EXPECT(mudiff_matvec_workspace_size(nullptr, 1) == 0, "matvec ws");
  STATUS(mudiff_matvec(nullptr, 1, dummy, dummy, 1, dummy, 256, nullptr), MUDIFF_ERR_INVALID);
  STATUS(mudiff_matvec_noalloc(nullptr, 1, dummy, dummy, 1, nullptr), MUDIFF_ERR_INVALID);
  STATUS(mudiff_rhs(nullptr, 1, (double*)dummy, dummy, 0, nullptr), MUDIFF_ERR_INVALID);
  STATUS(mudiff_rhs_point(nullptr, 1, (double*)dummy, dummy, 0, nullptr), MUDIFF_ERR_INVALID);
  EXPECT(mudiff_gmres_workspace_size(nullptr, 1, 10, 0) == 0, "gmres ws");
  STATUS(mudiff_gmres(nullptr, 1, nullptr, dummy, dummy, 10, 1e-8, 10, 0, dummy, 256, nullptr,
                      nullptr, nullptr, nullptr, nullptr),
         MUDIFF_ERR_INVALID);
  STATUS(mudiff_farfield(nullptr, 1, dummy, 4, (double*)dummy, dummy, nullptr), MUDIFF_ERR_INVALID);
  EXPECT(mudiff_gmres_workspace_size(nullptr, 8, 10, MUDIFF_BLOCK | MUDIFF_BLOCK_SIZE(8)) == 0,
         "block gmres ws");
  STATUS(mudiff_nearfield(nullptr, 1, dummy, 4, (double*)dummy, nullptr, 0, dummy, nullptr),
         MUDIFF_ERR_INVALID);
  EXPECT(mudiff_grad_workspace_size(nullptr, 1, 4, 10, 0) == 0, "grad ws");
  EXPECT(mudiff_operator_workspace_size(nullptr) == 0, "operator ws");
  STATUS(mudiff_set_operator(nullptr, nullptr, nullptr, nullptr, dummy, 256, nullptr),
         MUDIFF_ERR_INVALID);
  STATUS(mudiff_set_formulation(nullptr, MUDIFF_FORM_MFIE, 0.5, 0, 1, dummy, 256, nullptr),
         MUDIFF_ERR_INVALID);
  STATUS(mudiff_set_penetrable(nullptr, (double*)dummy, nullptr, dummy, 256, nullptr),
         MUDIFF_ERR_INVALID);
  EXPECT(mudiff_interior_workspace_size(nullptr, 1) == 0, "interior ws");
  STATUS(mudiff_profile_begin(nullptr, 4), MUDIFF_ERR_INVALID);
  STATUS(mudiff_profile_end(nullptr, &i32, ms), MUDIFF_ERR_INVALID);

  step("handle-free calls: argument checks");
  STATUS(mudiff_tro(0, 4, dummy, dummy, nullptr), MUDIFF_ERR_INVALID);
  STATUS(mudiff_tro(4, 4, nullptr, dummy, nullptr), MUDIFF_ERR_INVALID);
  EXPECT(mudiff_tro_eigh_workspace_size(0, 4) == 0, "eigh ws");
  int32_t sweeps = 0;
  STATUS(mudiff_tro_eigh(4, 4, dummy, (double*)dummy, dummy, 0, 1e-12, dummy, 256, &sweeps, nullptr),
         MUDIFF_ERR_INVALID);
  STATUS(mudiff_herglotz(0, (double*)dummy, 1, dummy, 1.0, 0.1, 4, (double*)dummy, dummy, nullptr),
         MUDIFF_ERR_INVALID);
  EXPECT(mudiff_probe_workspace_size(7, 0) == 0, "probe kind");
  double rate = 0;
  STATUS(mudiff_probe(7, 0, dummy, 256, &rate, nullptr), MUDIFF_ERR_INVALID);
}

// ------------------------------------------------------------------ gpu mode

// Uniform orders (one-lane kernel at R < 8), two instances.
static void gpu_uniform(std::mt19937_64& g) {
  Dev dev;
  Batch b;
  add_instance(b, g, 12, 3.0, 0.5, 1.0, 4.0, 0, 8);
  add_instance(b, g, 9, 3.0, 0.5, 1.0, 3.0, 0, 8);
  Handle H;
  make(H, dev, b, 0);

  step("uniform batch: applies L, A, L^T at R = 1 and 3; no-allocation apply");
  for (int R : {1, 3}) {
    const auto x = random_vec(g, (size_t)R * H.total);
    for (int op : {MUDIFF_OP_L, MUDIFF_OP_A, MUDIFF_OP_LT}) {
      const auto y = apply(H, dev, R, x, op);
      EXPECT(all_finite(y), "apply R=%d op=%d", R, op);
      cd* xd = dev.put(x);
      cd* yd = (cd*)dev.get(x.size() * sizeof(cd));
      STATUS(mudiff_matvec_noalloc(H.h, R, xd, yd, op, nullptr), MUDIFF_OK);
      HIPCHK(hipDeviceSynchronize());
      const auto y2 = fetch<cd>(yd, x.size());
      EXPECT(rel_diff(y2, y) < 1e-13, "noalloc R=%d op=%d: %g", R, op, rel_diff(y2, y));
    }
    int kind = -1;
    STATUS(mudiff_apply_config(H.h, R, &kind, nullptr, nullptr, nullptr, nullptr, nullptr),
           MUDIFF_OK);
  }
  STATUS(mudiff_matvec_noalloc(H.h, 8, dev.get(16), dev.get(16), 1, nullptr), MUDIFF_ERR_INVALID);

  step("uniform batch: tables copies, right-hand sides, GMRES (eager and graph), far and near field");
  int64_t npairs = 0;
  STATUS(mudiff_pair_tables(H.h, nullptr, &npairs, nullptr), MUDIFF_OK);
  void* t = dev.get((size_t)npairs * 16);
  STATUS(mudiff_pair_tables(H.h, t, &npairs, nullptr), MUDIFF_OK);
  void* Jd = dev.get(b.M() * 10 * 8), * Hd = dev.get(b.M() * 10 * 16);
  STATUS(mudiff_disk_tables(H.h, (double*)Jd, Hd, nullptr), MUDIFF_OK);
  const int R = 2;
  std::vector<double> beta{0.1, 1.3, -0.4, 2.2};
  double* betad = dev.put(beta);
  void* U = dev.get((size_t)R * H.total * 16);
  STATUS(mudiff_rhs(H.h, R, betad, U, 1, nullptr), MUDIFF_OK);
  for (int flags : {0, (int)MUDIFF_GRAPH}) {
    const size_t ws = mudiff_gmres_workspace_size(H.h, R, 20, flags);
    void* w = dev.get(ws);
    void* rho = dev.get((size_t)R * H.total * 16);
    int32_t* fl = (int32_t*)dev.get(4 * 4);
    double* rr = (double*)dev.get(4 * 8);
    int32_t* it = (int32_t*)dev.get(4 * 4);
    double* rv = (double*)dev.get(4 * 8 * 501);
    STATUS(mudiff_gmres(H.h, R, betad, nullptr, rho, 20, 1e-10, 500, flags, w, ws, fl, rr, it, rv,
                        nullptr),
           MUDIFF_OK);
    HIPCHK(hipDeviceSynchronize());
    for (int32_t f : fetch<int32_t>(fl, 4)) EXPECT(f == 0, "gmres flag %d (flags %d)", f, flags);
    std::vector<double> th{0.0, 0.7, 2.0, 4.1, 5.5};
    double* thd = dev.put(th);
    void* ff = dev.get((size_t)2 * R * th.size() * 16);
    STATUS(mudiff_farfield(H.h, R, rho, (int)th.size(), thd, ff, nullptr), MUDIFF_OK);
    std::vector<double> pts{-5.0, -5.0, 1.5, 1.5, 40.0, 2.0};
    double* ptd = dev.put(pts);
    void* nf = dev.get((size_t)2 * R * 3 * 16);
    STATUS(mudiff_nearfield(H.h, R, rho, 3, ptd, betad, 0, nf, nullptr), MUDIFF_OK);
    HIPCHK(hipDeviceSynchronize());
    EXPECT(all_finite(fetch<cd>(ff, 2 * R * th.size())), "far field");
  }

  step("uniform batch: point sources, formulations, penetrable disks, interior field");
  std::vector<double> src{-6.0, -6.0, 30.0, -3.0, -6.0, 25.0, 28.0, 27.0};
  double* srcd = dev.put(src);
  STATUS(mudiff_rhs_point(H.h, R, srcd, U, 0, nullptr), MUDIFF_OK);
  const size_t ows = mudiff_operator_workspace_size(H.h);
  void* ow = dev.get(ows);
  for (int kind = MUDIFF_FORM_MFIE; kind <= MUDIFF_FORM_SOUND_HARD_DOUBLE + 1; ++kind) {
    const int want = kind <= MUDIFF_FORM_SOUND_HARD_DOUBLE ? MUDIFF_OK : MUDIFF_ERR_INVALID;
    STATUS(mudiff_set_formulation(H.h, kind, 0.5, 0.0, 4.0, ow, ows, nullptr), want);
    if (want != MUDIFF_OK) continue;
    const size_t ws = std::max(mudiff_gmres_workspace_size(H.h, R, 20, 0),
                               mudiff_gmres_workspace_size(H.h, R, 20, MUDIFF_NO_PRECOND));
    void* w = dev.get(ws);
    void* rho = dev.get((size_t)R * H.total * 16);
    int32_t* fl = (int32_t*)dev.get(16);
    double* rr = (double*)dev.get(32);
    int32_t* it = (int32_t*)dev.get(16);
    STATUS(mudiff_gmres(H.h, R, betad, nullptr, rho, 20, 1e-8, 2000, 0, w, ws, fl, rr, it, nullptr,
                        nullptr),
           MUDIFF_OK);
    STATUS(mudiff_gmres(H.h, R, betad, nullptr, rho, 20, 1e-8, 2000, MUDIFF_NO_PRECOND, w, ws, fl,
                        rr, it, nullptr, nullptr),
           MUDIFF_OK);
    STATUS(mudiff_matvec(H.h, R, rho, dev.get((size_t)R * H.total * 16), MUDIFF_OP_LT, w, ws,
                         nullptr),
           MUDIFF_ERR_INVALID);
  }
  STATUS(mudiff_set_formulation(H.h, MUDIFF_FORM_CFIE, 0.5, 0.0, 0.0, ow, ows, nullptr),
         MUDIFF_ERR_INVALID);
  STATUS(mudiff_set_formulation(H.h, MUDIFF_FORM_EFIE, 0, 0, 0, ow, ows, nullptr), MUDIFF_OK);
  std::vector<double> kin(b.M(), 6.0), mu(b.M(), 1.5);
  STATUS(mudiff_set_penetrable(H.h, kin.data(), mu.data(), ow, ows, nullptr), MUDIFF_OK);
  {
    const size_t ws = mudiff_gmres_workspace_size(H.h, R, 30, MUDIFF_POINT_SOURCE);
    void* w = dev.get(ws);
    void* rho = dev.get((size_t)R * H.total * 16);
    int32_t* fl = (int32_t*)dev.get(16);
    double* rr = (double*)dev.get(32);
    int32_t* it = (int32_t*)dev.get(16);
    STATUS(mudiff_gmres(H.h, R, srcd, nullptr, rho, 30, 1e-8, 3000, MUDIFF_POINT_SOURCE, w, ws, fl,
                        rr, it, nullptr, nullptr),
           MUDIFF_OK);
    std::vector<double> pts{b.xy[0], b.xy[1], b.xy[0] + 0.1, b.xy[1], -20.0, -20.0};
    double* ptd = dev.put(pts);
    const size_t iws = mudiff_interior_workspace_size(H.h, R);
    void* iw = dev.get(iws);
    void* out = dev.get((size_t)2 * R * 3 * 16);
    STATUS(mudiff_interior_field(H.h, R, rho, srcd, MUDIFF_POINT_SOURCE, 3, ptd, out, iw, iws,
                                 nullptr),
           MUDIFF_OK);
    HIPCHK(hipDeviceSynchronize());
  }
  std::vector<double> kbad(b.M(), -1.0);
  STATUS(mudiff_set_penetrable(H.h, kbad.data(), nullptr, ow, ows, nullptr), MUDIFF_ERR_INVALID);
  STATUS(mudiff_set_operator(H.h, nullptr, nullptr, nullptr, ow, ows, nullptr), MUDIFF_OK);

  step("uniform batch: adjoint gradient");
  {
    const int nrec = 6;
    std::vector<double> th(nrec);
    for (int j = 0; j < nrec; ++j) th[j] = 2 * M_PI * j / nrec;
    double* thd = dev.put(th);
    void* target = dev.get((size_t)2 * R * nrec * 16);
    const size_t ws = mudiff_grad_workspace_size(H.h, R, nrec, 20, 0);
    void* w = dev.get(ws);
    double* loss = (double*)dev.get(16);
    double* dc = (double*)dev.get(b.M() * 16);
    double* dr = (double*)dev.get(b.M() * 8);
    double* dk = (double*)dev.get(16);
    STATUS(mudiff_grad(H.h, R, betad, nrec, thd, target, 20, 1e-10, 500, 0, w, ws, loss, dc, dr, dk,
                       nullptr),
           MUDIFF_OK);
    HIPCHK(hipDeviceSynchronize());
    for (double v : fetch<double>(dr, b.M())) EXPECT(std::isfinite(v), "radius gradient");
  }
}

// Mixed orders with the circulant flag: MFMA and circulant applies, tiles,
// profiling, lockstep GMRES with graphs and a straggler.
static void gpu_circulant(std::mt19937_64& g) {
  Dev dev;
  Batch b;
  add_instance(b, g, 30, 3.2, 0.3, 1.0, 6.0, 4, -1);
  add_instance(b, g, 10, 2.2, 0.5, 0.9, 1.0, 6, -1);
  add_instance(b, g, 18, 4.0, 0.2, 0.8, 9.0, 3, -1);
  add_instance(b, g, 1, 3.0, 0.7, 0.7, 6.0, 0, 6);
  Handle H;
  make(H, dev, b, MUDIFF_TABLES_CIRCULANT);
  int64_t far = 0, near = 0;
  int Lmax = 0;
  STATUS(mudiff_circulant_info(H.h, &far, &near, &Lmax), MUDIFF_OK);
  EXPECT(far > 0 && near > 0 && Lmax > 0, "classification %lld %lld %d", (long long)far,
         (long long)near, Lmax);

  for (int R : {8, 13, 40, 64}) {
    char msg[96];
    std::snprintf(msg, sizeof msg, "mixed batch R = %d: autotuned, direct, circulant, every tile", R);
    step(msg);
    const auto x = random_vec(g, (size_t)R * H.total);
    const auto y_auto = apply(H, dev, R, x, MUDIFF_OP_A);
    STATUS(mudiff_set_circulant(H.h, R, 0), MUDIFF_OK);
    const auto y_dir = apply(H, dev, R, x, MUDIFF_OP_A);
    STATUS(mudiff_set_circulant(H.h, R, 1), MUDIFF_OK);
    const auto y_circ = apply(H, dev, R, x, MUDIFF_OP_A);
    EXPECT(rel_diff(y_auto, y_dir) < 1e-12 && rel_diff(y_circ, y_dir) < 1e-12,
           "forms disagree at R=%d: %g %g", R, rel_diff(y_auto, y_dir), rel_diff(y_circ, y_dir));
    int kind = -1, ct = 0, rp = 0, qs = 0, th = 0;
    float ms = 0;
    STATUS(mudiff_apply_config(H.h, R, &kind, &ct, &rp, &qs, &th, &ms), MUDIFF_OK);
    EXPECT(kind == 3, "circulant kind at R=%d: %d", R, kind);
    static const int tiles[][6] = {{64, 64, 16, 1, 256, 4},  {64, 64, 16, 2, 256, 4},
                                   {64, 32, 32, 2, 256, 4},  {128, 32, 16, 3, 512, 4},
                                   {64, 32, 16, 3, 256, 4},  {128, 16, 16, 2, 256, 4},
                                   {128, 16, 16, 3, 256, 4}, {128, 8, 16, 2, 256, 4},
                                   {64, 8, 16, 2, 256, 4},   {128, 32, 8, 3, 512, 4},
                                   {128, 64, 8, 3, 512, 4},  {128, 32, 8, 2, 1024, 4},
                                   {256, 32, 8, 2, 512, 4},  {128, 8, 8, 2, 256, 4},
                                   {128, 32, 8, 2, 512, 3},  {128, 64, 8, 2, 512, 3},
                                   {128, 16, 8, 2, 256, 3},  {64, 32, 8, 2, 256, 3}};
    for (const auto& tile : tiles) {
      const int st = mudiff_set_circulant_tile(H.h, R, tile[0], tile[1], tile[2], tile[3], tile[4],
                                               tile[5]);
      if (st != MUDIFF_OK) continue;  // not a candidate for this R
      const auto y = apply(H, dev, R, x, MUDIFF_OP_A);
      EXPECT(rel_diff(y, y_dir) < 1e-12, "tile %dx%d (%d products) at R=%d", tile[0], tile[1], tile[5], R);
      int r2 = 0, c2 = 0, k2 = 0, s2 = 0, t2 = 0, m2 = 0;
      STATUS(mudiff_circulant_tile(H.h, R, &r2, &c2, &k2, &s2, &t2, &m2), MUDIFF_OK);
      EXPECT(r2 == tile[0] && c2 == tile[1] && m2 == tile[5], "tile readback");
    }
    STATUS(mudiff_set_circulant_tile(H.h, R, 48, 48, 16, 2, 256, 4), MUDIFF_ERR_INVALID);
    STATUS(mudiff_set_circulant_tile(H.h, R, 128, 32, 8, 2, 512, 2), MUDIFF_ERR_INVALID);
    STATUS(mudiff_set_apply_config(H.h, R, 1, 8, 32, 512), MUDIFF_OK);
    const auto y_cfg = apply(H, dev, R, x, MUDIFF_OP_A);
    EXPECT(rel_diff(y_cfg, y_dir) < 1e-12, "apply config at R=%d", R);
    STATUS(mudiff_set_apply_config(H.h, R, 3, 1, 0, 256), MUDIFF_ERR_INVALID);
    STATUS(mudiff_matvec_noalloc(H.h, R, dev.get(16), dev.get(16), 1, nullptr), MUDIFF_ERR_INVALID);
  }

  step("mixed batch: phase profile");
  {
    const int R = 16;
    STATUS(mudiff_set_circulant(H.h, R, 1), MUDIFF_OK);
    const auto x = random_vec(g, (size_t)R * H.total);
    (void)apply(H, dev, R, x, MUDIFF_OP_A);  // plan and tiles first
    STATUS(mudiff_profile_begin(H.h, 3), MUDIFF_OK);
    for (int i = 0; i < 5; ++i) (void)apply(H, dev, R, x, MUDIFF_OP_L);
    int n = 0;
    double ms[MUDIFF_N_PHASES];
    STATUS(mudiff_profile_end(H.h, &n, ms), MUDIFF_OK);
    EXPECT(n == 3, "profiled applies %d", n);
    STATUS(mudiff_profile_end(H.h, &n, ms), MUDIFF_OK);  // nothing recorded since
    EXPECT(n == 0, "second profile end %d", n);
  }

  step("mixed batch: lockstep, block and s-step GMRES, circulant form, eager then graph");
  {
    const int R = 8;
    std::vector<double> beta((size_t)b.B() * R);
    for (size_t i = 0; i < beta.size(); ++i) beta[i] = 0.37 * (double)i;
    double* betad = dev.put(beta);
    std::vector<int32_t> it0, its0;
    const int ssf = (int)(MUDIFF_SSTEP | MUDIFF_SSTEP_SIZE(5));
    for (int flags : {0, (int)MUDIFF_GRAPH, (int)(MUDIFF_BLOCK | MUDIFF_BLOCK_SIZE(4)), ssf,
                      ssf | (int)MUDIFF_GRAPH}) {
      const size_t ws = mudiff_gmres_workspace_size(H.h, R, 30, flags);
      void* w = dev.get(ws);
      void* rho = dev.get((size_t)R * H.total * 16);
      int32_t* fl = (int32_t*)dev.get(b.B() * R * 4);
      int32_t* it = (int32_t*)dev.get(b.B() * R * 4);
      double* rr = (double*)dev.get(b.B() * R * 8);
      STATUS(mudiff_gmres(H.h, R, betad, nullptr, rho, 30, 1e-12, 3000, flags, w, ws, fl, rr, it,
                          nullptr, nullptr),
             MUDIFF_OK);
      HIPCHK(hipDeviceSynchronize());
      for (int32_t f : fetch<int32_t>(fl, b.B() * R)) EXPECT(f == 0, "gmres flag %d (flags %d)", f, flags);
      const auto its = fetch<int32_t>(it, b.B() * R);
      std::vector<int32_t>& ref = (flags & MUDIFF_SSTEP) ? its0 : it0;
      if (flags & MUDIFF_BLOCK) continue;
      if (ref.empty())
        ref = its;
      else
        EXPECT(its == ref, "graph replay iteration counts (flags %d)", flags);
    }
  }
}

// Many easy instances and one hard one: the straggler phase of lockstep GMRES.
static void gpu_straggler(std::mt19937_64& g) {
  step("straggler phase: 31 easy instances and one hard one, R = 8");
  Dev dev;
  Batch b;
  for (int i = 0; i < 32; ++i) {
    if (i == 16)
      add_instance(b, g, 26, 3.0, 0.5, 1.0, 6.0, 4, -1);
    else
      add_instance(b, g, 4, 20.0, 0.3, 0.5, 2.0, 3, -1);
  }
  Handle H;
  make(H, dev, b, MUDIFF_TABLES_CIRCULANT);
  const int R = 8;
  std::vector<double> beta((size_t)b.B() * R, 0.3);
  double* betad = dev.put(beta);
  const size_t ws = mudiff_gmres_workspace_size(H.h, R, 10, 0);
  void* w = dev.get(ws);
  void* rho = dev.get((size_t)R * H.total * 16);
  int32_t* fl = (int32_t*)dev.get(b.B() * R * 4);
  double* rr = (double*)dev.get(b.B() * R * 8);
  int32_t* it = (int32_t*)dev.get(b.B() * R * 4);
  STATUS(mudiff_gmres(H.h, R, betad, nullptr, rho, 10, 1e-12, 5000, 0, w, ws, fl, rr, it, nullptr,
                      nullptr),
         MUDIFF_OK);
  HIPCHK(hipDeviceSynchronize());
  for (int32_t f : fetch<int32_t>(fl, b.B() * R)) EXPECT(f == 0, "straggler flag %d", f);
}

static void gpu_handle_free(std::mt19937_64& g) {
  step("time reversal: T, Jacobi eigen-decomposition, Herglotz waves; probes");
  Dev dev;
  for (int n : {5, 40}) {
    const int m = n + 3;
    const auto X = random_vec(g, (size_t)n * m);
    cd* Xd = dev.put(X);
    void* T = dev.get((size_t)n * n * 16);
    STATUS(mudiff_tro(n, m, Xd, T, nullptr), MUDIFF_OK);
    const size_t ws = mudiff_tro_eigh_workspace_size(n, m);
    void* w = dev.get(ws);
    double* ev = (double*)dev.get(n * 8);
    void* V = dev.get((size_t)n * n * 16);
    int32_t sweeps = 0;
    STATUS(mudiff_tro_eigh(n, m, Xd, ev, V, 30, 1e-14, w, ws, &sweeps, nullptr), MUDIFF_OK);
    EXPECT(sweeps > 0, "sweeps %d", sweeps);
    std::vector<double> al(n);
    for (int j = 0; j < n; ++j) al[j] = 2 * M_PI * j / n;
    double* ald = dev.put(al);
    std::vector<double> pts{0.0, 0.0, 3.0, -1.0};
    double* ptd = dev.put(pts);
    void* u = dev.get((size_t)2 * 2 * 16);
    STATUS(mudiff_herglotz(n, ald, 2, V, 6.28, 2 * M_PI / n, 2, ptd, u, nullptr), MUDIFF_OK);
    HIPCHK(hipDeviceSynchronize());
  }
  for (int kind : {MUDIFF_PROBE_FP64_FMA, MUDIFF_PROBE_FP64_MFMA, MUDIFF_PROBE_COPY}) {
    const size_t bytes = kind == MUDIFF_PROBE_COPY ? (size_t)64 << 20 : 0;
    const size_t ws = mudiff_probe_workspace_size(kind, bytes);
    void* w = dev.get(ws);
    double rate = 0;
    STATUS(mudiff_probe(kind, bytes, w, ws, &rate, nullptr), MUDIFF_OK);
    EXPECT(rate > 0, "probe %d", kind);
  }
}

int main(int argc, char** argv) {
  const char* mode = argc > 1 ? argv[1] : "cpu";
  cpu_mode();
  if (std::strcmp(mode, "gpu") == 0) {
    std::mt19937_64 g(20240901);
    gpu_uniform(g);
    gpu_circulant(g);
    gpu_straggler(g);
    gpu_handle_free(g);
  }
  std::printf("%s mode: %d failure(s)\n", mode, g_fail);
  std::fflush(stdout);  // the leak check may end the process without flushing
  // Leaks are checked here rather than at exit: once a device has been used, the
  // ROCm runtime's own finalizers free memory after the sanitizer has released its
  // device-side allocator, which trips an internal check of the sanitizer.  Every
  // handle and buffer of the library has been released by now, so the explicit
  // check covers the same allocations; then the process leaves without running
  // the runtime's finalizers.
  __lsan_do_leak_check();
  std::fflush(stderr);
  _exit(g_fail ? 1 : 0);
}
