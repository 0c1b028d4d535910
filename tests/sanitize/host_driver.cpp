// Drives the host logic of the C ABI (parameter validation, workspace
// layouts, batch headers, the surrogate's workspace carve, argument checks
// of every handle entry point, the per-thread error text) in a build of the
// library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// Every call here returns before the library touches the HIP runtime or any
// device memory: the checks it exercises all precede the first HIP call of
// their entry point, so the program behaves the same with or without a GPU
// and never launches a kernel.  Pointers passed as "device workspace" are
// never dereferenced by those paths.
//
// PLANT=1 (a compile-time switch) adds one read past the end of a heap
// buffer, so that a test can show the sanitizer is live in the sanitized binary.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <thread>
#include <vector>

#include "cosmolat.h"
#include "surrogate.h"

static int failures = 0;
static int checks = 0;

static void expect(bool ok, const char* what, int line) {
  ++checks;
  if (!ok) {
    std::fprintf(stderr, "line %d: %s (last error: %s)\n", line, what, lattice_last_error());
    ++failures;
  }
}
#define EXPECT(c) expect((c), #c, __LINE__)

// a failing call must also leave a message
#define EXPECT_RC(call, code)                                           \
  do {                                                                  \
    const int rc_ = (call);                                             \
    expect(rc_ == (code), #call " == " #code, __LINE__);                \
    if ((code) != LAT_OK) expect(std::strlen(lattice_last_error()) > 0, \
                                 "error text after " #call, __LINE__);  \
  } while (0)

static lattice_params params(int model, int nf, int N, int integ, int prec) {
  lattice_params p;
  std::memset(&p, 0, sizeof p);
  p.model = model; p.nf = nf; p.N = N; p.integrator = integ; p.precision = prec;
  p.expansion = 1; p.ic = LAT_IC_VACUUM; p.seed = 7;
  p.kIR = 0.6; p.dt = 0.005; p.alpha = 1.0; p.fstar_over_mp = 0.1; p.omega_over_f = 0.01;
  p.lambda = 1.0; p.q = 100.0; p.e = 0.5; p.g = 0.2; p.a0 = 1.0;
  p.phi0[0] = 1.0;
  return p;
}

struct Model { int model, nf; };
static const Model kModels[] = {{LAT_MODEL_SCALAR, 1}, {LAT_MODEL_SCALAR, 2}, {LAT_MODEL_U1, 2},
                                {LAT_MODEL_U1_NC, 2}, {LAT_MODEL_SU2U1, 4}};

static void workspace_sizes() {
  for (const Model& m : kModels)
    for (int prec : {LAT_FP64, LAT_FP32})
      for (int integ : {LAT_LF2, LAT_VV2, LAT_VV4, LAT_VV10}) {
        size_t prev = 0;
        for (int N : {32, 64, 96, 256, 1024}) {
          lattice_params p = params(m.model, m.nf, N, integ, prec);
          size_t b = 0;
          EXPECT_RC(lattice_workspace_size(&p, &b), LAT_OK);
          // at least the fields and momenta, in the storage precision
          const size_t V = (size_t)N * N * N;
          EXPECT(b >= 2 * (size_t)m.nf * V * (prec == LAT_FP32 ? 4 : 8));
          EXPECT(b > prev);
          EXPECT(b % 256 == 0);
          prev = b;
        }
      }
}

static void invalid_params() {
  const lattice_params ok = params(LAT_MODEL_SCALAR, 2, 64, LAT_VV2, LAT_FP32);
  const double nan = std::numeric_limits<double>::quiet_NaN();
  std::vector<lattice_params> bad;
  auto add = [&](auto edit) { lattice_params p = ok; edit(p); bad.push_back(p); };
  add([](lattice_params& p) { p.model = 7; });
  add([](lattice_params& p) { p.model = -1; });
  add([](lattice_params& p) { p.nf = 3; });
  add([](lattice_params& p) { p.nf = 0; });
  add([](lattice_params& p) { p.model = LAT_MODEL_U1; p.nf = 1; });
  add([](lattice_params& p) { p.model = LAT_MODEL_SU2U1; p.nf = 2; });
  add([](lattice_params& p) { p.model = LAT_MODEL_SU2U1; p.nf = 4; p.g = 0.0; });
  add([nan](lattice_params& p) { p.model = LAT_MODEL_SU2U1; p.nf = 4; p.e = nan; });
  add([](lattice_params& p) { p.N = 0; });
  add([](lattice_params& p) { p.N = -32; });
  add([](lattice_params& p) { p.N = 33; });
  add([](lattice_params& p) { p.N = 2048; });
  add([](lattice_params& p) { p.N = std::numeric_limits<int32_t>::max(); });
  add([](lattice_params& p) { p.integrator = -1; });
  add([](lattice_params& p) { p.integrator = LAT_VV10 + 1; });
  add([](lattice_params& p) { p.precision = 2; });
  add([](lattice_params& p) { p.kIR = 0.0; });
  add([nan](lattice_params& p) { p.kIR = nan; });
  add([](lattice_params& p) { p.dt = -0.005; });
  add([nan](lattice_params& p) { p.dt = nan; });
  add([](lattice_params& p) { p.dt = 1.0; });   // above the Courant bound dx/sqrt(3)
  add([](lattice_params& p) { p.ic = 9; });
  add([](lattice_params& p) { p.fstar_over_mp = 0.0; });
  add([](lattice_params& p) { p.a0 = 0.0; });
  add([nan](lattice_params& p) { p.a0 = nan; });
  for (const lattice_params& p : bad) {
    size_t b = 12345;
    EXPECT_RC(lattice_workspace_size(&p, &b), LAT_EINVAL);
    EXPECT(b == 12345);
    lattice_t* h = nullptr;
    char ws[512];
    EXPECT_RC(lattice_init(&p, ws, sizeof ws, nullptr, &h), LAT_EINVAL);
    EXPECT(h == nullptr);
  }
  size_t b = 0;
  EXPECT_RC(lattice_workspace_size(nullptr, &b), LAT_EINVAL);
  EXPECT_RC(lattice_workspace_size(&ok, nullptr), LAT_EINVAL);
}

static void init_argument_checks() {
  const lattice_params p = params(LAT_MODEL_U1, 2, 64, LAT_LF2, LAT_FP32);
  size_t need = 0;
  EXPECT_RC(lattice_workspace_size(&p, &need), LAT_OK);
  alignas(256) static char ws[1024];
  lattice_t* h = nullptr;
  EXPECT_RC(lattice_init(nullptr, ws, need, nullptr, &h), LAT_EINVAL);
  EXPECT_RC(lattice_init(&p, nullptr, need, nullptr, &h), LAT_EINVAL);
  EXPECT_RC(lattice_init(&p, ws, need, nullptr, nullptr), LAT_EINVAL);
  EXPECT_RC(lattice_init(&p, ws, need - 1, nullptr, &h), LAT_ENOMEM);
  EXPECT(std::string(lattice_last_error()).find(std::to_string(need)) != std::string::npos);
  EXPECT_RC(lattice_init(&p, ws + 8, need, nullptr, &h), LAT_EINVAL);   // not 256-byte aligned
  EXPECT(h == nullptr);
}

static void batch_checks() {
  std::vector<lattice_params> runs;
  size_t sum = 0;
  for (int N : {32, 64, 96}) {
    lattice_params p = params(LAT_MODEL_SCALAR, 2, N, LAT_VV2, LAT_FP32);
    p.q = 10.0 * N;
    p.seed = 100 + N;
    size_t b = 0;
    EXPECT_RC(lattice_workspace_size(&p, &b), LAT_OK);
    sum += b;
    runs.push_back(p);
  }
  size_t total = 0;
  EXPECT_RC(lattice_batch_workspace_size(runs.data(), (int)runs.size(), &total), LAT_OK);
  EXPECT(total > sum);
  // a large ensemble: the header's tile tables grow with it
  std::vector<lattice_params> many(2000, params(LAT_MODEL_SCALAR, 2, 256, LAT_VV4, LAT_FP32));
  size_t big = 0;
  EXPECT_RC(lattice_batch_workspace_size(many.data(), (int)many.size(), &big), LAT_OK);
  EXPECT(big > 2000 * (size_t)256 * 256 * 256 * 16);

  EXPECT_RC(lattice_batch_workspace_size(nullptr, 3, &total), LAT_EINVAL);
  EXPECT_RC(lattice_batch_workspace_size(runs.data(), 0, &total), LAT_EINVAL);
  EXPECT_RC(lattice_batch_workspace_size(runs.data(), -4, &total), LAT_EINVAL);
  EXPECT_RC(lattice_batch_workspace_size(runs.data(), 3, nullptr), LAT_EINVAL);
  auto bad = [&](auto edit) {
    std::vector<lattice_params> r = runs;
    edit(r[2]);
    size_t b = 0;
    EXPECT_RC(lattice_batch_workspace_size(r.data(), (int)r.size(), &b), LAT_EINVAL);
    lattice_batch_t* B = nullptr;
    alignas(256) static char ws[512];
    EXPECT_RC(lattice_batch_init(r.data(), (int)r.size(), ws, sizeof ws, nullptr, &B), LAT_EINVAL);
    EXPECT(B == nullptr);
  };
  bad([](lattice_params& p) { p.nf = 1; });
  bad([](lattice_params& p) { p.precision = LAT_FP64; });
  bad([](lattice_params& p) { p.integrator = LAT_VV4; });
  bad([](lattice_params& p) { p.integrator = LAT_LF2; });
  bad([](lattice_params& p) { p.dt = 0.004; });
  bad([](lattice_params& p) { p.model = LAT_MODEL_U1; });
  bad([](lattice_params& p) { p.N = 48; });

  alignas(256) static char ws[1024];
  lattice_batch_t* B = nullptr;
  EXPECT_RC(lattice_batch_init(runs.data(), 3, nullptr, total, nullptr, &B), LAT_EINVAL);
  EXPECT_RC(lattice_batch_init(runs.data(), 3, ws, total, nullptr, nullptr), LAT_EINVAL);
  EXPECT_RC(lattice_batch_init(runs.data(), 3, ws, total - 1, nullptr, &B), LAT_ENOMEM);
  EXPECT_RC(lattice_batch_init(runs.data(), 3, ws + 64, total, nullptr, &B), LAT_EINVAL);
  EXPECT(B == nullptr);
}

static surrogate_params surr() {
  surrogate_params p;
  std::memset(&p, 0, sizeof p);
  p.max_batch = 256;
  p.beta1 = 0.9; p.beta2 = 0.999; p.eps = 1e-8;
  for (int c = 0; c < SURR_N_IN; ++c) { p.in_scale[c] = 1.0f; p.enc_freq[c] = 0.5f; }
  for (int c = 0; c < SURR_N_OUT; ++c) p.out_scale[c] = 1.0f;
  return p;
}

static void surrogate_checks() {
  size_t prev = 0;
  for (int mb : {64, 256, 4096, 16384}) {
    surrogate_params p = surr();
    p.max_batch = mb;
    size_t b = 0;
    EXPECT_RC(surrogate_workspace_size(&p, &b), LAT_OK);
    // master weights, two Adam moments and the gradient, FP32
    EXPECT(b >= 4 * (size_t)SURR_NPARAMS * 4);
    EXPECT(b > prev);
    prev = b;
  }
  const float inf = std::numeric_limits<float>::infinity(), fnan = std::numeric_limits<float>::quiet_NaN();
  std::vector<surrogate_params> bad;
  auto add = [&](auto edit) { surrogate_params p = surr(); edit(p); bad.push_back(p); };
  add([](surrogate_params& p) { p.max_batch = 0; });
  add([](surrogate_params& p) { p.max_batch = 63; });
  add([](surrogate_params& p) { p.max_batch = 100; });
  add([](surrogate_params& p) { p.max_batch = 16384 + 64; });
  add([](surrogate_params& p) { p.max_batch = -64; });
  add([](surrogate_params& p) { p.beta1 = 1.0; });
  add([](surrogate_params& p) { p.beta2 = -0.1; });
  add([](surrogate_params& p) { p.eps = 0.0; });
  add([](surrogate_params& p) { p.in_scale[1] = 0.0f; });
  add([inf](surrogate_params& p) { p.in_shift[0] = inf; });
  add([fnan](surrogate_params& p) { p.enc_freq[1] = fnan; });
  add([inf](surrogate_params& p) { p.out_scale[63] = inf; });
  add([fnan](surrogate_params& p) { p.out_shift[10] = fnan; });
  for (const surrogate_params& p : bad) {
    size_t b = 777;
    EXPECT_RC(surrogate_workspace_size(&p, &b), LAT_EINVAL);
    EXPECT(b == 777);
    surrogate_t* h = nullptr;
    alignas(256) static char ws[512];
    EXPECT_RC(surrogate_init(&p, ws, sizeof ws, nullptr, &h), LAT_EINVAL);
    EXPECT(h == nullptr);
  }
  const surrogate_params p = surr();
  size_t need = 0;
  EXPECT_RC(surrogate_workspace_size(&p, &need), LAT_OK);
  alignas(256) static char ws[512];
  surrogate_t* h = nullptr;
  EXPECT_RC(surrogate_workspace_size(nullptr, &need), LAT_EINVAL);
  EXPECT_RC(surrogate_workspace_size(&p, nullptr), LAT_EINVAL);
  EXPECT_RC(surrogate_init(&p, nullptr, need, nullptr, &h), LAT_EINVAL);
  EXPECT_RC(surrogate_init(&p, ws, need, nullptr, nullptr), LAT_EINVAL);
  EXPECT_RC(surrogate_init(&p, ws, need - 1, nullptr, &h), LAT_ENOMEM);
  EXPECT(h == nullptr);
}

static void null_handles() {
  double d[4] = {0, 0, 0, 0};
  float f[4] = {0, 0, 0, 0};
  int32_t i32[4] = {0, 0, 0, 0};
  int64_t i64[4] = {0, 0, 0, 0};
  int nb = 0;
  void* ptr = nullptr;
  lattice_obs obs;
  lattice_scalars sc;
  std::memset(&sc, 0, sizeof sc);
  lattice_t* run = nullptr;
  EXPECT_RC(lattice_set_state(nullptr, d, d, nullptr, nullptr, &sc), LAT_EINVAL);
  EXPECT_RC(lattice_get_state(nullptr, d, d, nullptr, nullptr, &sc), LAT_EINVAL);
  EXPECT_RC(lattice_step(nullptr, 1), LAT_EINVAL);
  EXPECT_RC(lattice_energies(nullptr, &obs), LAT_EINVAL);
  EXPECT_RC(lattice_energies_noalloc(nullptr, &obs), LAT_EINVAL);
  EXPECT_RC(lattice_spectrum(nullptr, 0, 4, d, d, d, i64, &nb), LAT_EINVAL);
  EXPECT_RC(lattice_spectrum_logk(nullptr, 0, 64, f), LAT_EINVAL);
  EXPECT_RC(lattice_get_tiling(nullptr, i32, i32 + 1, i32 + 2, i32 + 3), LAT_EINVAL);
  EXPECT_RC(lattice_set_tiling(nullptr, 32, 8, 2, 1), LAT_EINVAL);
  EXPECT_RC(lattice_pass_timer(nullptr, 10), LAT_EINVAL);
  EXPECT_RC(lattice_pass_timer_read(nullptr, d, i64), LAT_EINVAL);
  EXPECT_RC(lattice_field_device_ptr(nullptr, 0, &ptr, i32), LAT_EINVAL);
  EXPECT_RC(lattice_destroy(nullptr), LAT_OK);
  EXPECT_RC(lattice_batch_step(nullptr, 1), LAT_EINVAL);
  EXPECT_RC(lattice_batch_energies(nullptr, &obs), LAT_EINVAL);
  EXPECT_RC(lattice_batch_run(nullptr, 0, &run), LAT_EINVAL);
  EXPECT_RC(lattice_batch_get_tiling(nullptr, i32, i32 + 1, i32 + 2, i32 + 3), LAT_EINVAL);
  EXPECT_RC(lattice_batch_set_tiling(nullptr, 32, 8, 2, 1), LAT_EINVAL);
  EXPECT_RC(lattice_batch_use_graph(nullptr, 1), LAT_EINVAL);
  EXPECT_RC(lattice_batch_destroy(nullptr), LAT_OK);
  EXPECT_RC(surrogate_set_weights(nullptr, f), LAT_EINVAL);
  EXPECT_RC(surrogate_get_weights(nullptr, f), LAT_EINVAL);
  EXPECT_RC(surrogate_fit_output_scale(nullptr, f, 4, d, d), LAT_EINVAL);
  EXPECT_RC(surrogate_loss_grad(nullptr, f, f, nullptr, 1, f, d), LAT_EINVAL);
  EXPECT_RC(surrogate_train_epoch(nullptr, f, f, i32, 1, 1e-3, d), LAT_EINVAL);
  EXPECT_RC(surrogate_predict(nullptr, f, 1, f), LAT_EINVAL);
  EXPECT_RC(surrogate_use_graph(nullptr, 1), LAT_EINVAL);
  EXPECT_RC(surrogate_destroy(nullptr), LAT_OK);
}

// the error text belongs to the calling thread
static void error_text_per_thread() {
  std::atomic<int> arrived{0};
  std::string seen[2];
  auto worker = [&](int t) {
    lattice_params p = params(LAT_MODEL_SCALAR, 2, 64, LAT_VV2, LAT_FP32);
    if (t == 0) p.N = 33; else p.model = 9;
    size_t b = 0;
    lattice_workspace_size(&p, &b);
    arrived.fetch_add(1);
    while (arrived.load() < 2) std::this_thread::yield();
    seen[t] = lattice_last_error();
  };
  std::thread a(worker, 0), b(worker, 1);
  a.join();
  b.join();
  EXPECT(seen[0].find("N must be") != std::string::npos);
  EXPECT(seen[1].find("unknown model") != std::string::npos);
}

#ifndef PLANT
#define PLANT 0
#endif

int main() {
  if (PLANT == 1) {
    double* buf = new double[4]();
    double* volatile opaque = buf;   // hides the size from compile-time checks
    const double past = opaque[4];
    std::printf("%g\n", past);
    delete[] buf;
  }
  workspace_sizes();
  invalid_params();
  init_argument_checks();
  batch_checks();
  surrogate_checks();
  null_handles();
  error_text_per_thread();
  if (failures) {
    std::fprintf(stderr, "%d of %d checks failed\n", failures, checks);
    return 1;
  }
  std::printf("host driver ok: %d checks\n", checks);
  return 0;
}
