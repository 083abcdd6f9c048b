// libdda host driver: the C ABI of include/dda.h.
//
// Every step of the DDA matrix-vector product, the spectrum build, the Krylov
// solvers, the refinement loop, the cross sections and the gradient runs in
// the HIP kernels of kernels_fft.hpp / kernels_solver.hpp; this file only
// plans sizes, owns device memory and enqueues launches on the caller's
// stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>
#include <atomic>
#include <sstream>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <string>
#include <vector>

#include "dda.h"
#include "common.hpp"
#include "kernels_fft.hpp"
#include "kernels_solver.hpp"
#include "kernels_krylov.hpp"
#include "fft_fast.hpp"
#include "fft_reg.hpp"
#include "kernels_farfield.hpp"

using namespace dda;

// ----------------------------------------------------------------------------
// errors
// ----------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(x)                                                                         \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess) return fail(DDA_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)
#define CHK(x)              \
  do {                      \
    int rc_ = (x);          \
    if (rc_ != DDA_OK) return rc_; \
  } while (0)
#define LAUNCHCHK() HIPCHK(hipGetLastError())

// ----------------------------------------------------------------------------
// device buffers
// ----------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t b) {
    if (b <= bytes && p) return DDA_OK;
    release();
    if (b == 0) return DDA_OK;
    if (hipMalloc(&p, b) != hipSuccess) {
      p = nullptr;
      bytes = 0;
      (void)hipGetLastError();
      return fail(DDA_ENOMEM, "hipMalloc(%zu) failed", b);
    }
    bytes = b;
    return DDA_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T* as() const { return reinterpret_cast<T*>(p); }
  ~DevBuf() { release(); }
};

// ----------------------------------------------------------------------------
// FFT planning
// ----------------------------------------------------------------------------
static bool smooth235(int n) {
  for (int f : {2, 3, 5})
    while (n % f == 0) n /= f;
  return n == 1;
}

// lengths with a register-resident kernel (fft_fast.hpp)
#define DDA_FAST_SIZES(X) X(16) X(32) X(64) X(128) X(256) X(512) X(24) X(48) X(96) X(192) X(384)
static bool fast_size(int n) {
  switch (n) {
#define DDA_CASE(N) case N:
    DDA_FAST_SIZES(DDA_CASE)
#undef DDA_CASE
    return true;
    default:
      return false;
  }
}
// ... and those with register-resident y passes and transposing x passes
// (the z-contiguous schedule): the above and 5 2^k, 25 2^k
#define DDA_FAST_Y_SIZES(X) DDA_FAST_SIZES(X) X(80) X(160) X(320) X(100) X(200) X(400)
static bool fast_y_size(int n) {
  switch (n) {
#define DDA_CASE(N) case N:
    DDA_FAST_Y_SIZES(DDA_CASE)
#undef DDA_CASE
    return true;
    default:
      return false;
  }
}

// lengths with a two-level z pass (fft_reg.hpp) in precision R
template <typename R = float>
static bool z2_size(int n) {
  switch (n) {
#define DDA_CASE(N) \
  case N:           \
    return Z2Shape<R, N, true>::ok;
    DDA_FAST_SIZES(DDA_CASE)
#undef DDA_CASE
    default:
      return false;
  }
}

// columns per tile of the tile-blocked layout (and of its two-level z pass)
template <typename R>
static int z2_cols(int n) {
  switch (n) {
#define DDA_CASE(N) \
  case N:           \
    return Z2Shape<R, N, true>::C;
    DDA_FAST_SIZES(DDA_CASE)
#undef DDA_CASE
    default:
      return 1;
  }
}

// Padded FFT length for a lattice extent: any n'' >= 2n - 1 embeds the
// Toeplitz matrix in a circulant (Sec. 3).  Take the smallest 2^a 3^b 5^c
// length, or the smallest length with a register-resident kernel when it is
// at most 30% longer (for y, `yax`: a register-resident y pass).
static int fft_size_at_least(int m, bool yax = false) {
  auto fast = [yax](int v) { return yax ? fast_y_size(v) : fast_size(v); };
  int n = std::max(1, m);
  while (!smooth235(n)) ++n;
  int f = std::max(1, m);
  while (!fast(f) && f < 4 * n) ++f;
  if (fast(f) && 10 * f <= 13 * n) return f;  // register-resident kernels beat generic ones up to +30%
  return n;
}

static FftDesc make_desc(int n) {
  FftDesc d;
  d.n = n;
  d.nst = 0;
  int r = n;
  int twos = 0;
  while (r % 2 == 0) { r /= 2; ++twos; }
  while (twos >= 3) { d.radix[d.nst++] = 8; twos -= 3; }
  if (twos == 2) d.radix[d.nst++] = 4;
  if (twos == 1) d.radix[d.nst++] = 2;
  while (r % 5 == 0) { r /= 5; d.radix[d.nst++] = 5; }
  while (r % 3 == 0) { r /= 3; d.radix[d.nst++] = 3; }
  return d;
}

static int pow2_floor(long v) {
  int p = 1;
  while ((long)p * 2 <= v) p *= 2;
  return p;
}

// ----------------------------------------------------------------------------
// handles
// ----------------------------------------------------------------------------
// Optional per-pass kernel timing: HIP events recorded on the launch stream
// around every matrix-vector pass.
// PASS_MATVEC brackets the whole product (every pass and the gaps between).
enum { PASS_YFWD = 0, PASS_XFWD, PASS_ZMUL, PASS_XINV, PASS_YINV, PASS_XYFWD, PASS_XYINV, PASS_MATVEC, PASS_PER_PREC };
static_assert(PASS_PER_PREC == DDA_PROF_SLOTS, "profiling slots of the header");
constexpr int PASS_COUNT = 2 * PASS_PER_PREC;  // second half: FP32 vectors

// Device scratch of the allocation-free product (dda_matvec_noalloc): the
// orientation factors and the FFT workspaces of one call.  One copy per
// device, held until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns with that device current (dda_open).
static constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct dda_lib {
  int device = 0;
  unsigned char* scratch_dev = nullptr;  // this device's copy of `scratch`
  std::string tune_path;
  std::map<std::string, int> tuned;  // schedule per (lattice, padding, nrhs, precision)
  std::mutex tune_mu;                // guards `tuned` and the tune file (batch workers)
  std::vector<hipStream_t> workers;  // streams of dda_batch_solve's workers
  int prof = 0;  // 0 off, 1 every pass and product, 2 whole products only
  std::vector<hipEvent_t> ev_pool;                 // free events
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;  // (pass, start, stop)
  double prof_ms[PASS_COUNT] = {0};
  long prof_n[PASS_COUNT] = {0};
};

static hipEvent_t take_event(dda_lib* l) {
  if (!l->ev_pool.empty()) {
    hipEvent_t e = l->ev_pool.back();
    l->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct PassTimer {
  dda_lib* l;
  int pass;
  hipStream_t st;
  bool on;
  hipEvent_t a = nullptr, b = nullptr;
  PassTimer(dda_lib* l_, int p, hipStream_t s, bool enabled = true)
      : l(l_), pass(p), st(s), on(enabled && (l_->prof == 1 || (l_->prof == 2 && p % PASS_PER_PREC == PASS_MATVEC))) {
    if (on) {
      a = take_event(l);
      b = take_event(l);
      if (a) (void)hipEventRecord(a, st);
    }
  }
  ~PassTimer() {
    if (on && a && b) {
      (void)hipEventRecord(b, st);
      l->pending.push_back({pass, {a, b}});
    }
  }
};

template <typename R>
struct PrecBufs {
  DevBuf Y;                 // spectrum [6][Ph][Jh][Kh]
  DevBuf Yz;                // the same, z fastest: [6][Jh][Kh][Ph]
  DevBuf tw[3];             // twiddles for K'', J'', P''
  DevBuf a0, a1;            // diagonal alpha^{-1} = a0 + S a1
  DevBuf mt0, mt1;          // composition: the materials' alpha^{-1} = mt0 + S mt1
  DevBuf G1, G2;            // matvec workspaces
  int cap = 0;              // right-hand sides the workspaces hold
  DevBuf vec;               // solver vectors: vec_slots x [vec_cap][3][vec_nd]
  int vec_cap = 0, vec_slots = 0;
  int64_t vec_nd = 0;
};

struct dda_target {
  dda_lib* lib = nullptr;
  int device = 0;  // the library's device, kept so that destruction needs no library
  int K = 0, J = 0, P = 0;
  double kd = 0;
  int Kpp = 0, Jpp = 0, Ppp = 0, Kh = 0, Jh = 0, Ph = 0;
  FftDesc fx{}, fy{}, fz{};
  int64_t nd = 0;
  int occ_words = 0;  // W of the bit-fielded occupancy
  DevBuf occ;    // uint2 [P][J][W] (bits, occupied sites before the word), W = ceil(K / 32)
  DevBuf sites;  // int [nd] linear index
  bool have_alpha = false, have_eps = false, has_a1 = false;
  bool aniso = false;  // the three components' diagonals differ (dda_set_composition)
  // bit-fielded composition (dda_set_composition): material index of entry
  // c N_d + n at 2^mlb bits each; the matrix-vector passes read these and the
  // materials' table instead of per-dipole diagonals
  bool comp_bits = false;
  bool uniform_diag = false;  // one permittivity for every dipole: the passes read a one-entry table
  int mlb = 0;
  DevBuf mbits;
  int prescription = -1;
  DevBuf d0, d1;  // d alpha^{-1} / d eps = d0 + S d1 (FP64)
  PrecBufs<double> p64;
  PrecBufs<float> p32;
  bool spec_ready = false;
  int forced_sched = -1;     // -1: tuned; 0: five passes; D > 0: fused xy passes with split D
  int forced_ylog = -1;      // -1: tuned; L >= 0: y tile 2^L times the default
  int forced_xsel = -1;      // -1: tuned; 0, 1, 2: x-pass rows per block default, half, twice
  int inject_bad_step = 0;   // fault injection: refinement steps applied with the wrong sign
  int inject_breakdown = 0;  // BiCGSTAB inner solves still to start from a zero shadow vector
  int canary = 0;            // dda_matvec fills its workspaces with NaN first (debug)
  int fuse_qmr = 1;          // QMR_sym step fused into the y-forward pass where possible
  int z_rb = 0;              // right-hand sides per block of the two-level z pass (0: by size)
  // dda_matvec_noalloc: FFT workspaces in the device scratch, no profiling
  void* ws_over[2] = {nullptr, nullptr};
  int sched_override = -1;   // autotuner: schedule under trial (-1: none)
  // per-solve scratch
  DevBuf S;       // double [cap]
  DevBuf active;  // int [cap]
  DevBuf active_outer;
  DevBuf state;   // solver states
  DevBuf part;    // reduction partials
  DevBuf part_mv; // partials of the inner products fused into the matvec
  DevBuf scal;    // double [cap] scale factors
  DevBuf tolv;    // double [cap] inner tolerances
  DevBuf outer;   // FP64 outer vectors: E, r, y  (3 x [cap][3][nd])
  DevBuf khat, ehat;
  DevBuf far_dirs, far_part, far_F, far_w, far_tp;  // far-field scratch
  double extent = 0;  // diameter of the occupied sites' bounding box (units of d)
  int scap = 0;
  // LDR orientation factor S per right-hand side of the last dda_solve (the
  // values passed, or those derived from khat/ehat); empty before a solve
  std::vector<double> solve_S;
  std::vector<int> h_active;
  int matvecs = 0;
  // captured inner iteration
  // captured inner iteration, one per vector precision (FP64 index 0, FP32 1):
  // a batched mixed solve can run both kinds of inner solve in one step
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  std::vector<uintptr_t> graph_key[2];
  hipStream_t cap_stream = nullptr;
  ~dda_target() {
    for (hipGraphExec_t g : graph_exec)
      if (g) (void)hipGraphExecDestroy(g);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

template <typename R>
static PrecBufs<R>& bufs(dda_target* t);
template <>
PrecBufs<double>& bufs<double>(dda_target* t) { return t->p64; }
template <>
PrecBufs<float>& bufs<float>(dda_target* t) { return t->p32; }

// the occupancy as the expand / compress passes read it
static OccBits occ_of(const dda_target* t) {
  OccBits o;
  o.words = (const uint2*)t->occ.p;
  o.W = t->occ_words;
  return o;
}

template <typename R>
static std::vector<int> xy_candidates(const dda_target* t);

// ----------------------------------------------------------------------------
// launch helpers
// ----------------------------------------------------------------------------
static const int kThreads = 256;
static const size_t kLdsBudget = 64 * 1024;

template <typename R>
static int launch_contig(const cx<R>* in, cx<R>* out, long nlines, long lin_stride, long lout_stride, int Lin,
                         int Lout, const FftDesc& d, const cx<R>* tw, bool inv, bool mirror, long lines_per_comp,
                         int axis, long lines_per_rhs, const int* active, double scale, hipStream_t st) {
  ContigArgs a;
  a.nlines = nlines;
  a.lin_stride = lin_stride;
  a.lout_stride = lout_stride;
  a.Lin = Lin;
  a.Lout = Lout;
  a.ls = d.n;
  a.lines_per_comp = lines_per_comp > 0 ? lines_per_comp : 1;
  a.axis = axis;
  a.lines_per_rhs = active ? lines_per_rhs : 0;
  a.scale = scale;
  const size_t per = 2 * (size_t)d.n * sizeof(cx<R>);
  int rows = (int)std::max<size_t>(1, std::min<size_t>(64, kLdsBudget / per));
  if (a.lines_per_rhs) {
    while (rows > 1 && a.lines_per_rhs % rows != 0) --rows;
  }
  a.rows = rows;
  const size_t lds = rows * per;
  dim3 grid((unsigned)((nlines + rows - 1) / rows));
  if (inv) {
    if (mirror) hipLaunchKernelGGL((k_lines_contig<R, true, true>), grid, dim3(kThreads), lds, st, in, out, a, d, tw, active);
    else hipLaunchKernelGGL((k_lines_contig<R, true, false>), grid, dim3(kThreads), lds, st, in, out, a, d, tw, active);
  } else {
    if (mirror) hipLaunchKernelGGL((k_lines_contig<R, false, true>), grid, dim3(kThreads), lds, st, in, out, a, d, tw, active);
    else hipLaunchKernelGGL((k_lines_contig<R, false, false>), grid, dim3(kThreads), lds, st, in, out, a, d, tw, active);
  }
  LAUNCHCHK();
  return DDA_OK;
}

template <typename R>
static int tile_width(int NX, int n, int nbuf) {
  const size_t per = (size_t)nbuf * n * sizeof(cx<R>);
  int tx = (int)std::min<size_t>(64, std::max<size_t>(1, kLdsBudget / per));
  tx = pow2_floor(tx);
  while (tx > 1 && tx / 2 >= NX) tx /= 2;
  return tx;
}

template <typename R>
static int launch_strided_mirror(const cx<R>* in, cx<R>* out, StridedArgs a, int NO, int NB, const FftDesc& d,
                                 const cx<R>* tw, hipStream_t st) {
  a.TX = tile_width<R>(a.NX, d.n, 2);
  const size_t lds = 2 * (size_t)d.n * a.TX * sizeof(cx<R>);
  dim3 grid((a.NX + a.TX - 1) / a.TX, NO, NB);
  hipLaunchKernelGGL((k_lines_strided<R, false, true>), grid, dim3(kThreads), lds, st, in, out, a, d, tw);
  LAUNCHCHK();
  return DDA_OK;
}

// ----------------------------------------------------------------------------
// C ABI
// ----------------------------------------------------------------------------
template <typename R>
static int ylog_max(const dda_target* t);

static const char* schedule_missing(int value, int K, int J, int Kpp, int Jpp, int Ppp);

// the captured inner iterations (their launches bake in sizes and addresses)
static void drop_graphs(dda_target* t) {
  for (int g = 0; g < 2; ++g) {
    if (t->graph_exec[g]) (void)hipGraphExecDestroy(t->graph_exec[g]);
    t->graph_exec[g] = nullptr;
    t->graph_key[g].clear();
  }
}

// Padded lengths K'', J'', P'' and what follows from them: half lengths,
// radix plans and the twiddle tables exp(-2 pi i m / n) (host libm in FP64,
// FP32 by rounding).  What was built or captured for other lengths goes: the
// spectrum, the product workspaces and the captured iterations.
static int set_lengths(dda_target* t, int Kpp, int Jpp, int Ppp) {
  const int ns[3] = {Kpp, Jpp, Ppp};
  for (int a = 0; a < 3; ++a) {
    const int n = ns[a];
    std::vector<c64> w(n);
    std::vector<c32> wf(n);
    for (int m = 0; m < n; ++m) {
      const double ang = 2.0 * M_PI * (double)m / (double)n;
      w[m] = mk(std::cos(ang), -std::sin(ang));
      wf[m] = mk((float)w[m].x, (float)w[m].y);
    }
    CHK(t->p64.tw[a].ensure(n * sizeof(c64)));
    CHK(t->p32.tw[a].ensure(n * sizeof(c32)));
    if (hipMemcpy(t->p64.tw[a].p, w.data(), n * sizeof(c64), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t->p32.tw[a].p, wf.data(), n * sizeof(c32), hipMemcpyHostToDevice) != hipSuccess)
      return fail(DDA_EDEVICE, "twiddle upload failed");
  }
  t->Kpp = Kpp;
  t->Jpp = Jpp;
  t->Ppp = Ppp;
  t->Kh = Kpp / 2 + 1;
  t->Jh = Jpp / 2 + 1;
  t->Ph = Ppp / 2 + 1;
  t->fx = make_desc(Kpp);
  t->fy = make_desc(Jpp);
  t->fz = make_desc(Ppp);
  t->spec_ready = false;
  t->p32.cap = t->p64.cap = 0;
  drop_graphs(t);
  return DDA_OK;
}

// a padded length the transforms take for lattice extent n: at least 2n - 1
// (Sec. 3), of the form 2^a 3^b 5^c, and at most max(16, 4 (2n - 1))
static bool padding_ok(int n, int npp) {
  const long m = 2L * n - 1;
  return npp >= m && smooth235(npp) && npp <= std::max(16L, 4 * m);
}

extern "C" {

const char* dda_last_error(void) { return g_err.c_str(); }

int dda_profile_enable(dda_lib* lib, int enable) {
  if (!lib) return fail(DDA_EINVAL, "dda_profile_enable: NULL lib");
  if (enable < 0 || enable > 2) return fail(DDA_EINVAL, "dda_profile_enable: enable must be 0, 1 or 2");
  lib->prof = enable;
  return DDA_OK;
}

int dda_profile_read(dda_lib* lib, double* ms, int64_t* count) {
  if (!lib || !ms || !count) return fail(DDA_EINVAL, "dda_profile_read: NULL argument");
  HIPCHK(hipSetDevice(lib->device));
  for (auto& pe : lib->pending) {
    HIPCHK(hipEventSynchronize(pe.second.second));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, pe.second.first, pe.second.second));
    lib->prof_ms[pe.first] += t;
    lib->prof_n[pe.first] += 1;
    lib->ev_pool.push_back(pe.second.first);
    lib->ev_pool.push_back(pe.second.second);
  }
  lib->pending.clear();
  for (int p = 0; p < PASS_COUNT; ++p) {
    ms[p] = lib->prof_ms[p];
    count[p] = lib->prof_n[p];
  }
  return DDA_OK;
}

int dda_profile_reset(dda_lib* lib) {
  if (!lib) return fail(DDA_EINVAL, "dda_profile_reset: NULL lib");
  double ms[PASS_COUNT];
  int64_t n[PASS_COUNT];
  CHK(dda_profile_read(lib, ms, n));
  for (int p = 0; p < PASS_COUNT; ++p) {
    lib->prof_ms[p] = 0;
    lib->prof_n[p] = 0;
  }
  return DDA_OK;
}

int dda_open(int hip_device, const char* tune_cache_path, dda_lib** out) {
  if (!out) return fail(DDA_EINVAL, "dda_open: out is NULL");
  *out = nullptr;
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (hip_device < 0 || hip_device >= n) return fail(DDA_EINVAL, "dda_open: device %d of %d", hip_device, n);
  HIPCHK(hipSetDevice(hip_device));
  dda_lib* l = new dda_lib();
  l->device = hip_device;
  {
    const hipError_t e = hipGetSymbolAddress((void**)&l->scratch_dev, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !l->scratch_dev) {
      delete l;
      return fail(DDA_EDEVICE, "dda_open: scratch address on device %d: %s", hip_device, hipGetErrorString(e));
    }
  }
  if (tune_cache_path) {
    l->tune_path = tune_cache_path;
    std::ifstream f(tune_cache_path);
    std::string line;
    while (std::getline(f, line)) {
      const size_t eq = line.rfind(" = ");
      if (eq == std::string::npos) continue;
      l->tuned[line.substr(0, eq)] = std::atoi(line.c_str() + eq + 3);
    }
  }
  *out = l;
  return DDA_OK;
}

void dda_close(dda_lib* lib) {
  if (!lib) return;
  (void)hipSetDevice(lib->device);
  for (auto& pe : lib->pending) {
    (void)hipEventSynchronize(pe.second.second);
    lib->ev_pool.push_back(pe.second.first);
    lib->ev_pool.push_back(pe.second.second);
  }
  for (hipEvent_t e : lib->ev_pool) (void)hipEventDestroy(e);
  for (hipStream_t w : lib->workers) (void)hipStreamDestroy(w);
  delete lib;
  (void)hipGetLastError();  // leave no error state behind for later launches
}

int dda_target_create(dda_lib* lib, int K, int J, int P, double kd, dda_target** out) {
  if (!lib || !out) return fail(DDA_EINVAL, "dda_target_create: NULL argument");
  *out = nullptr;
  if (K < 1 || J < 1 || P < 1) return fail(DDA_EINVAL, "dda_target_create: lattice %dx%dx%d", K, J, P);
  if (!(kd > 0.0) || !std::isfinite(kd)) return fail(DDA_EINVAL, "dda_target_create: kd = %g", kd);
  if ((long)K * J * P > (1L << 30)) return fail(DDA_EINVAL, "dda_target_create: lattice too large");
  HIPCHK(hipSetDevice(lib->device));
  dda_target* t = new dda_target();
  t->lib = lib;
  t->device = lib->device;
  t->K = K;
  t->J = J;
  t->P = P;
  t->kd = kd;
  const int rc = set_lengths(t, fft_size_at_least(2 * K - 1), fft_size_at_least(2 * J - 1, true),
                             fft_size_at_least(2 * P - 1));
  if (rc != DDA_OK) {
    delete t;
    return rc;
  }
  *out = t;
  return DDA_OK;
}

void dda_target_destroy(dda_target* t) {
  if (!t) return;
  (void)hipSetDevice(t->device);
  delete t;
  (void)hipGetLastError();  // leave no error state behind for later launches
}

int dda_target_set_option(dda_target* t, int option, int value) {
  if (!t) return fail(DDA_EINVAL, "dda_target_set_option: NULL target");
  switch (option) {
    case DDA_OPT_SCHEDULE: {
      if (value > 0)
        if (const char* why = schedule_missing(value, t->K, t->J, t->Kpp, t->Jpp, t->Ppp))
          return fail(DDA_EINVAL, "dda_target_set_option: schedule %d: %s for this lattice", value, why);
      t->forced_sched = value < 0 ? -1 : value;
      return DDA_OK;
    }
    case DDA_OPT_INJECT_BREAKDOWN:
      if (value < 0) return fail(DDA_EINVAL, "dda_target_set_option: inject count %d", value);
      t->inject_breakdown = value;
      return DDA_OK;
    case DDA_OPT_FUSE_QMR_STEP:
      if (value != 0 && value != 1) return fail(DDA_EINVAL, "dda_target_set_option: fuse %d", value);
      t->fuse_qmr = value;
      return DDA_OK;
    case DDA_OPT_X_ROWS:
      if (value < -1 || value > 2) return fail(DDA_EINVAL, "dda_target_set_option: x rows variant %d", value);
      t->forced_xsel = value;
      return DDA_OK;
    case DDA_OPT_INJECT_BAD_STEP:
      if (value < 0) return fail(DDA_EINVAL, "dda_target_set_option: inject count %d", value);
      t->inject_bad_step = value;
      return DDA_OK;
    case DDA_OPT_Y_TILE:
      if (value < -1 || value > 2) return fail(DDA_EINVAL, "dda_target_set_option: y tile variant %d", value);
      if (value > 0 && value > ylog_max<float>(t))
        return fail(DDA_EINVAL, "dda_target_set_option: no y tile variant %d for this lattice", value);
      t->forced_ylog = value;
      return DDA_OK;
    case DDA_OPT_RHS_PER_BLOCK:
      if (value < 0 || value > 8) return fail(DDA_EINVAL, "dda_target_set_option: right-hand sides per block %d", value);
      t->z_rb = value;
      return DDA_OK;
    case DDA_OPT_CANARY:
      if (value != 0 && value != 1) return fail(DDA_EINVAL, "dda_target_set_option: canary %d", value);
      t->canary = value;
      return DDA_OK;
    default:
      return fail(DDA_EINVAL, "dda_target_set_option: option %d", option);
  }
}

int dda_target_info(const dda_target* t, int64_t* dims) {
  if (!t || !dims) return fail(DDA_EINVAL, "dda_target_info: NULL argument");
  dims[0] = t->Kpp;
  dims[1] = t->Jpp;
  dims[2] = t->Ppp;
  dims[3] = t->Kh;
  dims[4] = t->Jh;
  dims[5] = t->Ph;
  dims[6] = t->nd;
  // 1D transforms per matrix-vector product and right-hand side, forward and
  // inverse (Sec. 3): y on K*P lines, x on J''*P lines, z on K''*J'' lines,
  // for each of the 3 components, both directions.
  dims[7] = 2L * 3 * ((long)t->K * t->P + (long)t->Jpp * t->P + (long)t->Kpp * t->Jpp);
  // spectrum build: x on J*P, y on K_h*P, z on K_h*J_h lines, 6 components
  dims[8] = 6L * ((long)t->J * t->P + (long)t->Kh * t->P + (long)t->Kh * t->Jh);
  return DDA_OK;
}

int dda_target_set_padding(dda_target* t, int Kpp, int Jpp, int Ppp) {
  if (!t) return fail(DDA_EINVAL, "dda_target_set_padding: NULL target");
  const int n[3] = {t->K, t->J, t->P};
  int v[3] = {Kpp, Jpp, Ppp};
  for (int a = 0; a < 3; ++a) {
    if (v[a] == 0) v[a] = fft_size_at_least(2 * n[a] - 1, a == 1);
    if (!padding_ok(n[a], v[a]))
      return fail(DDA_EINVAL, "dda_target_set_padding: length %d for extent %d (needs >= %d, 2^a 3^b 5^c, <= %ld)",
                  v[a], n[a], 2 * n[a] - 1, std::max(16L, 4 * (2L * n[a] - 1)));
  }
  if (t->forced_sched > 0)
    if (const char* why = schedule_missing(t->forced_sched, t->K, t->J, v[0], v[1], v[2]))
      return fail(DDA_EINVAL, "dda_target_set_padding: forced schedule %d: %s at %dx%dx%d", t->forced_sched, why,
                  v[0], v[1], v[2]);
  if (v[0] == t->Kpp && v[1] == t->Jpp && v[2] == t->Ppp) return DDA_OK;
  HIPCHK(hipSetDevice(t->lib->device));
  return set_lengths(t, v[0], v[1], v[2]);
}

int dda_set_occupancy(dda_target* t, const uint8_t* occ, int64_t* nd_out) {
  if (!t || !occ) return fail(DDA_EINVAL, "dda_set_occupancy: NULL argument");
  HIPCHK(hipSetDevice(t->lib->device));
  const long N = (long)t->K * t->J * t->P;
  const int W = (t->K + 31) / 32;
  const long nrow = (long)t->J * t->P;
  std::vector<uint32_t> words((size_t)nrow * W * 2, 0u);  // (bits, base) pairs
  std::vector<int> sites;
  for (long r = 0; r < nrow; ++r)
    for (int w = 0; w < W; ++w) {
      uint32_t* wd = &words[((size_t)r * W + w) * 2];
      wd[1] = (uint32_t)sites.size();
      for (int b = 0; b < 32 && 32 * w + b < t->K; ++b) {
        const long s = r * t->K + 32 * w + b;
        if (occ[s]) {
          wd[0] |= 1u << b;
          sites.push_back((int)s);
        }
      }
    }
  if (sites.empty()) return fail(DDA_EINVAL, "dda_set_occupancy: no occupied site");
  (void)N;
  CHK(t->occ.ensure(words.size() * sizeof(uint32_t)));
  CHK(t->sites.ensure(sites.size() * sizeof(int)));
  HIPCHK(hipMemcpy(t->occ.p, words.data(), words.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  t->occ_words = W;
  HIPCHK(hipMemcpy(t->sites.p, sites.data(), sites.size() * sizeof(int), hipMemcpyHostToDevice));
  t->nd = (int64_t)sites.size();
  t->have_alpha = t->have_eps = false;
  t->comp_bits = false;
  t->uniform_diag = false;
  // everything sized or captured for the previous N_d goes: solver vectors
  // (ensure_solver_ws grows them by count, not bytes), the captured
  // iteration (its launches bake in N_d, block counts and slot offsets) and
  // the orientation factors of the last solve
  t->p32.vec.release();
  t->p64.vec.release();
  t->p32.vec_cap = t->p32.vec_slots = 0;
  t->p64.vec_cap = t->p64.vec_slots = 0;
  t->p32.vec_nd = t->p64.vec_nd = 0;
  drop_graphs(t);
  t->solve_S.clear();
  {
    int lo[3] = {t->K, t->J, t->P}, hi[3] = {-1, -1, -1};
    for (int sv : sites) {
      const int c[3] = {sv % t->K, (sv / t->K) % t->J, sv / (t->K * t->J)};
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], c[a]);
        hi[a] = std::max(hi[a], c[a]);
      }
    }
    double e2 = 0;
    for (int a = 0; a < 3; ++a) e2 += (double)(hi[a] - lo[a]) * (hi[a] - lo[a]);
    t->extent = std::sqrt(e2);
  }
  if (nd_out) *nd_out = t->nd;
  return DDA_OK;
}

// Diagonal alpha^{-1} = a0 + S a1 as [3][N_d] (one value per component and
// dipole); per-dipole (isotropic) inputs of N_d entries are repeated.
static int upload_diag(dda_target* t, std::vector<c64> a0, const std::vector<c64>* a1_in) {
  const size_t nd = (size_t)t->nd * 3;
  std::vector<c64> a1v;
  const std::vector<c64>* a1 = a1_in;
  if (a0.size() * 3 == nd) {
    std::vector<c64> r(nd);
    for (int c = 0; c < 3; ++c) std::copy(a0.begin(), a0.end(), r.begin() + (size_t)c * t->nd);
    a0.swap(r);
    if (a1_in) {
      a1v.resize(nd);
      for (int c = 0; c < 3; ++c) std::copy(a1_in->begin(), a1_in->end(), a1v.begin() + (size_t)c * t->nd);
      a1 = &a1v;
    }
  }
  CHK(t->p64.a0.ensure(nd * sizeof(c64)));
  CHK(t->p32.a0.ensure(nd * sizeof(c32)));
  std::vector<c32> f(nd);
  for (size_t n = 0; n < nd; ++n) f[n] = mk((float)a0[n].x, (float)a0[n].y);
  HIPCHK(hipMemcpy(t->p64.a0.p, a0.data(), nd * sizeof(c64), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(t->p32.a0.p, f.data(), nd * sizeof(c32), hipMemcpyHostToDevice));
  t->has_a1 = a1 != nullptr;
  if (a1) {
    CHK(t->p64.a1.ensure(nd * sizeof(c64)));
    CHK(t->p32.a1.ensure(nd * sizeof(c32)));
    for (size_t n = 0; n < nd; ++n) f[n] = mk((float)(*a1)[n].x, (float)(*a1)[n].y);
    HIPCHK(hipMemcpy(t->p64.a1.p, a1->data(), nd * sizeof(c64), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(t->p32.a1.p, f.data(), nd * sizeof(c32), hipMemcpyHostToDevice));
  }
  return DDA_OK;
}

// alpha^{-1}(eps) = v + S s1 and its eps-derivative dv + S ds1 for the
// published prescriptions (CM; Draine 1988 radiative reaction; Draine &
// Goodman 1993 lattice dispersion relation), d = 1.  False at a pole.
static bool alpha_inv_of(c64 e, int prescription, double kd, c64& v, c64& s1, c64& dv, c64& ds1) {
  const double b1 = -1.8915316, b2 = 0.1648469, b3 = -1.7700004;
  const double kd2 = kd * kd, kd3 = kd2 * kd;
  const c64 em1 = e - mk(1.0, 0.0);
  if (!(abs2(em1) > 0.0)) return false;
  v = (4.0 * M_PI / 3.0) * cdiv(e + mk(2.0, 0.0), em1);
  dv = (-4.0 * M_PI) * cdiv(mk(1.0, 0.0), em1 * em1);
  s1 = mk(0.0, 0.0);
  ds1 = mk(0.0, 0.0);
  if (prescription >= DDA_POL_RR) v = v + mk(0.0, -(2.0 / 3.0) * kd3);
  if (prescription == DDA_POL_LDR) {
    v = v + kd2 * (mk(b1, 0.0) + b2 * e);
    dv = dv + mk(b2 * kd2, 0.0);
    s1 = (b3 * kd2) * e;
    ds1 = mk(b3 * kd2, 0.0);
  }
  return std::isfinite(v.x) && std::isfinite(v.y) && abs2(v) > 0.0;
}

int dda_set_permittivity(dda_target* t, const double* eps, int prescription) {
  if (!t || !eps) return fail(DDA_EINVAL, "dda_set_permittivity: NULL argument");
  if (t->nd <= 0) return fail(DDA_ESTATE, "dda_set_permittivity: occupancy not set");
  if (prescription < DDA_POL_CM || prescription > DDA_POL_LDR)
    return fail(DDA_EINVAL, "dda_set_permittivity: prescription %d", prescription);
  HIPCHK(hipSetDevice(t->lib->device));
  const size_t nd = (size_t)t->nd;
  std::vector<c64> a0(nd), a1(nd), d0(nd), d1(nd);
  for (size_t n = 0; n < nd; ++n) {
    const c64 e = mk(eps[2 * n], eps[2 * n + 1]);
    if (!(abs2(e - mk(1.0, 0.0)) > 0.0)) return fail(DDA_EINVAL, "dda_set_permittivity: eps = 1 at dipole %zu", n);
    if (!alpha_inv_of(e, prescription, t->kd, a0[n], a1[n], d0[n], d1[n]))
      return fail(DDA_EINVAL, "dda_set_permittivity: alpha^-1 not finite at dipole %zu", n);
  }
  const bool ldr = prescription == DDA_POL_LDR;
  CHK(upload_diag(t, a0, ldr ? &a1 : nullptr));
  CHK(t->d0.ensure(nd * sizeof(c64)));
  HIPCHK(hipMemcpy(t->d0.p, d0.data(), nd * sizeof(c64), hipMemcpyHostToDevice));
  if (ldr) {
    CHK(t->d1.ensure(nd * sizeof(c64)));
    HIPCHK(hipMemcpy(t->d1.p, d1.data(), nd * sizeof(c64), hipMemcpyHostToDevice));
  }
  // one permittivity for all dipoles (a homogeneous target): the
  // matrix-vector passes take alpha^{-1} from a one-entry table instead of
  // gathering the per-dipole arrays (the solver's outer kernels keep those)
  bool uniform = true;
  for (size_t n = 1; n < nd && uniform; ++n) uniform = eps[2 * n] == eps[0] && eps[2 * n + 1] == eps[1];
  t->uniform_diag = false;
  if (uniform) {
    const c32 f0 = mk((float)a0[0].x, (float)a0[0].y), f1 = mk((float)a1[0].x, (float)a1[0].y);
    CHK(t->p64.mt0.ensure(sizeof(c64)));
    CHK(t->p64.mt1.ensure(sizeof(c64)));
    CHK(t->p32.mt0.ensure(sizeof(c32)));
    CHK(t->p32.mt1.ensure(sizeof(c32)));
    HIPCHK(hipMemcpy(t->p64.mt0.p, &a0[0], sizeof(c64), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(t->p64.mt1.p, &a1[0], sizeof(c64), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(t->p32.mt0.p, &f0, sizeof(c32), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(t->p32.mt1.p, &f1, sizeof(c32), hipMemcpyHostToDevice));
    t->uniform_diag = true;
  }
  t->prescription = prescription;
  t->have_alpha = t->have_eps = true;
  t->aniso = false;
  t->comp_bits = false;
  return DDA_OK;
}

int dda_set_polarizability(dda_target* t, const double* alpha) {
  if (!t || !alpha) return fail(DDA_EINVAL, "dda_set_polarizability: NULL argument");
  if (t->nd <= 0) return fail(DDA_ESTATE, "dda_set_polarizability: occupancy not set");
  HIPCHK(hipSetDevice(t->lib->device));
  const size_t nd = (size_t)t->nd;
  std::vector<c64> a0(nd);
  for (size_t n = 0; n < nd; ++n) {
    const c64 a = mk(alpha[2 * n], alpha[2 * n + 1]);
    if (!(abs2(a) > 0.0)) return fail(DDA_EINVAL, "dda_set_polarizability: alpha = 0 at dipole %zu", n);
    a0[n] = cdiv(mk(1.0, 0.0), a);
    if (!std::isfinite(a0[n].x) || !std::isfinite(a0[n].y))
      return fail(DDA_EINVAL, "dda_set_polarizability: alpha^-1 not finite at dipole %zu", n);
  }
  CHK(upload_diag(t, a0, nullptr));
  t->prescription = -1;
  t->have_alpha = true;
  t->have_eps = false;
  t->aniso = false;
  t->comp_bits = false;
  t->uniform_diag = false;
  return DDA_OK;
}

int dda_set_composition(dda_target* t, int nmat, const double* eps, const uint8_t* flags, int prescription) {
  if (!t || !eps || !flags || nmat < 1 || nmat > 256) return fail(DDA_EINVAL, "dda_set_composition: bad arguments");
  if (t->nd <= 0) return fail(DDA_ESTATE, "dda_set_composition: occupancy not set");
  if (prescription < DDA_POL_CM || prescription > DDA_POL_LDR)
    return fail(DDA_EINVAL, "dda_set_composition: prescription %d", prescription);
  HIPCHK(hipSetDevice(t->lib->device));
  std::vector<c64> mv(nmat), ms(nmat);
  for (int q = 0; q < nmat; ++q) {
    c64 dv, ds;
    if (!alpha_inv_of(mk(eps[2 * q], eps[2 * q + 1]), prescription, t->kd, mv[q], ms[q], dv, ds))
      return fail(DDA_EINVAL, "dda_set_composition: material %d has no finite alpha^-1 (eps = 1 or a pole)", q);
  }
  const size_t nd = (size_t)t->nd;
  std::vector<c64> a0(3 * nd), a1(3 * nd);
  for (size_t e = 0; e < 3 * nd; ++e) {
    const int q = flags[e];
    if (q >= nmat) return fail(DDA_EINVAL, "dda_set_composition: flag %d at entry %zu (nmat %d)", q, e, nmat);
    a0[e] = mv[q];
    a1[e] = ms[q];
  }
  const bool ldr = prescription == DDA_POL_LDR;
  // per-dipole FP64 diagonals for the solver's outer kernels (scaling,
  // refinement, cross sections), once per refinement step
  CHK(upload_diag(t, a0, ldr ? &a1 : nullptr));
  // the matrix-vector passes read the flags at the minimal power-of-two bit
  // width (Sec. 2: 4 materials need 2 bits) and the nmat-entry table
  int fb = 1;
  while ((1 << fb) < nmat) ++fb;
  int mlb = 0;
  while ((1 << mlb) < fb) ++mlb;
  const size_t nbits = 3 * nd << mlb;
  std::vector<uint32_t> words((nbits + 31) / 32, 0u);
  for (size_t e = 0; e < 3 * nd; ++e) {
    const size_t bit = e << mlb;
    words[bit >> 5] |= (uint32_t)flags[e] << (bit & 31);
  }
  CHK(t->mbits.ensure(words.size() * sizeof(uint32_t)));
  HIPCHK(hipMemcpy(t->mbits.p, words.data(), words.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
  std::vector<c32> mf0(nmat), mf1(nmat);
  for (int q = 0; q < nmat; ++q) {
    mf0[q] = mk((float)mv[q].x, (float)mv[q].y);
    mf1[q] = mk((float)ms[q].x, (float)ms[q].y);
  }
  CHK(t->p64.mt0.ensure(nmat * sizeof(c64)));
  CHK(t->p64.mt1.ensure(nmat * sizeof(c64)));
  CHK(t->p32.mt0.ensure(nmat * sizeof(c32)));
  CHK(t->p32.mt1.ensure(nmat * sizeof(c32)));
  HIPCHK(hipMemcpy(t->p64.mt0.p, mv.data(), nmat * sizeof(c64), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(t->p64.mt1.p, ms.data(), nmat * sizeof(c64), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(t->p32.mt0.p, mf0.data(), nmat * sizeof(c32), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(t->p32.mt1.p, mf1.data(), nmat * sizeof(c32), hipMemcpyHostToDevice));
  t->mlb = mlb;
  t->comp_bits = true;
  t->uniform_diag = false;
  t->prescription = prescription;
  t->have_alpha = true;
  t->have_eps = false;  // the permittivity gradient is defined per isotropic dipole
  t->aniso = true;
  return DDA_OK;
}

int dda_build_spectrum(dda_target* t, void* hip_stream) {
  if (!t) return fail(DDA_EINVAL, "dda_build_spectrum: NULL target");
  HIPCHK(hipSetDevice(t->lib->device));
  hipStream_t st = (hipStream_t)hip_stream;
  const int K = t->K, J = t->J, P = t->P, Kh = t->Kh, Jh = t->Jh, Ph = t->Ph;
  DevBuf T, S1, S2;
  CHK(T.ensure(6L * K * J * P * sizeof(c64)));
  CHK(S1.ensure(6L * P * J * Kh * sizeof(c64)));
  CHK(S2.ensure(6L * P * Jh * Kh * sizeof(c64)));
  CHK(t->p64.Y.ensure(6L * Ph * Jh * Kh * sizeof(c64)));
  CHK(t->p32.Y.ensure(6L * Ph * Jh * Kh * sizeof(c32)));
  CHK(t->p64.Yz.ensure(6L * Ph * Jh * Kh * sizeof(c64)));
  CHK(t->p32.Yz.ensure(6L * Ph * Jh * Kh * sizeof(c32)));
  const long N = (long)K * J * P;
  hipLaunchKernelGGL(k_tensor_column, dim3((unsigned)std::min<long>((N + 255) / 256, 65535)), dim3(256), 0, st,
                     T.as<c64>(), K, J, P, t->kd);
  LAUNCHCHK();
  // x: 6*J*P lines of K -> K'' (mirrored with Table 1 signs), keep K_h
  CHK(launch_contig<double>(T.as<c64>(), S1.as<c64>(), 6L * J * P, K, Kh, K, Kh, t->fx, t->p64.tw[0].as<c64>(),
                            false, true, (long)J * P, 0, 0, nullptr, 1.0, st));
  // y: lines along y of [6][P][J][K_h] -> [6][P][J_h][K_h]
  StridedArgs ya;
  ya.sb = (long)P * J * Kh;
  ya.so = (long)J * Kh;
  ya.se = Kh;
  ya.tb = (long)P * Jh * Kh;
  ya.to = (long)Jh * Kh;
  ya.te = Kh;
  ya.NX = Kh;
  ya.Lin = J;
  ya.Lout = Jh;
  ya.axis = 1;
  CHK(launch_strided_mirror<double>(S1.as<c64>(), S2.as<c64>(), ya, P, 6, t->fy, t->p64.tw[1].as<c64>(), st));
  // z: lines along z of [6][P][J_h][K_h] -> [6][P_h][J_h][K_h]
  StridedArgs za;
  za.sb = (long)P * Jh * Kh;
  za.so = Kh;
  za.se = (long)Jh * Kh;
  za.tb = (long)Ph * Jh * Kh;
  za.to = Kh;
  za.te = (long)Jh * Kh;
  za.NX = Kh;
  za.Lin = P;
  za.Lout = Ph;
  za.axis = 2;
  CHK(launch_strided_mirror<double>(S2.as<c64>(), t->p64.Y.as<c64>(), za, Jh, 6, t->fz, t->p64.tw[2].as<c64>(),
                                    st));
  const long ny = 6L * Ph * Jh * Kh;
  hipLaunchKernelGGL(k_round_to_f32, dim3((unsigned)std::min<long>((ny + 255) / 256, 65535)), dim3(256), 0, st,
                     t->p64.Y.as<c64>(), t->p32.Y.as<c32>(), ny);
  LAUNCHCHK();
  {
    const unsigned g = (unsigned)std::min<long>((ny + 255) / 256, 65535);
    hipLaunchKernelGGL((k_spec_zfast<double>), dim3(g), dim3(256), 0, st, t->p64.Y.as<c64>(), t->p64.Yz.as<c64>(), Kh,
                       Jh, Ph);
    hipLaunchKernelGGL((k_spec_zfast<float>), dim3(g), dim3(256), 0, st, t->p32.Y.as<c32>(), t->p32.Yz.as<c32>(), Kh,
                       Jh, Ph);
    LAUNCHCHK();
  }
  // temporaries are freed on return: wait for the kernels that use them
  HIPCHK(hipStreamSynchronize(st));
  t->spec_ready = true;
  return DDA_OK;
}

int dda_get_spectrum(dda_target* t, int precision, void* out_dev, void* hip_stream) {
  if (!t || !out_dev) return fail(DDA_EINVAL, "dda_get_spectrum: NULL argument");
  if (!t->spec_ready) return fail(DDA_ESTATE, "dda_get_spectrum: spectrum not built");
  HIPCHK(hipSetDevice(t->lib->device));
  const long ny = 6L * t->Ph * t->Jh * t->Kh;
  if (precision == DDA_FP64)
    HIPCHK(hipMemcpyAsync(out_dev, t->p64.Y.p, ny * sizeof(c64), hipMemcpyDeviceToDevice, (hipStream_t)hip_stream));
  else
    HIPCHK(hipMemcpyAsync(out_dev, t->p32.Y.p, ny * sizeof(c32), hipMemcpyDeviceToDevice, (hipStream_t)hip_stream));
  return DDA_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// matrix-vector product
// ----------------------------------------------------------------------------
static int ensure_scratch(dda_target* t, int nrhs) {
  if (nrhs <= t->scap) return DDA_OK;
  const int cap = nrhs;
  CHK(t->S.ensure(cap * sizeof(double)));
  CHK(t->active.ensure(cap * sizeof(int)));
  CHK(t->active_outer.ensure(cap * sizeof(int)));
  CHK(t->scal.ensure(cap * sizeof(double)));
  CHK(t->tolv.ensure(cap * sizeof(double)));
  CHK(t->state.ensure(2 * cap * std::max({sizeof(BcgState), sizeof(QmrState), sizeof(CgState), sizeof(CgsState),
                                             sizeof(TfqState), sizeof(GenState)})));
  CHK(t->khat.ensure(cap * 3 * sizeof(double)));
  CHK(t->ehat.ensure(cap * 6 * sizeof(double)));
  t->h_active.resize(cap);
  t->scap = cap;
  return DDA_OK;
}

// Bytes of the two FFT workspaces of a product (every schedule): the
// y-transformed array [nrhs][3][P][J''][K] and the x-transformed one (K''
// padded to whole tiles where the tile-blocked layout exists).
template <typename R>
static void matvec_ws_bytes(const dda_target* t, int nrhs, size_t& g1, size_t& g2) {
  size_t e2 = (size_t)t->P * t->Jpp * t->Kpp;
  if (z2_size<R>(t->Ppp)) {
    const int C = z2_cols<R>(t->Ppp);
    e2 = std::max(e2, (size_t)t->P * t->Jpp * ((t->Kpp + C - 1) / C) * C);
  }
  g1 = (size_t)nrhs * 3 * t->P * t->Jpp * t->K * sizeof(cx<R>);
  g2 = (size_t)nrhs * 3 * e2 * sizeof(cx<R>);
}

template <typename R>
static int ensure_matvec_ws(dda_target* t, int nrhs) {
  PrecBufs<R>& b = bufs<R>(t);
  if (nrhs <= b.cap) return DDA_OK;
  size_t g1, g2;
  matvec_ws_bytes<R>(t, nrhs, g1, g2);
  CHK(b.G1.ensure(g1));
  CHK(b.G2.ensure(g2));
  b.cap = nrhs;
  return DDA_OK;
}

// ---- register-resident passes -------------------------------------------
template <int N>
constexpr int fast_tx() {
  constexpr int T = FastPlan<N>::T;
  if (FastPlan<N>::five) {
    // (y passes only) a power-of-two tile of at least 128 threads, within
    // 64 KB of FP64 LDS
    int tx = 1;
    while (T * tx < 128 && N * (2 * tx) * 16 <= 64 * 1024) tx *= 2;
    return tx;
  }
  int tx = 256 / T;
  if (tx < 16) tx = 512 / T < 16 ? 512 / T : 16;  // rows of >= 128 B where a 512-thread block allows
  return tx < 8 ? 8 : (tx > 64 ? 64 : tx);
}
template <typename R, int N>
constexpr int fast_txz() {
  int tx = fast_tx<N>();
  while (tx > 2 && 3 * N * tx * (int)sizeof(cx<R>) > 48 * 1024) tx /= 2;
  return tx;
}
// y-pass tiles wider than fast_tx: 2^L times as many x positions per block,
// up to 1024 threads and 64 KB of LDS (longer contiguous runs in the strided
// rows of the y-transformed array, fewer blocks)
template <typename R, int N>
constexpr int ytx_max_log() {
  int L = 0;
  while (L < 2 && FastPlan<N>::T * (fast_tx<N>() << (L + 1)) <= 1024 &&
         N * (fast_tx<N>() << (L + 1)) * (int)sizeof(cx<R>) <= 64 * 1024)
    ++L;
  return L;
}
template <int N>
constexpr int fast_rw() {
  constexpr int T = FastPlan<N>::T;
  constexpr int rw = 256 / T;
  return rw < 1 ? 1 : (rw > 64 ? 64 : rw);
}

// Rows per block of an x pass for variant xsel: 0 the base count, 1 half of
// it, 2 twice it (within 1024 threads and 64 KB of LDS; a variant that does
// not fit is the base count)
template <typename R, int N>
constexpr int xrows_variant(int base, int xsel) {
  constexpr int T = FastPlan<N>::T, LS = N + N / 8 + 1;
  const int rw = xsel == 1 ? base / 2 : xsel == 2 ? base * 2 : base;
  if (rw < 1 || rw * T > 1024 || rw * LS * (int)sizeof(cx<R>) > 65536) return base;
  return rw;
}

template <typename R>
struct FastLaunch {
  template <int N>
  static void xT(bool inv, int nrhs, hipStream_t st, const cx<R>* in, cx<R>* out, const dda_target* t,
                 const int* act, const cx<R>* tw) {
    constexpr int RK = xt_rows<R, N>();
    dim3 grid((t->P + RK - 1) / RK, t->Jpp, nrhs * 3);
    if (inv)
      hipLaunchKernelGGL((k_xT_inv<R, N, RK>), grid, dim3(FastPlan<N>::T * RK), 0, st, in, out, t->K, t->P, t->Jpp,
                         act, tw);
    else
      hipLaunchKernelGGL((k_xT_fwd<R, N, RK>), grid, dim3(FastPlan<N>::T * RK), 0, st, in, out, t->K, t->P, t->Jpp,
                         act, tw);
  }
  template <int N>
  static void zline(int nrhs, hipStream_t st, cx<R>* G2t, const cx<R>* Yz, const int* act, ZArgs za,
                    const cx<R>* tw) {
    constexpr int RL = zline_rows<R, N>();
    ZMap zm;
    zm.NX = (za.Kpp + RL - 1) / RL;
    zm.ngx = (zm.NX + 1) / 2;
    zm.ngy = za.Jpp / 2 + 1;
    zm.ngroups = nrhs * zm.ngx * zm.ngy;
    dim3 grid(32 * ((zm.ngroups + 7) / 8));
    hipLaunchKernelGGL((k_zline<R, N, RL>), grid, dim3(FastPlan<N>::T * RL), 0, st, G2t, Yz, act, za, zm, tw);
  }
  // y tile of variant ylog (clamped to the widest that exists)
  template <int N>
  static int ytx(int ylog) {
    return fast_tx<N>() << std::min(std::max(ylog, 0), ytx_max_log<R, N>());
  }
  template <int N, int L>
  static void yfwd_L(hipStream_t st, const cx<R>* x, cx<R>* G1, OccBits map, const cx<R>* a0,
                     const cx<R>* a1, const double* S, const int* act, VecArgs va, const cx<R>* tw,
                     const QmrFuse<R>* qf) {
    constexpr int TX = fast_tx<N>() << L;
    dim3 grid((unsigned)ytile_blocks((long)((va.K + TX - 1) / TX) * va.P * va.nrhs));
    if (qf)
      hipLaunchKernelGGL((k_fast_yfwd<R, N, TX, true>), grid, dim3(FastPlan<N>::T * TX), 0, st, x, G1, map, a0, a1,
                         S, act, va, tw, *qf);
    else
      hipLaunchKernelGGL((k_fast_yfwd<R, N, TX, false>), grid, dim3(FastPlan<N>::T * TX), 0, st, x, G1, map, a0,
                         a1, S, act, va, tw, QmrFuse<R>{});
  }
  template <int N>
  static void yfwd(int ylog, hipStream_t st, const cx<R>* x, cx<R>* G1, OccBits map, const cx<R>* a0,
                   const cx<R>* a1, const double* S, const int* act, VecArgs va, const cx<R>* tw,
                   const QmrFuse<R>* qf) {
    constexpr int LM = ytx_max_log<R, N>();
    const int L = std::min(std::max(ylog, 0), LM);
    if constexpr (LM >= 2)
      if (L == 2) return yfwd_L<N, 2>(st, x, G1, map, a0, a1, S, act, va, tw, qf);
    if constexpr (LM >= 1)
      if (L == 1) return yfwd_L<N, 1>(st, x, G1, map, a0, a1, S, act, va, tw, qf);
    yfwd_L<N, 0>(st, x, G1, map, a0, a1, S, act, va, tw, qf);
  }
  // y-forward blocks per right-hand side (3 components x P planes x x tiles)
  template <int N>
  static int yfwd_blocks(const dda_target* t, int ylog) {
    const int TX = ytx<N>(ylog);
    return 3 * t->P * ((t->K + TX - 1) / TX);
  }
  template <int N, int L>
  static void yinv_L(hipStream_t st, const cx<R>* G1, const cx<R>* x, cx<R>* y, OccBits map,
                     const cx<R>* a0, const cx<R>* a1, const double* S, const int* act, VecArgs va,
                     const cx<R>* tw, DotArgs dot) {
    constexpr int TX = fast_tx<N>() << L;
    dim3 grid((unsigned)ytile_blocks((long)((va.K + TX - 1) / TX) * va.P * va.nrhs));
    hipLaunchKernelGGL((k_fast_yinv<R, N, TX>), grid, dim3(FastPlan<N>::T * TX), 0, st, G1, x, y, map, a0, a1, S,
                       act, va, tw, dot);
  }
  template <int N>
  static void yinv(int ylog, hipStream_t st, const cx<R>* G1, const cx<R>* x, cx<R>* y, OccBits map,
                   const cx<R>* a0, const cx<R>* a1, const double* S, const int* act, VecArgs va, const cx<R>* tw,
                   DotArgs dot) {
    constexpr int LM = ytx_max_log<R, N>();
    const int L = std::min(std::max(ylog, 0), LM);
    if constexpr (LM >= 2)
      if (L == 2) return yinv_L<N, 2>(st, G1, x, y, map, a0, a1, S, act, va, tw, dot);
    if constexpr (LM >= 1)
      if (L == 1) return yinv_L<N, 1>(st, G1, x, y, map, a0, a1, S, act, va, tw, dot);
    yinv_L<N, 0>(st, G1, x, y, map, a0, a1, S, act, va, tw, dot);
  }
  template <int N, bool INV, int RW>
  static void xpass_rw(hipStream_t st, const cx<R>* in, cx<R>* out, long nrows, int lin_stride, int lout_stride,
                       int Lin, int Lout, long rows_per_rhs, const int* act, const cx<R>* tw) {
    dim3 grid((unsigned)((nrows + RW - 1) / RW));
    hipLaunchKernelGGL((k_fast_x<R, INV, N, RW>), grid, dim3(FastPlan<N>::T * RW), 0, st, in, out, nrows, lin_stride,
                       lout_stride, Lin, Lout, rows_per_rhs, act, tw);
  }
  template <int N, bool INV>
  static void xpass(int xsel, hipStream_t st, const cx<R>* in, cx<R>* out, long nrows, int lin_stride,
                    int lout_stride, int Lin, int Lout, long rows_per_rhs, const int* act, const cx<R>* tw) {
    constexpr int B = fast_rw<N>(), R1 = xrows_variant<R, N>(B, 1), R2 = xrows_variant<R, N>(B, 2);
    if (xsel == 1 && R1 != B)
      return xpass_rw<N, INV, R1>(st, in, out, nrows, lin_stride, lout_stride, Lin, Lout, rows_per_rhs, act, tw);
    if (xsel == 2 && R2 != B)
      return xpass_rw<N, INV, R2>(st, in, out, nrows, lin_stride, lout_stride, Lin, Lout, rows_per_rhs, act, tw);
    xpass_rw<N, INV, B>(st, in, out, nrows, lin_stride, lout_stride, Lin, Lout, rows_per_rhs, act, tw);
  }
  template <int N>
  static void zsplit(int nrhs, hipStream_t st, cx<R>* G2, const cx<R>* Y, const int* act, ZArgs za,
                     const cx<R>* tw) {
    constexpr int TX = fast_txz<R, N>();
    ZMap zm;
    zm.NX = (za.Kpp + TX - 1) / TX;
    zm.ngx = (zm.NX + 1) / 2;
    zm.ngy = za.Jpp / 2 + 1;
    zm.ngroups = nrhs * zm.ngx * zm.ngy;
    dim3 grid(32 * ((zm.ngroups + 7) / 8));
    hipLaunchKernelGGL((k_fast_zsplit<R, N, TX>), grid, dim3(3 * FastPlan<N>::T * TX), 0, st, G2, Y, act, za, zm, tw);
  }
  // two-level z pass: one right-hand side per block unless the target asks
  // for more (DDA_OPT_RHS_PER_BLOCK).  Several per block reuse the spectrum
  // tile from the caches (8% faster on a full 128-RHS batch of the 96^3
  // ellipsoid), but inside a solve the active right-hand sides thin out and a
  // block then runs its few active ones in turn where one block each would
  // run side by side (the batched solve took 21.5 s instead of 16.7 s).
  // x passes to and from the tile-blocked layout of the two-level z pass
  // rows per block of the x passes to and from the tile-blocked layout:
  // enough that a block's share of a tile (RW x C values) is a run of at
  // least 512 bytes, within 1024 threads and 64 KB of LDS
  template <int N>
  static constexpr int xb_rows() {
    constexpr int C = Z2Shape<R, N, true>::C, T = FastPlan<N>::T, LS = N + N / 8 + 1;
    int rw = fast_rw<N>();
    while (rw * C * (int)sizeof(cx<R>) < 512 && 2 * rw * T <= 1024 && 2 * rw * LS * (int)sizeof(cx<R>) <= 65536)
      rw *= 2;
    return rw;
  }
  template <int N, bool INV>
  static void xb(int xsel, const dda_target* t, int nrhs, int C, hipStream_t st, const cx<R>* in, cx<R>* out,
                 const int* act, const cx<R>* tw) {
    constexpr int B = xb_rows<N>(), R1 = xrows_variant<R, N>(B, 1), R2 = xrows_variant<R, N>(B, 2);
    if (xsel == 1 && R1 != B) return xb_rw<N, INV, R1>(t, nrhs, C, st, in, out, act, tw);
    if (xsel == 2 && R2 != B) return xb_rw<N, INV, R2>(t, nrhs, C, st, in, out, act, tw);
    xb_rw<N, INV, B>(t, nrhs, C, st, in, out, act, tw);
  }
  template <int N, bool INV, int RW>
  static void xb_rw(const dda_target* t, int nrhs, int C, hipStream_t st, const cx<R>* in, cx<R>* out,
                    const int* act, const cx<R>* tw) {
    int lc = 0;
    while ((1 << lc) < C) ++lc;
    const int NT = (t->Kpp + C - 1) / C;
    dim3 grid((t->P + RW - 1) / RW, t->Jpp, nrhs * 3);
    hipLaunchKernelGGL((k_xb<R, INV, N, RW>), grid, dim3(FastPlan<N>::T * RW), 0, st, in, out, t->K, t->P, t->Jpp,
                       NT, lc, act, tw);
  }
  template <int N, bool BLK>
  static void z2(int nrhs, int rb, hipStream_t st, cx<R>* G2, const cx<R>* Y, const int* act, ZArgs za,
                 const cx<R>* tw) {
    using SH = Z2Shape<R, N, BLK>;
    if constexpr (SH::ok) {
      constexpr int T = SH::T, C = SH::C, W = SH::W;
      Z2Map zm;
      zm.NX = (za.Kpp + C - 1) / C;
      zm.ngx = (zm.NX + 1) / 2;
      zm.ngy = za.Jpp / 2 + 1;
      const int per = zm.ngx * zm.ngy;
      zm.nrhs = nrhs;
      zm.RB = rb > 0 ? std::min(rb, nrhs) : 1;
      zm.ngroups = ((nrhs + zm.RB - 1) / zm.RB) * per;
      dim3 grid(32 * ((zm.ngroups + 7) / 8));
      hipLaunchKernelGGL((k_z2<R, N, T, W, BLK, SH::WPE>), grid, dim3(64 * W), 0, st, G2, Y, act, za, zm, tw);
    }
  }
  template <int N>
  static void zmul(int nrhs, hipStream_t st, cx<R>* G2, const cx<R>* Y, const int* act, ZArgs za, const cx<R>* tw) {
    constexpr int TX = fast_txz<R, N>();
    ZMap zm;
    zm.NX = (za.Kpp + TX - 1) / TX;
    zm.ngx = (zm.NX + 1) / 2;
    zm.ngy = za.Jpp / 2 + 1;
    zm.ngroups = nrhs * zm.ngx * zm.ngy;
    dim3 grid(32 * ((zm.ngroups + 7) / 8));
    hipLaunchKernelGGL((k_fast_zmul<R, N, TX>), grid, dim3(FastPlan<N>::T * TX), 0, st, G2, Y, act, za, zm, tw);
  }
};

// y = A x (jacobi = 0) or D^{-1/2} A D^{-1/2} x (jacobi = 1); S and active are
// device arrays [nrhs] (nullable).
// ---- fused xy-plane passes ------------------------------------------------
#define DDA_XY_SIZES(X) X(32, 2) X(64, 2) X(64, 4) X(128, 2) X(128, 4) X(128, 8) X(256, 2) X(256, 4) \
  X(256, 8) X(96, 2) X(96, 4) X(192, 2) X(192, 4) X(192, 8)
static const size_t kXYLds = 80 * 1024;

template <typename R, int NN, int D>
static size_t xy_fwd_lds(int K) {
  using PL = XYPlan<R, NN, D>;
  const int KP = ((K + PL::CA - 1) / PL::CA) * PL::CA;
  return ((size_t)PL::M * KP + (size_t)PL::RB * PL::LSB) * sizeof(cx<R>);
}
template <typename R, int NN, int D>
static size_t xy_inv_lds(int K) {
  constexpr int M = NN / D;
  constexpr int TXT = FastPlan<M>::T, RX = 256 / TXT, LSX = M + M / 8 + 1;
  constexpr int CY = 256 / FastPlan<NN>::T;
  const int Q = (K + D - 1) / D;
  const int QP = ((Q + CY - 1) / CY) * CY;
  return ((size_t)NN * QP + (size_t)RX * LSX) * sizeof(cx<R>);
}

// Residue splits D of the fused xy-plane passes that exist for this lattice
// and fit the LDS budget (both directions).
template <typename R>
static std::vector<int> xy_candidates_of(int K, int J, int Kpp, int Jpp) {
  std::vector<int> out;
  if (Kpp != Jpp || 2 * K > Kpp || 2 * J > Jpp) return out;
#define DDA_CASE(NN, D)                                                                      \
  if (Kpp == NN && xy_fwd_lds<R, NN, D>(K) <= kXYLds && xy_inv_lds<R, NN, D>(K) <= kXYLds) \
    out.push_back(D);
  DDA_XY_SIZES(DDA_CASE)
#undef DDA_CASE
  return out;
}
template <typename R>
static std::vector<int> xy_candidates(const dda_target* t) {
  return xy_candidates_of<R>(t->K, t->J, t->Kpp, t->Jpp);
}

// why schedule `value` does not exist for a lattice padded to Kpp x Jpp x
// Ppp (nullptr: it exists in both precisions)
static const char* schedule_missing(int value, int K, int J, int Kpp, int Jpp, int Ppp) {
  if (value == 1 && !(fast_y_size(Kpp) && fast_size(Ppp))) return "no z-contiguous schedule";
  if (value == 3 && !fast_size(Ppp)) return "no component-split z pass";
  if (value == 5 && !z2_size(Ppp)) return "no two-level z pass";
  if (value == 6 && !(z2_size(Ppp) && fast_size(Kpp))) return "no tile-blocked schedule";
  if (value >= 2 && value != 3 && value != 5 && value != 6) {
    const std::vector<int> c64c = xy_candidates_of<double>(K, J, Kpp, Jpp),
                           c32c = xy_candidates_of<float>(K, J, Kpp, Jpp);
    if (std::find(c64c.begin(), c64c.end(), value) == c64c.end() ||
        std::find(c32c.begin(), c32c.end(), value) == c32c.end())
      return "no fused schedule with this split";
  }
  return nullptr;
}

template <typename R, int NN, int D>
static int launch_xy_fwd(dda_target* t, int nrhs, hipStream_t st, const cx<R>* x, cx<R>* G2, const cx<R>* a0,
                         const cx<R>* a1, const double* dS, const int* act, const VecArgs& va) {
  const size_t lds = xy_fwd_lds<R, NN, D>(t->K);
  static std::atomic<bool> attr{false};  // set once per process (idempotent)
  if (!attr.load()) {
    HIPCHK(hipFuncSetAttribute((const void*)k_xy_fwd<R, NN, D>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kXYLds));
    attr = true;
  }
  const int ngroups = nrhs * 3 * t->P;
  dim3 grid(8 * D * ((ngroups + 7) / 8));
  hipLaunchKernelGGL((k_xy_fwd<R, NN, D>), grid, dim3(256), lds, st, x, G2, occ_of(t), a0, a1, dS, act, va,
                     ngroups, bufs<R>(t).tw[1].template as<cx<R>>(), bufs<R>(t).tw[0].template as<cx<R>>());
  LAUNCHCHK();
  return DDA_OK;
}

template <typename R, int NN, int D>
static int launch_xy_inv(dda_target* t, int nrhs, hipStream_t st, const cx<R>* G2, const cx<R>* x, cx<R>* y,
                         const cx<R>* a0, const cx<R>* a1, const double* dS, const int* act, const VecArgs& va,
                         DotArgs dot) {
  const size_t lds = xy_inv_lds<R, NN, D>(t->K);
  static std::atomic<bool> attr{false};  // set once per process (idempotent)
  if (!attr.load()) {
    HIPCHK(hipFuncSetAttribute((const void*)k_xy_inv<R, NN, D>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kXYLds));
    attr = true;
  }
  const int ngroups = nrhs * 3 * t->P;
  dim3 grid(8 * D * ((ngroups + 7) / 8));
  hipLaunchKernelGGL((k_xy_inv<R, NN, D>), grid, dim3(256), lds, st, G2, x, y, occ_of(t), a0, a1, dS, act,
                     va, ngroups, bufs<R>(t).tw[1].template as<cx<R>>(), bufs<R>(t).tw[0].template as<cx<R>>(), dot);
  LAUNCHCHK();
  return DDA_OK;
}

// Schedules: 0 five passes (strided z tiles), 1 five passes (z-contiguous),
// 3 five passes (z pass on three component groups), D in {2, 4, 8} fused xy.
static inline bool is_fused(int s) { return s == 2 || s == 4 || s == 8; }

// blocks per right-hand side of the last matvec pass (fused-dot partials)
template <typename R>
static int schedule_of(const dda_target* t, int nrhs);
template <typename R>
static int ylog_of(const dda_target* t, int nrhs);
template <typename R>
static int xsel_of(const dda_target* t, int nrhs);

template <typename R>
static int yinv_blocks(const dda_target* t, int nrhs) {
  const int sc = schedule_of<R>(t, nrhs);
  if (is_fused(sc)) return 3 * t->P * sc;
  int tx = 0;
  switch (t->Jpp) {
#define DDA_CASE(N)                                           \
  case N:                                                     \
    tx = FastLaunch<R>::template ytx<N>(ylog_of<R>(t, nrhs)); \
    break;
    DDA_FAST_Y_SIZES(DDA_CASE)
#undef DDA_CASE
    default:
      tx = tile_width<R>(t->K, t->Jpp, 2);
  }
  return 3 * t->P * ((t->K + tx - 1) / tx);
}

// qf (fused QMR_sym step): the y-forward pass forms its input from the
// step's vectors (qmr_fusable schedules only).
template <typename R>
static int matvec_passes(dda_target* t, int nrhs, const double* dS, int jacobi, const cx<R>* x, cx<R>* y,
                         const int* active, hipStream_t st, DotArgs dot, const QmrFuse<R>* qf);

template <typename R>
static int matvec_T(dda_target* t, int nrhs, const double* dS, int jacobi, const cx<R>* x, cx<R>* y,
                    const int* active, hipStream_t st, DotArgs dot = DotArgs(), const QmrFuse<R>* qf = nullptr) {
  PassTimer pt(t->lib, PASS_MATVEC + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, !t->ws_over[0]);
  return matvec_passes<R>(t, nrhs, dS, jacobi, x, y, active, st, dot, qf);
}

template <typename R>
static int matvec_passes(dda_target* t, int nrhs, const double* dS, int jacobi, const cx<R>* x, cx<R>* y,
                         const int* active, hipStream_t st, DotArgs dot, const QmrFuse<R>* qf) {
  const bool own_ws = !t->ws_over[0];
  if (own_ws) CHK(ensure_matvec_ws<R>(t, nrhs));
  PrecBufs<R>& b = bufs<R>(t);
  const int K = t->K, J = t->J, P = t->P, Jpp = t->Jpp, Kpp = t->Kpp, Ppp = t->Ppp;
  cx<R>* G1 = own_ws ? b.G1.template as<cx<R>>() : (cx<R>*)t->ws_over[0];
  cx<R>* G2 = own_ws ? b.G2.template as<cx<R>>() : (cx<R>*)t->ws_over[1];
  const cx<R>* a0 = b.a0.template as<cx<R>>();
  const cx<R>* a1 = t->has_a1 ? b.a1.template as<cx<R>>() : nullptr;
  VecArgs va;
  va.nrhs = nrhs;
  va.K = K;
  va.J = J;
  va.P = P;
  va.Jpp = Jpp;
  va.Kpp = Kpp;
  va.Ppp = Ppp;
  va.nd = t->nd;
  va.dstride = t->aniso ? t->nd : 0;
  if (t->comp_bits) {
    va.mbits = t->mbits.as<uint32_t>();
    va.mlb = t->mlb;
    va.mt0 = b.mt0.p;
    va.mt1 = t->has_a1 ? b.mt1.p : nullptr;
  } else if (t->uniform_diag) {
    va.uniform = 1;
    va.mt0 = b.mt0.p;
    va.mt1 = t->has_a1 ? b.mt1.p : nullptr;
  }
  va.jacobi = jacobi;
  va.scale = 1.0 / ((double)Kpp * Jpp * Ppp);
  va.TX = tile_width<R>(K, Jpp, 2);
  const int sched = schedule_of<R>(t, nrhs), ylog = ylog_of<R>(t, nrhs), xsel = xsel_of<R>(t, nrhs);
  const int dfwd = is_fused(sched) ? sched : 0, dinv = dfwd;
  if (dfwd && qf) return fail(DDA_EINVAL, "matvec: fused QMR step needs the register-resident y pass");
  if (dfwd) {
    // fused: xy forward -> z with product -> xy inverse
    {
      PassTimer pt(t->lib, PASS_XYFWD + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
      int rc = DDA_EINVAL;
#define DDA_CASE(NN, D)                                                                          \
  if (Kpp == NN && dfwd == D) rc = launch_xy_fwd<R, NN, D>(t, nrhs, st, x, G2, a0, a1, dS, active, va);
      DDA_XY_SIZES(DDA_CASE)
#undef DDA_CASE
      CHK(rc);
    }
    {
      PassTimer pt(t->lib, PASS_ZMUL + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
      ZArgs za;
      za.Kpp = Kpp;
      za.Jpp = Jpp;
      za.P = P;
      za.Ppp = Ppp;
      za.Kh = t->Kh;
      za.Jh = t->Jh;
      za.Ph = t->Ph;
      if (fast_size(Ppp)) {
        switch (Ppp) {
#define DDA_CASE(N)                                                                                      \
  case N:                                                                                                \
    FastLaunch<R>::template zmul<N>(nrhs, st, G2, b.Y.template as<cx<R>>(), active, za,                   \
                                    b.tw[2].template as<cx<R>>());                                        \
    break;
          DDA_FAST_SIZES(DDA_CASE)
#undef DDA_CASE
        }
      } else {
        za.TX = tile_width<R>(Kpp, Ppp, 4);
        const size_t lds = 4 * (size_t)Ppp * za.TX * sizeof(cx<R>);
        dim3 grid((Kpp + za.TX - 1) / za.TX, Jpp, nrhs);
        hipLaunchKernelGGL((k_vec_zmul<R>), grid, dim3(kThreads), lds, st, G2, b.Y.template as<cx<R>>(), active,
                           za, t->fz, b.tw[2].template as<cx<R>>());
      }
      LAUNCHCHK();
    }
    {
      PassTimer pt(t->lib, PASS_XYINV + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
      int rc = DDA_EINVAL;
#define DDA_CASE(NN, D)                                                                                   \
  if (Kpp == NN && dinv == D) rc = launch_xy_inv<R, NN, D>(t, nrhs, st, G2, x, y, a0, a1, dS, active, va, dot);
      DDA_XY_SIZES(DDA_CASE)
#undef DDA_CASE
      CHK(rc);
    }
    t->matvecs += 1;
    return DDA_OK;
  }
  {
    PassTimer pt(t->lib, PASS_YFWD + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
    if (fast_y_size(Jpp)) {
      switch (Jpp) {
#define DDA_CASE(N)                                                                                         \
  case N:                                                                                                   \
    FastLaunch<R>::template yfwd<N>(ylog, st, x, G1, occ_of(t), a0, a1, dS, active, va, \
                                    b.tw[1].template as<cx<R>>(), qf);                                        \
    break;
        DDA_FAST_Y_SIZES(DDA_CASE)
#undef DDA_CASE
      }
    } else {
      if (qf) return fail(DDA_EINVAL, "matvec: fused QMR step needs the register-resident y pass");
      const size_t lds = 2 * (size_t)Jpp * va.TX * sizeof(cx<R>);
      dim3 grid((K + va.TX - 1) / va.TX, P, nrhs * 3);
      hipLaunchKernelGGL((k_vec_yfwd<R>), grid, dim3(kThreads), lds, st, x, G1, occ_of(t), a0, a1, dS,
                         active, va, t->fy, b.tw[1].template as<cx<R>>());
    }
    LAUNCHCHK();
  }
  const long rows = (long)nrhs * 3 * P * Jpp;
  if (sched == 6) {
    // tile-blocked layout: x forward into z tiles -> two-level z pass -> x inverse
    const int C = z2_cols<R>(Ppp);
    ZArgs za;
    za.Kpp = Kpp;
    za.Jpp = Jpp;
    za.P = P;
    za.Ppp = Ppp;
    za.Kh = t->Kh;
    za.Jh = t->Jh;
    za.Ph = t->Ph;
    {
      PassTimer pt(t->lib, PASS_XFWD + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
      switch (Kpp) {
#define DDA_CASE(N)                                                                                          \
  case N:                                                                                                    \
    FastLaunch<R>::template xb<N, false>(xsel, t, nrhs, C, st, G1, G2, active, b.tw[0].template as<cx<R>>());    \
    break;
        DDA_FAST_SIZES(DDA_CASE)
#undef DDA_CASE
      }
      LAUNCHCHK();
    }
    {
      PassTimer pt(t->lib, PASS_ZMUL + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
      switch (Ppp) {
#define DDA_CASE(N)                                                                                      \
  case N:                                                                                                \
    FastLaunch<R>::template z2<N, true>(nrhs, t->z_rb, st, G2, b.Yz.template as<cx<R>>(), active, za,     \
                                        b.tw[2].template as<cx<R>>());                                    \
    break;
        DDA_FAST_SIZES(DDA_CASE)
#undef DDA_CASE
      }
      LAUNCHCHK();
    }
    {
      PassTimer pt(t->lib, PASS_XINV + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
      switch (Kpp) {
#define DDA_CASE(N)                                                                                         \
  case N:                                                                                                   \
    FastLaunch<R>::template xb<N, true>(xsel, t, nrhs, C, st, G2, G1, active, b.tw[0].template as<cx<R>>());     \
    break;
        DDA_FAST_SIZES(DDA_CASE)
#undef DDA_CASE
      }
      LAUNCHCHK();
    }
  } else if (sched == 1) {
    // z-contiguous layout: x forward (transposed out) -> z lines -> x inverse (transposed in)
    {
      PassTimer pt(t->lib, PASS_XFWD + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
      switch (Kpp) {
#define DDA_CASE(N)                                                                               \
  case N:                                                                                         \
    FastLaunch<R>::template xT<N>(false, nrhs, st, G1, G2, t, active, b.tw[0].template as<cx<R>>()); \
    break;
        DDA_FAST_Y_SIZES(DDA_CASE)
#undef DDA_CASE
        default:
          return fail(DDA_EINVAL, "matvec: no transposing x pass of length %d", Kpp);
      }
      LAUNCHCHK();
    }
    {
      PassTimer pt(t->lib, PASS_ZMUL + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
      ZArgs za;
      za.Kpp = Kpp;
      za.Jpp = Jpp;
      za.P = P;
      za.Ppp = Ppp;
      za.Kh = t->Kh;
      za.Jh = t->Jh;
      za.Ph = t->Ph;
      switch (Ppp) {
#define DDA_CASE(N)                                                                                        \
  case N:                                                                                                  \
    FastLaunch<R>::template zline<N>(nrhs, st, G2, b.Yz.template as<cx<R>>(), active, za,                   \
                                     b.tw[2].template as<cx<R>>());                                         \
    break;
        DDA_FAST_SIZES(DDA_CASE)
#undef DDA_CASE
      }
      LAUNCHCHK();
    }
    {
      PassTimer pt(t->lib, PASS_XINV + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
      switch (Kpp) {
#define DDA_CASE(N)                                                                              \
  case N:                                                                                        \
    FastLaunch<R>::template xT<N>(true, nrhs, st, G2, G1, t, active, b.tw[0].template as<cx<R>>()); \
    break;
        DDA_FAST_Y_SIZES(DDA_CASE)
#undef DDA_CASE
        default:
          return fail(DDA_EINVAL, "matvec: no transposing x pass of length %d", Kpp);
      }
      LAUNCHCHK();
    }
  } else {
  {
  PassTimer pt(t->lib, PASS_XFWD + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
  if (fast_size(Kpp)) {
    switch (Kpp) {
#define DDA_CASE(N)                                                                                          \
  case N:                                                                                                    \
    FastLaunch<R>::template xpass<N, false>(xsel, st, G1, G2, rows, K, Kpp, K, Kpp, 3L * P * Jpp, active,           \
                                            b.tw[0].template as<cx<R>>());                                   \
    break;
      DDA_FAST_SIZES(DDA_CASE)
#undef DDA_CASE
    }
    LAUNCHCHK();
  } else {
    CHK(launch_contig<R>(G1, G2, rows, K, Kpp, K, Kpp, t->fx, b.tw[0].template as<cx<R>>(), false, false, 0, 0,
                         3L * P * Jpp, active, 1.0, st));
  }
  }
  {
    PassTimer pt(t->lib, PASS_ZMUL + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
    ZArgs za;
    za.Kpp = Kpp;
    za.Jpp = Jpp;
    za.P = P;
    za.Ppp = Ppp;
    za.Kh = t->Kh;
    za.Jh = t->Jh;
    za.Ph = t->Ph;
    if (sched == 5 && z2_size<R>(Ppp)) {
      switch (Ppp) {
#define DDA_CASE(N)                                                                                      \
  case N:                                                                                                \
    FastLaunch<R>::template z2<N, false>(nrhs, t->z_rb, st, G2, b.Yz.template as<cx<R>>(), active, za,    \
                                  b.tw[2].template as<cx<R>>());                                          \
    break;
        DDA_FAST_SIZES(DDA_CASE)
#undef DDA_CASE
      }
    } else if (fast_size(Ppp) && sched == 3) {
      switch (Ppp) {
#define DDA_CASE(N)                                                                                      \
  case N:                                                                                                \
    FastLaunch<R>::template zsplit<N>(nrhs, st, G2, b.Y.template as<cx<R>>(), active, za,                 \
                                      b.tw[2].template as<cx<R>>());                                      \
    break;
        DDA_FAST_SIZES(DDA_CASE)
#undef DDA_CASE
      }
    } else if (fast_size(Ppp)) {
      switch (Ppp) {
#define DDA_CASE(N)                                                                                      \
  case N:                                                                                                \
    FastLaunch<R>::template zmul<N>(nrhs, st, G2, b.Y.template as<cx<R>>(), active, za,                   \
                                    b.tw[2].template as<cx<R>>());                                        \
    break;
        DDA_FAST_SIZES(DDA_CASE)
#undef DDA_CASE
      }
    } else {
      za.TX = tile_width<R>(Kpp, Ppp, 4);
      const size_t lds = 4 * (size_t)Ppp * za.TX * sizeof(cx<R>);
      dim3 grid((Kpp + za.TX - 1) / za.TX, Jpp, nrhs);
      hipLaunchKernelGGL((k_vec_zmul<R>), grid, dim3(kThreads), lds, st, G2, b.Y.template as<cx<R>>(), active, za,
                         t->fz, b.tw[2].template as<cx<R>>());
    }
    LAUNCHCHK();
  }
  {
  PassTimer pt(t->lib, PASS_XINV + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
  if (fast_size(Kpp)) {
    switch (Kpp) {
#define DDA_CASE(N)                                                                                         \
  case N:                                                                                                   \
    FastLaunch<R>::template xpass<N, true>(xsel, st, G2, G1, rows, Kpp, K, Kpp, K, 3L * P * Jpp, active,           \
                                           b.tw[0].template as<cx<R>>());                                   \
    break;
      DDA_FAST_SIZES(DDA_CASE)
#undef DDA_CASE
    }
    LAUNCHCHK();
  } else {
    CHK(launch_contig<R>(G2, G1, rows, Kpp, K, Kpp, K, t->fx, b.tw[0].template as<cx<R>>(), true, false, 0, 0,
                         3L * P * Jpp, active, 1.0, st));
  }
  }
  }
  {
    PassTimer pt(t->lib, PASS_YINV + (sizeof(R) == 4 ? PASS_PER_PREC : 0), st, own_ws);
    if (fast_y_size(Jpp)) {
      switch (Jpp) {
#define DDA_CASE(N)                                                                                             \
  case N:                                                                                                       \
    FastLaunch<R>::template yinv<N>(ylog, st, G1, x, y, occ_of(t), a0, a1, dS, active, va, \
                                    b.tw[1].template as<cx<R>>(), dot);                                           \
    break;
        DDA_FAST_Y_SIZES(DDA_CASE)
#undef DDA_CASE
      }
    } else {
      const size_t lds = 2 * (size_t)Jpp * va.TX * sizeof(cx<R>);
      dim3 grid((K + va.TX - 1) / va.TX, P, nrhs * 3);
      hipLaunchKernelGGL((k_vec_yinv<R>), grid, dim3(kThreads), lds, st, G1, x, y, occ_of(t), a0, a1, dS,
                         active, va, t->fy, b.tw[1].template as<cx<R>>(), dot);
    }
    LAUNCHCHK();
  }
  t->matvecs += 1;
  return DDA_OK;
}

// ----------------------------------------------------------------------------
// Autotuner: the matrix-vector schedule (five passes, or fused xy-plane
// passes with residue split D) is chosen per (lattice, padded sizes, number of
// right-hand sides, precision) by timing each candidate on the first product
// of that kind (HIP events, 2 warm-up + 3 timed products on the caller's
// stream), the analogue of planning by measurement.  Choices are kept in the
// library handle and appended to the tune-cache file when one was given.
// ----------------------------------------------------------------------------
template <typename R>
static std::string tune_key(const dda_target* t, int nrhs) {
  std::ostringstream k;
  k << "mv " << t->K << "x" << t->J << "x" << t->P << " pad " << t->Kpp << "x" << t->Jpp << "x" << t->Ppp << " nrhs "
    << nrhs << " " << (sizeof(R) == 4 ? "fp32" : "fp64");
  return k.str();
}

// A plan is the schedule in its low 4 bits, the y-tile variant (log2 of the
// multiple of the default y tile) in bits 4-5 and the x-pass rows variant
// (0 the default rows per block, 1 half, 2 twice) in bits 6-7.
template <typename R>
static int plan_of(const dda_target* t, int nrhs) {
  if (t->sched_override >= 0) return t->sched_override;
  int v = 0;  // untuned: the strided five-pass schedule, default y tile
  if (t->forced_sched >= 0) {
    // the two-level z pass is not built for every length in FP64: the
    // five plain passes stand in for it there
    v = ((t->forced_sched == 5 || t->forced_sched == 6) && !z2_size<R>(t->Ppp)) ? 0 : t->forced_sched;
  } else {
    const std::string key = tune_key<R>(t, nrhs);
    std::lock_guard<std::mutex> g(t->lib->tune_mu);
    auto it = t->lib->tuned.find(key);
    if (it != t->lib->tuned.end()) v = it->second;
  }
  if (t->forced_ylog >= 0) v = (v & ~(3 << 4)) | (t->forced_ylog << 4);
  if (t->forced_xsel >= 0) v = (v & ~(3 << 6)) | (t->forced_xsel << 6);
  return v;
}
template <typename R>
static int schedule_of(const dda_target* t, int nrhs) {
  return plan_of<R>(t, nrhs) & 15;
}
template <typename R>
static int ylog_of(const dda_target* t, int nrhs) {
  return (plan_of<R>(t, nrhs) >> 4) & 3;
}
template <typename R>
static int xsel_of(const dda_target* t, int nrhs) {
  return (plan_of<R>(t, nrhs) >> 6) & 3;
}

// widest y-tile variant of this lattice's y length in precision R (0 where
// the y pass is not register-resident)
template <typename R>
static int ylog_max(const dda_target* t) {
  switch (t->Jpp) {
#define DDA_CASE(N) \
  case N:           \
    return ytx_max_log<R, N>();
    DDA_FAST_Y_SIZES(DDA_CASE)
#undef DDA_CASE
  }
  return 0;
}

template <typename R>
static int autotune(dda_target* t, int nrhs, const double* dS, int jacobi, const cx<R>* x, cx<R>* y,
                    hipStream_t st) {
  if (t->forced_sched >= 0) return DDA_OK;
  const std::string key = tune_key<R>(t, nrhs);
  {
    std::lock_guard<std::mutex> g(t->lib->tune_mu);
    if (t->lib->tuned.count(key)) return DDA_OK;
  }
  std::vector<int> cand = {0};
  if (fast_y_size(t->Kpp) && fast_size(t->Ppp)) cand.push_back(1);
  if (fast_size(t->Ppp)) cand.push_back(3);
  // the tile-blocked schedule before the strided one: it measured as fast or
  // faster on every workload here, so near-ties keep it
  if (z2_size<R>(t->Ppp) && fast_size(t->Kpp)) cand.push_back(6);
  if (z2_size<R>(t->Ppp)) cand.push_back(5);
  for (int d : xy_candidates<R>(t)) cand.push_back(d);
  int best = 0;
  if (cand.size() > 1) {
    const int prof = t->lib->prof;
    if (prof) t->lib->prof = 0;  // (profiling runs single-threaded)
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // candidates timed round-robin (three rounds of three matvecs after two
    // warm-ups each); each keeps its fastest round, so a cold start or a
    // disturbance in one round does not decide
    std::vector<float> best_c(cand.size(), 1e30f);
    int rc = DDA_OK;
    for (size_t ci = 0; ci < cand.size() && rc == DDA_OK; ++ci) {
      t->sched_override = cand[ci];
      for (int w = 0; w < 2 && rc == DDA_OK; ++w) rc = matvec_T<R>(t, nrhs, dS, jacobi, x, y, nullptr, st);
    }
    for (int round = 0; round < 3 && rc == DDA_OK; ++round)
      for (size_t ci = 0; ci < cand.size() && rc == DDA_OK; ++ci) {
        t->sched_override = cand[ci];
        (void)hipEventRecord(e0, st);
        for (int w = 0; w < 3 && rc == DDA_OK; ++w) rc = matvec_T<R>(t, nrhs, dS, jacobi, x, y, nullptr, st);
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        best_c[ci] = std::min(best_c[ci], ms);
      }
    // a later candidate must win by more than 3% (near-ties keep the earlier,
    // simpler schedule, so that repeated tunings agree; the five-pass
    // schedules also let QMR_sym fuse its step into the y pass)
    float best_ms = best_c[0];
    best = cand[0];
    for (size_t ci = 1; ci < cand.size(); ++ci)
      if (best_c[ci] < 0.97f * best_ms) {
        best_ms = best_c[ci];
        best = cand[ci];
      }
    t->matvecs -= 11 * (int)cand.size();
    // then the variants of the chosen schedule's y tiles and x-pass rows,
    // the same way, one dimension after the other
    auto time_plan = [&](int plan) -> float {
      t->sched_override = plan;
      float bl = 1e30f;
      for (int w = 0; w < 2 && rc == DDA_OK; ++w) rc = matvec_T<R>(t, nrhs, dS, jacobi, x, y, nullptr, st);
      for (int round = 0; round < 3 && rc == DDA_OK; ++round) {
        (void)hipEventRecord(e0, st);
        for (int w = 0; w < 3 && rc == DDA_OK; ++w) rc = matvec_T<R>(t, nrhs, dS, jacobi, x, y, nullptr, st);
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        bl = std::min(bl, ms);
      }
      t->matvecs -= 11;
      return bl;
    };
    if (!is_fused(best) && t->forced_ylog < 0) {
      const int base = best;
      for (int L = 1; L <= ylog_max<R>(t) && rc == DDA_OK; ++L) {
        const float bl = time_plan(base | (L << 4));
        if (bl < 0.97f * best_ms) {
          best_ms = bl;
          best = base | (L << 4);
        }
      }
    }
    if (!is_fused(best) && fast_size(t->Kpp) && t->forced_xsel < 0) {
      const int base = best;
      for (int xs = 1; xs <= 2 && rc == DDA_OK; ++xs) {
        const float bl = time_plan(base | (xs << 6));
        if (bl < 0.97f * best_ms) {
          best_ms = bl;
          best = base | (xs << 6);
        }
      }
    }
    t->sched_override = -1;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (prof) t->lib->prof = prof;
    CHK(rc);
  }
  std::lock_guard<std::mutex> g(t->lib->tune_mu);
  if (t->lib->tuned.count(key)) return DDA_OK;  // another worker tuned it meanwhile
  t->lib->tuned[key] = best;
  if (!t->lib->tune_path.empty()) {
    std::ofstream f(t->lib->tune_path, std::ios::app);
    if (f) f << key << " = " << best << "\n";
  }
  return DDA_OK;
}

// Padded lengths tried for lattice extent n: the smallest 2^a 3^b 5^c length
// >= 2n - 1, and the smallest length with register-resident kernels for
// every pass when it is at most twice that; the default rule's choice (for
// y, `yax`, counting the register-resident y passes) first.
static std::vector<int> padding_candidates(int n, bool yax) {
  const int m = 2 * n - 1;
  std::vector<int> c = {fft_size_at_least(m, yax)};
  int sm = m;
  while (!smooth235(sm)) ++sm;
  int f = m;
  while (!fast_size(f) && f <= 2 * sm) ++f;
  for (int v : {sm, f})
    if (padding_ok(n, v) && (v == sm || fast_size(v)) && std::find(c.begin(), c.end(), v) == c.end())
      c.push_back(v);
  return c;
}

// (a forced schedule narrows the candidate list, so it is part of the key:
// the recorded value is an index into that list)
static std::string padding_key(const dda_target* t, int nrhs, int precision) {
  std::ostringstream k;
  k << "pad " << t->K << "x" << t->J << "x" << t->P << " nrhs " << nrhs << " "
    << (precision == DDA_FP32 ? "fp32" : "fp64");
  if (t->forced_sched > 0) k << " schedule " << t->forced_sched;
  return k.str();
}

// One padding's product time: spectrum built for it, schedule tuned for it,
// then the fastest of three rounds of three products (after two warm-ups).
template <typename R>
static int time_padding(dda_target* t, int nrhs, const cx<R>* x, cx<R>* y, hipStream_t st, hipEvent_t e0,
                        hipEvent_t e1, float* out_ms) {
  CHK(dda_build_spectrum(t, st));
  CHK(ensure_matvec_ws<R>(t, nrhs));
  const double* dS = t->S.as<double>();
  CHK(autotune<R>(t, nrhs, dS, 1, x, y, st));
  for (int w = 0; w < 2; ++w) CHK(matvec_T<R>(t, nrhs, dS, 1, x, y, nullptr, st));
  float best = 1e30f;
  for (int round = 0; round < 3; ++round) {
    HIPCHK(hipEventRecord(e0, st));
    for (int w = 0; w < 3; ++w) CHK(matvec_T<R>(t, nrhs, dS, 1, x, y, nullptr, st));
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    best = std::min(best, ms);
  }
  *out_ms = best;
  return DDA_OK;
}

template <typename R>
static int tune_padding_T(dda_target* t, int nrhs, int precision, hipStream_t st) {
  const std::vector<int> ck = padding_candidates(t->K, false), cj = padding_candidates(t->J, true),
                         cp = padding_candidates(t->P, false);
  std::vector<std::array<int, 3>> combos;
  for (int a : ck)
    for (int b : cj)
      for (int c : cp)
        if (!(t->forced_sched > 0 && schedule_missing(t->forced_sched, t->K, t->J, a, b, c)))
          combos.push_back({a, b, c});
  if (combos.empty()) return DDA_OK;  // no candidate carries the forced schedule: the lengths stay
  const std::string key = padding_key(t, nrhs, precision);
  int pick = -1;
  {
    std::lock_guard<std::mutex> g(t->lib->tune_mu);
    auto it = t->lib->tuned.find(key);
    if (it != t->lib->tuned.end() && it->second >= 0 && it->second < (int)combos.size()) pick = it->second;
  }
  if (pick < 0 && combos.size() == 1) pick = 0;
  if (pick < 0) {
    const int k0 = t->Kpp, j0 = t->Jpp, p0 = t->Ppp;
    // product inputs: a fixed finite byte pattern (timing only), S = 0
    DevBuf xb, yb;
    const size_t vb = (size_t)nrhs * 3 * t->nd * sizeof(cx<R>);
    CHK(xb.ensure(vb));
    CHK(yb.ensure(vb));
    HIPCHK(hipMemsetAsync(xb.p, 0x3F, vb, st));
    CHK(ensure_scratch(t, nrhs));
    HIPCHK(hipMemsetAsync(t->S.p, 0, nrhs * sizeof(double), st));
    const int prof = t->lib->prof, mv = t->matvecs;
    t->lib->prof = 0;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int rc = DDA_OK;
    float best_ms = 1e30f;
    for (size_t i = 0; i < combos.size() && rc == DDA_OK; ++i) {
      rc = set_lengths(t, combos[i][0], combos[i][1], combos[i][2]);
      float ms = 1e30f;
      if (rc == DDA_OK) rc = time_padding<R>(t, nrhs, xb.as<cx<R>>(), yb.as<cx<R>>(), st, e0, e1, &ms);
      // a later padding must win by more than 3% (near-ties keep the
      // default rule's lengths, so that repeated tunings agree)
      if (rc == DDA_OK && (pick < 0 || ms < 0.97f * best_ms)) {
        best_ms = ms;
        pick = (int)i;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    t->lib->prof = prof;
    t->matvecs = mv;
    if (rc != DDA_OK) {  // back to the lengths the target had (its spectrum dropped)
      (void)hipStreamSynchronize(st);
      const std::string err = g_err;
      (void)set_lengths(t, k0, j0, p0);
      g_err = err;
      return rc;
    }
    HIPCHK(hipStreamSynchronize(st));  // the timing buffers are freed on return
    std::lock_guard<std::mutex> g(t->lib->tune_mu);
    if (!t->lib->tuned.count(key)) {
      t->lib->tuned[key] = pick;
      if (!t->lib->tune_path.empty()) {
        std::ofstream f(t->lib->tune_path, std::ios::app);
        if (f) f << key << " = " << pick << "\n";
      }
    }
  }
  const std::array<int, 3>& v = combos[pick];
  if (v[0] != t->Kpp || v[1] != t->Jpp || v[2] != t->Ppp) CHK(set_lengths(t, v[0], v[1], v[2]));
  if (!t->spec_ready) CHK(dda_build_spectrum(t, st));
  return DDA_OK;
}

extern "C" int dda_tune_padding(dda_target* t, int nrhs, int precision, int* lengths, void* hip_stream) {
  if (!t) return fail(DDA_EINVAL, "dda_tune_padding: NULL target");
  if (nrhs < 1) return fail(DDA_EINVAL, "dda_tune_padding: nrhs = %d", nrhs);
  if (precision != DDA_FP64 && precision != DDA_FP32)
    return fail(DDA_EINVAL, "dda_tune_padding: precision %d", precision);
  if (t->nd <= 0) return fail(DDA_ESTATE, "dda_tune_padding: occupancy not set");
  if (!t->have_alpha) return fail(DDA_ESTATE, "dda_tune_padding: polarisability not set");
  HIPCHK(hipSetDevice(t->lib->device));
  hipStream_t st = (hipStream_t)hip_stream;
  CHK(precision == DDA_FP64 ? tune_padding_T<double>(t, nrhs, precision, st)
                            : tune_padding_T<float>(t, nrhs, precision, st));
  if (lengths) {
    lengths[0] = t->Kpp;
    lengths[1] = t->Jpp;
    lengths[2] = t->Ppp;
  }
  return DDA_OK;
}

static int check_ready(dda_target* t, const char* who) {
  if (!t) return fail(DDA_EINVAL, "%s: NULL target", who);
  if (t->nd <= 0) return fail(DDA_ESTATE, "%s: occupancy not set", who);
  if (!t->have_alpha) return fail(DDA_ESTATE, "%s: polarisability not set", who);
  if (!t->spec_ready) return fail(DDA_ESTATE, "%s: spectrum not built", who);
  return DDA_OK;
}

extern "C" int dda_matvec(dda_target* t, int precision, int nrhs, const double* S, int jacobi, const void* x_dev,
                          void* y_dev, void* hip_stream) {
  CHK(check_ready(t, "dda_matvec"));
  if (nrhs < 1) return fail(DDA_EINVAL, "dda_matvec: nrhs = %d", nrhs);
  if (!x_dev || !y_dev) return fail(DDA_EINVAL, "dda_matvec: NULL vector");
  if (x_dev == y_dev) return fail(DDA_EINVAL, "dda_matvec: x and y must not alias");
  HIPCHK(hipSetDevice(t->lib->device));
  hipStream_t st = (hipStream_t)hip_stream;
  CHK(ensure_scratch(t, nrhs));
  std::vector<double> hs(nrhs, 0.0);
  if (S)
    for (int r = 0; r < nrhs; ++r) hs[r] = S[r];
  HIPCHK(hipMemcpyAsync(t->S.p, hs.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  // canaries: every workspace element starts as NaN (all bits set), so a pass
  // that reads what no earlier pass wrote poisons the product
  auto fill_canaries = [&](auto& b) -> int {
    if (!t->canary) return DDA_OK;
    HIPCHK(hipMemsetAsync(b.G1.p, 0xFF, b.G1.bytes, st));
    HIPCHK(hipMemsetAsync(b.G2.p, 0xFF, b.G2.bytes, st));
    return DDA_OK;
  };
  if (precision == DDA_FP64) {
    CHK(ensure_matvec_ws<double>(t, nrhs));
    CHK(autotune<double>(t, nrhs, t->S.as<double>(), jacobi ? 1 : 0, (const c64*)x_dev, (c64*)y_dev, st));
    CHK(fill_canaries(t->p64));
    return matvec_T<double>(t, nrhs, t->S.as<double>(), jacobi ? 1 : 0, (const c64*)x_dev, (c64*)y_dev, nullptr, st);
  }
  if (precision == DDA_FP32) {
    CHK(ensure_matvec_ws<float>(t, nrhs));
    CHK(autotune<float>(t, nrhs, t->S.as<double>(), jacobi ? 1 : 0, (const c32*)x_dev, (c32*)y_dev, st));
    CHK(fill_canaries(t->p32));
    return matvec_T<float>(t, nrhs, t->S.as<double>(), jacobi ? 1 : 0, (const c32*)x_dev, (c32*)y_dev, nullptr, st);
  }
  return fail(DDA_EINVAL, "dda_matvec: precision %d", precision);
}

// The product of dda_matvec with every device buffer it needs beyond x and y
// (the orientation factors and the FFT workspaces) in the device scratch:
// no allocation, no autotuning (the schedule is the tuned one if the library
// has it, else the five plain passes), no profiling events.
template <typename R>
static int matvec_noalloc_T(dda_target* t, int nrhs, const double* S, int jacobi, const cx<R>* x, cx<R>* y,
                            hipStream_t st) {
  const size_t sb = ((size_t)nrhs * sizeof(double) + 255) & ~(size_t)255;
  size_t g1, g2;
  matvec_ws_bytes<R>(t, nrhs, g1, g2);
  g1 = (g1 + 255) & ~(size_t)255;
  g2 = (g2 + 255) & ~(size_t)255;
  if (sb + g1 + g2 > kScratchBytes)
    return fail(DDA_EINVAL, "dda_matvec_noalloc: %d right-hand sides of this lattice need %zu bytes of scratch, "
                "the maximum is %zu", nrhs, sb + g1 + g2, kScratchBytes);
  unsigned char* base = t->lib->scratch_dev;
  double* dS = (double*)base;
  if (S) HIPCHK(hipMemcpyAsync(dS, S, nrhs * sizeof(double), hipMemcpyHostToDevice, st));
  else HIPCHK(hipMemsetAsync(dS, 0, nrhs * sizeof(double), st));
  if (t->canary) {
    HIPCHK(hipMemsetAsync(base + sb, 0xFF, g1, st));
    HIPCHK(hipMemsetAsync(base + sb + g1, 0xFF, g2, st));
  }
  t->ws_over[0] = base + sb;
  t->ws_over[1] = base + sb + g1;
  const int rc = matvec_T<R>(t, nrhs, dS, jacobi, x, y, nullptr, st);
  t->ws_over[0] = t->ws_over[1] = nullptr;
  CHK(rc);
  HIPCHK(hipStreamSynchronize(st));  // the caller's S may be reused at return
  return DDA_OK;
}

extern "C" int dda_matvec_noalloc(dda_target* t, int precision, int nrhs, const double* S, int jacobi,
                                  const void* x_dev, void* y_dev, void* hip_stream) {
  CHK(check_ready(t, "dda_matvec_noalloc"));
  if (nrhs < 1) return fail(DDA_EINVAL, "dda_matvec_noalloc: nrhs = %d", nrhs);
  if (!x_dev || !y_dev) return fail(DDA_EINVAL, "dda_matvec_noalloc: NULL vector");
  if (x_dev == y_dev) return fail(DDA_EINVAL, "dda_matvec_noalloc: x and y must not alias");
  if (!t->lib->scratch_dev) return fail(DDA_ESTATE, "dda_matvec_noalloc: no device scratch");
  HIPCHK(hipSetDevice(t->lib->device));
  hipStream_t st = (hipStream_t)hip_stream;
  if (precision == DDA_FP64)
    return matvec_noalloc_T<double>(t, nrhs, S, jacobi ? 1 : 0, (const c64*)x_dev, (c64*)y_dev, st);
  if (precision == DDA_FP32)
    return matvec_noalloc_T<float>(t, nrhs, S, jacobi ? 1 : 0, (const c32*)x_dev, (c32*)y_dev, st);
  return fail(DDA_EINVAL, "dda_matvec_noalloc: precision %d", precision);
}

// ----------------------------------------------------------------------------
// Krylov solvers
// ----------------------------------------------------------------------------
struct InnerResult {
  std::vector<int> iters, converged, breakdown;
  std::vector<double> rnorm2, bnorm2;
};

static int nblocks_for(long n3) {
  long b = (n3 + 2L * kRedThreads - 1) / (2L * kRedThreads);
  return (int)std::max(1L, std::min(b, 256L));
}

template <typename R>
static int ensure_solver_ws(dda_target* t, int nrhs, int nslots) {
  PrecBufs<R>& b = bufs<R>(t);
  if (b.vec_nd != t->nd) {  // sized for another occupancy: start over
    b.vec_cap = b.vec_slots = 0;
    b.vec_nd = t->nd;
  }
  if (nrhs <= b.vec_cap && nslots <= b.vec_slots) return DDA_OK;
  const int cap = std::max(nrhs, b.vec_cap), ns = std::max(nslots, b.vec_slots);
  CHK(b.vec.ensure((size_t)ns * cap * 3 * t->nd * sizeof(cx<R>)));
  b.vec_cap = cap;
  b.vec_slots = ns;
  return DDA_OK;
}

// Solver vectors a scheme needs (slot 0 = right-hand side, 1 = solution).
static int solver_slots(int solver, int param) {
  switch (solver) {
    case DDA_BICG: return 8;
    case DDA_QMR: return 11;
    case DDA_RBICGSTAB: return 5 + 2 * param;
    case DDA_MLBICGSTAB: return 4 + 3 * param;
    default: return 10;
  }
}

static int solver_param(const dda_solve_opts& o) {
  return o.solver_param > 0 ? o.solver_param : 2;
}

// Read the device `active` flags; returns the number still active.
static int read_active(dda_target* t, int nrhs, hipStream_t st, int& n_active) {
  HIPCHK(hipMemcpyAsync(t->h_active.data(), t->active.p, nrhs * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  n_active = 0;
  for (int r = 0; r < nrhs; ++r) n_active += t->h_active[r] != 0;
  return DDA_OK;
}

// QMR_sym runs its step fused into the y-forward pass when the product's
// y pass is the register-resident one (schedules 0, 1 and 3) and the target
// fills its lattice (>= 90% of the sites occupied): the fused pass reaches
// the step's seven vectors through the occupancy, which is a coalesced
// stream only where consecutive sites hold consecutive dipoles (measured:
// faster at the filled 64^3 cube, slower at the 200^3 sphere, the 96^3
// ellipsoid and the aggregates).  Returns the y-forward blocks per
// right-hand side, or 0 if the step stays separate.
template <typename R>
static int qmr_fused_blocks(dda_target* t, int nrhs) {
  if (is_fused(schedule_of<R>(t, nrhs)) || !fast_y_size(t->Jpp)) return 0;
  if ((double)t->nd < 0.9 * (double)t->K * t->J * t->P) return 0;
  switch (t->Jpp) {
#define DDA_CASE(N) \
  case N:           \
    return FastLaunch<R>::template yfwd_blocks<N>(t, ylog_of<R>(t, nrhs));
    DDA_FAST_Y_SIZES(DDA_CASE)
#undef DDA_CASE
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Host programs of the generic solvers (BiCG, QMR, BiCGSTAB(l), IDR(s) for
// ML(n)BiCGSTAB): each iteration is a fixed sequence of k_gen_dot,
// k_gen_scalar, k_gen_lin and matrix-vector launches.
// ---------------------------------------------------------------------------
static_assert(GEN_BICG == DDA_BICG && GEN_QMR == DDA_QMR && GEN_BICGSTAB_L == DDA_RBICGSTAB &&
                  GEN_IDR == DDA_MLBICGSTAB,
              "generic solver ids follow the C ABI");

struct LinB {
  GenLin L{};
  bool overflow = false;
  LinB& out(int slot) {
    if (L.nout >= kGenOut) {
      overflow = true;
      return *this;
    }
    L.out[L.nout] = (signed char)slot;
    L.nt[L.nout] = 0;
    ++L.nout;
    return *this;
  }
  LinB& term(int src, int code = kGenOne) {
    const int q = L.nout - 1;
    if (q < 0 || L.nt[q] >= kGenTerms) {
      overflow = true;
      return *this;
    }
    L.src[q][L.nt[q]] = (signed char)src;
    L.coef[q][L.nt[q]] = (short)code;
    ++L.nt[q];
    return *this;
  }
};

struct DotB {
  GenDots D{};
  bool overflow = false;
  DotB& add(int a, int b, int herm) {
    if (D.n >= kGenDots) {
      overflow = true;
      return *this;
    }
    D.a[D.n] = (signed char)a;
    D.b[D.n] = (signed char)b;
    D.herm[D.n] = (signed char)herm;
    ++D.n;
    return *this;
  }
  DotB& h(int a, int b) { return add(a, b, 1); }    // a^H b
  DotB& bil(int a, int b) { return add(a, b, 0); }  // a^T b
};

template <typename R>
struct GenRun {
  dda_target* t;
  int nrhs, solver, param, mvpi, jacobi;
  cx<R>* V;
  long vsz;
  SolverDims dm;
  c64* part;
  GenState* st;
  int* act;
  const double* tolv;
  const double* dS;

  int dot(hipStream_t s, const DotB& d) {
    if (d.overflow) return fail(DDA_EINVAL, "solver program: too many inner products");
    hipLaunchKernelGGL((k_gen_dot<R>), dim3(dm.nblk, nrhs), dim3(kRedThreads), 0, s, V, vsz, d.D, act, dm, part);
    return DDA_OK;
  }
  int scal(hipStream_t s, int step, int sub = 0) {
    GenStep g{solver, step, sub, param, mvpi};
    hipLaunchKernelGGL((k_gen_scalar<R>), dim3(nrhs), dim3(kRedThreads), 0, s, part, dm.nblk, g, st, act, tolv);
    return DDA_OK;
  }
  int lin(hipStream_t s, const LinB& b) {
    if (b.overflow) return fail(DDA_EINVAL, "solver program: too many terms");
    const unsigned gx = (unsigned)std::min<long>((dm.n3 + 255) / 256, 2048);
    hipLaunchKernelGGL((k_gen_lin<R>), dim3(gx, nrhs), dim3(256), 0, s, V, vsz, b.L, st, act, dm.n3);
    return DDA_OK;
  }
  int rnd(hipStream_t s, int slot, uint64_t seed) {
    const unsigned gx = (unsigned)std::min<long>((dm.n3 + 255) / 256, 2048);
    hipLaunchKernelGGL((k_gen_random<R>), dim3(gx, nrhs), dim3(256), 0, s, V, vsz, slot, seed, act, dm.n3);
    return DDA_OK;
  }
  int mv(hipStream_t s, int src, int dst) {
    return matvec_T<R>(t, nrhs, dS, jacobi, V + src * vsz, V + dst * vsz, act, s);
  }

  // ---- BiCG: 0 b, 1 u, 2 r, 3 rh, 4 p, 5 ph, 6 q, 7 qh (h: conjugated shadow)
  int init(hipStream_t s) {
    const int B = 0, X = 1;
    if (solver == GEN_BICG) {
      CHK(lin(s, LinB().out(2).term(B).out(3).term(B, kGenOne | kGenConj).out(X).out(4).out(5)));
    } else if (solver == GEN_QMR) {
      // 2 r, 3 vt, 4 wt (conj), 5 p, 6 qh, 7 pt = A p, 8 t = A qh, 9 d, 10 s
      CHK(lin(s, LinB().out(2).term(B).out(3).term(B).out(4).term(B, kGenOne | kGenConj).out(X).out(5).out(6).out(9)
                     .out(10)));
    } else if (solver == GEN_BICGSTAB_L) {
      // 2 rt, r_j = 3 + j, u_j = 4 + l + j
      CHK(lin(s, LinB().out(2).term(B).out(3).term(B).out(X).out(4 + param)));
    } else {
      // 2 r, 3 t, P_j = 4 + j, G_j = 4 + n + j, U_j = 4 + 2n + j
      CHK(lin(s, LinB().out(2).term(B).out(X).out(4).term(B)));
      LinB z;
      for (int j = 0; j < param; ++j) z.out(4 + param + j).out(4 + 2 * param + j);
      CHK(lin(s, z));
      for (int j = 1; j < param; ++j) CHK(rnd(s, 4 + j, 0x1d2a7b3cull));
    }
    CHK(dot(s, DotB().h(B, B)));
    return scal(s, GS_INIT);
  }

  int body(hipStream_t s) {
    const int X = 1;
    if (solver == GEN_BICG) {
      const int Rr = 2, RH = 3, P = 4, PH = 5, Q = 6, QH = 7;
      CHK(dot(s, DotB().h(Rr, Rr).bil(RH, Rr)));
      CHK(scal(s, GS_A));
      CHK(lin(s, LinB().out(P).term(Rr).term(P, BG_BETA).out(PH).term(RH).term(PH, BG_BETA)));
      CHK(mv(s, P, Q));
      CHK(mv(s, PH, QH));
      CHK(dot(s, DotB().bil(PH, Q)));
      CHK(scal(s, GS_B));
      return lin(s, LinB()
                        .out(X).term(X).term(P, BG_ALPHA)
                        .out(Rr).term(Rr).term(Q, BG_ALPHA | kGenNeg)
                        .out(RH).term(RH).term(QH, BG_ALPHA | kGenNeg));
    }
    if (solver == GEN_QMR) {
      const int Rr = 2, VT = 3, WT = 4, P = 5, QH = 6, PT = 7, T = 8, D = 9, S = 10;
      CHK(dot(s, DotB().h(Rr, Rr).h(WT, WT).bil(WT, VT)));
      CHK(scal(s, GS_A));
      CHK(lin(s, LinB()
                     .out(P).term(VT, QM_INVRHO).term(P, QM_CP | kGenNeg)
                     .out(VT).term(VT, QM_INVRHO)
                     .out(QH).term(WT, QM_INVXI).term(QH, QM_CQ | kGenNeg)
                     .out(WT).term(WT, QM_INVXI)));
      CHK(mv(s, P, PT));
      CHK(mv(s, QH, T));
      CHK(dot(s, DotB().bil(QH, PT)));
      CHK(scal(s, GS_B));
      CHK(lin(s, LinB().out(VT).term(PT).term(VT, QM_BETA | kGenNeg).out(WT).term(T).term(WT, QM_BETA | kGenNeg)));
      CHK(dot(s, DotB().h(VT, VT)));
      CHK(scal(s, GS_C));
      return lin(s, LinB()
                        .out(D).term(P, QM_ETA).term(D, QM_CD)
                        .out(S).term(PT, QM_ETA).term(S, QM_CD)
                        .out(X).term(X).term(D)
                        .out(Rr).term(Rr).term(S, kGenOne | kGenNeg));
    }
    if (solver == GEN_BICGSTAB_L) {
      const int l = param, RT = 2;
      auto r = [&](int j) { return 3 + j; };
      auto u = [&](int j) { return 4 + l + j; };
      for (int j = 0; j < l; ++j) {
        DotB d;
        if (j == 0) d.h(r(0), r(0));
        d.h(RT, r(j));
        CHK(dot(s, d));
        CHK(scal(s, GS_A, j));
        LinB a;
        for (int i = 0; i <= j; ++i) a.out(u(i)).term(r(i)).term(u(i), BL_BETA | kGenNeg);
        CHK(lin(s, a));
        CHK(mv(s, u(j), u(j + 1)));
        CHK(dot(s, DotB().h(RT, u(j + 1))));
        CHK(scal(s, GS_B, j));
        LinB b;
        for (int i = 0; i <= j; ++i) b.out(r(i)).term(r(i)).term(u(i + 1), BL_ALPHA | kGenNeg);
        b.out(X).term(X).term(u(0), BL_ALPHA);
        CHK(lin(s, b));
        CHK(mv(s, r(j), r(j + 1)));
      }
      DotB g;
      for (int i = 1; i <= l; ++i)
        for (int k = i; k <= l; ++k) g.h(r(i), r(k));
      for (int i = 1; i <= l; ++i) g.h(r(i), r(0));
      CHK(dot(s, g));
      CHK(scal(s, GS_C));
      LinB m;
      m.out(X).term(X);
      for (int j = 1; j <= l; ++j) m.term(r(j - 1), BL_GAM + j - 1);
      m.out(r(0)).term(r(0));
      for (int j = 1; j <= l; ++j) m.term(r(j), (BL_GAM + j - 1) | kGenNeg);
      m.out(u(0)).term(u(0));
      for (int j = 1; j <= l; ++j) m.term(u(j), (BL_GAM + j - 1) | kGenNeg);
      return lin(s, m);
    }
    // IDR(s), s = n
    const int n = param, Rr = 2, T = 3;
    auto P = [&](int j) { return 4 + j; };
    auto G = [&](int j) { return 4 + n + j; };
    auto U = [&](int j) { return 4 + 2 * n + j; };
    {
      DotB d;
      for (int j = 0; j < n; ++j) d.h(P(j), Rr);
      d.h(Rr, Rr);
      CHK(dot(s, d));
      CHK(scal(s, GS_A));
    }
    for (int k = 0; k < n; ++k) {
      // U_k = sum_{i>=k} c_i U_i + omega (r - sum_{i>=k} c_i G_i);  G_k = A U_k
      LinB a;
      a.out(U(k));
      for (int i = k; i < n; ++i) a.term(U(i), ID_C + i);
      a.term(Rr, ID_OMEGA);
      for (int i = k; i < n; ++i) a.term(G(i), (ID_OC + i) | kGenNeg);
      CHK(lin(s, a));
      CHK(mv(s, U(k), G(k)));
      DotB d;
      for (int j = 0; j < n; ++j) d.h(P(j), G(k));
      CHK(dot(s, d));
      CHK(scal(s, GS_B, k));
      LinB b;
      b.out(G(k)).term(G(k));
      for (int i = 0; i < k; ++i) b.term(G(i), (ID_AL + i) | kGenNeg);
      b.out(U(k)).term(U(k));
      for (int i = 0; i < k; ++i) b.term(U(i), (ID_AL + i) | kGenNeg);
      b.out(Rr).term(Rr).term(G(k), ID_BETA | kGenNeg);
      b.out(X).term(X).term(U(k), ID_BETA);
      CHK(lin(s, b));
    }
    CHK(mv(s, Rr, T));
    CHK(dot(s, DotB().h(T, Rr).h(T, T)));
    CHK(scal(s, GS_C));
    return lin(s, LinB().out(X).term(X).term(Rr, ID_OMEGA).out(Rr).term(Rr).term(T, ID_OMEGA | kGenNeg));
  }
};

// Solve (jacobi-scaled) A u = b for the right-hand sides flagged in
// t->active; b and u are slots 0 and 1 of the solver vectors.  The
// iteration is enqueued as a fixed kernel sequence; with use_graph a chunk of
// `check` iterations is captured once into a HIP graph (on a private stream)
// and replayed on the caller's stream, the host reading the `active` flags
// only between chunks.
template <typename R>
static int inner_solve(dda_target* t, int solver, int param, int nrhs, const double* tolv, int max_iter, int jacobi,
                       int check_every, int use_graph, hipStream_t st, InnerResult& res) {
  PrecBufs<R>& B = bufs<R>(t);
  const long n3 = 3 * t->nd;
  const size_t vsz = (size_t)nrhs * n3;
  CHK(ensure_matvec_ws<R>(t, nrhs));
  cx<R>* V = B.vec.template as<cx<R>>();
  auto slot = [&](int k) { return V + k * vsz; };
  cx<R>* b = slot(0);
  cx<R>* u = slot(1);
  SolverDims dm;
  dm.n3 = n3;
  dm.nblk = nblocks_for(n3);
  int* act = t->active.as<int>();
  const double* dS = t->S.as<double>();
  // ---- schedule: tune on scratch slots (4 -> 5, both rewritten below)
  CHK(autotune<R>(t, nrhs, dS, jacobi, slot(0), slot(4), st));
  // QMR_sym: step fused into the y-forward pass where the schedule allows
  const int nblk_f = (solver == DDA_QMR_SYM && t->fuse_qmr) ? qmr_fused_blocks<R>(t, nrhs) : 0;
  const bool qfuse = nblk_f > 0;
  // four regions of partial sums (each nrhs x nblk x 2, nblk_f when fused)
  const size_t preg = (size_t)nrhs * std::max(dm.nblk, nblk_f) * 2;
  CHK(t->part.ensure(std::max(4 * preg, (size_t)nrhs * dm.nblk * kGenDots) * sizeof(c64)));
  c64* part = t->part.as<c64>();
  c64 *R0 = part, *R1 = part + preg, *R2 = part + 2 * preg, *R3 = part + 3 * preg;
  dim3 vg(dm.nblk, nrhs), fg(nrhs);
  int check = check_every > 0 ? check_every : 8;
  if (check % 2) ++check;  // vector rings and state buffers have period 2
  int n_active = 0;
  const bool bcg = solver == DDA_BICGSTAB;
  const bool cgs = solver == DDA_BICG_SYM;
  const bool sq = solver == DDA_CGS;
  const bool tf = solver == DDA_TFQMR;
  const bool gen = solver >= DDA_BICG;
  int mv_per_iter = (bcg || sq || tf) ? 2 : 1;
  if (solver == DDA_BICG || solver == DDA_QMR) mv_per_iter = 2;
  if (solver == DDA_RBICGSTAB) mv_per_iter = 2 * param;
  if (solver == DDA_MLBICGSTAB) mv_per_iter = param + 1;
  GenRun<R> gr{t, nrhs, solver, param, mv_per_iter, jacobi, V, (long)vsz, dm, part, t->state.as<GenState>(), act,
               tolv, dS};

  // ---- initialisation (eager); state buffer 0 receives the initial state
  const int nblk_mv = yinv_blocks<R>(t, nrhs);
  CHK(t->part_mv.ensure((size_t)2 * nrhs * nblk_mv * 2 * sizeof(c64)));
  c64* M0 = t->part_mv.as<c64>();
  c64* M1 = M0 + (size_t)nrhs * nblk_mv * 2;
  if (gen) {
    CHK(gr.init(st));
  } else if (bcg) {
    BcgState* S0 = t->state.as<BcgState>();
    hipLaunchKernelGGL((k_bcg_init<R>), vg, dim3(kRedThreads), 0, st, b, slot(2), slot(3), slot(4), slot(5), u, act, dm,
                       R3);
    hipLaunchKernelGGL(k_bcg_fin_init, fg, dim3(kRedThreads), 0, st, R3, dm.nblk, S0, act, tolv);
    if (t->inject_breakdown > 0) {
      // fault injection: rhat = 0 makes rhat^H v vanish in the first step
      --t->inject_breakdown;
      HIPCHK(hipMemsetAsync(slot(3), 0, vsz * sizeof(cx<R>), st));
    }
  } else if (tf) {
    // slot 2 = rt, 3 = w, 4 = ue, 5 = uo, 6 = v, 7 = d, 8 = A ue, 9 = A uo;
    // the first product A ue (with rt^H A ue) completes the initialisation
    TfqState* S0 = t->state.as<TfqState>();
    hipLaunchKernelGGL((k_tfq_init<R>), vg, dim3(kRedThreads), 0, st, b, u, slot(2), slot(3), slot(4), slot(5),
                       slot(6), slot(7), slot(9), act, dm, R3);
    hipLaunchKernelGGL(k_tfq_fin_init, fg, dim3(kRedThreads), 0, st, R3, dm.nblk, S0, act, tolv);
    DotArgs d0;
    d0.mode = DOT_HA;
    d0.a = slot(2);
    d0.part = M1;
    CHK(matvec_T<R>(t, nrhs, dS, jacobi, slot(4), slot(8), act, st, d0));
  } else if (sq) {
    // slot 2 = r, 3 = rt, 4 = p, 5 = q, 6 = uu, 7 = v and t, 8 = w
    CgsState* S0 = t->state.as<CgsState>();
    hipLaunchKernelGGL((k_cgs_init<R>), vg, dim3(kRedThreads), 0, st, b, slot(2), slot(3), slot(4), slot(5), u, act,
                       dm, R3);
    hipLaunchKernelGGL(k_cgs_fin_init, fg, dim3(kRedThreads), 0, st, R3, dm.nblk, S0, act, tolv);
  } else if (cgs) {
    // slot 2 = r, 3 = p, 4 = q
    CgState* S0 = t->state.as<CgState>();
    hipLaunchKernelGGL((k_cg_init<R>), vg, dim3(kRedThreads), 0, st, b, slot(2), slot(3), u, act, dm, R3);
    hipLaunchKernelGGL(k_cg_fin_init, fg, dim3(kRedThreads), 0, st, R3, dm.nblk, S0, act, tolv);
  } else {
    QmrState* S0 = t->state.as<QmrState>();
    // slot 2 = vt_1 = b, slot 3 = vt_0 = 0, slots 5, 6 = p ring, slot 7 = QMR residual;
    // fused: the partials take the y-forward pass's block count, and the
    // first product A vt_1 is formed here (each iteration then runs step n
    // and the product of vt_{n+1})
    SolverDims dmi = dm;
    if (qfuse) dmi.nblk = nblk_f;
    hipLaunchKernelGGL((k_qmr_init<R>), dim3(dmi.nblk, nrhs), dim3(kRedThreads), 0, st, b, u, slot(2), slot(3),
                       slot(5), slot(6), slot(7), act, dmi, R1);
    hipLaunchKernelGGL(k_qmr_fin_init, fg, dim3(kRedThreads), 0, st, R1, dmi.nblk, S0, act, tolv);
    if (qfuse) {
      DotArgs d0;
      d0.mode = DOT_BIL;
      d0.part = M0;
      CHK(matvec_T<R>(t, nrhs, dS, jacobi, slot(2), slot(4), act, st, d0));
    }
  }
  LAUNCHCHK();

  // ---- one iteration; `par` selects the roles of the ring and state buffers
  auto body = [&](hipStream_t s, int par) -> int {
    if (gen) {
      CHK(gr.body(s));
    } else if (bcg) {
      BcgState* SA = t->state.as<BcgState>() + (par ? nrhs : 0);
      BcgState* SB = t->state.as<BcgState>() + (par ? 0 : nrhs);
      cx<R>*r = slot(2), *rhat = slot(3), *p = slot(4), *v = slot(5), *tt = slot(6);
      hipLaunchKernelGGL((k_bcg_p<R>), vg, dim3(kRedThreads), 0, s, r, p, v, R3, SA, SB, act, dm);
      DotArgs d1;
      d1.mode = DOT_HA;
      d1.a = rhat;
      d1.part = M0;
      CHK(matvec_T<R>(t, nrhs, dS, jacobi, p, v, act, s, d1));
      hipLaunchKernelGGL((k_bcg_s<R>), vg, dim3(kRedThreads), 0, s, r, v, M0, nblk_mv, SB, SA, act, dm, R1);
      DotArgs d2;
      d2.mode = DOT_TS;
      d2.part = M1;
      CHK(matvec_T<R>(t, nrhs, dS, jacobi, r, tt, act, s, d2));
      hipLaunchKernelGGL((k_bcg_update<R>), vg, dim3(kRedThreads), 0, s, u, r, p, tt, rhat, R1, M1, nblk_mv, SA, SB, act, dm,
                         R3);
    } else if (tf) {
      TfqState* SA = t->state.as<TfqState>() + (par ? nrhs : 0);
      TfqState* SB = t->state.as<TfqState>() + (par ? 0 : nrhs);
      cx<R>*rt = slot(2), *w = slot(3), *ue = slot(4), *uo = slot(5), *v = slot(6), *d = slot(7), *aue = slot(8),
           *auo = slot(9);
      hipLaunchKernelGGL((k_tfq_a<R>), vg, dim3(kRedThreads), 0, s, ue, aue, auo, v, uo, w, d, M1, nblk_mv, SA, SB,
                         act, dm, R1);
      DotArgs d1;
      d1.mode = DOT_HA;
      d1.a = rt;
      d1.part = M0;
      CHK(matvec_T<R>(t, nrhs, dS, jacobi, uo, auo, act, s, d1));
      hipLaunchKernelGGL((k_tfq_b<R>), vg, dim3(kRedThreads), 0, s, u, uo, auo, rt, w, d, R1, M0, nblk_mv, SB, SA,
                         act, dm, R3);
      hipLaunchKernelGGL((k_tfq_c<R>), vg, dim3(kRedThreads), 0, s, u, d, w, uo, ue, R3, SA, SB, act, dm);
      DotArgs d2;
      d2.mode = DOT_HA;
      d2.a = rt;
      d2.part = M1;
      CHK(matvec_T<R>(t, nrhs, dS, jacobi, ue, aue, act, s, d2));
    } else if (sq) {
      // two state writes per iteration: the newest state is back in SA
      CgsState* SA = t->state.as<CgsState>();
      CgsState* SB = t->state.as<CgsState>() + nrhs;
      cx<R>*r = slot(2), *rt = slot(3), *p = slot(4), *q = slot(5), *uu = slot(6), *v = slot(7), *w = slot(8);
      hipLaunchKernelGGL((k_cgs_p<R>), vg, dim3(kRedThreads), 0, s, r, q, uu, p, R3, SA, SB, act, dm);
      DotArgs d1;
      d1.mode = DOT_HA;
      d1.a = rt;
      d1.part = M0;
      CHK(matvec_T<R>(t, nrhs, dS, jacobi, p, v, act, s, d1));
      hipLaunchKernelGGL((k_cgs_q<R>), vg, dim3(kRedThreads), 0, s, uu, v, q, w, u, M0, nblk_mv, SB, SA, act, dm);
      CHK(matvec_T<R>(t, nrhs, dS, jacobi, w, v, act, s, DotArgs{}));
      hipLaunchKernelGGL((k_cgs_update<R>), vg, dim3(kRedThreads), 0, s, r, v, rt, SA, act, dm, R3);
    } else if (cgs) {
      // two state writes per iteration: the newest state is back in SA
      CgState* SA = t->state.as<CgState>();
      CgState* SB = t->state.as<CgState>() + nrhs;
      cx<R>*r = slot(2), *p = slot(3), *q = slot(4);
      hipLaunchKernelGGL((k_cg_p<R>), vg, dim3(kRedThreads), 0, s, r, p, R3, SA, SB, act, dm);
      DotArgs d;
      d.mode = DOT_BIL;
      d.part = M0;
      CHK(matvec_T<R>(t, nrhs, dS, jacobi, p, q, act, s, d));
      hipLaunchKernelGGL((k_cg_update<R>), vg, dim3(kRedThreads), 0, s, u, r, p, q, M0, nblk_mv, SB, SA, act, dm, R3);
    } else if (qfuse) {
      QmrState* SA = t->state.as<QmrState>() + (par ? nrhs : 0);
      QmrState* SB = t->state.as<QmrState>() + (par ? 0 : nrhs);
      cx<R>* w = slot(4);
      cx<R>* vn = par ? slot(3) : slot(2);
      cx<R>* vp = par ? slot(2) : slot(3);
      cx<R>* p1 = par ? slot(6) : slot(5);
      cx<R>* p2 = par ? slot(5) : slot(6);
      c64* pn_in = par ? R3 : R1;
      c64* pn_out = par ? R1 : R3;
      QmrFuse<R> f{w, vn, vp, p1, p2, u, slot(7), pn_out, nblk_f, pn_in, nblk_f, M0, nblk_mv, SA, SB, act};
      DotArgs d;
      d.mode = DOT_BIL;
      d.part = M0;
      // vt_{n+1} lands in vp's slot and is the product's input
      CHK(matvec_T<R>(t, nrhs, dS, jacobi, vp, w, act, s, d, &f));
    } else {
      QmrState* SA = t->state.as<QmrState>() + (par ? nrhs : 0);
      QmrState* SB = t->state.as<QmrState>() + (par ? 0 : nrhs);
      cx<R>* w = slot(4);
      cx<R>* vn = par ? slot(3) : slot(2);
      cx<R>* vp = par ? slot(2) : slot(3);
      cx<R>* p1 = par ? slot(6) : slot(5);
      cx<R>* p2 = par ? slot(5) : slot(6);
      c64* pn_in = par ? R3 : R1;
      c64* pn_out = par ? R1 : R3;
      DotArgs d;
      d.mode = DOT_BIL;
      d.part = M0;
      CHK(matvec_T<R>(t, nrhs, dS, jacobi, vn, w, act, s, d));
      // vt_{n+1} lands in vp's slot and p_{n-1} in p2's: roles swap next time
      hipLaunchKernelGGL((k_qmr_step<R>), vg, dim3(kRedThreads), 0, s, w, vn, vp, p1, p2, u, slot(7), pn_in, M0, nblk_mv, SA,
                         SB, act, dm, pn_out);
    }
    LAUNCHCHK();
    return DDA_OK;
  };

  int it = 0;
  bool done = false;
  if (use_graph && !t->lib->prof) {
    std::vector<uintptr_t> key = {sizeof(R),
                                  (uintptr_t)solver,
                                  (uintptr_t)param,
                                  (uintptr_t)nblk_f,
                                  (uintptr_t)nrhs,
                                  (uintptr_t)jacobi,
                                  (uintptr_t)check,
                                  (uintptr_t)schedule_of<R>(t, nrhs),
                                  (uintptr_t)V,
                                  (uintptr_t)part,
                                  (uintptr_t)t->part_mv.p,
                                  (uintptr_t)act,
                                  (uintptr_t)dS,
                                  (uintptr_t)t->state.p,
                                  (uintptr_t)B.G1.p,
                                  (uintptr_t)B.G2.p,
                                  (uintptr_t)B.Y.p,
                                  (uintptr_t)B.a0.p,
                                  (uintptr_t)B.a1.p,
                                  (uintptr_t)t->has_a1,
                                  (uintptr_t)t->aniso,
                                  (uintptr_t)t->nd,
                                  (uintptr_t)t->occ.p,
                                  (uintptr_t)t->fuse_qmr,
                                  (uintptr_t)t->comp_bits,
                                  (uintptr_t)t->uniform_diag,
                                  (uintptr_t)t->mbits.p,
                                  (uintptr_t)B.mt0.p,
                                  (uintptr_t)B.mt1.p};
    hipGraphExec_t& gexec = t->graph_exec[sizeof(R) == 4 ? 1 : 0];
    std::vector<uintptr_t>& gkey = t->graph_key[sizeof(R) == 4 ? 1 : 0];
    if (!gexec || gkey != key) {
      if (gexec) {
        (void)hipGraphExecDestroy(gexec);
        gexec = nullptr;
      }
      if (!t->cap_stream) HIPCHK(hipStreamCreateWithFlags(&t->cap_stream, hipStreamNonBlocking));
      const int mv_save = t->matvecs;
      HIPCHK(hipStreamBeginCapture(t->cap_stream, hipStreamCaptureModeRelaxed));
      int rc = DDA_OK;
      for (int g = 0; g < check && rc == DDA_OK; ++g) rc = body(t->cap_stream, g & 1);
      hipGraph_t graph = nullptr;
      hipError_t ec = hipStreamEndCapture(t->cap_stream, &graph);
      t->matvecs = mv_save;
      if (rc != DDA_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (ec != hipSuccess) return fail(DDA_EDEVICE, "graph capture failed: %s", hipGetErrorString(ec));
      ec = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ec != hipSuccess) {
        gexec = nullptr;
        return fail(DDA_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(ec));
      }
      gkey = key;
    }
    while (it + check <= max_iter) {
      HIPCHK(hipGraphLaunch(gexec, st));
      it += check;
      t->matvecs += check * mv_per_iter;
      CHK(read_active(t, nrhs, st, n_active));
      if (n_active == 0) {
        done = true;
        break;
      }
    }
  }
  for (; !done && it < max_iter; ++it) {
    CHK(body(st, it & 1));
    if ((it + 1) % check == 0 || it + 1 == max_iter) {
      CHK(read_active(t, nrhs, st, n_active));
      if (n_active == 0) break;
    }
  }

  auto collect = [&](auto* hs_dev, auto tag) -> int {
    using S = decltype(tag);
    std::vector<S> hs(2 * nrhs);
    HIPCHK(hipMemcpyAsync(hs.data(), hs_dev, 2 * nrhs * sizeof(S), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int q = 0; q < nrhs; ++q) {
      const S& a = hs[q].ver >= hs[nrhs + q].ver ? hs[q] : hs[nrhs + q];  // the later write
      res.iters[q] = a.iters < 0 ? 0 : a.iters;
      res.converged[q] = a.converged;
      res.breakdown[q] = a.breakdown;
      res.rnorm2[q] = a.rnorm2;
      res.bnorm2[q] = a.bnorm2;
    }
    return DDA_OK;
  };
  if (gen) {
    std::vector<GenState> hs(nrhs);
    HIPCHK(hipMemcpyAsync(hs.data(), t->state.p, nrhs * sizeof(GenState), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int q = 0; q < nrhs; ++q) {
      res.iters[q] = hs[q].iters < 0 ? 0 : hs[q].iters;
      res.converged[q] = hs[q].converged;
      res.breakdown[q] = hs[q].breakdown;
      res.rnorm2[q] = hs[q].rnorm2;
      res.bnorm2[q] = hs[q].bnorm2;
    }
    return DDA_OK;
  }
  if (bcg) return collect(t->state.as<BcgState>(), BcgState{});
  if (cgs) return collect(t->state.as<CgState>(), CgState{});
  if (sq) return collect(t->state.as<CgsState>(), CgsState{});
  if (tf) return collect(t->state.as<TfqState>(), TfqState{});
  return collect(t->state.as<QmrState>(), QmrState{});
}

// FP64 true residual r = E - A P for all right-hand sides; returns |r|^2 and
// |E|^2 per right-hand side on the host.
static int true_residual(dda_target* t, int nrhs, const c64* E, const c64* Pv, c64* r, c64* y, hipStream_t st,
                         std::vector<double>& rn2, std::vector<double>& en2, bool p_zero = false) {
  CHK(ensure_matvec_ws<double>(t, nrhs));
  CHK(autotune<double>(t, nrhs, t->S.as<double>(), 0, Pv, y, st));
  if (p_zero)  // A 0 = 0 (the product of a zero vector is exactly zero)
    HIPCHK(hipMemsetAsync(y, 0, (size_t)nrhs * 3 * t->nd * sizeof(c64), st));
  else
    CHK(matvec_T<double>(t, nrhs, t->S.as<double>(), 0, Pv, y, nullptr, st));
  SolverDims dm;
  dm.n3 = 3 * t->nd;
  dm.nblk = nblocks_for(dm.n3);
  CHK(t->part.ensure((size_t)nrhs * dm.nblk * 2 * sizeof(c64)));
  hipLaunchKernelGGL(k_residual, dim3(dm.nblk, nrhs), dim3(kRedThreads), 0, st, E, y, r, dm, t->part.as<c64>());
  LAUNCHCHK();
  std::vector<c64> hp((size_t)nrhs * dm.nblk * 2);
  HIPCHK(hipMemcpyAsync(hp.data(), t->part.p, hp.size() * sizeof(c64), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  rn2.assign(nrhs, 0.0);
  en2.assign(nrhs, 0.0);
  for (int q = 0; q < nrhs; ++q)
    for (int bk = 0; bk < dm.nblk; ++bk) {
      rn2[q] += hp[((size_t)q * dm.nblk + bk) * 2].x;
      en2[q] += hp[((size_t)q * dm.nblk + bk) * 2 + 1].x;
    }
  return DDA_OK;
}

// FP64 outer buffers, five slots of [nrhs][3][N_d]: (caller's), residual,
// product scratch, and the P and residual of the last accepted step
static int ensure_outer(dda_target* t, int nrhs) {
  return t->outer.ensure((size_t)5 * nrhs * 3 * t->nd * sizeof(c64));
}

static void orientation_S(dda_target* t, int nrhs, const double* khat, const double* ehat, const double* S,
                          std::vector<double>& hs) {
  hs.assign(nrhs, 0.0);
  for (int r = 0; r < nrhs; ++r) {
    if (S) {
      hs[r] = S[r];
    } else if (t->prescription == DDA_POL_LDR && khat && ehat) {
      double s = 0.0;
      for (int a = 0; a < 3; ++a) {
        // (khat_a ehat_a)^2 for a complex ehat: real part of the square
        const double kr = khat[3 * r + a];
        const double er = ehat[6 * r + 2 * a], ei = ehat[6 * r + 2 * a + 1];
        s += kr * kr * (er * er - ei * ei);
      }
      hs[r] = s;
    }
  }
}

// Refinement loop around the inner solves: P += D^{-1/2} u |r| where
// (D^{-1/2} A D^{-1/2}) u = D^{-1/2} r / |r|, until the FP64 true residual
// meets tol.  Inner precision FP64 (tol_in = tol) or FP32 (tol_in = inner_tol),
// chosen per right-hand side: FP32 inner solves while they make progress; a
// refinement step that cuts a right-hand side's true residual by less than 4x
// (FP32 Krylov recurrences can stagnate, e.g. QMR_sym on point sources) moves
// that right-hand side, and only it, to FP64 inner solves.  A step runs the
// FP32 group and the FP64 group as two masked multi-RHS inner solves.
static int solve_core(dda_target* t, const dda_solve_opts& o, int nrhs, const c64* E, c64* Pv, dda_solve_info* info,
                      hipStream_t st) {
  CHK(ensure_outer(t, nrhs));
  const long n3 = 3 * t->nd;
  c64* r64 = t->outer.as<c64>() + (size_t)nrhs * n3;
  c64* y64 = r64 + (size_t)nrhs * n3;
  c64* pkeep = y64 + (size_t)nrhs * n3;
  c64* rkeep = pkeep + (size_t)nrhs * n3;
  const bool mixed = o.precision == DDA_SOLVE_MIXED;
  std::vector<int> hi(nrhs, mixed ? 0 : 1);  // 1: FP64 inner solves for this right-hand side
  const int nslots = solver_slots(o.solver, solver_param(o));
  if (mixed) CHK(ensure_solver_ws<float>(t, nrhs, nslots));
  else CHK(ensure_solver_ws<double>(t, nrhs, nslots));
  const int max_iter = o.max_iter > 0 ? o.max_iter : 10000;
  const int max_outer = o.max_outer > 0 ? o.max_outer : 20;
  const double tol = o.tol > 0 ? o.tol : 1e-6;
  const double tol_in = mixed ? (o.inner_tol > 0 ? o.inner_tol : 1e-3) : tol;
  const int mv0 = t->matvecs;
  HIPCHK(hipMemsetAsync(Pv, 0, (size_t)nrhs * n3 * sizeof(c64), st));
  std::vector<double> rn2, en2;
  // P = 0: the residual is E (and no product is needed for it)
  CHK(true_residual(t, nrhs, E, Pv, r64, y64, st, rn2, en2, true));
  for (int q = 0; q < nrhs; ++q)
    if (!std::isfinite(en2[q])) return fail(DDA_EINVAL, "dda_solve: right-hand side %d is not finite", q);
  std::vector<int> iters(nrhs, 0), outer(nrhs, 0), done(nrhs, 0);
  auto new_result = [nrhs]() {
    InnerResult r;
    r.iters.assign(nrhs, 0);
    r.converged.assign(nrhs, 0);
    r.breakdown.assign(nrhs, 0);
    r.rnorm2.assign(nrhs, 0.0);
    r.bnorm2.assign(nrhs, 0.0);
    return r;
  };
  InnerResult ir = new_result(), irg = new_result();
  std::vector<int> hact(nrhs), hgrp[2] = {std::vector<int>(nrhs), std::vector<int>(nrhs)};
  std::vector<double> hsc(nrhs), hacc(nrhs), htol(nrhs);
  const unsigned gx = (unsigned)std::min<long>((n3 + 255) / 256, 4096);
  const c64* a0 = t->p64.a0.as<c64>();
  const c64* a1 = t->has_a1 ? t->p64.a1.as<c64>() : nullptr;
  for (int step = 0; step < max_outer; ++step) {
    int n_left = 0;
    for (int q = 0; q < nrhs; ++q) {
      done[q] = !(rn2[q] > tol * tol * en2[q]) || iters[q] >= max_iter;
      hact[q] = !done[q];
      n_left += hact[q];
      hsc[q] = rn2[q] > 0 ? 1.0 / std::sqrt(rn2[q]) : 0.0;
      // solve only as far as the outer target needs: ||r_new|| <= tol ||E|| / 2
      const double need = rn2[q] > 0 ? 0.5 * tol * std::sqrt(en2[q] / rn2[q]) : 1.0;
      htol[q] = std::min(0.5, std::max(hi[q] ? tol : tol_in, need));
    }
    if (n_left == 0) break;
    HIPCHK(hipMemcpyAsync(t->scal.p, hsc.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(t->tolv.p, htol.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    for (int q = 0; q < nrhs; ++q) hacc[q] = std::sqrt(rn2[q]);
    // g = 0: the FP32 group, g = 1: the FP64 group; each an inner solve over
    // the right-hand sides of its group, then P += |r| D^{-1/2} u for them
    for (int g = 0; g < 2; ++g) {
      std::vector<int>& m = hgrp[g];
      int nm = 0, budget = 0;
      for (int q = 0; q < nrhs; ++q) {
        m[q] = hact[q] && hi[q] == g;
        nm += m[q];
        if (m[q]) budget = std::max(budget, max_iter - iters[q]);
      }
      if (nm == 0) continue;
      HIPCHK(hipMemcpyAsync(t->active.p, m.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
      if (g == 0) {
        hipLaunchKernelGGL((k_scale_rhs<float>), dim3(gx, nrhs), dim3(256), 0, st, r64, t->p32.vec.as<c32>(), a0, a1,
                           t->S.as<double>(), t->scal.as<double>(), t->active.as<int>(), (long)t->nd,
                           o.jacobi ? 1 : 0);
        LAUNCHCHK();
        CHK(inner_solve<float>(t, o.solver, solver_param(o), nrhs, t->tolv.as<double>(), budget, o.jacobi ? 1 : 0,
                               o.check_every, o.use_graph, st, irg));
      } else {
        hipLaunchKernelGGL((k_scale_rhs<double>), dim3(gx, nrhs), dim3(256), 0, st, r64, t->p64.vec.as<c64>(), a0,
                           a1, t->S.as<double>(), t->scal.as<double>(), t->active.as<int>(), (long)t->nd,
                           o.jacobi ? 1 : 0);
        LAUNCHCHK();
        CHK(inner_solve<double>(t, o.solver, solver_param(o), nrhs, t->tolv.as<double>(), budget, o.jacobi ? 1 : 0,
                                o.check_every, o.use_graph, st, irg));
      }
      for (int q = 0; q < nrhs; ++q)
        if (m[q]) ir.iters[q] = irg.iters[q];
    }
    if (t->inject_bad_step > 0) {
      // fault injection: this step's correction goes the wrong way
      --t->inject_bad_step;
      for (int q = 0; q < nrhs; ++q) hacc[q] = -hacc[q];
    }
    HIPCHK(hipMemcpyAsync(t->scal.p, hacc.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    // keep P and the residual of this step's start, to take the step back
    HIPCHK(hipMemcpyAsync(pkeep, Pv, (size_t)nrhs * n3 * sizeof(c64), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(rkeep, r64, (size_t)nrhs * n3 * sizeof(c64), hipMemcpyDeviceToDevice, st));
    for (int g = 0; g < 2; ++g) {
      int nm = 0;
      for (int q = 0; q < nrhs; ++q) nm += hgrp[g][q];
      if (nm == 0) continue;
      HIPCHK(hipMemcpyAsync(t->active_outer.p, hgrp[g].data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
      const size_t vsz = (size_t)nrhs * n3;
      if (g == 0)
        hipLaunchKernelGGL((k_accumulate<float>), dim3(gx, nrhs), dim3(256), 0, st, Pv, t->p32.vec.as<c32>() + vsz, a0,
                           a1, t->S.as<double>(), t->scal.as<double>(), t->active_outer.as<int>(), (long)t->nd,
                           o.jacobi ? 1 : 0);
      else
        hipLaunchKernelGGL((k_accumulate<double>), dim3(gx, nrhs), dim3(256), 0, st, Pv, t->p64.vec.as<c64>() + vsz,
                           a0, a1, t->S.as<double>(), t->scal.as<double>(), t->active_outer.as<int>(), (long)t->nd,
                           o.jacobi ? 1 : 0);
      LAUNCHCHK();
    }
    for (int q = 0; q < nrhs; ++q)
      if (hact[q]) {
        iters[q] += ir.iters[q];
        outer[q] += 1;
      }
    const std::vector<double> prev = rn2;
    CHK(true_residual(t, nrhs, E, Pv, r64, y64, st, rn2, en2));
    for (int q = 0; q < nrhs; ++q)
      if (hact[q] && !(rn2[q] <= prev[q])) {
        // the correction made this right-hand side's true residual worse, or
        // not finite (an FP32 inner solve that overflowed): take the step
        // back; the rule below then moves it to FP64 inner solves
        const size_t off = (size_t)q * n3, bytes = (size_t)n3 * sizeof(c64);
        HIPCHK(hipMemcpyAsync(Pv + off, pkeep + off, bytes, hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(r64 + off, rkeep + off, bytes, hipMemcpyDeviceToDevice, st));
        rn2[q] = prev[q];
      }
    for (int q = 0; q < nrhs; ++q)
      if (hact[q] && !hi[q] && rn2[q] > tol * tol * en2[q] && rn2[q] > prev[q] / 16.0) {
        hi[q] = 1;
        CHK(ensure_solver_ws<double>(t, nrhs, nslots));
      }
  }
  bool all = true;
  for (int q = 0; q < nrhs; ++q) {
    const double rel = en2[q] > 0 ? std::sqrt(rn2[q] / en2[q]) : 0.0;
    const int conv = rel <= tol;
    all = all && conv;
    if (info) {
      info[q].converged = conv;
      info[q].iterations = iters[q];
      info[q].outer_iterations = outer[q];
      info[q].rel_residual = rel;
      info[q].matvecs = t->matvecs - mv0;
    }
  }
  if (!all) return fail(DDA_ENOTCONV, "dda_solve: a right-hand side missed tol %g", tol);
  return DDA_OK;
}

static int check_opts(const dda_solve_opts* opts, const char* who) {
  if (!opts) return fail(DDA_EINVAL, "%s: opts is NULL", who);
  if (opts->solver < DDA_BICGSTAB || opts->solver > DDA_MLBICGSTAB)
    return fail(DDA_EINVAL, "%s: solver %d", who, opts->solver);
  if (opts->solver_param > kGenMaxParam)
    return fail(DDA_EINVAL, "%s: solver_param %d (at most %d)", who, opts->solver_param, kGenMaxParam);
  if (opts->precision != DDA_SOLVE_FP64 && opts->precision != DDA_SOLVE_MIXED)
    return fail(DDA_EINVAL, "%s: precision %d", who, opts->precision);
  if (!(opts->tol > 0.0) || !(opts->tol < 1.0)) return fail(DDA_EINVAL, "%s: tol %g", who, opts->tol);
  return DDA_OK;
}

static int solve_one(dda_target* t, const dda_solve_opts* opts, int nrhs, const double* khat, const double* ehat,
                     const double* S, const void* einc_dev, void* p_dev, dda_solve_info* info, hipStream_t st) {
  CHK(check_ready(t, "dda_solve"));
  if (nrhs < 1) return fail(DDA_EINVAL, "dda_solve: nrhs = %d", nrhs);
  if (!p_dev) return fail(DDA_EINVAL, "dda_solve: p_dev is NULL");
  if (!einc_dev && (!khat || !ehat)) return fail(DDA_EINVAL, "dda_solve: need einc_dev or khat and ehat");
  HIPCHK(hipSetDevice(t->lib->device));
  CHK(ensure_scratch(t, nrhs));
  CHK(ensure_outer(t, nrhs));
  if (t->has_a1 && !S && (!khat || !ehat))
    return fail(DDA_EINVAL, "dda_solve: an LDR target needs S or khat and ehat (S depends on the orientation)");
  std::vector<double> hs;
  orientation_S(t, nrhs, khat, ehat, S, hs);
  HIPCHK(hipMemcpyAsync(t->S.p, hs.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
  t->solve_S = hs;
  const c64* E = (const c64*)einc_dev;
  if (!E) {
    c64* Eg = t->outer.as<c64>();
    HIPCHK(hipMemcpyAsync(t->khat.p, khat, nrhs * 3 * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(t->ehat.p, ehat, nrhs * 6 * sizeof(double), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_einc, dim3((unsigned)std::min<long>((t->nd + 255) / 256, 4096), nrhs), dim3(256), 0, st, Eg,
                       t->sites.as<int>(), (long)t->nd, t->K, t->J, t->kd, t->khat.as<double>(), t->ehat.as<double>());
    LAUNCHCHK();
    E = Eg;
  }
  HIPCHK(hipStreamSynchronize(st));
  return solve_core(t, *opts, nrhs, E, (c64*)p_dev, info, st);
}

extern "C" int dda_solve(dda_target* t, const dda_solve_opts* opts, int nrhs, const double* khat, const double* ehat,
                         const double* S, const void* einc_dev, void* p_dev, dda_solve_info* info, void* hip_stream) {
  CHK(check_opts(opts, "dda_solve"));
  return solve_one(t, opts, nrhs, khat, ehat, S, einc_dev, p_dev, info, (hipStream_t)hip_stream);
}

// Batch of targets: a longest-first queue drained by host workers, one HIP
// stream each.  Targets own all their workspaces, graphs and solver state, so
// workers share only the library's tuning table (locked).
extern "C" int dda_batch_solve(dda_lib* lib, const dda_solve_opts* opts, int nitems, const dda_batch_item* items,
                               int nworkers, void* hip_stream) {
  if (!lib) return fail(DDA_EINVAL, "dda_batch_solve: lib is NULL");
  CHK(check_opts(opts, "dda_batch_solve"));
  if (nitems < 0 || (nitems > 0 && !items)) return fail(DDA_EINVAL, "dda_batch_solve: %d items", nitems);
  if (nitems == 0) return DDA_OK;
  for (int i = 0; i < nitems; ++i) {
    const dda_target* t = items[i].target;
    if (!t) return fail(DDA_EINVAL, "dda_batch_solve: item %d has no target", i);
    if (t->lib != lib) return fail(DDA_EINVAL, "dda_batch_solve: item %d belongs to another library", i);
    for (int j = 0; j < i; ++j)
      if (items[j].target == t) return fail(DDA_EINVAL, "dda_batch_solve: items %d and %d share a target", j, i);
    if (items[i].nrhs < 1) return fail(DDA_EINVAL, "dda_batch_solve: item %d nrhs = %d", i, items[i].nrhs);
  }
  std::vector<int> order(nitems);
  std::iota(order.begin(), order.end(), 0);
  auto cost = [&](int i) {
    const dda_target* t = items[i].target;
    return (double)t->Kpp * t->Jpp * t->Ppp * items[i].nrhs;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  int nw = nworkers > 0 ? nworkers : 4;
  nw = std::min(nw, nitems);
  if (lib->prof) nw = 1;  // the pass timers are not shared between threads
  HIPCHK(hipSetDevice(lib->device));
  while ((int)lib->workers.size() < nw) {
    hipStream_t w = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&w, hipStreamNonBlocking));
    lib->workers.push_back(w);
  }
  hipEvent_t ready = nullptr;
  HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  HIPCHK(hipEventRecord(ready, (hipStream_t)hip_stream));
  std::atomic<int> next{0};
  std::atomic<bool> stop{false};
  std::atomic<bool> notconv{false};
  std::mutex emu;
  int err_code = DDA_OK;
  std::string err_msg;
  auto worker = [&](int w) {
    hipStream_t st = lib->workers[w];
    int rc = hipSetDevice(lib->device) == hipSuccess && hipStreamWaitEvent(st, ready, 0) == hipSuccess
                 ? DDA_OK
                 : fail(DDA_EDEVICE, "dda_batch_solve: worker %d could not start", w);
    while (rc == DDA_OK && !stop.load()) {
      const int k = next.fetch_add(1);
      if (k >= nitems) break;
      const dda_batch_item& it = items[order[k]];
      rc = solve_one(it.target, opts, it.nrhs, it.khat, it.ehat, it.S, it.einc_dev, it.p_dev, it.info, st);
      if (rc == DDA_ENOTCONV) {
        notconv = true;
        rc = DDA_OK;
      } else if (rc != DDA_OK) {
        char buf[64];
        snprintf(buf, sizeof buf, " (batch item %d)", order[k]);
        g_err += buf;
      }
    }
    if (rc != DDA_OK) {
      stop = true;
      std::lock_guard<std::mutex> g(emu);
      if (err_code == DDA_OK) {
        err_code = rc;
        err_msg = g_err;
      }
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < nw; ++w) pool.emplace_back(worker, w);
  worker(0);
  for (auto& th : pool) th.join();
  (void)hipEventDestroy(ready);
  if (err_code != DDA_OK) return fail(err_code, "%s", err_msg.c_str());
  if (notconv) return fail(DDA_ENOTCONV, "dda_batch_solve: a right-hand side missed tol %g", opts->tol);
  return DDA_OK;
}

extern "C" int dda_incident_field(dda_target* t, int nrhs, const double* khat, const double* ehat, void* e_dev,
                                  void* hip_stream) {
  if (!t || !khat || !ehat || !e_dev || nrhs < 1) return fail(DDA_EINVAL, "dda_incident_field: bad arguments");
  if (t->nd <= 0) return fail(DDA_ESTATE, "dda_incident_field: occupancy not set");
  HIPCHK(hipSetDevice(t->lib->device));
  hipStream_t st = (hipStream_t)hip_stream;
  CHK(ensure_scratch(t, nrhs));
  HIPCHK(hipMemcpyAsync(t->khat.p, khat, nrhs * 3 * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(t->ehat.p, ehat, nrhs * 6 * sizeof(double), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_einc, dim3((unsigned)std::min<long>((t->nd + 255) / 256, 4096), nrhs), dim3(256), 0, st,
                     (c64*)e_dev, t->sites.as<int>(), (long)t->nd, t->K, t->J, t->kd, t->khat.as<double>(),
                     t->ehat.as<double>());
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));
  return DDA_OK;
}

// S of a call after the solve: the caller's values, else (LDR targets) those
// of the last dda_solve on the target when it had the same right-hand-side
// count; an LDR target with neither is an error, since alpha^{-1} then
// depends on an orientation the library does not know.  Non-LDR targets
// have no S term (0).
static int resolve_S(const dda_target* t, int nrhs, const double* S, const char* who, std::vector<double>& hs) {
  hs.assign(nrhs, 0.0);
  if (S) {
    for (int r = 0; r < nrhs; ++r) hs[r] = S[r];
    return DDA_OK;
  }
  if (!t->has_a1) return DDA_OK;
  if ((int)t->solve_S.size() != nrhs)
    return fail(DDA_EINVAL, "%s: LDR target without S, and no solve of %d right-hand sides to take it from", who, nrhs);
  hs = t->solve_S;
  return DDA_OK;
}

extern "C" int dda_solve_orientation_factors(const dda_target* t, int nrhs, double* S_out) {
  if (!t || !S_out || nrhs < 1) return fail(DDA_EINVAL, "dda_solve_orientation_factors: bad arguments");
  if ((int)t->solve_S.size() != nrhs)
    return fail(DDA_ESTATE, "dda_solve_orientation_factors: the last solve had %d right-hand sides, not %d",
                (int)t->solve_S.size(), nrhs);
  for (int r = 0; r < nrhs; ++r) S_out[r] = t->solve_S[r];
  return DDA_OK;
}

extern "C" int dda_cross_sections(dda_target* t, int nrhs, const double* S, const void* einc_dev, const void* p_dev,
                                  double* cext, double* cabs, double* csca, void* hip_stream) {
  CHK(check_ready(t, "dda_cross_sections"));
  if (nrhs < 1 || !einc_dev || !p_dev) return fail(DDA_EINVAL, "dda_cross_sections: bad arguments");
  HIPCHK(hipSetDevice(t->lib->device));
  hipStream_t st = (hipStream_t)hip_stream;
  CHK(ensure_scratch(t, nrhs));
  std::vector<double> hs;
  CHK(resolve_S(t, nrhs, S, "dda_cross_sections", hs));
  HIPCHK(hipMemcpyAsync(t->S.p, hs.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
  SolverDims dm;
  dm.n3 = 3 * t->nd;
  dm.nblk = nblocks_for(dm.n3);
  CHK(t->part.ensure((size_t)nrhs * dm.nblk * 2 * sizeof(c64)));
  hipLaunchKernelGGL(k_cross_sums, dim3(dm.nblk, nrhs), dim3(kRedThreads), 0, st, (const c64*)einc_dev, (const c64*)p_dev,
                     t->p64.a0.as<c64>(), t->has_a1 ? t->p64.a1.as<c64>() : nullptr, t->S.as<double>(), (long)t->nd,
                     t->kd, dm, t->part.as<c64>());
  LAUNCHCHK();
  std::vector<c64> hp((size_t)nrhs * dm.nblk * 2);
  HIPCHK(hipMemcpyAsync(hp.data(), t->part.p, hp.size() * sizeof(c64), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double fk = 4.0 * M_PI * t->kd;
  for (int q = 0; q < nrhs; ++q) {
    double se = 0, sa = 0;
    for (int bk = 0; bk < dm.nblk; ++bk) {
      se += hp[((size_t)q * dm.nblk + bk) * 2].x;
      sa += hp[((size_t)q * dm.nblk + bk) * 2 + 1].x;
    }
    if (cext) cext[q] = fk * se;
    if (cabs) cabs[q] = fk * sa;
    if (csca) csca[q] = fk * (se - sa);
  }
  return DDA_OK;
}

// ---------------------------------------------------------------------------
// far field
// ---------------------------------------------------------------------------

// F = k^2 (I - n n) sum_m e^{-i k n.r_m} P_m for ndir device directions.
static int far_field_dev(dda_target* t, int nrhs, const c64* P, int ndir, const double* dirs_dev, c64* F,
                         hipStream_t st) {
  const int ntile = (ndir + kFarDirs - 1) / kFarDirs;
  // enough blocks to fill the chip: split the dipoles into chunks
  long nchunk = std::max<long>(1, std::min<long>(256, (2048 + (long)ntile * nrhs - 1) / ((long)ntile * nrhs)));
  nchunk = std::min<long>(nchunk, std::max<long>(1, t->nd / kRedThreads));
  CHK(t->far_part.ensure((size_t)nrhs * ntile * nchunk * kFarDirs * 3 * sizeof(c64)));
  const size_t lds = (size_t)kFarDirs * (t->K + t->J + t->P) * sizeof(c64);
  if (lds > 64 * 1024) return fail(DDA_EINVAL, "far field: lattice %dx%dx%d too long for the phase tables", t->K, t->J, t->P);
  hipLaunchKernelGGL(k_far_partial, dim3(ntile, (unsigned)nchunk, nrhs), dim3(kRedThreads), lds, st, P,
                     t->sites.as<int>(), (long)t->nd, t->K, t->J, t->P, t->kd, dirs_dev, ndir, (int)nchunk,
                     t->far_part.as<c64>());
  LAUNCHCHK();
  const long nt = (long)nrhs * ndir;
  hipLaunchKernelGGL(k_far_finish, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, t->far_part.as<c64>(), ntile,
                     (int)nchunk, dirs_dev, ndir, nrhs, t->kd, F);
  LAUNCHCHK();
  return DDA_OK;
}

extern "C" int dda_far_field(dda_target* t, int nrhs, const void* p_dev, int ndir, const double* dirs, void* f_dev,
                             void* hip_stream) {
  if (!t || !p_dev || !dirs || !f_dev || nrhs < 1 || ndir < 1)
    return fail(DDA_EINVAL, "dda_far_field: bad arguments");
  if (t->nd <= 0) return fail(DDA_ESTATE, "dda_far_field: occupancy not set");
  for (int d = 0; d < ndir; ++d) {
    const double n2 = dirs[3 * d] * dirs[3 * d] + dirs[3 * d + 1] * dirs[3 * d + 1] + dirs[3 * d + 2] * dirs[3 * d + 2];
    if (!(std::fabs(n2 - 1.0) < 1e-9)) return fail(DDA_EINVAL, "dda_far_field: direction %d is not a unit vector", d);
  }
  HIPCHK(hipSetDevice(t->lib->device));
  hipStream_t st = (hipStream_t)hip_stream;
  CHK(t->far_dirs.ensure((size_t)ndir * 3 * sizeof(double)));
  HIPCHK(hipMemcpyAsync(t->far_dirs.p, dirs, (size_t)ndir * 3 * sizeof(double), hipMemcpyHostToDevice, st));
  CHK(far_field_dev(t, nrhs, (const c64*)p_dev, ndir, t->far_dirs.as<double>(), (c64*)f_dev, st));
  HIPCHK(hipStreamSynchronize(st));  // the host direction array may be reused at return
  return DDA_OK;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n from the
// Chebyshev-like first guesses; weights 2 / ((1 - x^2) P_n'(x)^2)).
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int j = 2; j <= n; ++j) {
      const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

extern "C" int dda_csca_quadrature(dda_target* t, int nrhs, const void* p_dev, int ntheta, int nphi, double* csca,
                                   void* hip_stream) {
  if (!t || !p_dev || !csca || nrhs < 1) return fail(DDA_EINVAL, "dda_csca_quadrature: bad arguments");
  if (t->nd <= 0) return fail(DDA_ESTATE, "dda_csca_quadrature: occupancy not set");
  if (ntheta <= 0) {
    ntheta = (int)std::ceil(t->kd * (t->extent + 1.0)) + 16;
    nphi = 2 * ntheta;
  }
  if (nphi <= 0) nphi = 2 * ntheta;
  if ((long)ntheta * nphi > (1L << 24)) return fail(DDA_EINVAL, "dda_csca_quadrature: %d x %d nodes", ntheta, nphi);
  HIPCHK(hipSetDevice(t->lib->device));
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<double> gx, gw;
  gauss_legendre(ntheta, gx, gw);
  const int ndir = ntheta * nphi;
  std::vector<double> dirs((size_t)ndir * 3), wts(ndir);
  for (int a = 0; a < ntheta; ++a) {
    const double ct = gx[a], stv = std::sqrt(std::max(0.0, 1.0 - ct * ct));
    for (int b = 0; b < nphi; ++b) {
      const double ph = 2.0 * M_PI * b / nphi;
      const int d = a * nphi + b;
      dirs[3 * d] = stv * std::cos(ph);
      dirs[3 * d + 1] = stv * std::sin(ph);
      dirs[3 * d + 2] = ct;
      wts[d] = gw[a] * (2.0 * M_PI / nphi);
    }
  }
  CHK(t->far_dirs.ensure((size_t)ndir * 3 * sizeof(double)));
  CHK(t->far_w.ensure((size_t)ndir * sizeof(double)));
  CHK(t->far_F.ensure((size_t)nrhs * ndir * 3 * sizeof(c64)));
  HIPCHK(hipMemcpyAsync(t->far_dirs.p, dirs.data(), dirs.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(t->far_w.p, wts.data(), wts.size() * sizeof(double), hipMemcpyHostToDevice, st));
  CHK(far_field_dev(t, nrhs, (const c64*)p_dev, ndir, t->far_dirs.as<double>(), t->far_F.as<c64>(), st));
  const int nb = std::max(1, std::min(64, (ndir + kRedThreads - 1) / kRedThreads));
  CHK(t->part.ensure((size_t)nrhs * nb * sizeof(c64)));
  hipLaunchKernelGGL(k_far_power, dim3(nb, nrhs), dim3(kRedThreads), 0, st, t->far_F.as<c64>(), t->far_w.as<double>(),
                     ndir, t->part.as<c64>());
  LAUNCHCHK();
  std::vector<c64> hp((size_t)nrhs * nb);
  HIPCHK(hipMemcpyAsync(hp.data(), t->part.p, hp.size() * sizeof(c64), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int q = 0; q < nrhs; ++q) {
    double sum = 0.0;
    for (int b = 0; b < nb; ++b) sum += hp[(size_t)q * nb + b].x;
    csca[q] = sum;  // F already carries k^2, so |F|^2 carries k^4
  }
  return DDA_OK;
}

extern "C" int dda_mueller(dda_target* t, const void* p_dev, int ndir, const double* theta_phi, void* s_dev,
                           void* m_dev, void* hip_stream) {
  if (!t || !p_dev || !theta_phi || ndir < 1 || (!s_dev && !m_dev))
    return fail(DDA_EINVAL, "dda_mueller: bad arguments");
  if (t->nd <= 0) return fail(DDA_ESTATE, "dda_mueller: occupancy not set");
  HIPCHK(hipSetDevice(t->lib->device));
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<double> dirs((size_t)ndir * 3);
  for (int d = 0; d < ndir; ++d) {
    const double th = theta_phi[2 * d], ph = theta_phi[2 * d + 1];
    dirs[3 * d] = std::sin(th) * std::cos(ph);
    dirs[3 * d + 1] = std::sin(th) * std::sin(ph);
    dirs[3 * d + 2] = std::cos(th);
  }
  CHK(t->far_dirs.ensure((size_t)ndir * 3 * sizeof(double)));
  CHK(t->far_tp.ensure((size_t)ndir * 2 * sizeof(double)));
  CHK(t->far_F.ensure((size_t)2 * ndir * 3 * sizeof(c64)));
  HIPCHK(hipMemcpyAsync(t->far_dirs.p, dirs.data(), dirs.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(t->far_tp.p, theta_phi, (size_t)ndir * 2 * sizeof(double), hipMemcpyHostToDevice, st));
  CHK(far_field_dev(t, 2, (const c64*)p_dev, ndir, t->far_dirs.as<double>(), t->far_F.as<c64>(), st));
  const c64* F = t->far_F.as<c64>();
  hipLaunchKernelGGL(k_mueller, dim3((ndir + 255) / 256), dim3(256), 0, st, F, F + (size_t)ndir * 3,
                     t->far_tp.as<double>(), ndir, t->kd, (c64*)s_dev, (double*)m_dev);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));  // the host angle array may be reused at return
  return DDA_OK;
}

extern "C" int dda_grad_cabs_eps(dda_target* t, const dda_solve_opts* opts, int nrhs, const double* S,
                                 const void* p_dev, void* grad_dev, void* hip_stream) {
  CHK(check_ready(t, "dda_grad_cabs_eps"));
  CHK(check_opts(opts, "dda_grad_cabs_eps"));
  if (!t->have_eps) return fail(DDA_ESTATE, "dda_grad_cabs_eps: needs dda_set_permittivity");
  if (nrhs < 1 || !p_dev || !grad_dev) return fail(DDA_EINVAL, "dda_grad_cabs_eps: bad arguments");
  HIPCHK(hipSetDevice(t->lib->device));
  hipStream_t st = (hipStream_t)hip_stream;
  CHK(ensure_scratch(t, nrhs));
  CHK(ensure_outer(t, nrhs));
  std::vector<double> hs;
  CHK(resolve_S(t, nrhs, S, "dda_grad_cabs_eps", hs));
  HIPCHK(hipMemcpyAsync(t->S.p, hs.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
  const long n3 = 3 * t->nd;
  // adjoint right-hand side W conj(P) into a separate buffer (the outer slot 0
  // holds E for plane-wave solves; the adjoint uses its own allocation)
  DevBuf rhs, mu;
  CHK(rhs.ensure((size_t)nrhs * n3 * sizeof(c64)));
  CHK(mu.ensure((size_t)nrhs * n3 * sizeof(c64)));
  const c64* a1 = t->has_a1 ? t->p64.a1.as<c64>() : nullptr;
  hipLaunchKernelGGL(k_adjoint_rhs, dim3((unsigned)std::min<long>((nrhs * n3 + 255) / 256, 65535)), dim3(256), 0, st,
                     (const c64*)p_dev, rhs.as<c64>(), t->p64.a0.as<c64>(), a1, t->S.as<double>(), (long)t->nd, t->kd,
                     nrhs);
  LAUNCHCHK();
  int rc = solve_core(t, *opts, nrhs, rhs.as<c64>(), mu.as<c64>(), nullptr, st);
  if (rc != DDA_OK && rc != DDA_ENOTCONV) return rc;
  hipLaunchKernelGGL(k_gradient, dim3((unsigned)std::min<long>((nrhs * t->nd + 255) / 256, 65535)), dim3(256), 0, st,
                     (const c64*)p_dev, mu.as<c64>(), t->d0.as<c64>(), t->has_a1 ? t->d1.as<c64>() : nullptr,
                     t->S.as<double>(), (long)t->nd, t->kd, nrhs, (c64*)grad_dev);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(st));
  return rc;
}
