// lb_lib.hip - plan management and the C ABI of include/lb.h.
//
// Host code here only enqueues kernels and runs the O(1) scalar logic of the
// trust-region method (ratio test, radius updates, CG and Lanczos scalars);
// every array operation runs in the kernels of kernels.hpp / fft.hpp.
#define LB_MAIN_TU 1
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/lb.h"
#include "launch.hpp"

using lb::NFuncs;
using lb::PassArgs;
using lbk::ColGeo;
using lbk::Geo;
using lbk::Prm;
using lbk::RowGeo;
using lbk::SubState;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;
static int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}
#define LB_HIP(call)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess) return fail(LB_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)
#define LB_TRY(expr)         \
  do {                       \
    int rc_ = (expr);        \
    if (rc_ < 0) return rc_; \
  } while (0)

extern "C" const char *lb_last_error(void) { return g_last_error.c_str(); }
extern "C" int lb_version(void) { return 100; }

// ---------------------------------------------------------------------------
// kernels used only here
// ---------------------------------------------------------------------------
namespace lbk {
// Gamma'(psi) = tau - gamma psi + psi^2 / 2 pointwise, in FP64 and optionally FP32
__global__ __launch_bounds__(EW_NT) void k_gamma_p(long N, int batch, Prm p, const double *__restrict__ psi,
                                                   double *__restrict__ g64, float *__restrict__ g32) {
  const long total = N * batch;
  for (long i = (long)blockIdx.x * EW_NT + threadIdx.x; i < total; i += (long)gridDim.x * EW_NT) {
    const int b = (int)(i / N);
    const double s = psi[i];
    const double v = p.tau[b] - p.gamma[b] * s + 0.5 * s * s;
    g64[i] = v;
    if (g32) g32[i] = float(v);
  }
}
// out = x / sqrt(Lambda + c) (root != 0) or x / (Lambda + c) over the half
// spectrum (k = 0 removed)
__global__ __launch_bounds__(EW_NT) void k_prec_scale(Geo g, Prm p, const double2 *__restrict__ x, double c, int root,
                                                      double2 *__restrict__ out) {
  for (long h = (long)blockIdx.x * EW_NT + threadIdx.x; h < g.nh; h += (long)gridDim.x * EW_NT) {
    int kl;
    const double lam = lam_of(kk_at(g, (int)h, kl), p.xi[0], p.q[0]);
    const double s = (h == 0) ? 0.0 : (root ? 1.0 / sqrt(lam + c) : 1.0 / (lam + c));
    const double2 v = x[h];
    out[h] = double2{v.x * s, v.y * s};
  }
}
// parameter derivatives from the finalised sums [psi^2, psi^3, w psi, w psi^2]
// per instance: out[4 b + q] = c_q sums[4 b + q] / N with c = (1/2, -1/6, 1, -1/2)
__global__ void k_param_out(const double *sums, int batch, double inv_n, double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4 * batch) return;
  const int q = i & 3;
  const double c = q == 0 ? 0.5 : q == 1 ? -1.0 / 6.0 : q == 2 ? 1.0 : -0.5;
  out[i] = c * sums[i] * inv_n;
}
// out = (ct[2 b] psi - ct[2 b + 1] psi^2 / 2) / N over instance b's points
__global__ __launch_bounds__(EW_NT) void k_param_vjp(long N, int batch, const double *__restrict__ psi,
                                                     const double *__restrict__ ct, double *__restrict__ out) {
  const long total = N * batch;
  const double inv_n = 1.0 / (double)N;
  for (long i = (long)blockIdx.x * EW_NT + threadIdx.x; i < total; i += (long)gridDim.x * EW_NT) {
    const int b = (int)(i / N);
    const double x = psi[i];
    out[i] = (ct[2 * b] * x - 0.5 * ct[2 * b + 1] * x * x) * inv_n;
  }
}
// out = x + y (real)
__global__ __launch_bounds__(EW_NT) void k_add_real(long n, const double *__restrict__ x, const double *__restrict__ y,
                                                    double *__restrict__ out) {
  for (long i = (long)blockIdx.x * EW_NT + threadIdx.x; i < n; i += (long)gridDim.x * EW_NT) out[i] = x[i] + y[i];
}
}  // namespace lbk

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// kernel timing (measurement aid): events on the plan's stream around every
// launch whose name contains the filter; resolved at the next host sync
// ---------------------------------------------------------------------------
struct TimingEntry {
  std::string name;
  long count = 0;
  double total_ms = 0.0;
};
struct PendingTiming {
  hipEvent_t a, b;
  int idx;
};
struct TimingState {
  bool on = false;
  std::vector<std::string> names;  // kernels to time (all when empty)
  long every = 1;                  // time one launch in `every` of each kernel
  std::vector<long> seen;          // launches per entry since timing was set
  std::vector<TimingEntry> entries;
  std::vector<PendingTiming> pending;
  std::vector<hipEvent_t> pool;
};

struct AxisTab {
  int n = 0;
  const NFuncs *f64 = nullptr, *f32 = nullptr;
  double2 *tw64 = nullptr;
  float2 *tw32 = nullptr;
  double L = 1.0;  // box length along the axis
};

struct lb_plan {
  lb_grid grid{};
  int dim = 0, n0 = 0, n1 = 1, nl = 0, nhl = 0;
  long N = 0, nh = 0;
  int batch = 1;
  int prec = LB_FP64;
  hipStream_t stream = nullptr;
  hipStream_t own = nullptr;  // private stream for captured launch sequences (created on first use)
  int plane_nt = -1;          // autotuned plane-pass variant (index into plane_inner_nt), -1: built-in choice
  int plane_split = -1;       // parts K of the inner iteration's split order (1: none, 2, 4), -1: built-in choice
  int split_nt = -1;          // thread-count variant of its split-plane pass (index into plane_split_nt), -1: built-in
  int colv = 0;               // column variant (radix plan) of the inner iteration's axis-0 passes
  int hv_split = -1;          // parts K of lb_hessvec's split order (1: none, 2, 4), -1: built-in choice
  AxisTab ax[3];  // ax[0] leading axis, ax[1] middle axis (3D), ax[2] last axis
  // general Bravais lattice (lb_plan_set_lattice): the reciprocal metric
  // G = B^T B by axis slot (0 leading, 1 middle, 2 last); unused when 0
  int general = 0;
  double G[3][3] = {};
  double *mom = nullptr;  // moment partials of the update pass, MOM_NV x its blocks
  // FP64 spectral buffers (batch * nh complex each; SP holds 2 * batch)
  double2 *SP = nullptr, *GH = nullptr, *SH = nullptr, *W64 = nullptr;
  double2 *X = nullptr, *R = nullptr, *Pv = nullptr, *AP = nullptr;
  // inner-loop spectral buffers in the plan's precision
  void *B0 = nullptr, *B1 = nullptr, *WT = nullptr, *GHT = nullptr;
  // physical buffers (batch * N)
  double *gp64 = nullptr, *sphys = nullptr, *ptrial = nullptr;
  float *gp32 = nullptr;
  double *partial = nullptr;
  long partial_len = 0;
  double *sums = nullptr;  // small device scratch for finalised sums
  SubState *st = nullptr;
  // pinned host mirrors
  SubState *st_h = nullptr;
  double *sums_h = nullptr;
  // Lanczos basis, allocated on first use
  std::vector<double2 *> lz;
  TimingState timing;
  size_t bytes = 0;
  std::vector<void *> allocs;
};

static const NFuncs *funcs_for(int n, int prec) {
  switch (n) {
#define LB_CASE(k) \
  case k:          \
    return lb::funcs_##k(prec);
    LB_FOR_EACH_LENGTH(LB_CASE)
#undef LB_CASE
    default:
      return nullptr;
  }
}

template <typename T> static int dalloc(lb_plan *P, T **p, size_t count) {
  *p = nullptr;
  if (count == 0) return 0;
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return fail(LB_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  P->allocs.push_back(q);
  P->bytes += count * sizeof(T);
  *p = (T *)q;
  return 0;
}

// W[m] = exp(-2 pi i m / n), built quadrant by quadrant in long double so that
// the axis points are exact and every entry is rounded once.
static void twiddles(int n, std::vector<double2> &w64, std::vector<float2> &w32) {
  w64.resize(n);
  w32.resize(n);
  const long double halfpi = 1.570796326794896619231321691639751442L;
  for (int m = 0; m < n; ++m) {
    const long m4 = 4L * m;
    const int quad = (int)(m4 / n);
    const long rem = m4 % n;
    const long double th = halfpi * (long double)rem / (long double)n;
    const long double c = cosl(th), s = sinl(th);
    long double cc, ss;  // cos and sin of 2 pi m / n
    switch (quad) {
      case 0: cc = c; ss = s; break;
      case 1: cc = -s; ss = c; break;
      case 2: cc = -c; ss = -s; break;
      default: cc = s; ss = -c; break;
    }
    w64[m] = double2{(double)cc, (double)(-ss)};
    w32[m] = float2{(float)cc, (float)(-ss)};
  }
}



// Kernel-timing events only carry timestamps (results are read after stream
// synchronisation, never through them), so they are recorded without the
// system-scope fence, whose cache writeback and invalidation would otherwise
// slow every timed launch and the work after it.
static hipEvent_t timing_event(lb_plan *P) {
  hipEvent_t e = nullptr;
  if (!P->timing.pool.empty()) {
    e = P->timing.pool.back();
    P->timing.pool.pop_back();
  } else if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
    e = nullptr;
  }
  return e;
}
// Adds the first n pending kernel timings (all of them by default) to the
// totals and returns their events to the pool.
static void timing_flush(lb_plan *P, size_t n = (size_t)-1) {
  std::vector<PendingTiming> &pend = P->timing.pending;
  n = std::min(n, pend.size());
  for (size_t i = 0; i < n; ++i) {
    const PendingTiming &q = pend[i];
    float ms = 0.0f;
    if (hipEventSynchronize(q.b) == hipSuccess && hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
      P->timing.entries[q.idx].count += 1;
      P->timing.entries[q.idx].total_ms += ms;
    }
    P->timing.pool.push_back(q.a);
    P->timing.pool.push_back(q.b);
  }
  pend.erase(pend.begin(), pend.begin() + (long)n);
}
namespace lb {
thread_local hipEvent_t kt_ev[2] = {nullptr, nullptr};
}
using lb::kt_ev;

// Times the first LB_LAUNCH in its scope when timing is on for `name`.
struct KT {
  lb_plan *P;
  int idx = -1;
  hipEvent_t a = nullptr, b = nullptr;
  KT(lb_plan *P_, const char *name) : P(P_) {
    TimingState &T = P->timing;
    if (!T.on) return;
    if (!T.names.empty() && std::find(T.names.begin(), T.names.end(), name) == T.names.end()) return;
    for (size_t i = 0; i < T.entries.size(); ++i)
      if (T.entries[i].name == name) idx = (int)i;
    if (idx < 0) {
      T.entries.push_back(TimingEntry{name, 0, 0.0});
      T.seen.push_back(0);
      idx = (int)T.entries.size() - 1;
    }
    if (T.seen[idx]++ % T.every != 0) {  // not sampled
      idx = -1;
      return;
    }
    a = timing_event(P);
    b = timing_event(P);
    if (!a || !b) {
      if (a) P->timing.pool.push_back(a);
      if (b) P->timing.pool.push_back(b);
      idx = -1;
      return;
    }
    kt_ev[0] = a;
    kt_ev[1] = b;
  }
  ~KT() {
    if (idx < 0) return;
    if (kt_ev[0] == a) {  // no launch in the scope
      kt_ev[0] = kt_ev[1] = nullptr;
      P->timing.pool.push_back(a);
      P->timing.pool.push_back(b);
      return;
    }
    P->timing.pending.push_back(PendingTiming{a, b, idx});
    if (P->timing.pending.size() > 4096) timing_flush(P);
  }
};

extern "C" int lb_plan_set_timing(lb_plan *P, int enable, const char *filter) {
  return lb_plan_set_timing_sampled(P, enable, filter, 1);
}

extern "C" int lb_plan_set_timing_sampled(lb_plan *P, int enable, const char *filter, int every) {
  if (!P) return fail(LB_ERR_ARG, "null plan");
  if (every < 1) return fail(LB_ERR_ARG, "every must be >= 1");
  (void)hipStreamSynchronize(P->stream);
  timing_flush(P);
  TimingState &T = P->timing;
  T.on = enable != 0;
  T.every = every;
  T.names.clear();
  const std::string f = filter ? filter : "";
  size_t pos = 0;
  while (pos < f.size()) {
    size_t end = f.find(',', pos);
    if (end == std::string::npos) end = f.size();
    if (end > pos) T.names.push_back(f.substr(pos, end - pos));
    pos = end + 1;
  }
  T.entries.clear();
  T.seen.clear();
  return LB_OK;
}

extern "C" int lb_plan_timing_entry(lb_plan *P, int index, char *name, int name_len, long *count, double *total_ms) {
  if (!P || !name || name_len < 1 || !count || !total_ms) return fail(LB_ERR_ARG, "null argument");
  LB_HIP(hipStreamSynchronize(P->stream));
  timing_flush(P);
  if (index < 0 || index >= (int)P->timing.entries.size()) return fail(LB_ERR_ARG, "timing index out of range");
  const TimingEntry &e = P->timing.entries[index];
  std::snprintf(name, (size_t)name_len, "%s", e.name.c_str());
  *count = e.count;
  *total_ms = e.total_ms;
  return LB_OK;
}

extern "C" size_t lb_plan_workspace_bytes(const lb_plan *P) { return P ? P->bytes : 0; }

extern "C" int lb_plan_destroy(lb_plan *P) {
  if (!P) return LB_OK;
  for (void *q : P->allocs) (void)hipFree(q);
  for (double2 *q : P->lz) (void)hipFree(q);
  for (const PendingTiming &q : P->timing.pending) {
    (void)hipEventDestroy(q.a);
    (void)hipEventDestroy(q.b);
  }
  for (hipEvent_t e : P->timing.pool) (void)hipEventDestroy(e);
  if (P->st_h) (void)hipHostFree(P->st_h);
  if (P->sums_h) (void)hipHostFree(P->sums_h);
  if (P->own) (void)hipStreamDestroy(P->own);
  delete P;
  return LB_OK;
}

extern "C" int lb_plan_set_lattice(lb_plan *P, const double *A) {
  if (!P) return fail(LB_ERR_ARG, "null plan");
  const int d = P->dim;
  const int slot_of[3] = {0, d == 3 ? 1 : 2, 2};  // grid axis -> slot
  if (!A) {  // back to the grid's box
    P->general = 0;
    const int axis_of[3] = {0, d == 3 ? 1 : -1, d - 1};
    for (int s = 0; s < 3; ++s)
      if (axis_of[s] >= 0) P->ax[s].L = P->grid.box[axis_of[s]];
    return LB_OK;
  }
  for (int i = 0; i < d * d; ++i)
    if (!std::isfinite(A[i])) return fail(LB_ERR_ARG, "non-finite lattice matrix");
  bool diag = true;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j)
      if (i != j && A[i * d + j] != 0.0) diag = false;
  if (diag) {  // orthorhombic: the box path, bit for bit
    for (int a = 0; a < d; ++a)
      if (!(A[a * d + a] > 0.0)) return fail(LB_ERR_ARG, "lattice vectors must be nonzero");
    P->general = 0;
    for (int a = 0; a < d; ++a) P->ax[slot_of[a]].L = A[a * d + a];
    return LB_OK;
  }
  // reciprocal metric G = B^T B = 4 pi^2 (A^T A)^-1 (A B^T = 2 pi I)
  long double M[3][3] = {}, Inv[3][3] = {};
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j)
      for (int k = 0; k < d; ++k) M[i][j] += (long double)A[k * d + i] * (long double)A[k * d + j];
  long double det;
  if (d == 2) {
    det = M[0][0] * M[1][1] - M[0][1] * M[1][0];
    if (!(std::fabs((double)det) > 0.0)) return fail(LB_ERR_ARG, "singular lattice matrix");
    Inv[0][0] = M[1][1] / det;
    Inv[1][1] = M[0][0] / det;
    Inv[0][1] = Inv[1][0] = -M[0][1] / det;
  } else {
    det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
          M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
    if (!(std::fabs((double)det) > 0.0)) return fail(LB_ERR_ARG, "singular lattice matrix");
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
        Inv[i][j] = (M[i1][j1] * M[i2][j2] - M[i1][j2] * M[i2][j1]) / det;
      }
  }
  const long double fp2 = 4.0L * 3.141592653589793238462643383279502884L * 3.141592653589793238462643383279502884L;
  for (int s = 0; s < 3; ++s)
    for (int t = 0; t < 3; ++t) P->G[s][t] = 0.0;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) P->G[slot_of[i]][slot_of[j]] = (double)(fp2 * Inv[i][j]);
  P->general = 1;
  return LB_OK;
}

extern "C" int lb_plan_set_stream(lb_plan *P, void *stream) {
  if (!P) return fail(LB_ERR_ARG, "null plan");
  P->stream = (hipStream_t)stream;
  return LB_OK;
}

static long cdiv(long a, long b) { return (a + b - 1) / b; }

// workgroups of each pass kind, per instance
static long bpi_pairs(const lb_plan *P) {
  const long rpi = (P->dim == 3) ? (long)P->n0 * P->n1 : P->n0;
  return cdiv(rpi / 2, P->ax[2].f64->C);
}
static long bpi_rows(const lb_plan *P) {
  const long rpi = (P->dim == 3) ? (long)P->n0 * P->n1 : P->n0;
  return cdiv(rpi, P->ax[2].f64->C);
}
static long bpi_col1(const lb_plan *P) { return cdiv((long)P->n0 * P->nhl, P->ax[1].f64->C); }
static long bpi_col0(const lb_plan *P) {
  const long cpi = (P->dim == 3) ? (long)P->n1 * P->nhl : P->nhl;
  return cdiv(cpi, P->ax[0].f64->C);
}
static long bpi_ew(const lb_plan *P) { return std::min<long>(cdiv(P->nh, lbk::EW_NT * 4), 512); }

static int upload(lb_plan *P, void *dst, const void *src, size_t bytes) {
  LB_HIP(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
  return 0;
}

extern "C" int lb_plan_create(lb_plan **out, const lb_grid *g, int batch, int precision, void *stream) {
  if (!out || !g) return fail(LB_ERR_ARG, "null argument");
  *out = nullptr;
  if (g->dim != 2 && g->dim != 3) return fail(LB_ERR_ARG, "dim must be 2 or 3");
  if (batch < 1 || batch > lbk::MAXB) return fail(LB_ERR_ARG, "batch must be in [1, 8]");
  if (precision != LB_FP64 && precision != LB_FP32) return fail(LB_ERR_ARG, "precision must be LB_FP64 or LB_FP32");
  for (int a = 0; a < g->dim; ++a) {
    if (!(g->box[a] > 0.0) || !std::isfinite(g->box[a])) return fail(LB_ERR_ARG, "box sides must be positive");
    if (!funcs_for(g->n[a], 0)) return fail(LB_ERR_UNSUPPORTED, "axis length not supported (2^a 3^b, 8..512)");
  }
  lb_plan *P = new lb_plan();
  P->grid = *g;
  P->dim = g->dim;
  P->batch = batch;
  P->prec = precision;
  P->stream = (hipStream_t)stream;
  P->n0 = g->n[0];
  P->n1 = (g->dim == 3) ? g->n[1] : 1;
  P->nl = g->n[g->dim - 1];
  P->nhl = P->nl / 2 + 1;
  P->N = (long)P->n0 * P->n1 * P->nl;
  P->nh = (long)P->n0 * P->n1 * P->nhl;
  auto cleanup = [&](int rc) {
    lb_plan_destroy(P);
    return rc;
  };
  // per-axis tables: ax[0] leading, ax[1] middle (3D) or unused, ax[2] last
  const int axis_of[3] = {0, g->dim == 3 ? 1 : -1, g->dim - 1};
  for (int s = 0; s < 3; ++s) {
    const int a = axis_of[s];
    if (a < 0) {
      // 2D: the middle-axis slot is a single zero wavenumber
      P->ax[1].n = 1;
      continue;
    }
    AxisTab &A = P->ax[s];
    A.n = g->n[a];
    A.f64 = funcs_for(A.n, LB_FP64);
    A.f32 = funcs_for(A.n, LB_FP32);
    std::vector<double2> w64;
    std::vector<float2> w32;
    twiddles(A.n, w64, w32);
    int rc;
    if ((rc = dalloc(P, &A.tw64, A.n)) || (rc = dalloc(P, &A.tw32, A.n))) return cleanup(rc);
    if ((rc = upload(P, A.tw64, w64.data(), A.n * sizeof(double2)))) return cleanup(rc);
    if ((rc = upload(P, A.tw32, w32.data(), A.n * sizeof(float2)))) return cleanup(rc);
    A.L = g->box[a];
  }
  // the update pass reduces w |b|^2 over the +-k0 pairs of each axis-0
  // column: entries p = |k0| * columns + column, per instance
  const long S = (long)batch * P->nh, Np = (long)batch * P->N;
  int rc;
  if ((rc = dalloc(P, &P->SP, 2 * S)) || (rc = dalloc(P, &P->GH, S)) || (rc = dalloc(P, &P->SH, S)) ||
      (rc = dalloc(P, &P->W64, S)) || (rc = dalloc(P, &P->X, S)) || (rc = dalloc(P, &P->R, S)) ||
      (rc = dalloc(P, &P->Pv, S)) || (rc = dalloc(P, &P->AP, S)))
    return cleanup(rc);
  if (precision == LB_FP64) {
    double2 *b0, *b1;
    if ((rc = dalloc(P, &b0, S)) || (rc = dalloc(P, &b1, S))) return cleanup(rc);
    P->B0 = b0;
    P->B1 = b1;
    P->WT = P->W64;
    P->GHT = P->GH;
  } else {
    float2 *b0, *b1, *wt, *gt;
    if ((rc = dalloc(P, &b0, S)) || (rc = dalloc(P, &b1, S)) || (rc = dalloc(P, &wt, S)) || (rc = dalloc(P, &gt, S)))
      return cleanup(rc);
    P->B0 = b0;
    P->B1 = b1;
    P->WT = wt;
    P->GHT = gt;
    if ((rc = dalloc(P, &P->gp32, Np))) return cleanup(rc);
  }
  if ((rc = dalloc(P, &P->gp64, Np)) || (rc = dalloc(P, &P->sphys, Np)) || (rc = dalloc(P, &P->ptrial, Np)) ||
      (rc = dalloc(P, &P->mom, (long)lbk::MOM_NV * bpi_col0(P) * batch)))
    return cleanup(rc);
  const long mb = std::max({bpi_pairs(P), bpi_rows(P), bpi_col0(P), P->dim == 3 ? bpi_col1(P) : 1L, bpi_ew(P)});
  P->partial_len = 8 * mb * batch + 64;
  if ((rc = dalloc(P, &P->partial, P->partial_len)) || (rc = dalloc(P, &P->sums, 64 * lbk::MAXB)) ||
      (rc = dalloc(P, &P->st, lbk::MAXB)))
    return cleanup(rc);
  if (hipHostMalloc((void **)&P->st_h, sizeof(SubState) * lbk::MAXB, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&P->sums_h, sizeof(double) * 64 * lbk::MAXB, hipHostMallocDefault) != hipSuccess)
    return cleanup(fail(LB_ERR_HIP, "hipHostMalloc failed"));
  *out = P;
  return LB_OK;
}

// ---------------------------------------------------------------------------
// argument helpers
// ---------------------------------------------------------------------------
static int pack_params(const lb_plan *P, const lb_params *params, int count, Prm *p) {
  if (!params) return fail(LB_ERR_ARG, "null params");
  std::memset(p, 0, sizeof(Prm));
  for (int b = 0; b < count; ++b) {
    const lb_params &q = params[b];
    if (!std::isfinite(q.tau) || !std::isfinite(q.gamma) || !std::isfinite(q.xi) || !std::isfinite(q.q))
      return fail(LB_ERR_ARG, "non-finite model parameter");
    p->tau[b] = q.tau;
    p->gamma[b] = q.gamma;
    p->xi[b] = q.xi;
    p->q[b] = q.q;
  }
  return 0;
}
static Geo geo(const lb_plan *P, int batch) {
  Geo g{};
  g.dim = P->dim;
  g.n0 = P->n0;
  g.n1 = P->n1;
  g.nl = P->nl;
  g.nhl = P->nhl;
  g.N = P->N;
  g.nh = P->nh;
  g.batch = batch;
  if (!P->general) {
    g.c0 = 2.0 * M_PI / P->ax[0].L;
    g.c1 = 2.0 * M_PI / P->ax[1].L;
    g.cl = 2.0 * M_PI / P->ax[2].L;
    g.x01 = g.x0l = g.x1l = 0.0;
    g.general = 0;
  } else {
    g.c0 = std::sqrt(P->G[0][0]);
    g.c1 = P->dim == 3 ? std::sqrt(P->G[1][1]) : 2.0 * M_PI;
    g.cl = std::sqrt(P->G[2][2]);
    g.x01 = 2.0 * P->G[0][1];
    g.x0l = 2.0 * P->G[0][2];
    g.x1l = 2.0 * P->G[1][2];
    g.general = 1;
  }
  return g;
}

static const NFuncs *F(const lb_plan *P, int slot, int prec) { return prec == LB_FP64 ? P->ax[slot].f64 : P->ax[slot].f32; }
static const void *TW(const lb_plan *P, int slot, int prec) {
  return prec == LB_FP64 ? (const void *)P->ax[slot].tw64 : (const void *)P->ax[slot].tw32;
}

static PassArgs args_rows(const lb_plan *P, int prec, int batch, const Prm &p, bool pairs) {
  PassArgs a;
  a.stream = P->stream;
  a.g = geo(P, batch);
  a.p = p;
  a.rg.rpi = (P->dim == 3) ? (long)P->n0 * P->n1 : P->n0;
  a.rg.bpi = (int)(pairs ? bpi_pairs(P) : bpi_rows(P));
  a.nblocks = a.rg.bpi * batch;
  a.tw = TW(P, 2, prec);
  return a;
}
static PassArgs args_col(const lb_plan *P, int prec, int batch, const Prm &p, int axis) {
  PassArgs a;
  a.stream = P->stream;
  a.g = geo(P, batch);
  a.p = p;
  if (axis == 1) {
    a.cg.cpi = P->n0 * P->nhl;
    a.cg.inner = P->nhl;
    a.cg.outer = (long)P->n1 * P->nhl;
    a.cg.S = P->nhl;
    a.cg.bpi = (int)bpi_col1(P);
    a.tw = TW(P, 1, prec);
  } else {
    a.cg.cpi = (P->dim == 3) ? P->n1 * P->nhl : P->nhl;
    a.cg.inner = a.cg.cpi;
    a.cg.outer = P->nh;
    a.cg.S = a.cg.cpi;
    a.cg.bpi = (int)bpi_col0(P);
    a.tw = TW(P, 0, prec);
  }
  a.cg.inst = P->nh;
  a.nblocks = a.cg.bpi * batch;
  return a;
}

static int check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LB_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return 0;
}

// sum (or max) per-workgroup partials into P->sums[b * nq + q] (device)
static void finalize(lb_plan *P, const double *partial, int bpi, int nq, unsigned maxmask, int batch, double *out) {
  {
    KT kt_(P, "finalize");
    LB_LAUNCH(lbk::k_finalize, dim3(batch), dim3(256), 0, P->stream, partial, bpi, nq, maxmask, out);
  }
}
static int read_sums(lb_plan *P, const double *dev, int count) {
  LB_HIP(hipMemcpyAsync(P->sums_h, dev, sizeof(double) * count, hipMemcpyDeviceToHost, P->stream));
  LB_HIP(hipStreamSynchronize(P->stream));
  if (!P->timing.pending.empty()) timing_flush(P);
  return 0;
}

// ---------------------------------------------------------------------------
// transforms
// ---------------------------------------------------------------------------
// real (batch fields) -> half spectrum with the 1/N normalisation
static void fwd_r2c(lb_plan *P, int prec, int batch, const Prm &p, const double *in, void *out, int zero_dc) {
  PassArgs r = args_rows(P, prec, batch, p, true);
  r.in = in;
  r.out = out;
  {
    KT kt_(P, "rows_r2c");
    F(P, 2, prec)->rows_r2c(r, 0);
  }
  if (P->dim == 3) {
    PassArgs c1 = args_col(P, prec, batch, p, 1);
    c1.in = out;
    c1.out = out;
    {
      KT kt_(P, "col1_fwd");
      F(P, 1, prec)->cols_plain(c1, false);
    }
  }
  PassArgs c0 = args_col(P, prec, batch, p, 0);
  c0.in = out;
  c0.out = out;
  c0.scale = 1.0 / (double)P->N;
  c0.zero_dc = zero_dc;
  {
    KT kt_(P, "col0_fwd");
    F(P, 0, prec)->cols_plain(c0, false);
  }
}

// half spectrum -> real; `work` receives the partially inverted spectrum
static void inv_c2r(lb_plan *P, int prec, int batch, const Prm &p, const void *in, void *work, double *out, int mode,
                    const double *psi, double *partial) {
  PassArgs c0 = args_col(P, prec, batch, p, 0);
  c0.in = in;
  c0.out = work;
  {
    KT kt_(P, "col0_inv");
    F(P, 0, prec)->cols_plain(c0, true);
  }
  if (P->dim == 3) {
    PassArgs c1 = args_col(P, prec, batch, p, 1);
    c1.in = work;
    c1.out = work;
    {
      KT kt_(P, "col1_inv");
      F(P, 1, prec)->cols_plain(c1, true);
    }
  }
  PassArgs r = args_rows(P, prec, batch, p, true);
  r.in = work;
  r.out = out;
  r.psi = psi;
  r.partial = partial;
  {
    KT kt_(P, "rows_c2r");
    F(P, 2, prec)->rows_c2r(r, mode);
  }
}

// weighted spectral sums over the instances of a batch: MODE 0 <a,b>, MODE 1 sum Lambda |a|^2
template <typename TA, int MODE>
static void spec_reduce(lb_plan *P, int batch, const Prm &p, const void *a, const void *b, double *out_dev) {
  const int bpi = (int)bpi_ew(P);
  {
    KT kt_(P, "spec_reduce");
    LB_LAUNCH((lbk::k_spec_reduce<TA, MODE>), dim3(bpi * batch), dim3(lbk::EW_NT), 0, P->stream, geo(P, batch), p,
                       bpi, (const lbfft::c2<TA> *)a, (const lbfft::c2<TA> *)b, P->partial);
  }
  finalize(P, P->partial, bpi, 1, 0u, batch, out_dev);
}
static int spec_dot_host(lb_plan *P, const Prm &p, const double2 *a, const double2 *b, double *res) {
  spec_reduce<double, 0>(P, 1, p, a, b, P->sums);
  LB_TRY(read_sums(P, P->sums, 1));
  *res = P->sums_h[0];
  return 0;
}
static int spec_lam_host(lb_plan *P, const Prm &p, const double2 *a, double *res) {
  spec_reduce<double, 1>(P, 1, p, a, a, P->sums);
  LB_TRY(read_sums(P, P->sums, 1));
  *res = P->sums_h[0];
  return 0;
}

static void lincomb64(lb_plan *P, long n, double alpha, const double2 *x, double beta, const double2 *y, double2 *out) {
  const long nb = std::min<long>(cdiv(n, lbk::EW_NT), 4096);
  {
    KT kt_(P, "lincomb");
    LB_LAUNCH((lbk::k_lincomb<double, double, double>), dim3(nb), dim3(lbk::EW_NT), 0, P->stream, n, alpha, x,
                       beta, y, out);
  }
}

// ---------------------------------------------------------------------------
// energy and gradient
// ---------------------------------------------------------------------------
// After this call: GH holds g_hat (FP64), GHT its copy in the plan's precision,
// gp64/gp32 hold Gamma'(psi), and P->sums holds per instance
// [sum F, max |Gamma'|] at sums[0 .. 2B) and [G, ||g||^2, max |g|] at sums[32 ..).
static void energy_grad_core(lb_plan *P, int batch, const Prm &p, const double *psi, int raw = 0) {
  PassArgs r = args_rows(P, LB_FP64, batch, p, false);
  r.psi = psi;
  r.out = P->SP;
  r.out2 = P->SP + (long)batch * P->nh;
  r.gp64 = P->gp64;
  r.gp32 = P->gp32;
  r.partial = P->partial;
  {
    KT kt_(P, "rows_energy");
    F(P, 2, LB_FP64)->rows_energy(r);
  }
  finalize(P, P->partial, r.rg.bpi, 2, 0x2u, batch, P->sums);
  // psi and F'(psi) go through the column passes as 2 * batch stacked fields
  // (plain passes: the model parameters are not read)
  if (P->dim == 3) {
    PassArgs c1 = args_col(P, LB_FP64, 2 * batch, p, 1);
    c1.in = P->SP;
    c1.out = P->SP;
    {
      KT kt_(P, "col1_fwd");
      F(P, 1, LB_FP64)->cols_plain(c1, false);
    }
  }
  PassArgs c0 = args_col(P, LB_FP64, 2 * batch, p, 0);
  c0.in = P->SP;
  c0.out = P->SP;
  c0.scale = 1.0 / (double)P->N;
  {
    KT kt_(P, "col0_fwd");
    F(P, 0, LB_FP64)->cols_plain(c0, false);
  }
  const int bpi = (int)bpi_ew(P);
  double *part2 = P->partial + P->partial_len / 2;
  if (P->prec == LB_FP64)
    {
      KT kt_(P, "grad_assemble");
      LB_LAUNCH((lbk::k_grad_assemble<double>), dim3(bpi * batch), dim3(lbk::EW_NT), 0, P->stream,
                         geo(P, batch), p, bpi, (const double2 *)P->SP, (const double2 *)(P->SP + (long)batch * P->nh),
                         P->GH, (double2 *)nullptr, part2, raw);
    }
  else
    {
      KT kt_(P, "grad_assemble");
      LB_LAUNCH((lbk::k_grad_assemble<float>), dim3(bpi * batch), dim3(lbk::EW_NT), 0, P->stream,
                         geo(P, batch), p, bpi, (const double2 *)P->SP, (const double2 *)(P->SP + (long)batch * P->nh),
                         P->GH, (float2 *)P->GHT, part2, raw);
    }
  finalize(P, part2, bpi, 3, 0x4u, batch, P->sums + 32);
}

extern "C" int lb_energy_grad(lb_plan *P, const lb_params *params, const double *psi, double *energy, double *grad) {
  if (!P || !psi || !energy) return fail(LB_ERR_ARG, "null argument");
  Prm p;
  LB_TRY(pack_params(P, params, P->batch, &p));
  const int B = P->batch;
  energy_grad_core(P, B, p, psi);
  {
    KT kt_(P, "energy_out");
    LB_LAUNCH(lbk::k_energy_out, dim3(1), dim3(64), 0, P->stream, (const double *)(P->sums + 32), 3,
                       (const double *)P->sums, 2, 1.0 / (double)P->N, B, energy);
  }
  if (grad) inv_c2r(P, LB_FP64, B, p, P->GH, P->W64, grad, 0, nullptr, nullptr);
  return check_launch("lb_energy_grad");
}

// ---------------------------------------------------------------------------
// Hessian-vector product on physical fields
// The split order with K parts (2 or 4) exists on 3D grids with n1 = n_last
// whose split-plane kernels are built for K, and whose axis-0 workgroups
// hold whole groups of K columns without a ragged end ((n1/K) n_half columns
// per part, a multiple of C/K; four parts need C = 16: groups within rows of
// 16 lanes).
static int kidx(int K) { return K == 4 ? 1 : 0; }
static bool split_ok(const lb_plan *P, int prec, int K) {
  if (K != 2 && K != 4) return false;
  if (P->dim != 3 || P->n1 != P->nl || P->n1 % (2 * K)) return false;
  const NFuncs *f1 = F(P, 1, prec);
  const NFuncs *f0 = F(P, 0, prec);
  if (!f1 || f1->plane_split_default[kidx(K)] < 0 || !f0 || f0->C % K) return false;
  if (K == 4 && f0->C != 16) return false;
  const long hcols = (long)(P->n1 / K) * P->nhl;
  return hcols % (f0->C / K) == 0 && bpi_col0(P) * f0->C == K * hcols;
}
// the parts K of the inner iteration in use: pinned, or the built-in choice
// K = 1: one workgroup per plane where the plane fits in LDS, else the five
// passes of the column and row kernels (measured at 256^3: the split order's
// axis-0 passes, with groups of four 4-column runs per workgroup, cost more
// than its split planes save: 747 against 590 us per FP64 iteration); the
// autotuner may pick a split order
static int plane_k(const lb_plan *P, int prec) {
  if (P->plane_split == 2 || P->plane_split == 4) return split_ok(P, prec, P->plane_split) ? P->plane_split : 1;
  return 1;
}
// the parts K of lb_hessvec: pinned, or the built-in choice, as measured:
// where the plane fits, two parts for FP64 planes of 96 points and more
// (128^3: 3-5 % faster; in FP32 the pair steps cost the axis-0 pass more than
// the half planes save), else one workgroup per plane; where it does not fit,
// four parts in FP32 (256^3: 252 against 270 us per product) and the five
// passes in FP64 (378 against 363 us: the four-part axis-0 pass's 64 B runs)
static int hv_k(const lb_plan *P, int prec) {
  if (P->n0 > 512) return 1;
  if (P->hv_split == 2 || P->hv_split == 4) return split_ok(P, prec, P->hv_split) ? P->hv_split : 1;
  if (P->hv_split == 1) return 1;
  const NFuncs *f1 = P->dim == 3 ? F(P, 1, prec) : nullptr;
  if (f1 && f1->plane_fwd_phys && P->n1 == P->nl)
    return (prec == LB_FP64 && P->n1 >= 96 && split_ok(P, prec, 2)) ? 2 : 1;
  if (prec == LB_FP32 && split_ok(P, prec, 4)) return 4;
  return 1;
}
// the split order with K parts on an axis-0 pass's arguments
static void set_pair_split(const lb_plan *P, PassArgs &a, int prec, int K) {
  a.cg.hsplit = (P->n1 / K) * P->nhl;
  a.cg.kparts = K;
  a.tw1 = TW(P, 1, prec);
}
// column variant 3 (twice the columns per workgroup) takes one or two parts
// whose columns fill its workgroups exactly
static bool colv_ok(const lb_plan *P, int prec, int K, int cv) {
  if (cv != 3) return true;
  const int C3 = F(P, 0, prec)->C3;
  if (C3 <= 0 || K > 2) return false;
  if (K == 1) return true;
  const long hcols = (long)(P->n1 / K) * P->nhl;
  return hcols % (C3 / K) == 0 && cdiv((long)P->n1 * P->nhl, (long)C3) * C3 == K * hcols;
}
// the arguments of the inner iteration's axis-0 passes (inverse and update):
// the split order with K parts and the column variant in use
static PassArgs col0_args(const lb_plan *P, int prec, int B, const Prm &p, int K) {
  PassArgs a = args_col(P, prec, B, p, 0);
  if (K > 1) set_pair_split(P, a, prec, K);
  a.colv = colv_ok(P, prec, K, P->colv) ? P->colv : 0;
  if (a.colv == 3) {
    a.cg.bpi = (int)cdiv((long)a.cg.cpi, (long)F(P, 0, prec)->C3);
    a.nblocks = a.cg.bpi * B;
  }
  return a;
}

// ---------------------------------------------------------------------------
// mode 0: P(L v + Gamma' v); 1: P L v + Gamma' v; 2: (L v + Gamma' v) / N (raw coordinates)
static int hessvec_phys(lb_plan *P, const lb_params *params, const double *psi, const double *v, double *hv,
                        int mode) {
  if (!P || !psi || !v || !hv) return fail(LB_ERR_ARG, "null argument");
  Prm p;
  LB_TRY(pack_params(P, params, P->batch, &p));
  const int project = mode == 0;
  const int keep_dc = mode == 2;
  const double bscale = mode == 2 ? 1.0 / (double)P->N : 1.0;
  const int B = P->batch, prec = P->prec;
  void *work = P->WT;
  const NFuncs *f1 = P->dim == 3 ? F(P, 1, prec) : nullptr;
  const int hk = hv_k(P, prec);
  if (hk > 1) {
    // three passes in the split order: split planes forward, axis 0 with
    // Lambda and the first and last steps of the split axis-1 transforms,
    // split planes inverse
    PassArgs a = args_col(P, prec, B, p, 1);
    a.v = v;
    a.psi = psi;
    a.out = work;
    a.partial = project ? P->partial : nullptr;
    {
      KT kt_(P, "plane_fwd_phys");
      f1->plane_fwd_phys_split[kidx(hk)](a, P->n0);
    }
    PassArgs c0 = args_col(P, prec, B, p, 0);
    c0.out = work;
    c0.inv_n = bscale / (double)P->N;
    c0.keep_dc = keep_dc;
    set_pair_split(P, c0, prec, hk);
    {
      KT kt_(P, "col0_fwd_mul_inv");
      F(P, 0, prec)->cols_fwd_mul_inv(c0);
    }
    PassArgs o = args_col(P, prec, B, p, 1);
    o.in = work;
    o.out = hv;
    o.psi = psi;
    o.v = v;
    o.scale = bscale;
    o.mpart = project ? P->partial : nullptr;
    {
      KT kt_(P, "plane_inv_phys");
      f1->plane_inv_phys_split[kidx(hk)](o, P->n0);
    }
    return check_launch("lb_hessvec");
  }
  if (f1 && f1->plane_fwd_phys && P->n1 == P->nl) {
    // three passes: axes 2 and 1 forward per plane, axis 0 with Lambda, axes 1 and 2 inverse per plane
    PassArgs a = args_col(P, prec, B, p, 1);
    a.v = v;
    a.psi = psi;
    a.out = work;
    a.partial = project ? P->partial : nullptr;
    {
      KT kt_(P, "plane_fwd_phys");
      f1->plane_fwd_phys(a, P->n0);
    }
    PassArgs c0 = args_col(P, prec, B, p, 0);
    c0.out = work;
    c0.inv_n = bscale / (double)P->N;
    c0.keep_dc = keep_dc;
    {
      KT kt_(P, "col0_fwd_mul_inv");
      F(P, 0, prec)->cols_fwd_mul_inv(c0);
    }
    PassArgs o = args_col(P, prec, B, p, 1);
    o.in = work;
    o.out = hv;
    o.psi = psi;
    o.v = v;
    o.scale = bscale;
    o.mpart = project ? P->partial : nullptr;
    {
      KT kt_(P, "plane_inv_phys");
      f1->plane_inv_phys(o, P->n0);
    }
    return check_launch("lb_hessvec");
  }
  PassArgs r = args_rows(P, prec, B, p, true);
  r.in = v;
  r.psi = psi;
  r.out = work;
  r.partial = P->partial;
  {
    KT kt_(P, "rows_r2c");
    F(P, 2, prec)->rows_r2c(r, project ? 1 : 0);
  }
  if (P->dim == 3) {
    PassArgs c1 = args_col(P, prec, B, p, 1);
    c1.in = work;
    c1.out = work;
    {
      KT kt_(P, "col1_fwd");
      F(P, 1, prec)->cols_plain(c1, false);
    }
  }
  PassArgs c0 = args_col(P, prec, B, p, 0);
  c0.out = work;
  c0.inv_n = bscale / (double)P->N;
  c0.keep_dc = keep_dc;
  {
    KT kt_(P, "col0_fwd_mul_inv");
    F(P, 0, prec)->cols_fwd_mul_inv(c0);
  }
  if (P->dim == 3) {
    PassArgs c1 = args_col(P, prec, B, p, 1);
    c1.in = work;
    c1.out = work;
    {
      KT kt_(P, "col1_inv");
      F(P, 1, prec)->cols_plain(c1, true);
    }
  }
  PassArgs o = args_rows(P, prec, B, p, true);
  o.in = work;
  o.out = hv;
  o.psi = psi;
  o.v = v;
  o.mpart = project ? P->partial : nullptr;
  o.mbpi = r.rg.bpi;
  o.scale = bscale;
  {
    KT kt_(P, "rows_c2r_hv");
    F(P, 2, prec)->rows_c2r(o, 1);
  }
  return check_launch("lb_hessvec");
}

extern "C" int lb_hessvec(lb_plan *P, const lb_params *params, const double *psi, const double *v, double *hv,
                          int project) {
  return hessvec_phys(P, params, psi, v, hv, project ? 0 : 1);
}

extern "C" int lb_hessvec_raw(lb_plan *P, const lb_params *params, const double *psi, const double *v, double *hv) {
  return hessvec_phys(P, params, psi, v, hv, 2);
}

extern "C" int lb_energy_grad_raw(lb_plan *P, const lb_params *params, const double *psi, double *energy,
                                  double *grad) {
  if (!P || !psi || !energy || !grad) return fail(LB_ERR_ARG, "null argument");
  Prm p;
  LB_TRY(pack_params(P, params, P->batch, &p));
  const int B = P->batch;
  energy_grad_core(P, B, p, psi, 1);
  {
    KT kt_(P, "energy_out");
    LB_LAUNCH(lbk::k_energy_out, dim3(1), dim3(64), 0, P->stream, (const double *)(P->sums + 32), 3,
              (const double *)P->sums, 2, 1.0 / (double)P->N, B, energy);
  }
  inv_c2r(P, LB_FP64, B, p, P->GH, P->W64, grad, 0, nullptr, nullptr);
  return check_launch("lb_energy_grad_raw");
}

extern "C" int lb_field_moments(lb_plan *P, const double *psi, const double *w, double *out) {
  if (!P || !psi || !out) return fail(LB_ERR_ARG, "null argument");
  const int B = P->batch;
  const int bpi = (int)bpi_ew(P);
  {
    KT kt_(P, "field_moments");
    LB_LAUNCH(lbk::k_field_moments, dim3(bpi * B), dim3(lbk::EW_NT), 0, P->stream, P->N, bpi, psi, w, P->partial);
  }
  finalize(P, P->partial, bpi, 4, 0u, B, P->sums);
  {
    KT kt_(P, "scale_out");
    LB_LAUNCH(lbk::k_scale_out, dim3(1), dim3(64), 0, P->stream, (const double *)P->sums, 4 * B,
              1.0 / (double)P->N, out);
  }
  return check_launch("lb_field_moments");
}

// ---------------------------------------------------------------------------
// Hessian-vector product without allocation: the workspace (twiddles, the
// partial sums of the mean, the half spectrum) lives in a fixed device array,
// one per GPU, located once per device with hipGetSymbolAddress; the plan is
// a stack view onto it. Calls on one device share the array.
// ---------------------------------------------------------------------------
#define LB_NOALLOC_SCRATCH_BYTES (8u << 20)
static __device__ __align__(256) unsigned char scratch[LB_NOALLOC_SCRATCH_BYTES];
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
constexpr size_t kTwBytes = 3 * 512 * sizeof(double2);  // per-axis twiddles, n <= 512
constexpr size_t kPartialDoubles = 4096;
constexpr size_t kSpecOffset = kTwBytes + kPartialDoubles * sizeof(double);
}  // namespace
namespace lbk {
// W[m] = exp(-2 pi i m / n) by quadrant (the axis points exact), as the plan's host tables
__global__ void k_twiddles(int n, double2 *w) {
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < n; m += gridDim.x * blockDim.x) {
    const long m4 = 4L * m;
    const int quad = (int)(m4 / n);
    const long rem = m4 % n;
    double sn, cs;
    sincospi(0.5 * (double)rem / (double)n, &sn, &cs);
    double cc, ss;
    switch (quad) {
      case 0: cc = cs; ss = sn; break;
      case 1: cc = -sn; ss = cs; break;
      case 2: cc = -cs; ss = -sn; break;
      default: cc = sn; ss = -cs; break;
    }
    w[m] = double2{cc, -ss};
  }
}
}  // namespace lbk

// the device address of this GPU's scratch array (looked up once per device)
static int scratch_address(void **out) {
  int d = 0;
  LB_HIP(hipGetDevice(&d));
  if (d < 0 || d >= kMaxDevices) return fail(LB_ERR_HIP, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[d]) {
    void *ptr = nullptr;
    LB_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(LB_ERR_HIP, "hipGetSymbolAddress returned no address");
    g_scratch_ptr[d] = ptr;
  }
  *out = g_scratch_ptr[d];
  return 0;
}

extern "C" int lb_hessvec_noalloc(const lb_grid *g, const lb_params *params, const double *psi, const double *v,
                                  double *hv, int project, void *stream) {
  if (!g || !params || !psi || !v || !hv) return fail(LB_ERR_ARG, "null argument");
  if (g->dim != 2 && g->dim != 3) return fail(LB_ERR_ARG, "dim must be 2 or 3");
  for (int a = 0; a < g->dim; ++a) {
    if (!(g->box[a] > 0.0) || !std::isfinite(g->box[a])) return fail(LB_ERR_ARG, "box sides must be positive");
    if (!funcs_for(g->n[a], 0)) return fail(LB_ERR_UNSUPPORTED, "axis length not supported (2^a 3^b, 8..512)");
  }
  lb_plan V;  // a view: every buffer below points into the scratch array (no member allocates)
  V.grid = *g;
  V.dim = g->dim;
  V.batch = 1;
  V.prec = LB_FP64;
  V.stream = (hipStream_t)stream;
  V.n0 = g->n[0];
  V.n1 = (g->dim == 3) ? g->n[1] : 1;
  V.nl = g->n[g->dim - 1];
  V.nhl = V.nl / 2 + 1;
  V.N = (long)V.n0 * V.n1 * V.nl;
  V.nh = (long)V.n0 * V.n1 * V.nhl;
  if (kSpecOffset + (size_t)V.nh * sizeof(double2) > LB_NOALLOC_SCRATCH_BYTES)
    return fail(LB_ERR_ARG, "grid too large for the fixed workspace of lb_hessvec_noalloc (8 MiB: half spectrum of "
                            "at most 520 000 modes)");
  void *base = nullptr;
  LB_TRY(scratch_address(&base));
  unsigned char *sb = (unsigned char *)base;
  const int axis_of[3] = {0, g->dim == 3 ? 1 : -1, g->dim - 1};
  for (int sl = 0; sl < 3; ++sl) {
    AxisTab &A = V.ax[sl];
    if (axis_of[sl] < 0) {
      A.n = 1;
      continue;
    }
    A.n = g->n[axis_of[sl]];
    A.f64 = funcs_for(A.n, LB_FP64);
    A.f32 = funcs_for(A.n, LB_FP32);
    A.L = g->box[axis_of[sl]];
    A.tw64 = (double2 *)(sb + (size_t)sl * 512 * sizeof(double2));
    LB_LAUNCH(lbk::k_twiddles, dim3(2), dim3(256), 0, V.stream, A.n, A.tw64);
  }
  V.partial = (double *)(sb + kTwBytes);
  V.partial_len = (long)kPartialDoubles;
  const long need = std::max(bpi_pairs(&V), 4L * V.n0);  // K n0 (K <= 4): the split order's mean partials
  if (need > (long)kPartialDoubles) return fail(LB_ERR_ARG, "grid needs more partial sums than the fixed workspace holds");
  V.WT = (void *)(sb + kSpecOffset);
  const int rc = hessvec_phys(&V, params, psi, v, hv, project ? 0 : 1);
  V.ax[0].tw64 = V.ax[1].tw64 = V.ax[2].tw64 = nullptr;
  return rc;
}

extern "C" int lb_param_grad(lb_plan *P, const double *psi, const double *w, double *out) {
  if (!P || !psi || !out) return fail(LB_ERR_ARG, "null argument");
  const int B = P->batch;
  const int bpi = (int)bpi_ew(P);
  {
    KT kt_(P, "field_moments");
    LB_LAUNCH(lbk::k_field_moments, dim3(bpi * B), dim3(lbk::EW_NT), 0, P->stream, P->N, bpi, psi, w, P->partial);
  }
  finalize(P, P->partial, bpi, 4, 0u, B, P->sums);
  {
    KT kt_(P, "param_out");
    LB_LAUNCH(lbk::k_param_out, dim3(1), dim3(64), 0, P->stream, (const double *)P->sums, B, 1.0 / (double)P->N, out);
  }
  return check_launch("lb_param_grad");
}

extern "C" int lb_param_grad_vjp(lb_plan *P, const double *psi, const double *ct, double *out) {
  if (!P || !psi || !ct || !out) return fail(LB_ERR_ARG, "null argument");
  const long total = P->N * P->batch;
  {
    KT kt_(P, "param_vjp");
    LB_LAUNCH(lbk::k_param_vjp, dim3((unsigned)std::min<long>(cdiv(total, lbk::EW_NT), 4096)), dim3(lbk::EW_NT), 0,
              P->stream, P->N, P->batch, psi, ct, out);
  }
  return check_launch("lb_param_grad_vjp");
}

// the plane pass of the inner iteration, in the variant the autotuner chose

static void plane_pass(lb_plan *P, const NFuncs *f1, const PassArgs &a) {
  if (P->plane_nt >= 0 && f1->plane_inner_nt[P->plane_nt]) f1->plane_inner_nt[P->plane_nt](a, P->n0);
  else f1->plane_inner(a, P->n0);
}

// spectral Hessian-vector product in FP64: out = Lambda x + P F_N(Gamma' F_N^{-1} x) + shift x
static void hess_spec64(lb_plan *P, const Prm &p, const double2 *x, double2 *out, double shift,
                        const double *gp = nullptr) {
  if (!gp) gp = P->gp64;
  PassArgs c0 = args_col(P, LB_FP64, 1, p, 0);
  c0.in = x;
  c0.out = P->W64;
  {
    KT kt_(P, "col0_inv");
    F(P, 0, LB_FP64)->cols_plain(c0, true);
  }
  const NFuncs *f1 = P->dim == 3 ? F(P, 1, LB_FP64) : nullptr;
  if (f1 && f1->plane_inner && P->n1 == P->nl) {
    PassArgs pl = args_col(P, LB_FP64, 1, p, 1);
    pl.out = P->W64;
    pl.gp = gp;
    KT kt_(P, "plane_inner");
    plane_pass(P, f1, pl);
  } else {
    if (P->dim == 3) {
      PassArgs c1 = args_col(P, LB_FP64, 1, p, 1);
      c1.in = P->W64;
      c1.out = P->W64;
      KT kt_(P, "col1_inv");
      F(P, 1, LB_FP64)->cols_plain(c1, true);
    }
    PassArgs r = args_rows(P, LB_FP64, 1, p, true);
    r.out = P->W64;
    r.gp = gp;
    {
      KT kt_(P, "rows_inner");
      F(P, 2, LB_FP64)->rows_inner(r);
    }
    if (P->dim == 3) {
      PassArgs c1 = args_col(P, LB_FP64, 1, p, 1);
      c1.in = P->W64;
      c1.out = P->W64;
      KT kt_(P, "col1_fwd");
      F(P, 1, LB_FP64)->cols_plain(c1, false);
    }
  }
  PassArgs f = args_col(P, LB_FP64, 1, p, 0);
  f.in = P->W64;
  f.gh = x;
  f.out = out;
  f.inv_n = 1.0 / (double)P->N;
  f.shift = shift;
  {
    KT kt_(P, "col0_fwd_hess");
    F(P, 0, LB_FP64)->cols_fwd_hess(f);
  }
}

// ---------------------------------------------------------------------------
// Algorithm 3 on the device
// ---------------------------------------------------------------------------
struct SubOut {
  double lam = 0, resid = 0, dnorm = 0;
  int iters = 0, newton = 0, newton_direct = 0, status = 0;
};

// One iteration of Algorithm 3 for the B instances at the front of the plan's
// batch, as a launch sequence. The kernels take only the parity of the step
// (which b buffer and multiplier slot to use); the Newton kernel reads the
// step number itself from SubState, so the same two-step sequence serves
// every step pair and can be captured once.
template <typename T, bool GEN>
static void launch_newton(lb_plan *P, const PassArgs &u, const Prm &p, int B) {
  using C2 = lbfft::c2<T>;
  LB_LAUNCH((lbk::k_newton<T, GEN>), dim3(B), dim3(lbk::NW_NT), 0, P->stream, u.g, p, (const double *)P->mom,
            u.cg.bpi, (long)u.cg.bpi * B, (const double *)P->partial, u.cg.bpi, (const C2 *)P->B0, (const C2 *)P->B1,
            u.cg.cpi, P->st);
}
// the three passes of step t (inverse with the scale, axes 1 and 2 with
// Gamma', forward with the update); returns the update's arguments. fuse_t
// = t >= 1: the inverse pass first takes the multiplier step of t - 1 (the
// Newton kernel's work); -1: it reads lambda_t from the state
static PassArgs enqueue_passes(lb_plan *P, const Prm &p, int t, int B, int fuse_t = -1) {
  const int prec = P->prec;
  t &= 1;
  const int K = plane_k(P, prec);
  PassArgs a = col0_args(P, prec, B, p, K);
  a.step = t;
  a.b0 = P->B0;
  a.b1 = P->B1;
  a.out = P->WT;
  a.st = P->st;
  a.fuse_t = fuse_t;
  a.mom = P->mom;
  a.partial = P->partial;
  a.mstride = (long)a.cg.bpi * B;
  {
    KT kt_(P, "col0_inv_scale_d");
    F(P, 0, prec)->cols_inv_scale_d(a);
  }
  const NFuncs *f1 = P->dim == 3 ? F(P, 1, prec) : nullptr;
  if (K > 1) {
    // axis 1 split by x1 mod K, rows with Gamma': K workgroups per plane
    PassArgs pl = args_col(P, prec, B, p, 1);
    pl.out = P->WT;
    pl.gp = (prec == LB_FP64) ? (const void *)P->gp64 : (const void *)P->gp32;
    pl.st = P->st;
    const int ki = kidx(K);
    const int v = P->split_nt >= 0 && f1->plane_split_nt[ki][P->split_nt] ? P->split_nt : f1->plane_split_default[ki];
    KT kt_(P, "plane_inner");
    f1->plane_split_nt[ki][v](pl, P->n0);
  } else if (f1 && f1->plane_inner && P->n1 == P->nl) {
    // axis-1 inverse, rows with Gamma', axis-1 forward: one plane pass in LDS
    PassArgs pl = args_col(P, prec, B, p, 1);
    pl.out = P->WT;
    pl.gp = (prec == LB_FP64) ? (const void *)P->gp64 : (const void *)P->gp32;
    pl.st = P->st;
    KT kt_(P, "plane_inner");
    plane_pass(P, f1, pl);
  } else {
    if (P->dim == 3) {
      PassArgs c1 = args_col(P, prec, B, p, 1);
      c1.in = P->WT;
      c1.out = P->WT;
      c1.st = P->st;
      {
        KT kt_(P, "col1_inv");
        F(P, 1, prec)->cols_plain(c1, true);
      }
    }
    PassArgs r = args_rows(P, prec, B, p, true);
    r.out = P->WT;
    r.gp = (prec == LB_FP64) ? (const void *)P->gp64 : (const void *)P->gp32;
    r.st = P->st;
    {
      KT kt_(P, "rows_inner");
      F(P, 2, prec)->rows_inner(r);
    }
    if (P->dim == 3) {
      PassArgs c1 = args_col(P, prec, B, p, 1);
      c1.in = P->WT;
      c1.out = P->WT;
      c1.st = P->st;
      {
        KT kt_(P, "col1_fwd");
        F(P, 1, prec)->cols_plain(c1, false);
      }
    }
  }
  PassArgs u = col0_args(P, prec, B, p, K);
  u.in = P->WT;
  u.b0 = P->B0;
  u.b1 = P->B1;
  u.gh = P->GHT;
  u.partial = P->partial;
  u.mom = P->mom;
  u.st = P->st;
  u.inv_n = 1.0 / (double)P->N;
  u.step = t;
  {
    KT kt_(P, "col0_fwd_update");
    F(P, 0, prec)->cols_fwd_update(u);
  }
  return u;
}

// the Newton kernel after the update pass whose arguments are u
static void enqueue_newton(lb_plan *P, const Prm &p, const PassArgs &u, int B) {
  KT kt_(P, "newton");
  const bool gen = u.g.general != 0;
  if (P->prec == LB_FP64) {
    if (gen) launch_newton<double, true>(P, u, p, B);
    else launch_newton<double, false>(P, u, p, B);
  } else {
    if (gen) launch_newton<float, true>(P, u, p, B);
    else launch_newton<float, false>(P, u, p, B);
  }
}

static void enqueue_step(lb_plan *P, const Prm &p, int t, int B = 1) {
  const PassArgs u = enqueue_passes(P, p, t, B);
  enqueue_newton(P, p, u, B);
}

// Runs Algorithm 3 for the B instances at the front of the batch (radius r[b],
// step size eta[b], ||g_b|| = gnorm[b]) with g_hat in GH/GHT and Gamma' in
// gp64/gp32; the initial point is -r g/||g|| or d0_spec (FP64 spectral,
// nullable, B = 1 only). Leaves d in SH; out[b] per instance. The launches
// continue until every instance's stop test or cap has ended it (a stopped
// instance's passes compute but store nothing).
static int run_subproblem(lb_plan *P, const Prm &p, int B, const double *r, const lb_sub_opts &o, const double *eta,
                          const double *gnorm, const double2 *d0_spec, SubOut *out) {
  const int prec = P->prec;
  const long nb = std::min<long>(cdiv((long)B * P->nh, lbk::EW_NT), 4096);
  const Geo gB = geo(P, B);
  lbk::InitCoef ic{};
  for (int b = 0; b < B; ++b) {
    ic.coef[b] = d0_spec ? 1.0 : -r[b] / gnorm[b];
    ic.eta[b] = eta[b];
  }
  const void *src = d0_spec ? (const void *)d0_spec : (const void *)P->GH;
  if (prec == LB_FP64) {
    KT kt_(P, "init_b");
    LB_LAUNCH((lbk::k_init_b<double, double>), dim3(nb), dim3(lbk::EW_NT), 0, P->stream, gB, p, (const double2 *)src,
              ic, (double2 *)P->B1);
  } else {
    KT kt_(P, "init_b");
    LB_LAUNCH((lbk::k_init_b<float, double>), dim3(nb), dim3(lbk::EW_NT), 0, P->stream, gB, p, (const double2 *)src,
              ic, (float2 *)P->B1);
  }
  LB_HIP(hipStreamSynchronize(P->stream));  // the pinned mirror may still feed an earlier copy
  for (int b = 0; b < B; ++b) {
    SubState s{};
    s.lam[0] = 0.0;
    s.lam[1] = 0.0;
    s.eta = eta[b];
    s.r2 = r[b] * r[b];
    s.tol = std::max(o.eps_sub, o.eps_sub_rel * gnorm[b]);
    s.newton_rtol = o.newton_rtol;
    s.newton_steptol = o.newton_steptol;
    s.step = 0;
    s.done = 0;
    s.max_inner = o.max_inner;
    s.max_newton = o.max_newton;
    s.newton_phi = o.newton_phi;
    s.newton_direct_only = o.newton_direct;
    P->st_h[b] = s;
  }
  LB_HIP(hipMemcpyAsync(P->st, P->st_h, sizeof(SubState) * B, hipMemcpyHostToDevice, P->stream));
  const int chunk = std::max(1, o.poll_every);
  long launched = 0;
  const long max_steps = (long)o.max_inner + 1;
  const NFuncs *f0 = F(P, 0, prec);
  if (o.single_workgroup && P->dim == 2 && P->n0 == P->nl && f0->sub2d) {
    // square 2D grid that fits one workgroup: every iteration in one launch,
    // one workgroup per instance
    PassArgs a = args_col(P, prec, B, p, 0);
    a.b0 = P->B0;
    a.b1 = P->B1;
    a.gh = P->GHT;
    a.gp = (prec == LB_FP64) ? (const void *)P->gp64 : (const void *)P->gp32;
    a.st = P->st;
    {
      KT kt_(P, "sub2d");
      f0->sub2d(a);
    }
    LB_TRY(check_launch("subproblem (one workgroup)"));
    LB_HIP(hipMemcpyAsync(P->st_h, P->st, sizeof(SubState) * B, hipMemcpyDeviceToHost, P->stream));
    LB_HIP(hipStreamSynchronize(P->stream));
    launched = max_steps;
  }
  // long subproblems replay a captured two-step launch sequence (no timing:
  // its events are not captured)
  // restores the caller's stream and frees the graph on every exit
  struct GraphScope {
    lb_plan *P;
    hipStream_t user;
    hipGraphExec_t exec = nullptr;
    ~GraphScope() {
      if (exec) (void)hipGraphExecDestroy(exec);
      P->stream = user;
    }
  } gs{P, P->stream};
  hipGraphExec_t &gexec = gs.exec;
  const hipStream_t user = P->stream;
  const bool use_graph = o.graph && !P->timing.on && launched < max_steps && max_steps >= 128;
  if (use_graph) {
    // capture and replay on the plan's own stream (the null stream cannot be
    // captured), ordered after the work already on the caller's stream
    if (!P->own) LB_HIP(hipStreamCreateWithFlags(&P->own, hipStreamNonBlocking));
    hipEvent_t ev;
    LB_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    LB_HIP(hipEventRecord(ev, user));
    LB_HIP(hipStreamWaitEvent(P->own, ev, 0));
    (void)hipEventDestroy(ev);
    P->stream = P->own;
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal);
    if (ce == hipSuccess) {
      enqueue_step(P, p, 0, B);
      enqueue_step(P, p, 1, B);
      ce = hipStreamEndCapture(P->stream, &graph);
    }
    if (ce == hipSuccess) {
      ce = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
    }
    if (ce != hipSuccess) return fail(LB_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
  }
  // timings of launches the last stop-flag read has seen complete: read while
  // the GPU runs the next chunk, not while it waits for it
  size_t timed_done = 0;
  auto all_done = [&]() {
    for (int b = 0; b < B; ++b)
      if (!P->st_h[b].done) return false;
    return true;
  };
  // enqueues chunks of steps, then reads the stop flags (while the timings of
  // the chunk before are read)
  auto poll = [&]() -> int {
    LB_TRY(check_launch("subproblem step"));
    if (timed_done) {
      timing_flush(P, timed_done);
      timed_done = 0;
    }
    LB_HIP(hipMemcpyAsync(P->st_h, P->st, sizeof(SubState) * B, hipMemcpyDeviceToHost, P->stream));
    LB_HIP(hipStreamSynchronize(P->stream));
    timed_done = P->timing.pending.size();
    return 0;
  };
  // the multiplier step fused into the inverse pass costs every workgroup of
  // that pass a read of all the update pass's partials: nmb^2 (MOM_NV + 1)
  // doubles per instance over the pass. Measured per iteration: 1-1.7 us saved
  // up to 96^3 (15 MB of such reads), 3 us lost at 128^3 (48 MB); option 1
  // fuses below 16 MB, option 2 always
  const double nmb = (double)bpi_col0(P);
  const double red_bytes = (double)B * nmb * nmb * (lbk::MOM_NV + 1) * 8.0;
  const bool fuse = o.fused_newton == 2 || (o.fused_newton == 1 && red_bytes <= 16e6);
  if (!use_graph && fuse && !o.newton_direct && launched < max_steps) {
    // the multiplier step of step t - 1 runs in the first pass of step t, so
    // steps 0 .. max_inner + 1 are launched (the last one's first pass takes
    // the multiplier step of max_inner, which ends the subproblem at the cap)
    const long tend = (long)o.max_inner + 2;
    auto run_steps = [&](long t0, bool classic_first) -> int {
      for (long tn = t0; tn < tend;) {
        const int n = (int)std::min<long>(chunk, tend - tn);
        for (int i = 0; i < n; ++i) {
          const long ti = tn + i;
          enqueue_passes(P, p, (int)ti, B, (classic_first && ti == t0) ? -1 : (int)ti);
        }
        tn += n;
        LB_TRY(poll());
        if (all_done()) break;
      }
      return 0;
    };
    LB_TRY(run_steps(0, false));
    for (;;) {
      // an instance paused at a multiplier step whose series Newton needs
      // sums over the spectrum: that step in the Newton kernel (every other
      // instance has stopped or paused, so its workgroups return at once),
      // then the instance's next step reads the multiplier from the state
      int b = -1;
      for (int i = 0; i < B && b < 0; ++i)
        if (P->st_h[i].done == 3) b = i;
      if (b < 0) break;
      const long t1 = P->st_h[b].step;
      P->st_h[b].done = 0;
      LB_HIP(hipMemcpyAsync(P->st + b, P->st_h + b, sizeof(SubState), hipMemcpyHostToDevice, P->stream));
      PassArgs u = col0_args(P, prec, B, p, plane_k(P, prec));
      enqueue_newton(P, p, u, B);
      LB_TRY(run_steps(t1 + 1, true));
    }
    launched = max_steps;
  }
  while (launched < max_steps) {
    const int n = (int)std::min<long>(chunk, max_steps - launched);
    if (gexec) {
      for (int i = 0; i < n; i += 2) {
        const hipError_t le = hipGraphLaunch(gexec, P->stream);
        if (le != hipSuccess) return fail(LB_ERR_HIP, std::string("graph launch: ") + hipGetErrorString(le));
      }
      launched += n + (n & 1);
    } else {
      for (int i = 0; i < n; ++i) enqueue_step(P, p, (int)(launched + i), B);
      launched += n;
    }
    LB_TRY(poll());
    if (all_done()) break;
  }
  // the loop ended with a synchronisation of the stream it ran on, so the
  // caller's stream may go on
  P->stream = user;
  for (int b = 0; b < B; ++b) {
    if (!P->st_h[b].done) return fail(LB_ERR_HIP, "subproblem loop ended without a stop decision");
    if (P->st_h[b].nonfinite) return fail(LB_ERR_NONFINITE, "non-finite residual in the subproblem");
  }
  if (prec == LB_FP64) {
    KT kt_(P, "final_d");
    LB_LAUNCH((lbk::k_final_d<double>), dim3(nb), dim3(lbk::EW_NT), 0, P->stream, gB, p, (const double2 *)P->B0,
              (const double2 *)P->B1, (const SubState *)P->st, P->SH);
  } else {
    KT kt_(P, "final_d");
    LB_LAUNCH((lbk::k_final_d<float>), dim3(nb), dim3(lbk::EW_NT), 0, P->stream, gB, p, (const float2 *)P->B0,
              (const float2 *)P->B1, (const SubState *)P->st, P->SH);
  }
  spec_reduce<double, 0>(P, B, p, P->SH, P->SH, P->sums);
  LB_TRY(read_sums(P, P->sums, B));
  for (int b = 0; b < B; ++b) {
    const SubState &f = P->st_h[b];
    out[b].lam = f.lam_final;
    out[b].resid = f.resid;
    out[b].dnorm = std::sqrt(std::max(P->sums_h[b], 0.0));
    out[b].iters = f.final_step;
    out[b].newton = f.newton_total;
    out[b].newton_direct = f.newton_direct;
    out[b].status = (f.done == 1) ? LB_OK : LB_NOT_CONVERGED;
  }
  return 0;
}

extern "C" void lb_sub_opts_default(lb_sub_opts *o) {
  if (!o) return;
  o->eta = 0.1;
  o->eps_sub = 1e-13;
  o->eps_sub_rel = 0.0;
  o->max_inner = 10000;
  o->max_newton = 100;
  o->newton_rtol = 1e-14;
  o->newton_steptol = 1e-15;
  o->poll_every = 32;
  o->newton_phi = 0;
  o->newton_direct = 0;
  o->single_workgroup = 1;
  o->graph = 0;
  o->fused_newton = 1;
}

extern "C" void lb_tr_opts_default(lb_tr_opts *o) {
  if (!o) return;
  o->theta = 1e-4;
  o->gamma_c = 0.5;
  o->gamma_e = 2.0;
  o->gamma_lambda = 1.5;
  o->mu_lo = 1.0;
  o->mu_hi = 1e5;
  o->mu0 = 1.0;
  o->r0 = 1.0;
  o->nu0 = 5.0;
  o->eps = 1e-10;
  o->grad_norm_inf = 1;
  o->eta = 0.1;
  o->eta_safe = 1;
  o->rho_taylor = 1;
  o->contract_else_old_step = 0;
  o->nu_tol = 1e-12;
  o->max_outer = 500;
  lb_sub_opts_default(&o->sub);
  o->cg_rtol = 1e-12;
  o->cg_maxiter = 1000;
  o->cg_precond_shift = 1.0;
  o->capped_reject = 0;
  o->verbose = 0;
  o->hard_case = 0;
  o->hard_tol = 1e-12;
  o->hard_lanczos_steps = 30;
  o->hard_precond_shift = 1.0;
  o->seed = 0;
}

static int check_sub_opts(const lb_sub_opts &o) {
  if (!(o.eta > 0) || !(o.eps_sub >= 0) || !(o.eps_sub_rel >= 0) || o.max_inner < 1 || o.max_newton < 0)
    return fail(LB_ERR_ARG, "bad subproblem options");
  return 0;
}

extern "C" int lb_tr_subproblem(lb_plan *P, const lb_params *params, const double *psi, const double *grad,
                                double radius, const lb_sub_opts *opts, const double *d0, double *d_out,
                                lb_sub_info *info) {
  if (!P || !psi || !grad || !d_out || !info) return fail(LB_ERR_ARG, "null argument");
  if (P->batch != 1) return fail(LB_ERR_MISMATCH, "lb_tr_subproblem needs a plan with batch 1");
  if (!(radius > 0) || !std::isfinite(radius)) return fail(LB_ERR_ARG, "radius must be positive");
  lb_sub_opts o;
  if (opts) o = *opts;
  else lb_sub_opts_default(&o);
  LB_TRY(check_sub_opts(o));
  Prm p;
  LB_TRY(pack_params(P, params, 1, &p));
  {
    KT kt_(P, "gamma_p");
    LB_LAUNCH(lbk::k_gamma_p, dim3((unsigned)std::min<long>(cdiv(P->N, lbk::EW_NT), 4096)), dim3(lbk::EW_NT), 0,
                       P->stream, P->N, 1, p, psi, P->gp64, P->gp32);
  }
  fwd_r2c(P, LB_FP64, 1, p, grad, P->GH, 1);
  if (P->prec == LB_FP32)
    {
      KT kt_(P, "lincomb");
      LB_LAUNCH((lbk::k_lincomb<float, double, double>), dim3((unsigned)std::min<long>(cdiv(P->nh, lbk::EW_NT), 4096)),
                         dim3(lbk::EW_NT), 0, P->stream, P->nh, 1.0, (const double2 *)P->GH, 0.0, (const double2 *)nullptr,
                         (float2 *)P->GHT);
    }
  double gg = 0.0;
  LB_TRY(spec_dot_host(P, p, P->GH, P->GH, &gg));
  const double gnorm = std::sqrt(std::max(gg, 0.0));
  if (!(gnorm > 0) || !std::isfinite(gnorm)) return fail(gnorm == 0 ? LB_ERR_ARG : LB_ERR_NONFINITE, "gradient norm is zero or not finite");
  const double2 *d0s = nullptr;
  if (d0) {
    fwd_r2c(P, LB_FP64, 1, p, d0, P->X, 1);
    d0s = P->X;
  }
  SubOut so;
  LB_TRY(run_subproblem(P, p, 1, &radius, o, &o.eta, &gnorm, d0s, &so));
  inv_c2r(P, LB_FP64, 1, p, P->SH, P->W64, d_out, 0, nullptr, nullptr);
  LB_TRY(check_launch("lb_tr_subproblem"));
  LB_HIP(hipStreamSynchronize(P->stream));
  info->lambda = so.lam;
  info->resid = so.resid;
  info->dnorm = so.dnorm;
  info->gnorm = gnorm;
  info->iters = so.iters;
  info->newton_iters = so.newton;
  info->newton_direct = so.newton_direct;
  info->status = so.status;
  return so.status;
}

static void prec_scale(lb_plan *P, const Prm &p, const double2 *x, double c, double2 *out, int root);

// ---------------------------------------------------------------------------
// CG for (H + shift I) s = -g (Algorithm 2's linear systems), spectral FP64.
// g_hat in GH; solution in X. Stops when ||r|| <= rtol ||g|| or after maxiter
// steps. With pc > 0 the preconditioned form with the diagonal
// M = (Lambda + shift + pc)^-1, the interaction part of H + shift I, which
// spans the stiff range of the spectrum (z = M r lives in SP, free here);
// pc = 0 is plain CG.
// ---------------------------------------------------------------------------
static int cg_shifted(lb_plan *P, const Prm &p, double shift, double rtol, int maxiter, double pc, int *iters,
                      int inst = 0) {
  // instance `inst` of the batch: its g_hat and Gamma' (p holds its parameters
  // in entry 0); the CG vectors live in the first instance's workspace
  const double2 *GHi = P->GH + (long)inst * P->nh;
  const double *gpi = P->gp64 + (long)inst * P->N;
  const long n = P->nh;
  double2 *Z = pc > 0 ? P->SP : P->R;
  lincomb64(P, n, 0.0, GHi, 0.0, GHi, P->X);   // x = 0
  lincomb64(P, n, -1.0, GHi, 0.0, GHi, P->R);  // r = -g
  if (pc > 0) prec_scale(P, p, P->R, shift + pc, Z, 0);
  lincomb64(P, n, 1.0, Z, 0.0, Z, P->Pv);  // p = z
  double rr, rz;
  LB_TRY(spec_dot_host(P, p, P->R, P->R, &rr));
  if (pc > 0) LB_TRY(spec_dot_host(P, p, P->R, Z, &rz));
  else rz = rr;
  const double bn = std::sqrt(rr);
  int it = 0;
  while (it < maxiter && std::sqrt(rr) > rtol * bn) {
    hess_spec64(P, p, P->Pv, P->AP, shift, gpi);
    double pap;
    LB_TRY(spec_dot_host(P, p, P->Pv, P->AP, &pap));
    if (!(pap > 0)) return fail(LB_ERR_NONFINITE, "CG met a non-positive curvature; H + shift I is not positive definite");
    const double alpha = rz / pap;
    lincomb64(P, n, alpha, P->Pv, 1.0, P->X, P->X);
    lincomb64(P, n, -alpha, P->AP, 1.0, P->R, P->R);
    LB_TRY(spec_dot_host(P, p, P->R, P->R, &rr));
    double rzn = rr;
    if (pc > 0) {
      prec_scale(P, p, P->R, shift + pc, Z, 0);
      LB_TRY(spec_dot_host(P, p, P->R, Z, &rzn));
    }
    lincomb64(P, n, 1.0, Z, rzn / rz, P->Pv, P->Pv);
    rz = rzn;
    ++it;
  }
  *iters = it;
  return 0;
}

extern "C" int lb_shifted_solve(lb_plan *P, const lb_params *params, const double *psi, const double *grad,
                                double shift, double rtol, int maxiter, double precond_shift, double *s_out,
                                int *iters) {
  if (!P || !psi || !grad || !s_out || !iters) return fail(LB_ERR_ARG, "null argument");
  if (!(precond_shift >= 0) || !std::isfinite(precond_shift)) return fail(LB_ERR_ARG, "precond_shift must be finite and >= 0");
  if (P->batch != 1) return fail(LB_ERR_MISMATCH, "lb_shifted_solve needs a plan with batch 1");
  Prm p;
  LB_TRY(pack_params(P, params, 1, &p));
  {
    KT kt_(P, "gamma_p");
    LB_LAUNCH(lbk::k_gamma_p, dim3((unsigned)std::min<long>(cdiv(P->N, lbk::EW_NT), 4096)), dim3(lbk::EW_NT), 0,
                       P->stream, P->N, 1, p, psi, P->gp64, P->gp32);
  }
  fwd_r2c(P, LB_FP64, 1, p, grad, P->GH, 1);
  LB_TRY(cg_shifted(P, p, shift, rtol, maxiter, precond_shift, iters));
  inv_c2r(P, LB_FP64, 1, p, P->X, P->W64, s_out, 0, nullptr, nullptr);
  LB_TRY(check_launch("lb_shifted_solve"));
  LB_HIP(hipStreamSynchronize(P->stream));
  return LB_OK;
}

// ---------------------------------------------------------------------------
// Lanczos (full reorthogonalisation), spectral FP64, Gamma' in gp64
// ---------------------------------------------------------------------------
// eigenvalues / eigenvectors of a small symmetric matrix by cyclic Jacobi
static void jacobi_eig(int m, std::vector<double> &A, std::vector<double> &V) {
  V.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = i + 1; j < m; ++j) off += A[(size_t)i * m + j] * A[(size_t)i * m + j];
    if (off < 1e-300) break;
    for (int pi = 0; pi < m; ++pi)
      for (int q = pi + 1; q < m; ++q) {
        const double apq = A[(size_t)pi * m + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[(size_t)pi * m + pi], aqq = A[(size_t)q * m + q];
        const double th = 0.5 * (aqq - app) / apq;
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < m; ++k) {
          const double akp = A[(size_t)k * m + pi], akq = A[(size_t)k * m + q];
          A[(size_t)k * m + pi] = c * akp - s * akq;
          A[(size_t)k * m + q] = s * akp + c * akq;
        }
        for (int k = 0; k < m; ++k) {
          const double apk = A[(size_t)pi * m + k], aqk = A[(size_t)q * m + k];
          A[(size_t)pi * m + k] = c * apk - s * aqk;
          A[(size_t)q * m + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < m; ++k) {
          const double vkp = V[(size_t)k * m + pi], vkq = V[(size_t)k * m + q];
          V[(size_t)k * m + pi] = c * vkp - s * vkq;
          V[(size_t)k * m + q] = s * vkp + c * vkq;
        }
      }
  }
}

static void prec_scale(lb_plan *P, const Prm &p, const double2 *x, double c, double2 *out, int root = 1) {
  KT kt_(P, "prec_scale");
  LB_LAUNCH(lbk::k_prec_scale, dim3((unsigned)std::min<long>(cdiv(P->nh, lbk::EW_NT), 4096)), dim3(lbk::EW_NT), 0,
                     P->stream, geo(P, 1), p, x, c, root, out);
}

// Lanczos with full reorthogonalisation on H, or with c > 0 on K = S H S,
// S = (Lambda + c)^(-1/2) (congruent to H, same inertia, clustered spectrum);
// then the Rayleigh quotient of H at x = S y for the lowest Ritz vector y.
// vec_out (nullable, may alias v0): the unit Ritz vector (Psi_hat coordinates)
static int lanczos_core(lb_plan *P, const Prm &p, const double2 *v0, int steps, double c, double *ritz, double *resid,
                        double2 *vec_out = nullptr) {
  if ((int)P->lz.size() < steps + 1) {
    while ((int)P->lz.size() < steps + 1) {
      void *q = nullptr;
      LB_HIP(hipMalloc(&q, sizeof(double2) * P->nh));
      P->lz.push_back((double2 *)q);
    }
  }
  const long n = P->nh;
  const bool pc = c > 0.0;
  auto op = [&](const double2 *v, double2 *out) {
    if (pc) {
      prec_scale(P, p, v, c, P->Pv);
      hess_spec64(P, p, P->Pv, P->X, 0.0);
      prec_scale(P, p, P->X, c, out);
    } else {
      hess_spec64(P, p, v, out, 0.0);
    }
  };
  double nn;
  LB_TRY(spec_dot_host(P, p, v0, v0, &nn));
  if (!(nn > 0)) return fail(LB_ERR_ARG, "Lanczos start vector has no zero-mean component");
  lincomb64(P, n, 1.0 / std::sqrt(nn), v0, 0.0, v0, P->lz[0]);
  std::vector<double> alpha, beta;
  for (int i = 0; i < steps; ++i) {
    op(P->lz[i], P->AP);
    if (i > 0) lincomb64(P, n, 1.0, P->AP, -beta[i - 1], P->lz[i - 1], P->AP);
    double a;
    LB_TRY(spec_dot_host(P, p, P->AP, P->lz[i], &a));
    lincomb64(P, n, 1.0, P->AP, -a, P->lz[i], P->AP);
    for (int k = 0; k <= i; ++k) {
      double cc;
      LB_TRY(spec_dot_host(P, p, P->AP, P->lz[k], &cc));
      lincomb64(P, n, 1.0, P->AP, -cc, P->lz[k], P->AP);
    }
    alpha.push_back(a);
    double bb;
    LB_TRY(spec_dot_host(P, p, P->AP, P->AP, &bb));
    const double b = std::sqrt(std::max(bb, 0.0));
    beta.push_back(b);
    if (i == steps - 1 || b < 1e-300) break;
    lincomb64(P, n, 1.0 / b, P->AP, 0.0, P->AP, P->lz[i + 1]);
  }
  const int m = (int)alpha.size();
  std::vector<double> A((size_t)m * m, 0.0), V;
  for (int i = 0; i < m; ++i) {
    A[(size_t)i * m + i] = alpha[i];
    if (i + 1 < m) A[(size_t)i * m + i + 1] = A[(size_t)(i + 1) * m + i] = beta[i];
  }
  jacobi_eig(m, A, V);
  int imin = 0;
  for (int i = 1; i < m; ++i)
    if (A[(size_t)i * m + i] < A[(size_t)imin * m + imin]) imin = i;
  if (!pc) {
    *ritz = A[(size_t)imin * m + imin];
    *resid = std::fabs(beta[m - 1] * V[(size_t)(m - 1) * m + imin]);
    if (vec_out) {
      lincomb64(P, n, 0.0, P->lz[0], 0.0, P->lz[0], P->R);
      for (int i = 0; i < m; ++i) lincomb64(P, n, V[(size_t)i * m + imin], P->lz[i], 1.0, P->R, P->R);
      double yy;
      LB_TRY(spec_dot_host(P, p, P->R, P->R, &yy));
      lincomb64(P, n, 1.0 / std::sqrt(yy), P->R, 0.0, P->R, vec_out);
    }
    return 0;
  }
  // y = sum_i V[i, imin] q_i ; x = S y ; rho = <x, Hx> / <x, x>
  lincomb64(P, n, 0.0, P->lz[0], 0.0, P->lz[0], P->R);
  for (int i = 0; i < m; ++i) lincomb64(P, n, V[(size_t)i * m + imin], P->lz[i], 1.0, P->R, P->R);
  prec_scale(P, p, P->R, c, P->Pv);
  hess_spec64(P, p, P->Pv, P->AP, 0.0);
  double xx, xhx;
  LB_TRY(spec_dot_host(P, p, P->Pv, P->Pv, &xx));
  LB_TRY(spec_dot_host(P, p, P->Pv, P->AP, &xhx));
  const double rho = xhx / xx;
  lincomb64(P, n, 1.0, P->AP, -rho, P->Pv, P->AP);
  double rr;
  LB_TRY(spec_dot_host(P, p, P->AP, P->AP, &rr));
  *ritz = rho;
  *resid = std::sqrt(std::max(rr, 0.0) / xx);
  if (vec_out) lincomb64(P, n, 1.0 / std::sqrt(xx), P->Pv, 0.0, P->Pv, vec_out);
  return 0;
}

// Uniform point of the ball ||d|| <= r in the zero-mean subspace (physical
// field, batch 1): normals from Philox4x64-10 at counter (x, 0, 0, 0), key
// (seed, draw), centred, scaled to radius r u^(1/(N-1)), u from counter
// (0, 1, 0, 0).
static int ball_point(lb_plan *P, double r, unsigned long long seed, unsigned long long draw, double *out) {
  const int nb = (int)std::min<long>(cdiv(P->N, lbk::EW_NT), 1024);
  {
    KT kt_(P, "ball_normals");
    LB_LAUNCH(lbk::k_ball_normals, dim3(nb), dim3(lbk::EW_NT), 0, P->stream, P->N, (uint64_t)seed, (uint64_t)draw, out,
              P->partial);
  }
  finalize(P, P->partial, nb, 2, 0u, 1, P->sums);
  {
    KT kt_(P, "ball_factor");
    LB_LAUNCH(lbk::k_ball_factor, dim3(1), dim3(64), 0, P->stream, P->N, r, (uint64_t)seed, (uint64_t)draw,
              (const double *)P->sums, P->sums + 8);
  }
  {
    KT kt_(P, "ball_scale");
    LB_LAUNCH(lbk::k_ball_scale, dim3(nb), dim3(lbk::EW_NT), 0, P->stream, P->N, (const double *)(P->sums + 8), out);
  }
  return check_launch("ball_point");
}

extern "C" int lb_random_ball(lb_plan *P, double radius, unsigned long long seed, unsigned long long draw,
                              double *d_out) {
  if (!P || !d_out) return fail(LB_ERR_ARG, "null argument");
  if (P->batch != 1) return fail(LB_ERR_MISMATCH, "lb_random_ball needs a plan with batch 1");
  if (!(radius > 0) || !std::isfinite(radius)) return fail(LB_ERR_ARG, "radius must be positive");
  return ball_point(P, radius, seed, draw, d_out);
}

extern "C" int lb_lanczos_min(lb_plan *P, const lb_params *params, const double *psi, const double *v0, int steps,
                              double precond_shift, double *ritz_min, double *resid, double *evec) {
  if (!P || !psi || !v0 || !ritz_min || !resid) return fail(LB_ERR_ARG, "null argument");
  if (P->batch != 1) return fail(LB_ERR_MISMATCH, "lb_lanczos_min needs a plan with batch 1");
  if (steps < 1 || steps > 1000) return fail(LB_ERR_ARG, "steps must be in [1, 1000]");
  Prm p;
  LB_TRY(pack_params(P, params, 1, &p));
  {
    KT kt_(P, "gamma_p");
    LB_LAUNCH(lbk::k_gamma_p, dim3((unsigned)std::min<long>(cdiv(P->N, lbk::EW_NT), 4096)), dim3(lbk::EW_NT), 0,
                       P->stream, P->N, 1, p, psi, P->gp64, P->gp32);
  }
  fwd_r2c(P, LB_FP64, 1, p, v0, P->R, 1);
  if (!std::isfinite(precond_shift)) return fail(LB_ERR_ARG, "precond_shift must be finite");
  lincomb64(P, P->nh, 1.0, P->R, 0.0, P->R, P->SH);  // start vector out of the work buffers
  LB_TRY(lanczos_core(P, p, P->SH, steps, precond_shift, ritz_min, resid, evec ? P->SH : nullptr));
  if (evec) inv_c2r(P, LB_FP64, 1, p, P->SH, P->W64, evec, 0, nullptr, nullptr);
  return check_launch("lb_lanczos_min");
}

// ---------------------------------------------------------------------------
// Algorithms 1 and 2 (host-driven outer loop)
// ---------------------------------------------------------------------------
struct EG {
  double E, gnorm, gninf, gpmax;
};
// energy only at psi + s (s in sphys), for the direct ratio numerator; leaves
// the current iterate's g_hat and Gamma' untouched
static int energy_at_trial(lb_plan *P, const Prm &p, const double *psi, double *E) {
  const long nb = std::min<long>(cdiv(P->N, lbk::EW_NT), 4096);
  {
    KT kt_(P, "add_real");
    LB_LAUNCH(lbk::k_add_real, dim3(nb), dim3(lbk::EW_NT), 0, P->stream, P->N, psi, (const double *)P->sphys,
                       P->ptrial);
  }
  PassArgs r = args_rows(P, LB_FP64, 1, p, false);
  r.psi = P->ptrial;
  r.out = P->SP;
  r.out2 = P->SP + P->nh;
  r.partial = P->partial;
  {
    KT kt_(P, "rows_energy");
    F(P, 2, LB_FP64)->rows_energy(r);
  }
  finalize(P, P->partial, r.rg.bpi, 2, 0x2u, 1, P->sums);
  if (P->dim == 3) {
    PassArgs c1 = args_col(P, LB_FP64, 1, p, 1);
    c1.in = P->SP;
    c1.out = P->SP;
    {
      KT kt_(P, "col1_fwd");
      F(P, 1, LB_FP64)->cols_plain(c1, false);
    }
  }
  PassArgs c0 = args_col(P, LB_FP64, 1, p, 0);
  c0.in = P->SP;
  c0.out = P->SP;
  c0.scale = 1.0 / (double)P->N;
  {
    KT kt_(P, "col0_fwd");
    F(P, 0, LB_FP64)->cols_plain(c0, false);
  }
  spec_reduce<double, 1>(P, 1, p, P->SP, P->SP, P->sums + 32);
  LB_TRY(check_launch("trial energy"));
  LB_TRY(read_sums(P, P->sums, 40));
  *E = 0.5 * P->sums_h[32] + P->sums_h[0] / (double)P->N;
  if (!std::isfinite(*E)) return fail(LB_ERR_NONFINITE, "non-finite trial energy");
  return 0;
}

static int check_tr_opts(const lb_tr_opts &o) {
  LB_TRY(check_sub_opts(o.sub));
  if (!(o.theta > 0 && o.theta < 1) || !(o.gamma_c > 0 && o.gamma_c < 1) || !(o.gamma_e > 1) || !(o.gamma_lambda > 1) ||
      !(o.mu_lo > 0 && o.mu_lo <= o.mu_hi) || !(o.mu0 >= o.mu_lo) || !(o.r0 > 0 && o.r0 <= o.nu0) || !(o.eps > 0))
    return fail(LB_ERR_ARG, "bad trust-region options");
  if (o.hard_case && (o.hard_lanczos_steps < 1 || o.hard_lanczos_steps > 1000 || !(o.hard_tol >= 0)))
    return fail(LB_ERR_ARG, "bad hard-case options");
  if (!(o.cg_precond_shift >= 0) || !std::isfinite(o.cg_precond_shift)) return fail(LB_ERR_ARG, "bad cg_precond_shift");
  return 0;
}

// Prm whose entry 0 is entry s of q (one instance's view)
static Prm prm_one(const Prm &q, int s) {
  Prm p{};
  p.tau[0] = q.tau[s];
  p.gamma[0] = q.gamma[s];
  p.xi[0] = q.xi[s];
  p.q[0] = q.q[s];
  return p;
}

// Algorithm 2 (CONTRACT) for instance `inst` of the batch, whose g_j and
// Gamma'(psi_j) are in GH / gp64 (p: its parameters in entry 0): the new radius.
static int contract_radius(lb_plan *P, const Prm &p, int inst, const lb_tr_opts &o, double lam, double sn, double gnorm,
                           double *r_out, int *cg_total) {
  int it = 0;
  double xx;
  if (lam < o.mu_lo * sn) {
    const double lam_hat = lam + std::sqrt(o.mu_lo * gnorm);
    LB_TRY(cg_shifted(P, p, lam_hat, o.cg_rtol, o.cg_maxiter, o.cg_precond_shift, &it, inst));
    *cg_total += it;
    LB_TRY(spec_dot_host(P, p, P->X, P->X, &xx));
    double snew = std::sqrt(xx);
    if (lam_hat / snew > o.mu_hi) {
      // lambda~ / ||s(lambda~)|| increases with lambda~: bisect on (lambda_j, lambda_hat)
      double lo = lam, hi = lam_hat;
      for (int k = 0; k < 200; ++k) {
        const double mid = 0.5 * (lo + hi);
        LB_TRY(cg_shifted(P, p, mid, o.cg_rtol, o.cg_maxiter, o.cg_precond_shift, &it, inst));
        *cg_total += it;
        LB_TRY(spec_dot_host(P, p, P->X, P->X, &xx));
        snew = std::sqrt(xx);
        const double ratio = mid / snew;
        if (ratio < o.mu_lo) lo = mid;
        else if (ratio > o.mu_hi) hi = mid;
        else break;
      }
    }
    *r_out = snew;
    return 0;
  }
  const double lt = o.gamma_lambda * lam;
  LB_TRY(cg_shifted(P, p, lt, o.cg_rtol, o.cg_maxiter, o.cg_precond_shift, &it, inst));
  *cg_total += it;
  LB_TRY(spec_dot_host(P, p, P->X, P->X, &xx));
  const double snew = std::sqrt(xx);
  if (snew >= o.gamma_c * sn) *r_out = snew;
  else *r_out = o.contract_else_old_step ? o.gamma_c * sn : o.gamma_c * snew;
  return 0;
}

// real rows of instances: y[s] += coef[s] x[s] (coef by value, one per instance)
struct RowCoef {
  double c[lbk::MAXB];
};
namespace lbk {
__global__ __launch_bounds__(EW_NT) void k_axpy_rows(long N, int B, RowCoef a, const double *__restrict__ x, double *y) {
  const long total = N * B;
  for (long i = (long)blockIdx.x * EW_NT + threadIdx.x; i < total; i += (long)gridDim.x * EW_NT) {
    const double c = a.c[i / N];
    if (c != 0.0) y[i] += c * x[i];
  }
}
}  // namespace lbk

// swap the fields of batch slots s and t (device rows of N doubles; sphys is scratch)
static int swap_rows(lb_plan *P, double *psi, int s, int t) {
  if (s == t) return 0;
  const size_t bytes = sizeof(double) * P->N;
  double *a = psi + (long)s * P->N, *b = psi + (long)t * P->N, *tmp = P->sphys;
  LB_HIP(hipMemcpyAsync(tmp, a, bytes, hipMemcpyDeviceToDevice, P->stream));
  LB_HIP(hipMemcpyAsync(a, b, bytes, hipMemcpyDeviceToDevice, P->stream));
  LB_HIP(hipMemcpyAsync(b, tmp, bytes, hipMemcpyDeviceToDevice, P->stream));
  return 0;
}

// Algorithms 1 and 2 (host-driven outer loop) for the plan's `batch`
// instances together: every pass of every outer iteration is one launch for
// all instances still iterating (they are kept at the front of the batch;
// an instance that has converged or failed is swapped to the back and its
// field restored to its slot at the end). The scalar logic runs per instance
// exactly as for one instance, so each result equals its one-instance solve
// bit for bit. Nearly hard subproblems and the direct ratio numerator are
// supported for a batch of one.
static int solve_core(lb_plan *P, const lb_params *params, double *psi, const lb_tr_opts &o, lb_tr_info *infos,
                      int *status) {
  const int B = P->batch;
  LB_TRY(check_tr_opts(o));
  if (B > 1 && (o.hard_case || !o.rho_taylor))
    return fail(LB_ERR_UNSUPPORTED, "batched solves take the Taylor ratio numerator and no hard-case starts");
  Prm pall;
  LB_TRY(pack_params(P, params, B, &pall));
  struct Inst {
    double r, nu, mu, rho_prev = 0.0;
    bool have_prev = false;
    EG eg{};
  };
  std::vector<Inst> S(B);
  std::vector<int> slot_inst(B);  // instance held by each batch slot
  for (int b = 0; b < B; ++b) {
    S[b].r = o.r0;
    S[b].nu = o.nu0;
    S[b].mu = o.mu0;
    slot_inst[b] = b;
    std::memset(&infos[b], 0, sizeof(lb_tr_info));
    status[b] = LB_NOT_CONVERGED;
  }
  int nA = B;  // active slots [0, nA)
  Prm pA = pall;
  auto rebuild_params = [&]() {
    for (int s2 = 0; s2 < nA; ++s2) {
      const int i2 = slot_inst[s2];
      pA.tau[s2] = pall.tau[i2];
      pA.gamma[s2] = pall.gamma[i2];
      pA.xi[s2] = pall.xi[i2];
      pA.q[s2] = pall.q[i2];
    }
  };
  auto finish = [&](int slot, int st_code, int outer) {
    const int i2 = slot_inst[slot];
    lb_tr_info &inf = infos[i2];
    inf.energy = S[i2].eg.E;
    inf.gnorm = S[i2].eg.gnorm;
    inf.gnorm_inf = S[i2].eg.gninf;
    inf.outer = outer;
    inf.status = st_code;
    status[i2] = st_code;
  };
  // energy and gradient of the active slots, per instance
  auto energy_grads = [&]() -> int {
    energy_grad_core(P, nA, pA, psi);
    LB_TRY(check_launch("energy"));
    LB_TRY(read_sums(P, P->sums, 64));
    const double *sm = P->sums_h;
    for (int s2 = 0; s2 < nA; ++s2) {
      EG &eg = S[slot_inst[s2]].eg;
      eg.E = sm[32 + 3 * s2] + sm[2 * s2] / (double)P->N;
      eg.gnorm = std::sqrt(std::max(sm[33 + 3 * s2], 0.0));
      eg.gninf = sm[34 + 3 * s2];
      eg.gpmax = sm[2 * s2 + 1];
    }
    return 0;
  };
  // moves the slots flagged in `out` to the back of the active range
  std::vector<char> out(B, 0);
  auto compact = [&]() -> int {
    int s2 = 0;
    while (s2 < nA) {
      if (!out[s2]) {
        ++s2;
        continue;
      }
      const int last = nA - 1;
      LB_TRY(swap_rows(P, psi, s2, last));
      std::swap(slot_inst[s2], slot_inst[last]);
      std::swap(out[s2], out[last]);
      out[last] = 0;
      --nA;
    }
    rebuild_params();
    return 0;
  };
  int first_err = 0;
  std::string first_msg;
  int j = 0;
  bool eg_fresh = false;
  for (; j < o.max_outer && nA > 0; ++j) {
    // g_j of every active instance; those within the tolerance (or non-finite) leave
    if (!eg_fresh) LB_TRY(energy_grads());
    eg_fresh = false;
    bool any = false;
    for (int s2 = 0; s2 < nA; ++s2) {
      const EG &eg = S[slot_inst[s2]].eg;
      if (!std::isfinite(eg.E) || !std::isfinite(eg.gnorm)) {
        finish(s2, LB_ERR_NONFINITE, j);
        if (!first_err) {
          first_err = LB_ERR_NONFINITE;
          first_msg = "non-finite energy or gradient";
        }
        out[s2] = any = true;
      } else if ((o.grad_norm_inf ? eg.gninf : eg.gnorm) < o.eps) {
        finish(s2, LB_OK, j);
        out[s2] = any = true;
      }
    }
    if (any) {
      LB_TRY(compact());
      if (nA == 0) break;
      LB_TRY(energy_grads());  // the compacted slots' g_j and Gamma'
    }
    std::vector<double> r(nA), eta(nA), gn(nA);
    for (int s2 = 0; s2 < nA; ++s2) {
      const Inst &I = S[slot_inst[s2]];
      r[s2] = I.r;
      eta[s2] = o.eta_safe && I.eg.gpmax > 0 ? std::min(o.eta, 0.9 / I.eg.gpmax) : o.eta;
      gn[s2] = I.eg.gnorm;
    }
    lb_sub_opts so = o.sub;
    so.eta = eta[0];
    // nearly hard subproblem (Remark on the hard case; one instance): sigma_1 < 0
    // and |<xi, g>| <= hard_tol -> start Algorithm 3 from a random point of the ball
    const double2 *d0_spec = nullptr;
    if (o.hard_case) {
      LB_TRY(ball_point(P, 1.0, o.seed, 2ull * (unsigned long long)j + 1ull, P->sphys));
      fwd_r2c(P, LB_FP64, 1, pA, P->sphys, P->R, 1);
      lincomb64(P, P->nh, 1.0, P->R, 0.0, P->R, P->SH);
      double sig, res, g1;
      LB_TRY(lanczos_core(P, pA, P->SH, o.hard_lanczos_steps, o.hard_precond_shift, &sig, &res, P->SH));
      LB_TRY(spec_dot_host(P, pA, P->GH, P->SH, &g1));
      if (sig < 0.0 && std::fabs(g1) <= o.hard_tol) {
        LB_TRY(ball_point(P, r[0], o.seed, 2ull * (unsigned long long)j, P->sphys));
        fwd_r2c(P, LB_FP64, 1, pA, P->sphys, P->R, 1);
        d0_spec = P->R;
        infos[slot_inst[0]].hard_cases++;
      }
      if (o.verbose) std::fprintf(stderr, "[lb] j=%d sigma1~%.6e g1=%.3e%s\n", j, sig, g1, d0_spec ? " hard" : "");
    }
    std::vector<SubOut> sub(nA);
    LB_TRY(run_subproblem(P, pA, nA, r.data(), so, eta.data(), gn.data(), d0_spec, sub.data()));
    // the ratio numerator E(v) - E(v + s) of every active instance
    std::vector<double> dE(nA);
    if (o.rho_taylor) {
      spec_reduce<double, 0>(P, nA, pA, P->GH, P->SH, P->sums);
      spec_reduce<double, 1>(P, nA, pA, P->SH, P->SH, P->sums + 16);
      inv_c2r(P, LB_FP64, nA, pA, P->SH, P->W64, P->sphys, 2, psi, P->partial);
      finalize(P, P->partial, (int)bpi_pairs(P), 1, 0u, nA, P->sums + 32);
      LB_TRY(read_sums(P, P->sums, 48));
      for (int s2 = 0; s2 < nA; ++s2) {
        const double gs = P->sums_h[s2], quad = P->sums_h[16 + s2], pw = P->sums_h[32 + s2] / (double)P->N;
        dE[s2] = -(gs + 0.5 * quad + pw);
      }
    } else {  // one instance
      inv_c2r(P, LB_FP64, 1, pA, P->SH, P->W64, P->sphys, 0, nullptr, nullptr);
      double Et;
      LB_TRY(energy_at_trial(P, pA, psi, &Et));
      dE[0] = S[slot_inst[0]].eg.E - Et;
    }
    RowCoef acc{};
    bool any_accept = false;
    for (int s2 = 0; s2 < nA; ++s2) {
      const int i2 = slot_inst[s2];
      Inst &I = S[i2];
      lb_tr_info &inf = infos[i2];
      const SubOut &su = sub[s2];
      inf.inner_total += su.iters;
      inf.newton_total += su.newton;
      inf.newton_direct += su.newton_direct;
      if (su.status != LB_OK) inf.sub_capped++;
      const double lam = su.lam, sn = su.dnorm;
      if (!(sn > 0)) return fail(LB_ERR_NONFINITE, "zero trial step");
      if (o.capped_reject && su.status != LB_OK) {
        // no optimality conditions, no ratio test: the field stays, the radius shrinks
        I.r *= o.gamma_c;
        I.rho_prev = -1.0;  // a rejection for the next iteration's mu update
        I.have_prev = true;
        if (o.verbose)
          std::fprintf(stderr, "[lb] i=%d j=%d E=%.15e |g|=%.3e r=%.3e inner=%d resid=%.2e capped: rejected\n", i2, j,
                       I.eg.E, I.eg.gnorm, I.r, su.iters, su.resid);
        continue;
      }
      if (j > 0 && I.have_prev && I.rho_prev < o.theta) I.mu = std::max(I.mu, lam / sn);
      const double rho = dE[s2] / (sn * sn * sn);
      const char *branch;
      const bool on_nu = std::fabs(sn - I.nu) <= o.nu_tol * I.nu;
      // lambda <= mu ||s|| tested as lambda / ||s|| <= mu: after a contraction mu
      // was just raised to lambda / ||s||, and the sides must then compare equal
      // exactly, not by the rounding of (lambda / ||s||) ||s||
      if (rho >= o.theta && (lam / sn <= I.mu || on_nu)) {
        acc.c[s2] = 1.0;
        any_accept = true;
        I.nu = std::max(I.nu, o.gamma_e * sn);
        I.r = std::min(I.nu, std::max(I.r, o.gamma_e * sn));
        I.mu = std::max(I.mu, lam / sn);
        inf.accepted++;
        branch = "accept";
      } else if (rho < o.theta) {
        // Algorithm 2 (CONTRACT); needs Gamma'(psi_j) and g_j of this instance
        LB_TRY(contract_radius(P, prm_one(pA, s2), s2, o, lam, sn, I.eg.gnorm, &I.r, &inf.cg_total));
        inf.contracted++;
        branch = "contract";
      } else {
        I.r = std::min(I.nu, lam / I.mu);
        inf.expanded++;
        branch = "expand";
      }
      if (o.verbose)
        std::fprintf(stderr,
                     "[lb] i=%d j=%d E=%.15e |g|=%.3e |g|inf=%.3e r=%.3e nu=%.3e mu=%.3e lam=%.6e |s|=%.3e rho=%.6e "
                     "eta=%.4f inner=%d resid=%.2e %s\n",
                     i2, j, I.eg.E, I.eg.gnorm, I.eg.gninf, I.r, I.nu, I.mu, lam, sn, rho, eta[s2], su.iters, su.resid,
                     branch);
      I.rho_prev = rho;
      I.have_prev = true;
    }
    if (any_accept) {
      // v_{j+1} = v_j + s_j for the accepted instances (s_j in sphys)
      const long nb = std::min<long>(cdiv((long)nA * P->N, lbk::EW_NT), 4096);
      KT kt_(P, "axpy_real");
      LB_LAUNCH(lbk::k_axpy_rows, dim3(nb), dim3(lbk::EW_NT), 0, P->stream, P->N, nA, acc, (const double *)P->sphys,
                psi);
    } else if (!o.hard_case) {
      eg_fresh = true;  // no field moved: g_j and Gamma' still hold
    }
  }
  // instances still iterating at the cap: E and g at their last iterate
  if (nA > 0 && !eg_fresh) LB_TRY(energy_grads());
  for (int s2 = 0; s2 < nA; ++s2) finish(s2, LB_NOT_CONVERGED, j);
  // every field back to its own slot
  for (int s2 = 0; s2 < B; ++s2) {
    while (slot_inst[s2] != s2) {
      const int t = slot_inst[s2];
      LB_TRY(swap_rows(P, psi, s2, t));
      std::swap(slot_inst[s2], slot_inst[t]);
    }
  }
  LB_TRY(check_launch("lb_imex_tr_solve"));
  LB_HIP(hipStreamSynchronize(P->stream));
  if (first_err) return fail(first_err, first_msg);
  return 0;
}

extern "C" int lb_imex_tr_solve(lb_plan *P, const lb_params *params, double *psi, const lb_tr_opts *opts,
                                lb_tr_info *info) {
  if (!P || !psi || !info) return fail(LB_ERR_ARG, "null argument");
  if (P->batch != 1) return fail(LB_ERR_MISMATCH, "lb_imex_tr_solve needs a plan with batch 1");
  lb_tr_opts o;
  if (opts) o = *opts;
  else lb_tr_opts_default(&o);
  int st = 0;
  LB_TRY(solve_core(P, params, psi, o, info, &st));
  return st;
}

extern "C" int lb_imex_tr_solve_batch(lb_plan *P, const lb_params *params, double *psi, const lb_tr_opts *opts,
                                      lb_tr_info *infos, int *status) {
  if (!P || !params || !psi || !infos || !status) return fail(LB_ERR_ARG, "null argument");
  lb_tr_opts o;
  if (opts) o = *opts;
  else lb_tr_opts_default(&o);
  LB_TRY(solve_core(P, params, psi, o, infos, status));
  for (int b = 0; b < P->batch; ++b)
    if (status[b] < 0) return status[b];
  return LB_OK;
}

// ---------------------------------------------------------------------------
// Many independent solves at once (instances of different sizes and
// parameters): a pool of host threads, each with its own HIP stream, takes
// jobs largest first and runs the host-driven outer loop of each on its own
// plan, so that the small, latency-bound launches of different instances
// overlap on the GPU.
// ---------------------------------------------------------------------------
extern "C" int lb_imex_tr_solve_many(lb_plan *const *plans, const lb_params *params, double *const *psi, int count,
                                     const lb_tr_opts *opts, int workers, lb_tr_info *infos, int *status) {
  if (count < 0 || (count > 0 && (!plans || !params || !psi || !infos || !status)))
    return fail(LB_ERR_ARG, "null argument");
  if (count == 0) return LB_OK;
  if (workers < 1) return fail(LB_ERR_ARG, "workers must be >= 1");
  workers = std::min(workers, count);
  // job i solves the plans[i]->batch instances starting at instance off[i]
  std::vector<long> off(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    if (!plans[i] || !psi[i]) return fail(LB_ERR_ARG, "null plan or field");
    for (int k = 0; k < i; ++k)
      if (plans[k] == plans[i]) return fail(LB_ERR_ARG, "a plan appears in two jobs");
    off[i + 1] = off[i] + plans[i]->batch;
  }
  lb_tr_opts o;
  if (opts) o = *opts;
  else lb_tr_opts_default(&o);
  // the fields are ready on each plan's stream: the workers wait for that point
  std::vector<hipEvent_t> ready(count, nullptr);
  for (int i = 0; i < count; ++i) {
    LB_HIP(hipEventCreateWithFlags(&ready[i], hipEventDisableTiming));
    LB_HIP(hipEventRecord(ready[i], plans[i]->stream));
  }
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return plans[a]->N * plans[a]->batch > plans[b]->N * plans[b]->batch; });
  std::atomic<int> next{0};
  std::vector<std::string> errs(count);
  std::vector<int> job_rc(count, LB_OK);
  auto work = [&]() {
    hipStream_t ws = nullptr;
    if (hipStreamCreateWithFlags(&ws, hipStreamNonBlocking) != hipSuccess) ws = nullptr;
    for (int q = next.fetch_add(1); q < count; q = next.fetch_add(1)) {
      const int i = order[q];
      lb_plan *P = plans[i];
      if (!ws) {
        job_rc[i] = LB_ERR_HIP;
        errs[i] = "hipStreamCreate failed";
        for (long k = off[i]; k < off[i + 1]; ++k) status[k] = LB_ERR_HIP;
        continue;
      }
      const hipStream_t orig = P->stream;
      int rc = hipStreamWaitEvent(ws, ready[i], 0) == hipSuccess ? LB_OK : LB_ERR_HIP;
      if (rc == LB_OK) {
        P->stream = ws;
        rc = solve_core(P, &params[off[i]], psi[i], o, &infos[off[i]], &status[off[i]]);
        if (rc < 0) {
          errs[i] = g_last_error;
          for (long k = off[i]; k < off[i + 1]; ++k)
            if (status[k] >= 0) status[k] = rc;
        }
        // later work on the plan's own stream sees the result
        hipEvent_t done;
        if (hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess) {
          (void)hipEventRecord(done, ws);
          (void)hipStreamWaitEvent(orig, done, 0);
          (void)hipEventDestroy(done);
        }
        P->stream = orig;
      } else {
        errs[i] = "hipStreamWaitEvent failed";
        for (long k = off[i]; k < off[i + 1]; ++k) status[k] = rc;
      }
      job_rc[i] = rc;
    }
    if (ws) {
      (void)hipStreamSynchronize(ws);
      (void)hipStreamDestroy(ws);
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < workers; ++w) pool.emplace_back(work);
  work();
  for (auto &t : pool) t.join();
  for (int i = 0; i < count; ++i) (void)hipEventDestroy(ready[i]);
  for (int i = 0; i < count; ++i) {
    if (job_rc[i] < 0) return fail(job_rc[i], "job " + std::to_string(i) + ": " + errs[i]);
    for (long k = off[i]; k < off[i + 1]; ++k)
      if (status[k] < 0) return fail(status[k], "job " + std::to_string(i) + ": an instance failed");
  }
  return LB_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: the plane pass of the inner iteration (the dominant kernel on
// cubic grids) is built with 256, 512 and 1024 threads; time each on this
// plan's buffers and keep the fastest.
// ---------------------------------------------------------------------------
extern "C" int lb_plan_set_plane_threads(lb_plan *P, int threads) {
  if (!P) return fail(LB_ERR_ARG, "null plan");
  if (threads == 0) {
    P->plane_nt = -1;
    return LB_OK;
  }
  const int v = threads == 256 ? 0 : threads == 512 ? 1 : threads == 1024 ? 2 : -1;
  if (v < 0) return fail(LB_ERR_ARG, "plane threads must be 0, 256, 512 or 1024");
  const NFuncs *f1 = P->dim == 3 ? F(P, 1, P->prec) : nullptr;
  if (!f1 || !f1->plane_inner || P->n1 != P->nl || !f1->plane_inner_nt[v])
    return fail(LB_ERR_UNSUPPORTED, "this grid has no plane pass");
  P->plane_nt = v;
  return LB_OK;
}

extern "C" int lb_plan_autotune(lb_plan *P, const lb_params *params, const double *psi, int reps, int *threads) {
  if (!P || !psi || !threads) return fail(LB_ERR_ARG, "null argument");
  if (reps < 1 || reps > 10000) return fail(LB_ERR_ARG, "reps must be in [1, 10000]");
  *threads = 0;
  const int prec = P->prec;
  const NFuncs *f1 = P->dim == 3 ? F(P, 1, prec) : nullptr;
  const bool whole = f1 && f1->plane_inner && P->n1 == P->nl && f1->plane_inner_nt[0];
  if (!whole && !split_ok(P, prec, 2) && !split_ok(P, prec, 4)) return LB_OK;  // nothing to tune
  Prm p;
  LB_TRY(pack_params(P, params, P->batch, &p));
  {
    KT kt_(P, "gamma_p");
    LB_LAUNCH(lbk::k_gamma_p, dim3((unsigned)std::min<long>(cdiv(P->N * P->batch, lbk::EW_NT), 4096)), dim3(lbk::EW_NT),
              0, P->stream, P->N, P->batch, p, psi, P->gp64, P->gp32);
  }
  // a running subproblem state for instance 0 and zeroed b buffers: the three
  // passes of an inner iteration run on them as in a solve (the update pass
  // leaves the state alone; Newton is the same in every variant and not timed)
  SubState s0{};
  s0.eta = 0.05;
  s0.max_inner = 1 << 30;
  LB_HIP(hipMemcpyAsync(P->st, &s0, sizeof(SubState), hipMemcpyHostToDevice, P->stream));
  const size_t bbytes = (size_t)P->nh * (prec == LB_FP64 ? sizeof(double2) : sizeof(float2));
  LB_HIP(hipMemsetAsync(P->B0, 0, bbytes, P->stream));
  LB_HIP(hipMemsetAsync(P->B1, 0, bbytes, P->stream));
  hipEvent_t e0, e1;
  LB_HIP(hipEventCreate(&e0));
  LB_HIP(hipEventCreate(&e1));
  const int nts[3] = {256, 512, 1024};
  const int keep_split = P->plane_split, keep_nt = P->plane_nt, keep_snt = P->split_nt, keep_colv = P->colv;
  const int colv_built = F(P, 0, prec)->colv_built;
  // the built-in variant, which stays unless another is faster by more than
  // 2 % (near-ties are timing noise, and in FP32 the variants' rounding can
  // change a solve's path): plane_k's choice, its built-in threads, plan 0
  P->plane_split = -1;
  const int k0 = plane_k(P, prec);
  const int v0 = k0 > 1 ? f1->plane_split_default[kidx(k0)]
                        : !whole ? 0 : (f1->plane_nt_default == 256 ? 0 : f1->plane_nt_default == 512 ? 1 : 2);
  // every candidate (parts K, thread variant, column plan) is timed in two
  // rounds (interleaved, so that clock and cache drift hit all alike) and
  // keeps its faster round
  struct Cand {
    int k, v, cv;
    float ms;
  };
  std::vector<Cand> cands;
  for (int k : {1, 2, 4})
    for (int v = 0; v < 3; ++v) {
      // K = 1: the plane pass's thread variants, or once the five passes
      if (k == 1 && (whole ? !f1->plane_inner_nt[v] : v != 0)) continue;
      if (k > 1 && (!split_ok(P, prec, k) || !f1->plane_split_nt[kidx(k)][v])) continue;
      for (int cv = 0; cv < 4; ++cv)
        if ((colv_built >> cv & 1) && colv_ok(P, prec, k, cv)) cands.push_back(Cand{k, v, cv, 0.0f});
    }
  for (int round = 0; round < 2; ++round) {
    for (Cand &c : cands) {
      P->plane_split = c.k;
      if (c.k > 1) P->split_nt = c.v;
      else P->plane_nt = c.v;
      P->colv = c.cv;
      enqueue_passes(P, p, 1, 1);  // warm
      LB_HIP(hipEventRecord(e0, P->stream));
      for (int r = 0; r < reps; ++r) enqueue_passes(P, p, r + 2, 1);
      LB_HIP(hipEventRecord(e1, P->stream));
      LB_HIP(hipEventSynchronize(e1));
      float ms = 0.0f;
      LB_HIP(hipEventElapsedTime(&ms, e0, e1));
      c.ms = round == 0 ? ms : std::min(c.ms, ms);
    }
  }
  const Cand *pick = nullptr;
  for (const Cand &c : cands)
    if (!pick || c.ms < pick->ms) pick = &c;
  for (const Cand &c : cands)
    if (c.k == k0 && c.v == v0 && c.cv == 0 && c.ms <= 1.02f * pick->ms) pick = &c;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->plane_split = keep_split;
  P->plane_nt = keep_nt;
  P->split_nt = keep_snt;
  P->colv = keep_colv;
  LB_TRY(check_launch("lb_plan_autotune"));
  if (!pick) return LB_OK;
  P->plane_split = pick->k;
  if (pick->k > 1) P->split_nt = pick->v;
  else if (whole) P->plane_nt = pick->v;
  P->colv = pick->cv;
  *threads = (pick->k == 1 && !whole) ? 0 : nts[pick->v];
  return LB_OK;
}

// split codes of the API: 0 none, 1 two parts, 2 four parts
static int k_of_code(int code) { return code == 0 ? 1 : code == 1 ? 2 : code == 2 ? 4 : -1; }
static int code_of_k(int K) { return K == 2 ? 1 : K == 4 ? 2 : 0; }

extern "C" int lb_plan_set_plane_split(lb_plan *P, int split, int threads) {
  if (!P) return fail(LB_ERR_ARG, "null plan");
  const int K = k_of_code(split);
  if (K < 0) return fail(LB_ERR_ARG, "split must be 0, 1 or 2");
  const int v = threads == 0 ? -1 : threads == 256 ? 0 : threads == 512 ? 1 : threads == 1024 ? 2 : -2;
  if (v == -2) return fail(LB_ERR_ARG, "plane threads must be 0, 256, 512 or 1024");
  if (K > 1) {
    if (!split_ok(P, P->prec, K)) return fail(LB_ERR_UNSUPPORTED, "this grid has no split order with that many parts");
    if (v >= 0 && !F(P, 1, P->prec)->plane_split_nt[kidx(K)][v])
      return fail(LB_ERR_UNSUPPORTED, "split-plane pass not built with that thread count");
    P->split_nt = v;
  } else if (v >= 0) {
    // one workgroup per plane with a pinned thread count (without a plane
    // pass, split = 0 selects the column and row passes and takes no count)
    LB_TRY(lb_plan_set_plane_threads(P, threads));
  }
  P->plane_split = K;
  return LB_OK;
}

extern "C" int lb_plan_get_variant(lb_plan *P, int *split, int *threads, int *column_plan) {
  if (!P || !split || !threads || !column_plan) return fail(LB_ERR_ARG, "null argument");
  *split = 0;
  *threads = 0;
  const int prec = P->prec;
  const NFuncs *f1 = P->dim == 3 ? F(P, 1, prec) : nullptr;
  const int nts[3] = {256, 512, 1024};
  const int K = plane_k(P, prec);
  *column_plan = colv_ok(P, prec, K, P->colv) ? P->colv : 0;
  if (K > 1) {
    const int ki = kidx(K);
    *split = code_of_k(K);
    *threads = nts[P->split_nt >= 0 && f1->plane_split_nt[ki][P->split_nt] ? P->split_nt : f1->plane_split_default[ki]];
  } else if (f1 && f1->plane_inner && P->n1 == P->nl) {
    *threads = (P->plane_nt >= 0 && f1->plane_inner_nt[P->plane_nt]) ? nts[P->plane_nt] : f1->plane_nt_default;
  }
  return LB_OK;
}

extern "C" int lb_plan_set_hessvec_split(lb_plan *P, int split) {
  if (!P) return fail(LB_ERR_ARG, "null plan");
  if (split == -1) {
    P->hv_split = -1;
    return LB_OK;
  }
  const int K = k_of_code(split);
  if (K < 0) return fail(LB_ERR_ARG, "split must be -1, 0, 1 or 2");
  if (K > 1 && !split_ok(P, P->prec, K)) return fail(LB_ERR_UNSUPPORTED, "this grid has no split order with that many parts");
  P->hv_split = K;
  return LB_OK;
}

extern "C" int lb_plan_set_column_plan(lb_plan *P, int column_plan) {
  if (!P) return fail(LB_ERR_ARG, "null plan");
  if (column_plan < 0 || column_plan > 3) return fail(LB_ERR_ARG, "column plan must be 0, 1, 2 or 3");
  if (!(F(P, 0, P->prec)->colv_built >> column_plan & 1))
    return fail(LB_ERR_UNSUPPORTED, "column plan not built for this axis-0 length");
  P->colv = column_plan;
  return LB_OK;
}

