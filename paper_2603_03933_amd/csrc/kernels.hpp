// kernels.hpp - HIP kernels of the IMEX-TR hot path for gfx950.
//
// Spectral layout: the half spectrum of a real field, shape [n0][n1][nl/2+1]
// (3D) or [n0][nl/2+1] (2D), complex, last axis fastest, `batch` instances
// back to back. A mode with 0 < k_last < nl/2 stands for itself and its
// conjugate partner, so sums over the full spectrum weigh it by 2.
//
// A 3D transform is a row pass (last axis, real <-> complex, two real rows
// packed into one complex transform) plus column passes along axes 1 and 0
// (strided, C neighbouring columns per workgroup so that every global access
// is coalesced). The pointwise stages of the method ride on the row passes
// and the diagonal reciprocal-space stages on the axis-0 pass. Reductions
// write one partial per workgroup; a single workgroup sums them in a fixed
// order, so every result is bitwise reproducible.
#pragma once
#include <cstdint>
#include <type_traits>

#include "fft.hpp"

namespace lbk {
using namespace lbfft;

constexpr int MAXB = 8;  // instances per launch

struct Prm {  // model coefficients per instance (kernel argument, by value)
  double tau[MAXB], gamma[MAXB], xi[MAXB], q[MAXB];
};

struct Geo {
  int dim;       // 2 or 3
  int n0, n1;    // leading axes (n1 = 1 in 2D)
  int nl, nhl;   // last axis and its half-spectrum length nl/2 + 1
  long N;        // points per instance
  long nh;       // half-spectrum modes per instance
  int batch;
  // |Bk|^2 = sum_ab G_ab k_a k_b with G = B^T B (Section 2, A B^T = 2 pi I):
  // c_a = sqrt(G_aa) (2 pi / L_a for an orthorhombic box) and the cross
  // coefficients 2 G_ab of the leading, middle (3D) and last axes, all 0 for
  // an orthorhombic box
  double c0, c1, cl;
  double x01, x0l, x1l;
  int general;  // some cross coefficient is nonzero (uniform branch for the paired sums)
};

// |Bk|^2 along one axis, (c k)^2 with c = 2 pi / L, for storage index i of n
// points (signed k, except along the halved last axis): two multiplies, no
// table and so no memory round trip. Not contracted: the square is rounded
// before callers add the other axes.
__device__ __forceinline__ double kk_ax(int i, int n, double c, bool half) {
#pragma clang fp contract(off)
  const int k = (half || i < n / 2) ? i : i - n;
  const double t = c * (double)k;
  return t * t;
}
__device__ __forceinline__ double kk0_of(const Geo &g, int i0) { return kk_ax(i0, g.n0, g.c0, false); }
__device__ __forceinline__ double kk1_of(const Geo &g, int i1) { return kk_ax(i1, g.n1, g.c1, false); }
__device__ __forceinline__ double kkl_of(const Geo &g, int kl) { return kk_ax(kl, g.nl, g.cl, true); }

__device__ __forceinline__ double lam_of(double kk, double xi, double q) {
  const double t = q * q - kk;
  return xi * xi * t * t;
}

// instance-relative half-spectrum offset -> (i0, i1, kl); 32-bit arithmetic
__device__ __forceinline__ void decode(const Geo &g, int h, int &i0, int &i1, int &kl) {
  const int r = h / g.nhl;
  kl = h - r * g.nhl;
  i0 = r / g.n1;
  i1 = r - i0 * g.n1;
}

// The column part of |Bk|^2 for (k1, k_last) and the coefficients of k0 in
// the cross terms. The signed index set puts a Nyquist entry at -n/2; its
// conjugate partner is the entry with every Nyquist coordinate negated, and
// with cross terms the two would carry different |Bk|^2, so both take their
// mean: a cross term k_a k_b counts when axes a and b are both at Nyquist or
// both not. lin applies when k0 is not at Nyquist, lin_nyq when it is. On an
// orthorhombic box every cross coefficient is 0 and the sums below add zeros.
struct ColK {
  double kkc, lin, lin_nyq;
};
__device__ __forceinline__ ColK col_k(const Geo &g, int i1, int kl) {
  ColK c;
  c.kkc = g.dim == 3 ? kkl_of(g, kl) + kk1_of(g, i1) : kkl_of(g, kl);
  const bool n1q = g.dim == 3 && 2 * i1 == g.n1;
  const bool nlq = 2 * kl == g.nl;  // stored as +nl/2, signed -nl/2
  const double k1 = g.dim == 3 ? (double)(i1 < g.n1 / 2 ? i1 : i1 - g.n1) : 0.0;
  const double kls = nlq ? -(double)kl : (double)kl;
  c.kkc += (n1q == nlq) ? g.x1l * (k1 * kls) : 0.0;
  c.lin = (n1q ? 0.0 : g.x01 * k1) + (nlq ? 0.0 : g.x0l * kls);
  c.lin_nyq = (n1q ? g.x01 * k1 : 0.0) + (nlq ? g.x0l * kls : 0.0);
  return c;
}
// |Bk|^2 of axis-0 element e of a column: (kk0 + kkc) + k0 lin
__device__ __forceinline__ double kk_elem(const Geo &g, int e, double kkc, double lin, double lin_nyq) {
  const int k0 = e < g.n0 / 2 ? e : e - g.n0;
  return (kk0_of(g, e) + kkc) + (double)k0 * (2 * e == g.n0 ? lin_nyq : lin);
}
__device__ __forceinline__ double kk_at(const Geo &g, int h, int &kl) {
  int i0, i1;
  decode(g, h, i0, i1, kl);
  const ColK c = col_k(g, i1, kl);
  return kk_elem(g, i0, c.kkc, c.lin, c.lin_nyq);
}
__device__ __forceinline__ double herm_w(const Geo &g, int kl) { return (kl == 0 || 2 * kl == g.nl) ? 1.0 : 2.0; }

// 1 / x for x >= 1 to full FP64 accuracy: hardware estimate + two Newton steps
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Reciprocal-space data shared by all elements of one axis-0 column
struct ColInfo {
  double kkc;           // |Bk|^2 contribution of the column's (k1, k_last)
  double lin, lin_nyq;  // coefficients of k0 in the cross terms (0 on an orthorhombic box)
  double w;             // Hermitian weight of the column
  int dc;               // the column holds k = 0 at element 0
};
// GEN: the grid may have cross terms (general lattice); the orthorhombic
// instantiations keep |Bk|^2 = kk0 + kkc without them
template <bool GEN = true> __device__ __forceinline__ ColInfo col_info(const Geo &g, int ml) {
  int i1 = 0, kl = ml;
  if (g.dim == 3) {
    i1 = ml / g.nhl;
    kl = ml - i1 * g.nhl;
  }
  ColInfo c;
  if constexpr (GEN) {
    const ColK k = col_k(g, i1, kl);
    c.kkc = k.kkc;
    c.lin = k.lin;
    c.lin_nyq = k.lin_nyq;
  } else {
    c.kkc = g.dim == 3 ? kkl_of(g, kl) + kk1_of(g, i1) : kkl_of(g, kl);
    c.lin = c.lin_nyq = 0.0;
  }
  c.w = herm_w(g, kl);
  c.dc = (ml == 0);
  return c;
}
template <bool GEN = true> __device__ __forceinline__ double kk_e(const Geo &g, int e, const ColInfo &c) {
  if constexpr (GEN) return kk_elem(g, e, c.kkc, c.lin, c.lin_nyq);
  else return kk0_of(g, e) + c.kkc;
}

constexpr int pow2_floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}
// Column-pass shape. V = 0: radix plan 0 (8s first), TPF = N / 8 threads per
// transform; 256 threads per workgroup, or 512 for long transforms so that a
// workgroup still spans 16 adjacent columns (>= 128 B runs per row in FP32).
// V = 1: radix plan 2 (4s first: more threads per transform, one pass more at
// N = 128); V = 2: radix plan 1 (16 first: fewer threads, one pass fewer). The
// variants keep the C columns of V = 0 (autotuner candidates for the inner
// iteration's axis-0 passes; ok: they fit a workgroup).
template <int N, int V = 0> struct Cfg {
  static constexpr int PLAN = V == 0 || V == 3 ? 0 : (V == 1 ? 2 : 1);
  static constexpr int TPF0 = Shape<N>::TPF;
  static constexpr int C0 = pow2_floor((TPF0 >= 32 ? 512 : 256) / TPF0) * (V == 3 ? 2 : 1);  // V = 3: twice the columns
  static constexpr int C = C0 > 64 ? 64 : (C0 < 1 ? 1 : C0);  // transforms per workgroup
  static constexpr int TPF = N / lbfft::radix_p<PLAN>(N, 0);    // threads per transform
  static constexpr int NT = C * TPF;                             // threads per workgroup
  static constexpr bool ok = NT >= 64 && NT <= 1024 && lbfft::npass_p<PLAN>(N) > 0;
};

// ---------------------------------------------------------------------------
// Block reductions (wavefront shuffles, then LDS across waves)
// ---------------------------------------------------------------------------
// Wavefront reductions with DPP lane moves (no LDS round trips): row_shr 1, 2,
// 4, 8 leave each row's total in its lane 15, row_bcast15 / row_bcast31 fold
// the rows into lane 63, which is then read back as a uniform value. Lanes
// whose source is outside the row read 0, so wave_max needs values >= 0.
template <int CTRL, int ROW_MASK, bool BOUND_ZERO> __device__ __forceinline__ double dpp_d(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xf, BOUND_ZERO);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xf, BOUND_ZERO);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane63(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}
// sum over each row of 16 lanes, left in the row's lane 15
__device__ __forceinline__ double row_sum(double v) {
  v += dpp_d<0x111, 0xf, true>(v);  // row_shr:1
  v += dpp_d<0x112, 0xf, true>(v);  // row_shr:2
  v += dpp_d<0x114, 0xf, true>(v);  // row_shr:4
  v += dpp_d<0x118, 0xf, true>(v);  // row_shr:8
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
  v = row_sum(v);
  v += dpp_d<0x142, 0xa, false>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xc, false>(v);  // row_bcast:31 into rows 2 and 3
  return lane63(v);
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_d<0x111, 0xf, true>(v));
  v = fmax(v, dpp_d<0x112, 0xf, true>(v));
  v = fmax(v, dpp_d<0x114, 0xf, true>(v));
  v = fmax(v, dpp_d<0x118, 0xf, true>(v));
  v = fmax(v, dpp_d<0x142, 0xa, false>(v));
  v = fmax(v, dpp_d<0x143, 0xc, false>(v));
  return lane63(v);
}
// result valid in thread 0; `scratch` holds >= 16 doubles; all threads must call
template <int NT> __device__ __forceinline__ double block_sum(double v, double *scratch) {
  constexpr int NW = (NT + 63) / 64;
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NW; ++w) s += scratch[w];
  return s;
}
// sum over the block returned to every thread; `scratch` holds >= 17 doubles
template <int NT> __device__ __forceinline__ double block_sum_all(double v, double *scratch) {
  const double s = block_sum<NT>(v, scratch);
  if (threadIdx.x == 0) scratch[16] = s;
  __syncthreads();
  const double r = scratch[16];
  __syncthreads();
  return r;
}
template <int NT> __device__ __forceinline__ double block_max(double v, double *scratch) {
  constexpr int NW = (NT + 63) / 64;
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NW; ++w) s = fmax(s, scratch[w]);
  return s;
}

// ---------------------------------------------------------------------------
// Inner-iteration state (one per instance, device memory)
// ---------------------------------------------------------------------------
struct SubState {
  double lam[2];      // lambda_t for step t at lam[t & 1]
  double eta, r2, tol;
  double newton_rtol, newton_steptol;
  double resid;       // residual norm of the iterate tested last
  double lam_final;   // multiplier of the returned iterate
  int step;           // current step t
  int done;           // 0 running, 1 converged, 2 iteration cap, 3 paused (a multiplier step left to k_newton)
  int final_step;
  int newton_total;
  int max_inner, max_newton;
  int nonfinite;
  int newton_phi;     // 1: Newton on phi(lambda) = r^2; 0: on 1/sqrt(phi) = 1/r
  int newton_direct_only;  // 1: every Newton evaluation sums phi over the spectrum
  int newton_direct;       // Newton evaluations that summed phi over the spectrum
};

// ---------------------------------------------------------------------------
// The multiplier update of Algorithm 3 (eq. lambda_update_rule)
// ---------------------------------------------------------------------------
// phi(lambda) = sum_k w_k |b_k|^2 / (x_k + eta lambda)^2 with x_k = 1 + eta D_k.
// Rather than re-reading the spectrum for every Newton evaluation, one pass
// per step forms the power sums
//   M_j = sum_k w_k |b_k|^2 u_k^j,  u_k = 1 / (x_k + mu0),  j = 2 .. NMOM + 1,
// around mu0 = eta lambda_t, the previous multiplier. Every pole of phi as a
// function of mu = eta lambda lies at mu <= -1, so for D = mu - mu0
//   phi   = sum_{m >= 0} (m + 1) (-D)^m M_{m+2}
//   dphi/dmu = -sum_{m >= 0} (m + 1)(m + 2) (-D)^m M_{m+3},
// and since u_k <= 1 / (1 + mu0) the tail after NMOM terms is at most
// M_2 (NMOM + 1) rho^NMOM / (1 - rho)^2 with rho = |D| / (1 + mu0). A Newton
// evaluation uses the truncated series when that bound is below 1e-17 phi
// (far below rounding), and otherwise sums phi directly over the spectrum.
// phi(0), which decides whether the constraint is active, is summed exactly.
constexpr int NMOM = 20;          // series terms
constexpr int MOM_NV = NMOM + 1;  // phi(0) and M_2 .. M_{NMOM+1}

// Newton's method for the multiplier lambda_{t+1} (eq. lambda_update_rule)
// from the power sums M (M[0] = phi(0), M[1 + m] = M_{m+2} around
// mu0 = eta lambda_prev): the series with its tail bound where it holds,
// else direct(lam, phi, dphi), a block-collective sum over the spectrum. Every
// thread runs the same scalar iteration on the same values (uniform control
// flow) and gets the same result. it / ndirect count steps / direct sums.
struct NewtonPar {
  double eta, r2, lam_prev, rtol, steptol;
  int max_newton, form_phi, direct_only;
};
template <class Direct>
__device__ double multiplier_newton(const double *M, const NewtonPar &np, const Direct &direct, int &it,
                                    int &ndirect) {
  const double eta = np.eta, r2 = np.r2, lam_prev = np.lam_prev;
  const double mu0 = eta * lam_prev;
  auto eval = [&](double lam, double &phi, double &dphi) {
    const double D = eta * (lam - lam_prev);
    if (!np.direct_only && D == 0.0) {
      // the series at its centre (the warm start): the same values as the
      // Horner sums below with -D = 0, without their dependent chains
      phi = M[1];
      dphi = -eta * (2.0 * M[2]);
      return;
    }
    const double rho = fabs(D) / (1.0 + mu0);
    if (!np.direct_only && rho < 0.5) {
      double rn = 1.0;
#pragma unroll
      for (int j = 0; j < NMOM; ++j) rn *= rho;
      const double tail = M[1] * (NMOM + 1) * rn / ((1.0 - rho) * (1.0 - rho));
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int m = NMOM - 1; m >= 0; --m) a = fma(a, -D, (m + 1) * M[1 + m]);
#pragma unroll
      for (int m = NMOM - 2; m >= 0; --m) b = fma(b, -D, (double)((m + 1) * (m + 2)) * M[2 + m]);
      if (tail <= 1e-17 * a) {
        phi = a;
        dphi = -eta * b;
        return;
      }
    }
    ++ndirect;
    direct(lam, phi, dphi);
  };
  double lam = 0.0;
  it = 0;
  if (M[0] > r2) {  // phi(0) > r^2: the multiplier is the root of phi(lambda) = r^2
    double phi, dphi;
    if (np.form_phi || !(lam_prev > 0.0)) {
      lam = 0.0;  // the printed iteration: Newton from lambda = 0
      eval(0.0, phi, dphi);
    } else {
      lam = lam_prev;  // warm start at the previous multiplier
      eval(lam, phi, dphi);
    }
    const double rr = sqrt(r2);
    while (it < np.max_newton) {
      if (phi >= r2 && phi - r2 <= np.rtol * r2) break;
      double nl = np.form_phi ? lam - (phi - r2) / dphi : lam + 2.0 * phi * (1.0 - sqrt(phi) / rr) / dphi;
      if (nl < 0.0) nl = 0.0;
      ++it;
      if (fabs(nl - lam) <= np.steptol * fmax(1.0, fabs(lam))) {
        lam = nl;
        break;
      }
      lam = nl;
      eval(lam, phi, dphi);
    }
  }
  return lam;
}

// sums of two values over a block of NT threads, returned to every thread
template <int NT>
__device__ __forceinline__ void block_sum2_nt(double &a, double &b, double *scratch /* >= 2 * NT / 64 */) {
  constexpr int NW = NT / 64;
  const int w = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) {
    scratch[w] = a;
    scratch[NW + w] = b;
  }
  __syncthreads();
  a = b = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    a += scratch[i];
    b += scratch[NW + i];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Column passes
// ---------------------------------------------------------------------------
struct ColGeo {
  int cpi;    // columns per instance
  int bpi;    // workgroups per instance
  int inner;  // base(m) = (m / inner) * outer + m % inner
  long outer;
  long S;     // element stride along the transformed axis
  long inst;  // instance stride
  int hsplit = 0;  // > 0: split column order (col_of), hsplit = (n1/K) n_half columns per part
  int kparts = 2;  // K, the parts of the split order (2 or 4)
};

// Column of lane c in workgroup lb of an instance. Plain order: lb CC + c.
// Split order with K parts: lane c belongs to part q = c / (CC/K) and takes
// column q hsplit + lb CC/K + c mod CC/K, i.e. the column (k1 + q n1/K, k2) of
// the group whose first member is (k1, k2); the K members of a group sit in
// lanes CC/K apart in one wave (K = 2: lanes c and c ^ CC/2).
template <int CC> __device__ __forceinline__ int col_of(const ColGeo &cg, int lb, int c) {
  if (cg.hsplit == 0) return lb * CC + c;
  const int qc = CC / cg.kparts;
  const int q = c / qc;
  return q * cg.hsplit + lb * qc + (c - q * qc);
}
// the value lane ^ M holds (M = 8: row_ror:8 within rows of 16 lanes;
// otherwise a lane permute)
template <int M> __device__ __forceinline__ double lane_xor(double x) {
  if constexpr (M == 8) return dpp_d<0x128, 0xf, false>(x);
  else return __shfl_xor(x, M);
}
template <int M> __device__ __forceinline__ float lane_xor(float x) {
  if constexpr (M == 8)
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xf, 0xf, false));
  else return __shfl_xor(x, M);
}
template <int M, typename T> __device__ __forceinline__ c2<T> lane_xor2(c2<T> v) {
  return c2<T>{lane_xor<M>(v.x), lane_xor<M>(v.y)};
}
// DPP row_ror:R within rows of 16 lanes (lane i receives lane (i - R) mod 16)
template <int R> __device__ __forceinline__ double ror_d(double x) { return dpp_d<0x120 + R, 0xf, false>(x); }
template <int R> __device__ __forceinline__ float ror_d(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x120 + R, 0xf, 0xf, false));
}
template <int R, typename T> __device__ __forceinline__ c2<T> ror2(c2<T> v) {
  return c2<T>{ror_d<R>(v.x), ror_d<R>(v.y)};
}
// v times i^e (e in 0..3: quarter turns)
template <typename T> __device__ __forceinline__ c2<T> mul_iq(c2<T> v, int e) {
  const T x = (e & 1) ? -v.y : v.x, y = (e & 1) ? v.x : v.y;
  return (e & 2) ? c2<T>{-x, -y} : c2<T>{x, y};
}
// The K-point step of the split order across the K lanes of a group, for the
// lane of part q (its own value v = a_q). INV: s = sum_p a_p w^{p q} with
// w = e^{+2 pi i / K} (the first step of the inverse axis-1 transform split
// by x1 mod K); forward: Y = sum_p Z_p w^{-q p} (its last step). K = 2: lane
// ^ CC/2; K = 4 (CC = 16): DPP rotates by 4, 8 and 12 within rows of 16.
template <int K, int CC, bool INV, typename T> __device__ __forceinline__ c2<T> split_dft(c2<T> v, int q) {
  if constexpr (K == 2) {
    const c2<T> u = lane_xor2<CC / 2, T>(v);
    if (q == 0) return c2<T>{v.x + u.x, v.y + u.y};
    return c2<T>{u.x - v.x, u.y - v.y};  // a_0 - a_1 (INV) or Z_0 - Z_1 (forward)
  } else {
    static_assert(K == 4 && CC == 16, "four parts: groups within rows of 16 lanes");
    c2<T> a[4];  // a[r]: the value of part (q + r) mod 4
    a[0] = v;
    a[1] = ror2<12, T>(v);  // lane i + 4
    a[2] = ror2<8, T>(v);
    a[3] = ror2<4, T>(v);  // lane i - 4
    c2<T> s{T(0), T(0)};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pq = ((q + r) * q) & 3;
      const c2<T> t = mul_iq<T>(a[r], INV ? pq : (4 - pq) & 3);
      s = c2<T>{s.x + t.x, s.y + t.y};
    }
    return s;
  }
}

// pair butterfly of an axis-0 pass on the pair-split order: PAIR = 1 at the
// loads, 2 at the stores (Op::PAIR; 0 or absent: none)
template <class Op, class = void> struct OpPair {
  static constexpr int value = 0;
};
template <class Op> struct OpPair<Op, std::void_t<decltype(Op::PAIR)>> {
  static constexpr int value = Op::PAIR;
};
// ops with pre(bs, b, lb), run by every thread after begin() and before the
// transform's loads
template <class Op, class = void> struct OpHasPre {
  static constexpr bool value = false;
};
template <class Op> struct OpHasPre<Op, std::void_t<decltype(Op::HAS_PRE)>> {
  static constexpr bool value = Op::HAS_PRE;
};

// A twiddle table of N entries staged into LDS: load() reads it with a
// kernel's first loads, one scalar (real or imaginary part) per thread, and
// store() writes it to LDS before the first barrier (half the registers of
// holding whole complex entries in N threads). STRIDE 2 takes every other
// entry of a table of 2N (the twiddles of a half-length transform).
template <typename T, int N, int NT, int STRIDE = 1> struct TwStage {
  static constexpr int PER = (2 * N + NT - 1) / NT;
  T v[PER];
  __device__ __forceinline__ void load(const c2<T> *__restrict__ tw) {
    const T *s = reinterpret_cast<const T *>(tw);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = threadIdx.x + u * NT;
      v[u] = s[i < 2 * N ? 2 * STRIDE * (i >> 1) + (i & 1) : 0];
    }
  }
  __device__ __forceinline__ void store(c2<T> *twl) const {
    T *d = reinterpret_cast<T *>(twl);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = threadIdx.x + u * NT;
      if (i < 2 * N) d[i] = v[u];
    }
  }
};

// Ops are stateless: begin(b) returns per-workgroup state and column(...)
// per-column state by value; fetch(...) returns what the final store needs
// besides the transform output (loaded ahead of the last pass).
template <typename T, int N, bool INV, class Op, int V = 0>
__global__ __launch_bounds__((Cfg<N, V>::NT)) void k_cols(ColGeo cg, const c2<T> *__restrict__ tw, const Op op) {
  using C = c2<T>;
  constexpr int CC = Cfg<N, V>::C;
  constexpr int NT = Cfg<N, V>::NT;
  __shared__ C lds[N * CC];
  // the twiddle table in LDS: loaded with the first pass (which needs none),
  // stored before its barrier, so later passes read it without a memory round trip
  __shared__ C twl[N];
  TwStage<T, N, NT> tv;
  tv.load(tw);
  // a stopped subproblem's steps must not write; the flag is applied at the
  // stores, so that the data loads need not wait for it to arrive
  const int b = blockIdx.x / cg.bpi;
  const bool sk = op.skip(b);
  const int lb = blockIdx.x - b * cg.bpi;
  const int c = threadIdx.x % CC, t = threadIdx.x / CC;
  const int ml = col_of<CC>(cg, lb, c);
  const bool ok = ml < cg.cpi;
  // columns past the end (ragged last workgroup) address column 0; with
  // Op::eager_loads they also load it and discard the values, so that every
  // load is unconditional and all of a thread's loads are in flight together
  // (one branch, and one memory latency, per element otherwise). Ops whose
  // first pass holds many registers keep the branch (higher occupancy).
  const int mls = ok ? ml : 0;
  const int mo = mls / cg.inner;
  const long base = b * cg.inst + (long)mo * cg.outer + (mls - mo * cg.inner);
  auto bs = op.begin(b);
  if constexpr (OpHasPre<Op>::value) op.template pre<NT>(bs, b, lb);
  const auto cs = op.column(b, mls);
  double acc = 0.0;
  fft_run<T, N, INV, 0, Cfg<N, V>::PLAN>(
      t, c, lds, [](int cc, int e) { return e * CC + cc; }, twl,
      [&](int e) -> C {
        if constexpr (Op::eager_loads) {
          C v = op.load(bs, cs, base + e * cg.S, e);
          if constexpr (OpPair<Op>::value == 1) v = op.template pair_in<CC>(c, v);
          return ok ? v : C{T(0), T(0)};
        } else {
          return ok ? op.load(bs, cs, base + e * cg.S, e) : C{T(0), T(0)};
        }
      },
      [&](int e) { return op.fetch(bs, cs, ok, base + e * cg.S, e); },
      [&](int e, C v, const auto &aux) {
        if constexpr (OpPair<Op>::value == 2) v = op.template pair_out<CC>(cs, c, v);
        double *sq = reinterpret_cast<double *>(lds) + e * CC + c;
        if (ok && !sk) op.store(bs, cs, base + e * cg.S, e, v, aux, acc, sq);
        else *sq = 0.0;
      },
      [&]() {
        tv.store(twl);
      });
  if (!sk) op.template end<NT, N, CC>(bs, acc, reinterpret_cast<double *>(lds), b, ml, c);  // uniform
}

struct Empty {};

// plain pass: out = scale * FFT(in); optional removal of the k = 0 mode
// (zero_dc only on the final axis-0 pass)
template <typename T> struct OpPlain {
  static constexpr bool eager_loads = true;
  const c2<T> *in;
  c2<T> *out;
  T scale;
  int zero_dc;
  long nh;
  const SubState *st;  // non-null: skip once the subproblem has stopped
  __device__ bool skip(int b) const { return st && st[b].done; }
  __device__ Empty begin(int) const { return Empty{}; }
  __device__ int column(int, int ml) const { return zero_dc && ml == 0; }
  __device__ c2<T> load(const Empty &, int, long h, int) const { return in[h]; }
  __device__ Empty fetch(const Empty &, int, bool, long, int) const { return Empty{}; }
  __device__ void store(const Empty &, int dccol, long h, int e, c2<T> v, const Empty &, double &, double *) const {
    if (dccol && e == 0) v = c2<T>{T(0), T(0)};
    out[h] = c2<T>{v.x * scale, v.y * scale};
  }
  template <int NT, int N, int CC, class B> __device__ void end(const B &, double, double *, int, int, int) const {}
};

// per-workgroup subproblem state read from SubState
template <typename T> struct StepBlk {
  const c2<T> *bprev;
  c2<T> *bnext;
  double lam_t, eta, xi, q;
  int stop;  // the multiplier step taken at the start of the pass stopped (or paused) the subproblem
};

// column information plus the pair twiddle e^{-2 pi i k'/n1} of a
// pair-split partner column (k1 = k' + n1/2)
template <typename T> struct ColTw : ColInfo {
  c2<T> tw;
  int q;  // the column's part
};

// step t of the subproblem, axis-0 inverse pass: d_t = b_{t-1} / (1 + eta (Lambda + lambda_t)).
// KS > 1 (split order with KS parts, for the split-plane pass): the stores
// leave s_q(k') = e^{+2 pi i k' q/n1} sum_p a(k' + p n1/KS) e^{+2 pi i p q/KS}
// in row k' + q n1/KS (a: the axis-0 inverse of d_t), the first step of the
// axis-1 inverse transform split by x1 mod KS (KS = 2: s_0 = a(k') + a(k' +
// n1/2), s_1 = (a(k') - a(k' + n1/2)) e^{+2 pi i k'/n1})
//
// With tn >= 1 the pass first takes the multiplier step of iteration tn - 1
// (what k_newton does between the update pass and this one): every workgroup
// sums the update pass's nmb per-workgroup partials of its instance in the
// order k_newton uses, so all of them, and k_newton, get the same bits, runs
// the stop test and the series Newton, and scales with the resulting lambda;
// the instance's first workgroup records the step in the state. An iteration
// whose series Newton needs sums over the spectrum pauses the subproblem
// (done = 3, nothing stored) for the host to take that step with k_newton.
template <typename T, bool GEN, int KS = 1, bool FUSE = false> struct OpInvScaleD {
  static constexpr bool SPLIT = KS > 1;
  static constexpr bool eager_loads = true;
  static constexpr int PAIR = SPLIT ? 2 : 0;
  static constexpr bool HAS_PRE = FUSE;  // a separate instantiation: the step's registers stay out of the plain pass
  Geo g;
  Prm p;
  const c2<T> *b0, *b1;  // b buffers: b_{t-1} lives in (t - 1) & 1
  c2<T> *out;
  SubState *st;
  const c2<T> *twn;  // SPLIT: the axis-1 twiddle table (e^{-2 pi i k/n1})
  int t;  // step index (known to the host when it enqueues the step)
  int tn;  // >= 1: the step index, and the multiplier step of step tn - 1 runs first; else lambda_t from the state
  const double *mom;    // tn >= 1: the update pass's moment partials, value j of workgroup i at
  const double *rpart;  //   mom[j mstride + inst nmb + i]; residual partials at rpart[inst nmb + i]
  long mstride;
  int nmb;
  using CI = std::conditional_t<SPLIT, ColTw<T>, ColInfo>;
  // (with SPLIT, ColTw::q holds the column's part and tw = e^{-2 pi i k' q/n1})
  __device__ bool skip(int b) const { return st[b].done != 0; }
  __device__ StepBlk<T> begin(int b) const {
    StepBlk<T> s;
    s.bprev = ((t - 1) & 1) ? b1 : b0;
    s.bnext = nullptr;
    s.lam_t = (FUSE && tn >= 1) ? 0.0 : st[b].lam[t & 1];  // FUSE, tn >= 1: set by pre()
    s.eta = st[b].eta;
    s.xi = p.xi[b];
    s.q = p.q[b];
    s.stop = 0;
    return s;
  }
  // the multiplier step (tn >= 1), before the pass's loads (which need its
  // lambda); all threads of the workgroup call it
  template <int NT> __device__ void pre(StepBlk<T> &bs, int b, int lb) const {
    if (!FUSE || tn < 1) return;  // uniform
    constexpr int NW = NT / 64;                  // whole waves (NT = 96: the second wave, half full, idles)
    static_assert(NW >= 1, "one wave at least");
    constexpr int NV = MOM_NV + 1;               // phi(0), the power sums, the residual
    constexpr int VPW = (NV + NW - 1) / NW;      // values per wave: v = wave + u NW
    constexpr int KU = (40 / VPW) < 1 ? 1 : ((40 / VPW) > 9 ? 9 : 40 / VPW);  // loads per value per lane in flight
    __shared__ double M[NV];
    __shared__ SubState S0;
    __shared__ double lam_w;
    __shared__ int it_w, nd_w;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double *src[VPW];
    double acc[VPW];
#pragma unroll
    for (int u = 0; u < VPW; ++u) {
      const int v = wv + u * NW;
      src[u] = v < MOM_NV ? mom + (long)v * mstride + (long)b * nmb : rpart + (long)b * nmb;
      acc[u] = 0.0;
    }
    // the state as this workgroup sees it, read once and shared through LDS
    // (the instance's first workgroup may update it while others read)
    if (threadIdx.x == 0) S0 = st[b];
    // per lane, workgroups i = lane + 64 k in increasing k, then across the
    // wave: the summation order of k_newton
    for (int i0 = 0; wv < NW && i0 < nmb; i0 += 64 * KU) {
      double x[VPW][KU];
#pragma unroll
      for (int u = 0; u < VPW; ++u) {
#pragma unroll
        for (int k = 0; k < KU; ++k) {
          const int i = i0 + lane + 64 * k;
          x[u][k] = (wv + u * NW < NV) ? src[u][i < nmb ? i : 0] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < VPW; ++u) {
#pragma unroll
        for (int k = 0; k < KU; ++k) {
          const int i = i0 + lane + 64 * k;
          if (i < nmb) acc[u] += x[u][k];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < VPW; ++u) {
      const int v = wv + u * NW;
      if (wv < NW && v < NV) {  // uniform in the wave
        const double a = wave_sum(acc[u]);
        if (lane == 0) M[v] = a;
      }
    }
    __syncthreads();
    const bool writer = lb == 0 && threadIdx.x == 0;
    if (S0.done) {
      bs.stop = 1;
      return;
    }
    const int t1 = tn - 1;  // the iteration whose multiplier step this is
    const double resid = sqrt(M[MOM_NV]);
    const bool bad = !(resid == resid) || resid > 1e300;
    const double lam_prev = S0.lam[t1 & 1];
    if ((t1 >= 1 && resid < S0.tol) || t1 >= S0.max_inner || bad) {
      if (writer) {
        st[b].resid = resid;
        st[b].done = (resid < S0.tol) ? 1 : 2;
        if (bad) st[b].nonfinite = 1;
        st[b].final_step = t1;
        st[b].lam_final = lam_prev;
      }
      bs.stop = 1;
      return;
    }
    const NewtonPar np{S0.eta, S0.r2, lam_prev, S0.newton_rtol, S0.newton_steptol, S0.max_newton, S0.newton_phi,
                       S0.newton_direct_only};
    if (threadIdx.x < 64) {  // the series Newton in one wave, as k_newton runs it
      auto stub = [&](double, double &phi, double &dphi) {
        phi = np.r2;
        dphi = -1.0;
      };
      int it1 = 0, nd1 = 0;
      const double l1 = multiplier_newton(M, np, stub, it1, nd1);
      if (threadIdx.x == 0) {
        lam_w = l1;
        it_w = it1;
        nd_w = nd1;
      }
    }
    __syncthreads();
    if (nd_w != 0) {  // needs sums over the spectrum: pause for k_newton
      if (writer) st[b].done = 3;
      bs.stop = 1;
      return;
    }
    if (writer) {
      st[b].resid = resid;
      st[b].lam[tn & 1] = lam_w;
      st[b].newton_total = S0.newton_total + it_w;
      st[b].step = tn;
    }
    bs.lam_t = lam_w;
  }
  __device__ CI column(int, int ml) const {
    CI ci;
    static_cast<ColInfo &>(ci) = col_info<GEN>(g, ml);
    if constexpr (SPLIT) {
      const int k1 = ml / g.nhl, part = g.n1 / KS;
      const int q = k1 / part;
      ci.q = q;
      ci.tw = twn[(k1 - q * part) * q];
    }
    return ci;
  }
  // lane c holds a(k1) of its column, the other lanes of its group those of
  // the other parts
  template <int CC> __device__ c2<T> pair_out(const CI &ci, int c, c2<T> v) const {
    if constexpr (SPLIT) {
      const c2<T> d = split_dft<KS, CC, true, T>(v, ci.q);
      if (ci.q == 0) return d;
      return c2<T>{d.x * ci.tw.x + d.y * ci.tw.y, d.y * ci.tw.x - d.x * ci.tw.y};  // d conj(tw)
    } else {
      return v;
    }
  }
  __device__ c2<T> load(const StepBlk<T> &bs, const ColInfo &ci, long h, int e) const {
    const c2<T> v = bs.bprev[h];
    const double lam = lam_of(kk_e<GEN>(g, e, ci), bs.xi, bs.q);
    const double s = (ci.dc && e == 0) ? 0.0 : rcp64(1.0 + bs.eta * (lam + bs.lam_t));
    return c2<T>{T(double(v.x) * s), T(double(v.y) * s)};
  }
  __device__ Empty fetch(const StepBlk<T> &, const ColInfo &, bool, long, int) const { return Empty{}; }
  __device__ void store(const StepBlk<T> &bs, const ColInfo &, long h, int, c2<T> v, const Empty &, double &,
                        double *) const {
    if (!bs.stop) out[h] = v;
  }
  template <int NT, int N, int CC, class B> __device__ void end(const B &, double, double *, int, int, int) const {}
};

// step t, axis-0 forward pass of T d_t, then the diagonal update:
//   Td = P F_N(Gamma' d_t),  r_t = g + (Lambda + lambda_t) d_t + Td  (residual of d_t),
//   b_t = d_t - eta (g + Td),  w |b_t|^2 (for the secular function)
template <typename T> struct UpdAux {
  c2<T> bp, gg;
  double kk;  // |Bk|^2 of the element
};
// KS > 1 (split order with KS parts, after the split-plane pass): the loads
// form Y(k'' + q n1/KS) = sum_p Z_p(k'') e^{-2 pi i q p/KS} from Z_p in row
// k'' + p n1/KS, the last step of the axis-1 forward transform split by
// x1 mod KS (KS = 2: Y(k'') = Z_0 + Z_1, Y(k'' + n1/2) = Z_0 - Z_1)
template <typename T, bool GEN, int KS = 1> struct OpFwdUpdate {
  static constexpr bool SPLIT = KS > 1;
  static constexpr bool eager_loads = true;
  static constexpr int PAIR = SPLIT ? 1 : 0;
  Geo g;
  Prm p;
  const c2<T> *tmp;  // row/axis-1 transformed product Gamma' d_t
  c2<T> *b0, *b1;
  const c2<T> *gh;
  double *partial;  // one double per workgroup: sum w |r|^2
  double *mom;      // MOM_NV doubles per workgroup: phi(0), M_2 .. M_{NMOM+1}
  const SubState *st;
  double inv_n;
  int cpi;          // columns per instance
  int t;            // step index
  __device__ bool skip(int b) const { return st[b].done != 0; }
  __device__ StepBlk<T> begin(int b) const {
    StepBlk<T> s;
    s.bprev = ((t - 1) & 1) ? b1 : b0;
    s.bnext = (t & 1) ? b1 : b0;
    s.lam_t = st[b].lam[t & 1];
    s.eta = st[b].eta;
    s.xi = p.xi[b];
    s.q = p.q[b];
    s.stop = 0;
    return s;
  }
  __device__ ColInfo column(int, int ml) const { return col_info<GEN>(g, ml); }
  __device__ c2<T> load(const StepBlk<T> &, const ColInfo &, long h, int) const { return tmp[h]; }
  // lane c holds Z_q of its column (q = c / (CC/KS)), the other lanes of its
  // group the other parts
  template <int CC> __device__ c2<T> pair_in(int c, c2<T> v) const {
    return split_dft<KS, CC, false, T>(v, c / (CC / KS));
  }
  __device__ UpdAux<T> fetch(const StepBlk<T> &bs, const ColInfo &ci, bool ok, long h, int e) const {
    UpdAux<T> a;
    if (ok) {
      a.bp = bs.bprev[h];
      a.gg = gh[h];
    } else {
      a.bp = c2<T>{T(0), T(0)};
      a.gg = a.bp;
    }
    a.kk = kk_e<GEN>(g, e, ci);
    return a;
  }
  // the LDS buffer is free once the last pass has read it: w |b_t|^2 goes to
  // sq[e * CC + c] for the pair sums formed in end()
  __device__ void store(const StepBlk<T> &bs, const ColInfo &ci, long h, int e, c2<T> v, const UpdAux<T> &a,
                        double &acc, double *sq) const {
    if (ci.dc && e == 0) {
      bs.bnext[h] = c2<T>{T(0), T(0)};
      *sq = 0.0;
      return;
    }
    const double lam = lam_of(a.kk, bs.xi, bs.q);
    const double s = rcp64(1.0 + bs.eta * (lam + bs.lam_t));
    const double dx = double(a.bp.x) * s, dy = double(a.bp.y) * s;
    const double tx = double(v.x) * inv_n, ty = double(v.y) * inv_n;
    const double gx = double(a.gg.x), gy = double(a.gg.y);
    const double rx = gx + (lam + bs.lam_t) * dx + tx, ry = gy + (lam + bs.lam_t) * dy + ty;
    acc += ci.w * (rx * rx + ry * ry);
    const double bx = dx - bs.eta * (gx + tx), by = dy - bs.eta * (gy + ty);
    const c2<T> bn = c2<T>{T(bx), T(by)};
    bs.bnext[h] = bn;
    const double bxr = double(bn.x), byr = double(bn.y);
    *sq = ci.w * (bxr * bxr + byr * byr);
  }
  // From the pair sums w (|b(k0)|^2 + |b(-k0)|^2), the block's shares of
  // phi(0) and of the power sums M_j around mu0 = eta lambda_t, and of the
  // squared residual, go to mom[j * blocks + block] and partial[block].
  template <int NT, int N, int CC>
  __device__ void end(const StepBlk<T> &bs, double acc, double *sq, int b, int ml, int) const {
    static_assert(NT % CC == 0, "each thread keeps one column");
    __syncthreads();
    constexpr int NH0 = N / 2 + 1;
    const int cc = threadIdx.x % CC;
    const bool okc = ml < cpi;
    const double kkc = col_info<GEN>(g, okc ? ml : 0).kkc;
    const double mu0 = bs.eta * bs.lam_t;
    double m[MOM_NV];
#pragma unroll
    for (int j = 0; j < MOM_NV; ++j) m[j] = 0.0;
    auto add_moments = [&](double v, double kk) {
      const double x = 1.0 + bs.eta * lam_of(kk, bs.xi, bs.q);
      const double u0 = rcp64(x);
      m[0] = fma(v, u0 * u0, m[0]);
      const double u = rcp64(x + mu0);
      double pw = v * u * u;
#pragma unroll
      for (int j = 1; j < MOM_NV; ++j) {
        m[j] += pw;
        pw *= u;
      }
    };
    if constexpr (!GEN) {
      if (okc) {
        // +-k0 share Lambda on an orthorhombic box: one term per pair of rows.
        // Constant trip count, unrolled: the rows' power chains interleave
        constexpr int ES = NT / CC, NIT = (NH0 + ES - 1) / ES;
        const int e0 = threadIdx.x / CC;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
          const int e = e0 + it * ES;
          if (e >= NH0) break;
          double v = sq[e * CC + cc];
          if (e != 0 && 2 * e != N) v += sq[(N - e) * CC + cc];
          if (e != 0 || ml != 0) add_moments(v, kk0_of(g, e) + kkc);
        }
      }
    } else {
      if (okc) {
        // cross terms: every row with its own Lambda
        const ColInfo ci = col_info<true>(g, ml);
        constexpr int ES = NT / CC, NIT = (N + ES - 1) / ES;
        const int e0 = threadIdx.x / CC;
        for (int it = 0; it < NIT; ++it) {
          const int e = e0 + it * ES;
          if (e >= N) break;
          if (e != 0 || ml != 0) add_moments(sq[e * CC + cc], kk_e<true>(g, e, ci));
        }
      }
    }
    // each row of 16 lanes sums its 22 values (4 DPP steps each) and its lane
    // 15 leaves them in LDS; threads 0..21 then add the NT / 16 row sums
    constexpr int NROW = NT / 16;
    constexpr int RS = MOM_NV + 1;
    static_assert(N * CC >= NROW * RS, "LDS scratch of the row sums");
    const int row = threadIdx.x >> 4;
    const bool last = (threadIdx.x & 15) == 15;
    __syncthreads();  // sq becomes the reduction scratch [NROW][RS]
    {
      const double v = row_sum(acc);
      if (last) sq[row * RS + MOM_NV] = v;
    }
#pragma unroll
    for (int j = 0; j < MOM_NV; ++j) {
      const double v = row_sum(m[j]);
      if (last) sq[row * RS + j] = v;
    }
    __syncthreads();
    if (threadIdx.x < RS) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NROW; ++w) s += sq[w * RS + threadIdx.x];
      if (threadIdx.x == MOM_NV)
        partial[blockIdx.x] = s;
      else
        mom[(long)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
  }
};

// axis-0 forward pass completing a spectral Hessian-vector product:
//   out = Lambda x + P F_N(Gamma' F_N^{-1} x) + shift x
struct HessBlk {
  double xi, q;
};
template <typename T> struct HessAux {
  c2<T> xv;
  double kk;
};
template <typename T, bool GEN> struct OpFwdHess {
  static constexpr bool eager_loads = false;
  Geo g;
  Prm p;
  const c2<T> *tmp;
  const c2<T> *x;
  c2<T> *out;
  double inv_n, shift;
  __device__ bool skip(int) const { return false; }
  __device__ HessBlk begin(int b) const { return HessBlk{p.xi[b], p.q[b]}; }
  __device__ ColInfo column(int, int ml) const { return col_info<GEN>(g, ml); }
  __device__ c2<T> load(const HessBlk &, const ColInfo &, long h, int) const { return tmp[h]; }
  __device__ HessAux<T> fetch(const HessBlk &, const ColInfo &ci, bool ok, long h, int e) const {
    HessAux<T> a;
    const c2<T> xv = x[h];  // h is a valid address for every thread
    a.xv = ok ? xv : c2<T>{T(0), T(0)};
    a.kk = kk_e<GEN>(g, e, ci);
    return a;
  }
  __device__ void store(const HessBlk &hb, const ColInfo &ci, long h, int e, c2<T> v, const HessAux<T> &a,
                        double &, double *) const {
    if (ci.dc && e == 0) {
      out[h] = c2<T>{T(0), T(0)};
      return;
    }
    const double lam = lam_of(a.kk, hb.xi, hb.q) + shift;
    out[h] = c2<T>{T(lam * double(a.xv.x) + double(v.x) * inv_n), T(lam * double(a.xv.y) + double(v.y) * inv_n)};
  }
  template <int NT, int N, int CC, class B> __device__ void end(const B &, double, double *, int, int, int) const {}
};

// Hessian-vector product, axis-0: forward transform, multiply by Lambda / N
// (k = 0 removed unless keep_dc), inverse transform, all in one workgroup pass.
// KS > 1 (split order with KS parts, between the split-plane passes of the
// product): the loads form Y from the parts Z_p of a column group and the
// stores leave the parts s_q (the first and last steps of the axis-1
// transforms split by x1 mod KS, as in the inner iteration's axis-0 passes);
// tw1 is the axis-1 twiddle table
template <typename T, int N, bool GEN, int KS = 1>
__global__ __launch_bounds__(Cfg<N>::NT) void k_cols_fwd_mul_inv(ColGeo cg, Geo g, Prm p, const c2<T> *__restrict__ tw,
                                                                  c2<T> *data, double inv_n, int keep_dc,
                                                                  const c2<T> *__restrict__ tw1) {
  using C = c2<T>;
  constexpr int CC = Cfg<N>::C;
  __shared__ C lds[N * CC];
  __shared__ C twl[N];  // the twiddle table, stored during the first pass
  TwStage<T, N, Cfg<N>::NT> tv;
  tv.load(tw);
  const int b = blockIdx.x / cg.bpi;
  const int lb = blockIdx.x - b * cg.bpi;
  const int c = threadIdx.x % CC, t = threadIdx.x / CC;
  const int ml = col_of<CC>(cg, lb, c);
  const bool ok = ml < cg.cpi;
  const long base = b * cg.inst + (ok ? ml : 0);  // axis 0: every column starts in the first slab
  const ColInfo ci = col_info<GEN>(g, ok ? ml : 0);
  const double xi = p.xi[b], q = p.q[b];
  // KS > 1: the column's part and e^{-2 pi i k' part/n1} (k1 = k' + part n1/KS)
  int part = 0;
  C ptw{T(1), T(0)};
  if constexpr (KS > 1) {
    const int k1 = (ok ? ml : 0) / g.nhl, len = g.n1 / KS;
    part = c / (CC / KS);
    ptw = tw1[(k1 - part * len) * part];
  }
  auto lidx = [](int cc, int e) { return e * CC + cc; };
  fft_run<T, N, false>(
      t, c, lds, lidx, twl,
      [&](int e) -> C {
        C v = data[base + e * cg.S];
        if constexpr (KS > 1) v = split_dft<KS, CC, false, T>(v, part);
        return ok ? v : C{T(0), T(0)};
      },
      [&](int e) { return kk_e<GEN>(g, e, ci); },
      [&](int e, C v, double kk) {
        double m = lam_of(kk, xi, q) * inv_n;
        if (!ok || (ci.dc && e == 0 && !keep_dc)) m = 0.0;
        lds[lidx(c, e)] = C{T(double(v.x) * m), T(double(v.y) * m)};
      },
      [&]() {
        tv.store(twl);
      });
  __syncthreads();
  fft_run<T, N, true>(
      t, c, lds, lidx, twl, [&](int e) -> C { return lds[lidx(c, e)]; }, NoFetch{},
      [&](int e, C v, NoAux) {
        if constexpr (KS > 1) {
          const C d = split_dft<KS, CC, true, T>(v, part);
          v = part == 0 ? d : C{d.x * ptw.x + d.y * ptw.y, d.y * ptw.x - d.x * ptw.y};  // d conj(ptw)
        }
        if (ok) data[base + e * cg.S] = v;
      });
}

// ---------------------------------------------------------------------------
// Row passes (last axis). Two real rows a, b are packed as z = a + i b; the
// half spectra follow from Z_k and conj(Z_{N-k}).
// ---------------------------------------------------------------------------
struct RowGeo {
  long rpi;  // real rows per instance
  int bpi;   // workgroups per instance
};

template <int N> struct RowLds {
  static constexpr int LD = N + 1;  // padded row pitch in LDS
};

// Forward real-to-half-spectrum of pairs of rows with a fused prologue.
//   MODE 0 (plain): z = (in[a], in[b])
//   MODE 1 (hessian input): same, and partial sums of Gamma'(psi) v for the mean
template <typename T, int N, int MODE>
__global__ __launch_bounds__(Cfg<N>::NT) void k_rows_r2c(RowGeo rg, Geo g, Prm p, const c2<T> *__restrict__ tw,
                                                          const double *__restrict__ in, const double *__restrict__ psi,
                                                          c2<T> *__restrict__ out, double *partial) {
  using C = c2<T>;
  constexpr int CC = Cfg<N>::C, NT = Cfg<N>::NT, LD = RowLds<N>::LD, NHL = N / 2 + 1;
  __shared__ C lds[CC * LD];
  const int b = blockIdx.x / rg.bpi;
  const long pair0 = (long)(blockIdx.x % rg.bpi) * CC;
  const long ppi = rg.rpi / 2;
  const long rowbase = (long)b * rg.rpi;
  double acc = 0.0;
  const double tau = p.tau[b], gam = p.gamma[b];
  for (int i = threadIdx.x; i < CC * N; i += NT) {
    const int c = i / N, e = i % N;
    const long pr = pair0 + c;
    C z{T(0), T(0)};
    if (pr < ppi) {
      const long ia = (rowbase + 2 * pr) * N + e, ib = ia + N;
      const double va = in[ia], vb = in[ib];
      z = C{T(va), T(vb)};
      if constexpr (MODE == 1) {
        const double pa = psi[ia], pb = psi[ib];
        acc += (tau - gam * pa + 0.5 * pa * pa) * va + (tau - gam * pb + 0.5 * pb * pb) * vb;
      }
    }
    lds[c * LD + e] = z;
  }
  __syncthreads();
  const int c = threadIdx.x % CC, t = threadIdx.x / CC;
  auto lidx = [](int cc, int e) { return cc * LD + e; };
  fft_lds<T, N, false>(t, c, lds, lidx, tw);
  __syncthreads();
  for (int i = threadIdx.x; i < CC * NHL; i += NT) {
    const int cc = i / NHL, k = i % NHL;
    const long pr = pair0 + cc;
    if (pr < ppi) {
      const C zk = lds[cc * LD + k], zm = lds[cc * LD + ((N - k) % N)];
      const C A{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
      const C B{T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)};
      const long oa = (rowbase + 2 * pr) * NHL + k;
      out[oa] = A;
      out[oa + NHL] = B;
    }
  }
  if constexpr (MODE == 1) {
    const double s = block_sum<NT>(acc, reinterpret_cast<double *>(lds));
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// Energy row pass: one row per transform, z = psi + i F'(psi); writes the half
// spectra of psi (out0) and of F'(psi) (out1), Gamma'(psi) in T precision, and
// per-workgroup partials [sum F(psi), max |Gamma'|].
template <int N>
__global__ __launch_bounds__(Cfg<N>::NT) void k_rows_energy(RowGeo rg, Geo g, Prm p, const double2 *__restrict__ tw,
                                                            const double *__restrict__ psi, double2 *__restrict__ out0,
                                                            double2 *__restrict__ out1, double *__restrict__ gp64,
                                                            float *__restrict__ gp32, double *partial) {
  using C = double2;
  constexpr int CC = Cfg<N>::C, NT = Cfg<N>::NT, LD = RowLds<N>::LD, NHL = N / 2 + 1;
  __shared__ C lds[CC * LD];
  const int b = blockIdx.x / rg.bpi;
  const long row0 = (long)(blockIdx.x % rg.bpi) * CC;
  const long rowbase = (long)b * rg.rpi;
  const double tau = p.tau[b], gam = p.gamma[b];
  double accF = 0.0, mx = 0.0;
  for (int i = threadIdx.x; i < CC * N; i += NT) {
    const int c = i / N, e = i % N;
    const long rr = row0 + c;
    C z{0.0, 0.0};
    if (rr < rg.rpi) {
      const long ix = (rowbase + rr) * N + e;
      const double s = psi[ix];
      const double s2 = s * s;
      const double dF = tau * s - 0.5 * gam * s2 + s2 * s / 6.0;
      const double Fv = 0.5 * tau * s2 - gam * s2 * s / 6.0 + s2 * s2 / 24.0;
      const double gpv = tau - gam * s + 0.5 * s2;
      accF += Fv;
      mx = fmax(mx, fabs(gpv));
      if (gp64) gp64[ix] = gpv;
      if (gp32) gp32[ix] = float(gpv);
      z = C{s, dF};
    }
    lds[c * LD + e] = z;
  }
  __syncthreads();
  const int c = threadIdx.x % CC, t = threadIdx.x / CC;
  auto lidx = [](int cc, int e) { return cc * LD + e; };
  fft_lds<double, N, false>(t, c, lds, lidx, tw);
  __syncthreads();
  for (int i = threadIdx.x; i < CC * NHL; i += NT) {
    const int cc = i / NHL, k = i % NHL;
    const long rr = row0 + cc;
    if (rr < rg.rpi) {
      const C zk = lds[cc * LD + k], zm = lds[cc * LD + ((N - k) % N)];
      const long o = (rowbase + rr) * NHL + k;
      out0[o] = C{0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y)};
      out1[o] = C{0.5 * (zk.y + zm.y), 0.5 * (zm.x - zk.x)};
    }
  }
  const double sF = block_sum<NT>(accF, reinterpret_cast<double *>(lds));
  const double sM = block_max<NT>(mx, reinterpret_cast<double *>(lds) + 32);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sF;
    partial[2 * blockIdx.x + 1] = sM;
  }
}

// Load half rows a, b of a pair into LDS as Z = A + i B over the full length
// (Hermitian extension), dropping the imaginary parts that a real row's
// k = 0 and k = N/2 coefficients cannot have.
template <typename T, int N, class Src>
__device__ __forceinline__ void pack_pairs(c2<T> *lds, long pair0, long ppi, const Src &src) {
  using C = c2<T>;
  constexpr int CC = Cfg<N>::C, NT = Cfg<N>::NT, LD = RowLds<N>::LD, NHL = N / 2 + 1;
  for (int i = threadIdx.x; i < CC * NHL; i += NT) {
    const int c = i / NHL, k = i % NHL;
    const long pr = pair0 + c;
    C A{T(0), T(0)}, B{T(0), T(0)};
    if (pr < ppi) src(pr, k, A, B);
    if (k == 0 || 2 * k == N) {
      A.y = T(0);
      B.y = T(0);
    }
    lds[c * LD + k] = C{A.x - B.y, A.y + B.x};
    if (k > 0 && 2 * k < N) lds[c * LD + N - k] = C{A.x + B.y, B.x - A.y};
  }
}

// Inverse half-spectrum-to-real of pairs of rows with a fused epilogue.
//   MODE 0 (plain):    out = x
//   MODE 1 (hessian):  out = x + Gamma'(psi) v - mean, mean = (sum of the
//                      matching r2c pass's per-workgroup partials `mpart`) / N
//                      (mpart == nullptr: no mean removal)
//   MODE 2 (taylor):   out = s = x, partial sums of
//                      Gamma' s^2 / 2 + (psi - gamma) s^3 / 6 + s^4 / 24
template <typename T, int N, int MODE>
__global__ __launch_bounds__(Cfg<N>::NT) void k_rows_c2r(RowGeo rg, Geo g, Prm p, const c2<T> *__restrict__ tw,
                                                          const c2<T> *__restrict__ in, double *__restrict__ out,
                                                          const double *__restrict__ psi, const double *__restrict__ v,
                                                          const double *__restrict__ mpart, int mbpi, double *partial,
                                                          double bscale) {
  using C = c2<T>;
  constexpr int CC = Cfg<N>::C, NT = Cfg<N>::NT, LD = RowLds<N>::LD, NHL = N / 2 + 1;
  __shared__ C lds[CC * LD];
  const int b = blockIdx.x / rg.bpi;
  const long pair0 = (long)(blockIdx.x % rg.bpi) * CC;
  const long ppi = rg.rpi / 2;
  const long rowbase = (long)b * rg.rpi;
  double mean = 0.0;
  if constexpr (MODE == 1) {
    if (mpart) {
      double a = 0.0;
      for (int i = threadIdx.x; i < mbpi; i += NT) a += mpart[(long)b * mbpi + i];
      mean = block_sum_all<NT>(a, reinterpret_cast<double *>(lds)) / (double)g.N;
    }
  }
  pack_pairs<T, N>(lds, pair0, ppi, [&](long pr, int k, C &A, C &B) {
    const long ia = (rowbase + 2 * pr) * NHL + k;
    A = in[ia];
    B = in[ia + NHL];
  });
  __syncthreads();
  const int c = threadIdx.x % CC, t = threadIdx.x / CC;
  auto lidx = [](int cc, int e) { return cc * LD + e; };
  fft_lds<T, N, true>(t, c, lds, lidx, tw);
  __syncthreads();
  const double tau = p.tau[b], gam = p.gamma[b];
  double acc = 0.0;
  for (int i = threadIdx.x; i < CC * N; i += NT) {
    const int cc = i / N, e = i % N;
    const long pr = pair0 + cc;
    if (pr < ppi) {
      const C z = lds[cc * LD + e];
      const long ia = (rowbase + 2 * pr) * N + e, ib = ia + N;
      double xa = double(z.x), xb = double(z.y);
      if constexpr (MODE == 1) {
        const double pa = psi[ia], pb = psi[ib];
        xa += bscale * ((tau - gam * pa + 0.5 * pa * pa) * v[ia] - mean);
        xb += bscale * ((tau - gam * pb + 0.5 * pb * pb) * v[ib] - mean);
      }
      if constexpr (MODE == 2) {
        const double pa = psi[ia], pb = psi[ib];
        const double a2 = xa * xa, b2 = xb * xb;
        acc += 0.5 * (tau - gam * pa + 0.5 * pa * pa) * a2 + (pa - gam) * a2 * xa / 6.0 + a2 * a2 / 24.0;
        acc += 0.5 * (tau - gam * pb + 0.5 * pb * pb) * b2 + (pb - gam) * b2 * xb / 6.0 + b2 * b2 / 24.0;
      }
      out[ia] = xa;
      out[ib] = xb;
    }
  }
  if constexpr (MODE == 2) {
    const double s = block_sum<NT>(acc, reinterpret_cast<double *>(lds));
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// Row pass of one subproblem step: inverse row transform of d_t's partial
// spectrum, multiply by Gamma'(psi) pointwise, forward row transform back.
template <typename T, int N>
__global__ __launch_bounds__(Cfg<N>::NT) void k_rows_inner(RowGeo rg, const c2<T> *__restrict__ tw, c2<T> *data,
                                                            const T *__restrict__ gp, const SubState *st) {
  using C = c2<T>;
  constexpr int CC = Cfg<N>::C, NT = Cfg<N>::NT, LD = RowLds<N>::LD, NHL = N / 2 + 1;
  __shared__ C lds[CC * LD];
  const int b = blockIdx.x / rg.bpi;
  const bool sk = st && st[b].done;  // applied at the stores (the loads need not wait for it)
  const long pair0 = (long)(blockIdx.x % rg.bpi) * CC;
  const long ppi = rg.rpi / 2;
  const long rowbase = (long)b * rg.rpi;
  pack_pairs<T, N>(lds, pair0, ppi, [&](long pr, int k, C &A, C &B) {
    const long ia = (rowbase + 2 * pr) * NHL + k;
    A = data[ia];
    B = data[ia + NHL];
  });
  __syncthreads();
  const int c = threadIdx.x % CC, t = threadIdx.x / CC;
  auto lidx = [](int cc, int e) { return cc * LD + e; };
  fft_lds<T, N, true>(t, c, lds, lidx, tw);
  __syncthreads();
  for (int i = threadIdx.x; i < CC * N; i += NT) {
    const int cc = i / N, e = i % N;
    const long pr = pair0 + cc;
    if (pr < ppi) {
      const long ia = (rowbase + 2 * pr) * N + e;
      const C z = lds[cc * LD + e];
      lds[cc * LD + e] = C{z.x * gp[ia], z.y * gp[ia + N]};
    }
  }
  __syncthreads();
  fft_lds<T, N, false>(t, c, lds, lidx, tw);
  __syncthreads();
  for (int i = threadIdx.x; i < CC * NHL; i += NT) {
    const int cc = i / NHL, k = i % NHL;
    const long pr = pair0 + cc;
    if (pr < ppi && !sk) {
      const C zk = lds[cc * LD + k], zm = lds[cc * LD + ((N - k) % N)];
      const long oa = (rowbase + 2 * pr) * NHL + k;
      data[oa] = C{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
      data[oa + NHL] = C{T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)};
    }
  }
}

// ---------------------------------------------------------------------------
// Plane pass (3D grids with n1 = n_last = N whose half-spectrum plane fits in
// LDS): one workgroup per (instance, i0) plane does the axis-1 inverse, the row
// half-spectrum-to-real, the product with Gamma'(psi), the row real-to-half-
// spectrum and the axis-1 forward transform, in place in LDS. This replaces
// three passes through HBM in each subproblem step.
// ---------------------------------------------------------------------------
template <typename T, int N> struct PlaneCfg {
  static constexpr int NH = N / 2 + 1;
  // the plane must fit in LDS, and the butterflies plus the prefetched Gamma'
  // in registers (beyond N = 128 they spill)
  static constexpr bool fits = (long)N * NH * sizeof(c2<T>) <= 160 * 1024 && N <= 128;
  // 1024 threads from N = 96 (FP64 included: no spills with the odd packed-row
  // stride; 4 waves per SIMD hide the LDS and memory latency of the passes)
  static constexpr int NT = N >= 96 ? 1024 : (N >= 48 ? 512 : 256);
};

// One Stockham pass (radix plan 1) over NXF transforms of length N. Butterfly
// inputs come from load(f, e), outputs go to store(f, e, v, k, r) (k, r: the
// thread's butterfly slot and output, for per-output data held in registers).
// FAST puts consecutive threads on consecutive transforms, else on consecutive
// butterflies of one transform. MID: barrier between all loads and all stores
// (the pass updates one LDS buffer in place).
template <typename T, int N, bool INV, int NT, int NXF, bool FAST, int P> struct PassShape {
  static constexpr int R = lbfft::radix_p<1>(N, P);
  static constexpr int NS = lbfft::span_p<1>(N, P);
  static constexpr int NB = N / R;
  static constexpr int TOT = NXF * NB;
  static constexpr int K = (TOT + NT - 1) / NT;
  __device__ static int f_of(int bi) { return FAST ? bi % NXF : bi / NB; }
  __device__ static int j_of(int bi) { return FAST ? bi / NXF : bi % NB; }
};
template <typename T, int N, bool INV, int NT, int NXF, bool FAST, int P, bool MID, class Load, class Store>
__device__ __forceinline__ void sk_pass(const c2<T> *__restrict__ tw, const Load &load, const Store &store) {
  using C = c2<T>;
  using S = PassShape<T, N, INV, NT, NXF, FAST, P>;
  constexpr int R = S::R, NS = S::NS, NB = S::NB, K = S::K;
  C v[K][R];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int bi = threadIdx.x + k * NT;
    if (bi < S::TOT) {
      const int f = S::f_of(bi), j = S::j_of(bi);
#pragma unroll
      for (int r = 0; r < R; ++r) v[k][r] = load(f, j + r * NB);
    }
  }
  if constexpr (MID) __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int bi = threadIdx.x + k * NT;
    if (bi < S::TOT) {
      const int f = S::f_of(bi), j = S::j_of(bi);
      const int kk = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C w = tw[r * kk * (N / (NS * R))];
          if constexpr (INV) w.y = -w.y;
          v[k][r] = cmul(v[k][r], w);
        }
      }
      dft<T, R, INV>(v[k]);
      const int base = (j / NS) * NS * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) store(f, base + r * NS, v[k][r], k, r);
    }
  }
}
// LDS-to-LDS passes P .. PE - 1 of NXF transforms at buf[f * fs + e * es]
template <typename T, int N, bool INV, int NT, int NXF, bool FAST, int P, int PE>
__device__ __forceinline__ void sk_lds_passes(c2<T> *buf, int fs, int es, const c2<T> *__restrict__ tw) {
  if constexpr (P < PE) {
    using C = c2<T>;
    sk_pass<T, N, INV, NT, NXF, FAST, P, true>(
        tw, [&](int f, int e) -> C { return buf[f * fs + e * es]; },
        [&](int f, int e, C v, int, int) { buf[f * fs + e * es] = v; });
    __syncthreads();
    sk_lds_passes<T, N, INV, NT, NXF, FAST, P + 1, PE>(buf, fs, es, tw);
  }
}

// Stages of the plane kernels. A plane of fixed i0 is held in LDS as the
// half spectrum along the last axis: element (row e, column k) at L[e NH + k];
// row passes pack half rows 2p, 2p+1 as one complex row Z_p of length N at
// L[p PR + x]. Every pass reads all its elements into registers before it
// writes, so Z may use its own stride: PR = N + 1 is odd, so the rows that
// consecutive lanes hold start in distinct LDS banks (a stride of 2 NH, even,
// put every other lane on the same banks), and N/2 rows of N + 1 still fit in
// the N NH elements of the plane.
template <int N> constexpr int plane_pr() { return N + 1; }

// axis 1, inverse, first pass reading element (e, f) from load(f, e)
// (pre() runs after the first pass, before its barrier: the first pass reads
// no twiddles, so an LDS twiddle table stored there serves the later passes)
// (LEN: the axis-1 transform length, N or N/2 for the half-plane pass; tw
// is that length's table)
template <typename T, int N, int NT, int LEN, class Load, class Pre = lbfft::NoPre>
__device__ __forceinline__ void plane_cols_inv_load(c2<T> *L, const c2<T> *__restrict__ tw, const Load &load,
                                                    const Pre &pre = Pre{}) {
  using C = c2<T>;
  constexpr int NH = N / 2 + 1, NP = lbfft::npass_p<1>(LEN);
  sk_pass<T, LEN, true, NT, NH, true, 0, false>(tw, load, [&](int f, int e, C v, int, int) { L[e * NH + f] = v; });
  pre();
  __syncthreads();
  sk_lds_passes<T, LEN, true, NT, NH, true, 1, NP>(L, 1, NH, tw);
}
// ... from src (plane layout)
template <typename T, int N, int NT, class Pre = lbfft::NoPre>
__device__ __forceinline__ void plane_cols_inv_from(c2<T> *L, const c2<T> *src, const c2<T> *__restrict__ tw,
                                                    const Pre &pre = Pre{}) {
  plane_cols_inv_load<T, N, NT, N>(
      L, tw, [&](int f, int e) -> c2<T> { return src[e * (N / 2 + 1) + f]; }, pre);
}

// rows, inverse: the first pass packs half rows 2p, 2p+1 into Z_p = A + i B;
// the last pass (consecutive threads on consecutive outputs x = j + r NS of
// one row) hands its outputs to last(p, x, z, k, r)
// (NR packed rows: N/2, or N/4 in the half-plane pass)
template <typename T, int N, int NT, int NR, class Last>
__device__ __forceinline__ void plane_rows_inv(c2<T> *L, const c2<T> *__restrict__ tw, const Last &last) {
  using C = c2<T>;
  constexpr int NH = N / 2 + 1, NP = lbfft::npass_p<1>(N), PR = plane_pr<N>();
  auto packed = [&](int p, int e) -> C {
    const bool lo = 2 * e <= N;
    const int k = lo ? e : N - e;
    C A = L[2 * p * NH + k], B = L[(2 * p + 1) * NH + k];
    if (k == 0 || 2 * k == N) {
      A.y = T(0);
      B.y = T(0);
    }
    return lo ? C{A.x - B.y, A.y + B.x} : C{A.x + B.y, B.x - A.y};
  };
  if constexpr (NP == 1) {
    sk_pass<T, N, true, NT, NR, false, 0, true>(tw, packed, last);
  } else {
    sk_pass<T, N, true, NT, NR, true, 0, true>(tw, packed,
                                               [&](int f, int e, C v, int, int) { L[f * PR + e] = v; });
    __syncthreads();
    sk_lds_passes<T, N, true, NT, NR, true, 1, NP - 1>(L, PR, 1, tw);
    sk_pass<T, N, true, NT, NR, false, NP - 1, true>(
        tw, [&](int f, int e) -> C { return L[f * PR + e]; }, last);
  }
}

// axis 1, forward: the first pass unpacks Z_p into half rows 2p, 2p+1; the
// last pass hands element (e, f) to store_out(f, e, v, k, r)
// (LEN: the axis-1 transform length, as for plane_cols_inv_load)
template <typename T, int N, int NT, class Store, bool LAST_MID = false, int LEN = N>
__device__ __forceinline__ void plane_cols_fwd_store(c2<T> *L, const c2<T> *__restrict__ tw, const Store &store_mem) {
  using C = c2<T>;
  constexpr int NH = N / 2 + 1, NP = lbfft::npass_p<1>(LEN), PR = plane_pr<N>();
  auto unpacked = [&](int k, int e) -> C {
    const int p = e >> 1;
    const C zk = L[p * PR + k], zm = L[p * PR + ((N - k) % N)];
    return (e & 1) ? C{T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)}
                   : C{T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
  };
  auto store_lds = [&](int f, int e, C v, int, int) { L[e * NH + f] = v; };
  if constexpr (NP == 1) {
    sk_pass<T, LEN, false, NT, NH, true, 0, true>(tw, unpacked, store_mem);
  } else {
    sk_pass<T, LEN, false, NT, NH, true, 0, true>(tw, unpacked, store_lds);
    __syncthreads();
    sk_lds_passes<T, LEN, false, NT, NH, true, 1, NP - 1>(L, 1, NH, tw);
    sk_pass<T, LEN, false, NT, NH, true, NP - 1, LAST_MID>(
        tw, [&](int f, int e) -> C { return L[e * NH + f]; }, store_mem);
  }
}
// ... to dst (plane layout)
template <typename T, int N, int NT>
__device__ __forceinline__ void plane_cols_fwd_to(c2<T> *L, c2<T> *dst, const c2<T> *__restrict__ tw) {
  plane_cols_fwd_store<T, N, NT>(L, tw, [&](int f, int e, c2<T> v, int, int) { dst[e * (N / 2 + 1) + f] = v; });
}

// Axes 1 and 2 of the inner iteration for one plane of fixed k0: inverse
// along axis 1, inverse real row transforms, multiply by Gamma', forward real
// row transforms, forward along axis 1. Gamma' is applied by the last inverse
// row pass, its values loaded (coalesced) before the row passes start.
template <typename T, int N, int NT = PlaneCfg<T, N>::NT>
__global__ __launch_bounds__(NT) void k_plane_inner(int n0, long nh, long Np, const c2<T> *__restrict__ tw,
                                                    c2<T> *data, const T *__restrict__ gp, const SubState *st) {
  using C = c2<T>;
  constexpr int NH = N / 2 + 1, NP = lbfft::npass_p<1>(N), NR = N / 2, PR = plane_pr<N>();
  __shared__ C L[N * NH];
  __shared__ C twl[N];  // the twiddle table, stored during the first pass (which reads none)
  TwStage<T, N, NT> tv;
  tv.load(tw);
  const int b = blockIdx.x / n0, i0 = blockIdx.x - b * n0;
  const bool sk = st && st[b].done;  // applied at the stores (the loads need not wait for it)
  C *plane = data + b * nh + (long)i0 * (N * NH);
  const T *g = gp + b * Np + (long)i0 * (N * N);
  plane_cols_inv_from<T, N, NT>(L, plane, twl, [&]() {
    tv.store(twl);
  });
  __syncthreads();
  using LastS = PassShape<T, N, true, NT, NR, false, NP - 1>;
  T g0[LastS::K][LastS::R], g1[LastS::K][LastS::R];
#pragma unroll
  for (int k = 0; k < LastS::K; ++k) {
    const int bi = threadIdx.x + k * NT;
    if (bi < LastS::TOT) {
      const int f = LastS::f_of(bi), j = LastS::j_of(bi);
#pragma unroll
      for (int r = 0; r < LastS::R; ++r) {
        const int e = j + r * LastS::NS;
        g0[k][r] = g[(2 * f) * N + e];
        g1[k][r] = g[(2 * f + 1) * N + e];
      }
    }
  }
  plane_rows_inv<T, N, NT, N / 2>(L, twl, [&](int f, int e, C v, int k, int r) {
    L[f * PR + e] = C{v.x * g0[k][r], v.y * g1[k][r]};
  });
  __syncthreads();
  sk_lds_passes<T, N, false, NT, NR, true, 0, NP>(L, PR, 1, twl);  // rows, forward
  plane_cols_fwd_store<T, N, NT>(L, twl, [&](int f, int e, C v, int, int) {
    if (!sk) plane[e * NH + f] = v;
  });
}

// Split-plane pass of the inner iteration (split order with K parts, n1 =
// n_last = N): the axis-1 transform of length N split by x1 mod K, x1 = Km + p.
// The axis-0 inverse pass leaves s_p in rows p N/K .. (p + 1) N/K - 1 of each
// plane (OpInvScaleD with KS = K); values at x1 = Km + p are the length-N/K
// inverse transform of s_p. Workgroup (i0, p) transforms its part, does the
// row transforms with the product with Gamma' on rows x1 = Km + p, transforms
// back over m (length N/K) into Y_p and stores Z_p(k'') = e^{-2 pi i p k''/N}
// Y_p(k'') in the same rows (OpFwdUpdate with KS = K combines the parts). Each
// workgroup touches only its own rows and holds 1/K of a plane in LDS: K
// workgroups per plane (K = 2 at 128^3, K = 4 where a half plane does not fit,
// as at 256^3).
template <typename T, int N, int K> struct SplitCfg {
  static constexpr int L = N / K, NH = N / 2 + 1;
  static constexpr long LDS = (long)L * NH * sizeof(c2<T>) + (long)(N + L) * sizeof(c2<T>) + 256;
  static constexpr bool fits = (K == 2 || K == 4) && N % (2 * K) == 0 && L >= 8 && N <= 256 &&
                               LDS <= 160 * 1024 && lbfft::npass_p<1>(L) > 0 && lbfft::npass_p<1>(N) > 0;
  static constexpr int NT = N >= 96 ? 512 : 256;
};
template <typename T, int N, int K, int NT = SplitCfg<T, N, K>::NT>
__global__ __launch_bounds__(NT) void k_plane_inner_split(int n0, long nh, long Np, const c2<T> *__restrict__ tw,
                                                          c2<T> *data, const T *__restrict__ gp, const SubState *st) {
  using C = c2<T>;
  constexpr int L = N / K, NH = N / 2 + 1, NP = lbfft::npass_p<1>(N), NRW = L / 2, PR = plane_pr<N>();
  static_assert(NRW * PR <= L * NH, "packed rows fit in the part");
  __shared__ C Ls[L * NH];
  __shared__ C twl[N];  // length-N twiddles (rows, and Z_p's factor), stored during the first pass
  __shared__ C twh[L];  // length-N/K twiddles (axis 1)
  TwStage<T, N, NT> tv;
  TwStage<T, L, NT, K> th;
  tv.load(tw);
  th.load(tw);
  const int pl = blockIdx.x / K, par = blockIdx.x - pl * K;
  const int b = pl / n0, i0 = pl - b * n0;
  const bool sk = st && st[b].done;  // applied at the stores
  C *part = data + b * nh + (long)i0 * (N * NH) + (long)par * (L * NH);
  const T *g = gp + b * Np + (long)i0 * (N * N);
  plane_cols_inv_load<T, N, NT, L>(
      Ls, twh, [&](int f, int e) -> C { return part[e * NH + f]; },
      [&]() {
        tv.store(twl);
        th.store(twh);
      });
  __syncthreads();
  // Gamma' for the last inverse row pass: packed row f holds the local rows
  // 2f and 2f + 1, i.e. x1 = 2Kf + p and 2Kf + K + p
  using LastS = PassShape<T, N, true, NT, NRW, false, NP - 1>;
  T g0[LastS::K][LastS::R], g1[LastS::K][LastS::R];
#pragma unroll
  for (int k = 0; k < LastS::K; ++k) {
    const int bi = threadIdx.x + k * NT;
    if (bi < LastS::TOT) {
      const int f = LastS::f_of(bi), j = LastS::j_of(bi);
#pragma unroll
      for (int r = 0; r < LastS::R; ++r) {
        const int e = j + r * LastS::NS;
        g0[k][r] = g[(2 * K * f + par) * N + e];
        g1[k][r] = g[(2 * K * f + K + par) * N + e];
      }
    }
  }
  plane_rows_inv<T, N, NT, NRW>(Ls, twl, [&](int f, int e, C v, int k, int r) {
    Ls[f * PR + e] = C{v.x * g0[k][r], v.y * g1[k][r]};
  });
  __syncthreads();
  sk_lds_passes<T, N, false, NT, NRW, true, 0, NP>(Ls, PR, 1, twl);  // rows, forward
  auto store = [&](int f, int e, C v, int, int) {
    if (par) v = cmul(v, twl[par * e]);
    if (!sk) part[e * NH + f] = v;
  };
  plane_cols_fwd_store<T, N, NT, decltype(store), false, L>(Ls, twh, store);
}

// Hessian-vector product, axes 2 and 1 forward from the physical field v:
// real rows 2p, 2p+1 packed as Z_p, forward row transforms, forward along
// axis 1 into the half-spectrum plane of out. With partial non-null, the
// plane's share of sum Gamma'(psi) v goes to partial[block] (for the mean).
template <typename T, int N, int NT = PlaneCfg<T, N>::NT>
__global__ __launch_bounds__(NT) void k_plane_fwd_phys(int n0, long nh, long Np, Prm p, const c2<T> *__restrict__ tw,
                                                       const double *__restrict__ v, const double *__restrict__ psi,
                                                       c2<T> *out, double *partial) {
  using C = c2<T>;
  constexpr int NH = N / 2 + 1, NP = lbfft::npass_p<1>(N), NR = N / 2, PR = plane_pr<N>();
  __shared__ C L[N * NH];
  __shared__ C twl[N];  // the twiddle table, stored before the first pass
  TwStage<T, N, NT> tv;
  tv.load(tw);
  const int b = blockIdx.x / n0, i0 = blockIdx.x - b * n0;
  const long off = b * Np + (long)i0 * (N * N);
  const double tau = p.tau[b], gam = p.gamma[b];
  __shared__ double red[NT / 64];  // wave sums of the mean partial
  double acc = 0.0;
  for (int i = threadIdx.x; i < NR * N; i += NT) {
    const int q = i / N, x = i - q * N;
    const long ia = off + (long)(2 * q) * N + x, ib = ia + N;
    const double va = v[ia], vb = v[ib];
    if (partial) {
      const double pa = psi[ia], pb = psi[ib];
      acc += (tau - gam * pa + 0.5 * pa * pa) * va + (tau - gam * pb + 0.5 * pb * pb) * vb;
    }
    L[q * PR + x] = C{T(va), T(vb)};
  }
  tv.store(twl);
  if (partial) {  // the wave sums now; the passes' barriers order them before thread 0 adds them
    const double ws = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ws;
  }
  __syncthreads();
  sk_lds_passes<T, N, false, NT, NR, true, 0, NP>(L, PR, 1, twl);
  plane_cols_fwd_to<T, N, NT>(L, out + b * nh + (long)i0 * (N * NH), twl);
  if (partial && threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    partial[blockIdx.x] = s;
  }
}

// Hessian-vector product, axes 1 and 2 inverse into the physical result:
//   hv = F^-1(...) + bscale (Gamma'(psi) v - mean),  mean = sum of the n0
// partials / N (mean = 0 when mpart is null).
template <typename T, int N, int NT = PlaneCfg<T, N>::NT>
__global__ __launch_bounds__(NT) void k_plane_inv_phys(int n0, long nh, long Np, Prm p, const c2<T> *__restrict__ tw,
                                                       const c2<T> *__restrict__ in, const double *__restrict__ psi,
                                                       const double *__restrict__ v, const double *__restrict__ mpart,
                                                       double *hv, double bscale) {
  using C = c2<T>;
  constexpr int NH = N / 2 + 1, NP = lbfft::npass_p<1>(N), NR = N / 2;
  constexpr int NW = NT / 64;
  __shared__ C L[N * NH];
  __shared__ C twl[N];      // the twiddle table, stored during the first pass (which reads none)
  __shared__ double red[NW];  // wave sums of the mean
  TwStage<T, N, NT> tv;
  tv.load(tw);
  const int b = blockIdx.x / n0, i0 = blockIdx.x - b * n0;
  const long off = b * Np + (long)i0 * (N * N);
  const double tau = p.tau[b], gam = p.gamma[b];
  // the mean's partials (n0 <= 512 <= 4 NT) are loaded up front, and in FP32
  // also Gamma'(psi) v at this thread's outputs of the last row pass; the
  // plane's passes hide them (FP64 has no registers to spare: it loads them
  // at the stores)
  constexpr bool PREF = sizeof(T) == 4;
  double mv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = threadIdx.x + u * NT;
    mv[u] = (mpart && i < n0) ? mpart[(long)b * n0 + i] : 0.0;
  }
  using LastS = PassShape<T, N, true, NT, NR, false, NP - 1>;
  constexpr int KP = PREF ? LastS::K : 1, RP = PREF ? LastS::R : 1;
  double wa[KP][RP], wb[KP][RP];
  auto gpv = [&](long i) {
    const double ps = psi[i];
    return (tau - gam * ps + 0.5 * ps * ps) * v[i];
  };
  if constexpr (PREF) {
#pragma unroll
    for (int k = 0; k < LastS::K; ++k) {
      const int bi = threadIdx.x + k * NT;
      if (bi < LastS::TOT) {
        const int f = LastS::f_of(bi), j = LastS::j_of(bi);
#pragma unroll
        for (int r = 0; r < LastS::R; ++r) {
          const long ia = off + (long)(2 * f) * N + j + r * LastS::NS;
          wa[k][r] = gpv(ia);
          wb[k][r] = gpv(ia + N);
        }
      }
    }
  }
  plane_cols_inv_from<T, N, NT>(L, in + b * nh + (long)i0 * (N * NH), twl, [&]() {
    tv.store(twl);
  });
  {
    const double ws = wave_sum(mv[0] + mv[1] + mv[2] + mv[3]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ws;
  }
  __syncthreads();
  double msum = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) msum += red[w];
  const double mean = mpart ? msum / (double)Np : 0.0;
  plane_rows_inv<T, N, NT, N / 2>(L, twl, [&](int f, int x, C z, int k, int r) {
    const long ia = off + (long)(2 * f) * N + x, ib = ia + N;
    if constexpr (PREF) {
      hv[ia] = double(z.x) + bscale * (wa[k][r] - mean);
      hv[ib] = double(z.y) + bscale * (wb[k][r] - mean);
    } else {
      hv[ia] = double(z.x) + bscale * (gpv(ia) - mean);
      hv[ib] = double(z.y) + bscale * (gpv(ib) - mean);
    }
  });
}

// Hessian-vector product in the split order with K parts: workgroup (i0, p)
// of the forward pass takes the physical rows x1 = Km + p of its plane,
// transforms the rows, then over m (length N/K) and stores Z_p (rows p N/K
// ..); the axis-0 pass (k_cols_fwd_mul_inv with KS = K) forms Y, applies
// Lambda and leaves the parts s_q; workgroup (i0, p) of the inverse pass
// transforms s_p over k' (length N/K) into the rows x1 = Km + p, transforms
// them back to real values and writes those rows of hv. The mean of
// Gamma'(psi) v has K n0 partials per instance.
template <typename T, int N, int K, int NT = SplitCfg<T, N, K>::NT>
__global__ __launch_bounds__(NT) void k_plane_fwd_phys_split(int n0, long nh, long Np, Prm p,
                                                             const c2<T> *__restrict__ tw,
                                                             const double *__restrict__ v,
                                                             const double *__restrict__ psi, c2<T> *out,
                                                             double *partial) {
  using C = c2<T>;
  constexpr int L = N / K, NH = N / 2 + 1, NP = lbfft::npass_p<1>(N), NRW = L / 2, PR = plane_pr<N>();
  __shared__ C Ls[L * NH];
  __shared__ C twl[N];
  __shared__ C twh[L];
  __shared__ double red[NT / 64];  // wave sums of the mean partial
  TwStage<T, N, NT> tv;
  TwStage<T, L, NT, K> th;
  tv.load(tw);
  th.load(tw);
  const int pl = blockIdx.x / K, par = blockIdx.x - pl * K;
  const int b = pl / n0, i0 = pl - b * n0;
  const long off = b * Np + (long)i0 * (N * N);
  const double tau = p.tau[b], gam = p.gamma[b];
  double acc = 0.0;
  // packed row q holds the local rows 2q and 2q + 1: x1 = 2Kq + p and 2Kq + K + p
  for (int i = threadIdx.x; i < NRW * N; i += NT) {
    const int q = i / N, x = i - q * N;
    const long ia = off + (long)(2 * K * q + par) * N + x, ib = ia + (long)K * N;
    const double va = v[ia], vb = v[ib];
    if (partial) {
      const double pa = psi[ia], pb = psi[ib];
      acc += (tau - gam * pa + 0.5 * pa * pa) * va + (tau - gam * pb + 0.5 * pb * pb) * vb;
    }
    Ls[q * PR + x] = C{T(va), T(vb)};
  }
  tv.store(twl);
  th.store(twh);
  if (partial) {  // the wave sums now; the passes' barriers order them before thread 0 adds them
    const double ws = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ws;
  }
  __syncthreads();
  sk_lds_passes<T, N, false, NT, NRW, true, 0, NP>(Ls, PR, 1, twl);  // rows, forward
  C *part = out + b * nh + (long)i0 * (N * NH) + (long)par * (L * NH);
  auto store = [&](int f, int e, C val, int, int) {
    if (par) val = cmul(val, twl[par * e]);
    part[e * NH + f] = val;
  };
  plane_cols_fwd_store<T, N, NT, decltype(store), false, L>(Ls, twh, store);
  if (partial && threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    partial[blockIdx.x] = s;
  }
}

template <typename T, int N, int K, int NT = SplitCfg<T, N, K>::NT>
__global__ __launch_bounds__(NT) void k_plane_inv_phys_split(int n0, long nh, long Np, Prm p,
                                                             const c2<T> *__restrict__ tw,
                                                             const c2<T> *__restrict__ in,
                                                             const double *__restrict__ psi,
                                                             const double *__restrict__ v,
                                                             const double *__restrict__ mpart, double *hv,
                                                             double bscale) {
  using C = c2<T>;
  constexpr int L = N / K, NH = N / 2 + 1, NRW = L / 2;
  constexpr int NW = NT / 64, MV = (512 * K + NT - 1) / NT;  // K n0 <= 512 K partials
  __shared__ C Ls[L * NH];
  __shared__ C twl[N];
  __shared__ C twh[L];
  __shared__ double red[NW];
  TwStage<T, N, NT> tv;
  TwStage<T, L, NT, K> th;
  tv.load(tw);
  th.load(tw);
  const int pl = blockIdx.x / K, par = blockIdx.x - pl * K;
  const int b = pl / n0, i0 = pl - b * n0;
  const long off = b * Np + (long)i0 * (N * N);
  const double tau = p.tau[b], gam = p.gamma[b];
  const int np = K * n0;
  double mv = 0.0;
#pragma unroll
  for (int u = 0; u < MV; ++u) {
    const int i = threadIdx.x + u * NT;
    if (mpart && i < np) mv += mpart[(long)b * np + i];
  }
  auto gpv = [&](long i) {
    const double ps = psi[i];
    return (tau - gam * ps + 0.5 * ps * ps) * v[i];
  };
  const C *part = in + b * nh + (long)i0 * (N * NH) + (long)par * (L * NH);
  plane_cols_inv_load<T, N, NT, L>(
      Ls, twh, [&](int f, int e) -> C { return part[e * NH + f]; },
      [&]() {
        tv.store(twl);
        th.store(twh);
      });
  {
    const double ws = wave_sum(mv);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ws;
  }
  __syncthreads();
  double msum = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) msum += red[w];
  const double mean = mpart ? msum / (double)Np : 0.0;
  // packed row f holds the local rows 2f and 2f + 1: x1 = 2Kf + p and 2Kf + K + p
  plane_rows_inv<T, N, NT, NRW>(Ls, twl, [&](int f, int x, C z, int, int) {
    const long ia = off + (long)(2 * K * f + par) * N + x, ib = ia + (long)K * N;
    hv[ia] = double(z.x) + bscale * (gpv(ia) - mean);
    hv[ib] = double(z.y) + bscale * (gpv(ib) - mean);
  });
}

// Algorithm 3 for one square 2D instance (N x N, the half spectrum held in
// LDS like a plane) in a single workgroup that runs every iteration itself:
//   d_t = b_{t-1} / (1 + eta (Lambda + lambda_t)), T d_t = P F_N(Gamma' F_N^{-1} d_t),
//   residual of d_t, b_t = d_t - eta (g + T d_t), phi(0) and the power sums of
//   w |b_t|^2, then the stop test and Newton for lambda_{t+1},
// until the stop test holds or t reaches max_inner. b_t goes to b[t & 1]
// (global memory), so the result is read as for the multi-kernel iteration;
// SubState is read at the start and written at the end. b_t, g, Gamma',
// Lambda and the twiddles stay in LDS for the whole launch, so an iteration
// waits on no global load.
template <typename T, int N> struct Sub2dCfg {
  static constexpr int NH = N / 2 + 1;
  static constexpr long LDS = (long)N * NH * (sizeof(double2) + 2 * sizeof(c2<T>) + sizeof(double)) +
                              (long)N * N * sizeof(T) + (long)N * sizeof(c2<T>);
  static constexpr bool fits = N <= 64 && LDS <= 150 * 1024;  // the rest: M, scratch of the sums
};
template <typename T, int N, int NT = PlaneCfg<T, N>::NT>
__global__ __launch_bounds__(NT) void k_sub2d(Geo g, Prm p, const c2<T> *__restrict__ twg, c2<T> *b0, c2<T> *b1,
                                              const c2<T> *__restrict__ gh, const T *__restrict__ gp, SubState *st) {
  using C = c2<T>;
  constexpr int NH = N / 2 + 1, NP = lbfft::npass_p<1>(N), NR = N / 2, PR = plane_pr<N>();
  constexpr int NW = NT / 64, RS = MOM_NV + 1;
  static_assert(Sub2dCfg<T, N>::fits, "the LDS-resident subproblem");
  // the plane in LDS; after the last pass the same storage holds (w |b_t|^2, u) per element
  __shared__ double2 Lraw[N * NH];
  C *L = reinterpret_cast<C *>(Lraw);
  __shared__ C Bs[N * NH];  // b_t (b_{-1} on entry)
  __shared__ C Gs[N * NH];  // g
  __shared__ T Gp[N * N];   // Gamma'(psi)
  __shared__ double Lm[N * NH];  // Lambda
  __shared__ C tw[N];
  __shared__ double M[RS];
  __shared__ double scr[2 * NW];
  __shared__ double nw_lam;  // wave 0's Newton result, steps, direct sums
  __shared__ int nw_it[2];
  // row-sum scratch [NT / 16][RS]: the plane's storage where it is large
  // enough (not for N <= 16), else an array of its own
  constexpr int NROW = NT / 16;
  constexpr bool RED_IN_PLANE = 2 * N * NH >= NROW * RS;
  __shared__ double red_own[RED_IN_PLANE ? 1 : NROW * RS];
  double *red = RED_IN_PLANE ? reinterpret_cast<double *>(Lraw) : red_own;
  // one workgroup per instance of the batch
  const int inst = blockIdx.x;
  st += inst;
  b0 += (long)inst * N * NH;
  b1 += (long)inst * N * NH;
  gh += (long)inst * N * NH;
  gp += (long)inst * N * N;
  if (st->done) return;
  const double xi = p.xi[inst], q = p.q[inst];
  for (int h = threadIdx.x; h < N * NH; h += NT) {
    Bs[h] = b1[h];  // b_{t-1} of step 0 is b[1]
    Gs[h] = gh[h];
    const int e = h / NH, f = h - e * NH;
    const ColK ck = col_k(g, 0, f);
    Lm[h] = lam_of(kk_elem(g, e, ck.kkc, ck.lin, ck.lin_nyq), xi, q);
  }
  for (int i = threadIdx.x; i < N * N; i += NT) Gp[i] = gp[i];
  for (int i = threadIdx.x; i < N; i += NT) tw[i] = twg[i];
  __syncthreads();
  const double eta = st->eta, tol = st->tol;
  const int max_inner = st->max_inner;
  NewtonPar np{eta, st->r2, 0.0, st->newton_rtol, st->newton_steptol, st->max_newton, st->newton_phi,
               st->newton_direct_only};
  const double inv_n = 1.0 / ((double)N * (double)N);
  double lam_t = st->lam[0];
  int newton_total = 0, newton_direct = 0;
  for (int t = 0;; ++t) {
    C *bnext = (t & 1) ? b1 : b0;
    const double mu0 = eta * lam_t;
    // d_t, axis 0 inverse
    plane_cols_inv_load<T, N, NT, N>(L, tw, [&](int f, int e) -> C {
      const C v = Bs[e * NH + f];
      const double x = 1.0 + eta * Lm[e * NH + f] + mu0;
      const double sc = (e == 0 && f == 0) ? 0.0 : rcp64(x);
      return C{T(double(v.x) * sc), T(double(v.y) * sc)};
    });
    __syncthreads();
    // rows inverse, x Gamma' (rows 2f, 2f + 1), rows forward
    plane_rows_inv<T, N, NT, N / 2>(L, tw, [&](int f, int e, C v, int, int) {
      L[f * PR + e] = C{v.x * Gp[(2 * f) * N + e], v.y * Gp[(2 * f + 1) * N + e]};
    });
    __syncthreads();
    sk_lds_passes<T, N, false, NT, NR, true, 0, NP>(L, PR, 1, tw);
    // axis 0 forward; per output element: residual of d_t, b_t, and (w |b_t|^2, u)
    double res2 = 0.0;
    auto upd = [&](int f, int e, C v, int, int) {
      const int h = e * NH + f;
      const bool dc = (e == 0 && f == 0);
      const double lam = Lm[h];
      const double w = (f == 0 || 2 * f == N) ? 1.0 : 2.0;
      const C bp = Bs[h], gg = Gs[h];  // each element is read and rewritten by one thread
      const double u = rcp64(1.0 + eta * lam + mu0);
      const double sc = dc ? 0.0 : u;
      const double dx = double(bp.x) * sc, dy = double(bp.y) * sc;
      const double tx = double(v.x) * inv_n, ty = double(v.y) * inv_n;
      const double rx = double(gg.x) + (lam + lam_t) * dx + tx, ry = double(gg.y) + (lam + lam_t) * dy + ty;
      const C bn = dc ? C{T(0), T(0)} : C{T(dx - eta * (double(gg.x) + tx)), T(dy - eta * (double(gg.y) + ty))};
      bnext[h] = bn;
      Bs[h] = bn;
      if (!dc) res2 += w * (rx * rx + ry * ry);
      const double wb = dc ? 0.0 : w * (double(bn.x) * double(bn.x) + double(bn.y) * double(bn.y));
      Lraw[h] = double2{wb, u};
    };
    plane_cols_fwd_store<T, N, NT, decltype(upd), true>(L, tw, upd);
    __syncthreads();
    // phi(0) and the power sums M_2 .. M_{NMOM+1} from the stored pairs
    double acc[RS];
#pragma unroll
    for (int j = 0; j < RS; ++j) acc[j] = 0.0;
    acc[MOM_NV] = res2;
    for (int h = threadIdx.x; h < N * NH; h += NT) {
      const double2 wu = Lraw[h];
      const double u0 = rcp64(1.0 + eta * Lm[h]);
      acc[0] = fma(wu.x, u0 * u0, acc[0]);
      double pw = wu.x * wu.y * wu.y;
#pragma unroll
      for (int j = 1; j < MOM_NV; ++j) {
        acc[j] += pw;
        pw *= wu.y;
      }
    }
    __syncthreads();  // Lraw may become the row-sum scratch
    // sums over rows of 16 lanes (four DPP shifts each), row sums added in LDS
    const int row = threadIdx.x >> 4;
#pragma unroll
    for (int j = 0; j < RS; ++j) {
      const double v = row_sum(acc[j]);
      if ((threadIdx.x & 15) == 15) red[row * RS + j] = v;
    }
    __syncthreads();
    if (threadIdx.x < RS) {
      double a = 0.0;
#pragma unroll
      for (int w = 0; w < NROW; ++w) a += red[w * RS + threadIdx.x];
      M[threadIdx.x] = a;
    }
    __syncthreads();
    // stop test of d_t, then lambda_{t+1}
    const double resid = sqrt(M[MOM_NV]);
    const bool bad = !(resid == resid) || resid > 1e300;
    if ((t >= 1 && resid < tol) || t >= max_inner || bad) {
      if (threadIdx.x == 0) {
        st->resid = resid;
        st->done = (resid < tol) ? 1 : 2;
        if (bad) st->nonfinite = 1;
        st->final_step = t;
        st->lam_final = lam_t;
        st->lam[t & 1] = lam_t;
        st->newton_total += newton_total;
        st->newton_direct += newton_direct;
        st->step = t;
      }
      break;
    }
    np.lam_prev = lam_t;
    // direct sum of phi over the half spectrum of b_t
    auto direct = [&](double lam, double &phi, double &dphi) {
      const double e2 = eta * lam;
      double a = 0.0, b = 0.0;
      for (int h = threadIdx.x + 1; h < N * NH; h += NT) {
        const int e = h / NH, f = h - e * NH;
        const C bn = Bs[h];
        const double w = (f == 0 || 2 * f == N) ? 1.0 : 2.0;
        const double wb = w * (double(bn.x) * double(bn.x) + double(bn.y) * double(bn.y));
        const double r = rcp64(1.0 + eta * Lm[h] + e2);
        a = fma(wb, r * r, a);
        b = fma(wb, r * r * r, b);
      }
      block_sum2_nt<NT>(a, b, scr);
      phi = a;
      dphi = -2.0 * eta * b;
    };
    // Newton on the series in wave 0 alone; every thread runs it again with
    // the direct sum where an evaluation needs one (as in the Newton kernel)
    if (threadIdx.x < 64) {
      auto stub = [&](double, double &phi, double &dphi) {
        phi = np.r2;
        dphi = -1.0;
      };
      int it1 = 0, nd1 = 0;
      const double l1 = multiplier_newton(M, np, stub, it1, nd1);
      if (threadIdx.x == 0) {
        nw_lam = l1;
        nw_it[0] = it1;
        nw_it[1] = nd1;
      }
    }
    __syncthreads();
    int it = nw_it[0], nd = 0;
    lam_t = nw_lam;
    if (nw_it[1] != 0) {  // uniform
      it = 0;
      lam_t = multiplier_newton(M, np, direct, it, nd);
    }
    newton_total += it;
    newton_direct += nd;
    __syncthreads();  // M, the LDS, b_t and the Newton result are read again by the next iteration
  }
}

// ---------------------------------------------------------------------------
// Elementwise spectral kernels and reductions
// ---------------------------------------------------------------------------
constexpr int EW_NT = 256;

// gradient assembly after the forward transforms of psi and F'(psi):
//   g = P(Lambda psi_hat + F_N F'(psi)) and partials
//   [1/2 sum w Lambda |psi_hat|^2, sum w |g|^2, max |g|] per workgroup
// With raw != 0 the k = 0 entry is kept and g is scaled by 1/N: the gradient
// with respect to the N grid values of E as printed (no mass constraint).
template <typename TG>
__global__ __launch_bounds__(EW_NT) void k_grad_assemble(Geo g, Prm p, int bpi, const double2 *__restrict__ ph,
                                                         const double2 *__restrict__ fh, double2 *__restrict__ gh,
                                                         c2<TG> *__restrict__ gh_t, double *partial, int raw) {
  __shared__ double scratch[64];
  const int b = blockIdx.x / bpi;
  const long lb = blockIdx.x % bpi;
  double aG = 0.0, aN = 0.0, aM = 0.0;
  for (long hl = lb * EW_NT + threadIdx.x; hl < g.nh; hl += (long)bpi * EW_NT) {
    const long h = (long)b * g.nh + hl;
    int kl;
    const double lam = lam_of(kk_at(g, (int)hl, kl), p.xi[b], p.q[b]);
    const double w = herm_w(g, kl);
    const double2 a = ph[h], f = fh[h];
    aG += 0.5 * w * lam * (a.x * a.x + a.y * a.y);
    double2 gv{lam * a.x + f.x, lam * a.y + f.y};
    if (raw) {
      const double sN = 1.0 / (double)g.N;
      gv = double2{gv.x * sN, gv.y * sN};
    } else if (hl == 0) {
      gv = double2{0.0, 0.0};
    }
    const double m2 = gv.x * gv.x + gv.y * gv.y;
    aN += w * m2;
    aM = fmax(aM, sqrt(m2));
    gh[h] = gv;
    if (gh_t) gh_t[h] = c2<TG>{TG(gv.x), TG(gv.y)};
  }
  const double s0 = block_sum<EW_NT>(aG, scratch);
  const double s1 = block_sum<EW_NT>(aN, scratch + 16);
  const double s2 = block_max<EW_NT>(aM, scratch + 32);
  if (threadIdx.x == 0) {
    partial[3 * blockIdx.x + 0] = s0;
    partial[3 * blockIdx.x + 1] = s1;
    partial[3 * blockIdx.x + 2] = s2;
  }
}

// Spectral reductions over one instance's half spectrum (weights w):
//   MODE 0: sum w Re(a conj(b))          MODE 1: sum w Lambda |a|^2
template <typename TA, int MODE>
__global__ __launch_bounds__(EW_NT) void k_spec_reduce(Geo g, Prm p, int bpi, const c2<TA> *__restrict__ a,
                                                       const c2<TA> *__restrict__ bb, double *partial) {
  __shared__ double scratch[16];
  const int b = blockIdx.x / bpi;
  const long lb = blockIdx.x % bpi;
  double acc = 0.0;
  for (long hl = lb * EW_NT + threadIdx.x; hl < g.nh; hl += (long)bpi * EW_NT) {
    const long h = (long)b * g.nh + hl;
    int kl;
    const double kk = kk_at(g, (int)hl, kl);
    const double w = herm_w(g, kl);
    const c2<TA> x = a[h];
    if constexpr (MODE == 0) {
      const c2<TA> y = bb[h];
      acc += w * (double(x.x) * double(y.x) + double(x.y) * double(y.y));
    } else {
      acc += w * lam_of(kk, p.xi[b], p.q[b]) * (double(x.x) * double(x.x) + double(x.y) * double(x.y));
    }
  }
  const double s = block_sum<EW_NT>(acc, scratch);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out = alpha * x + beta * y over n complex entries (types may differ)
template <typename TO, typename TX, typename TY>
__global__ __launch_bounds__(EW_NT) void k_lincomb(long n, double alpha, const c2<TX> *__restrict__ x, double beta,
                                                   const c2<TY> *__restrict__ y, c2<TO> *__restrict__ out) {
  for (long i = (long)blockIdx.x * EW_NT + threadIdx.x; i < n; i += (long)gridDim.x * EW_NT) {
    double ox = 0.0, oy = 0.0;
    if (alpha != 0.0) {
      const c2<TX> a = x[i];
      ox += alpha * double(a.x);
      oy += alpha * double(a.y);
    }
    if (beta != 0.0) {
      const c2<TY> c = y[i];
      ox += beta * double(c.x);
      oy += beta * double(c.y);
    }
    out[i] = c2<TO>{TO(ox), TO(oy)};
  }
}

// Initial point of the subproblem, stored as b_{-1} = d_0 (1 + eta Lambda) so
// that step 0 recovers d_0 with lambda_0 = 0, per instance b:
//   d_0 = coef_b * src (coef_b = -r_b / ||g_b|| with src = g, or 1 with src = user d0)
struct InitCoef {
  double coef[MAXB], eta[MAXB];
};
template <typename T, typename TS>
__global__ __launch_bounds__(EW_NT) void k_init_b(Geo g, Prm p, const c2<TS> *__restrict__ src, InitCoef ic,
                                                  c2<T> *__restrict__ bm1) {
  const long total = (long)g.batch * g.nh;
  for (long h = (long)blockIdx.x * EW_NT + threadIdx.x; h < total; h += (long)gridDim.x * EW_NT) {
    const int b = (int)(h / g.nh);
    const long hl = h - (long)b * g.nh;
    int kl;
    const double lam = lam_of(kk_at(g, (int)hl, kl), p.xi[b], p.q[b]);
    const c2<TS> s = src[h];
    const double f = (hl == 0) ? 0.0 : ic.coef[b] * (1.0 + ic.eta[b] * lam);
    bm1[h] = c2<T>{T(f * double(s.x)), T(f * double(s.y))};
  }
}

// Final step of the subproblem: d = b_{t*-1} / (1 + eta (Lambda + lambda_{t*})) in FP64, per instance
template <typename T>
__global__ __launch_bounds__(EW_NT) void k_final_d(Geo g, Prm p, const c2<T> *__restrict__ b0, const c2<T> *__restrict__ b1,
                                                   const SubState *st, double2 *__restrict__ d) {
  const long total = (long)g.batch * g.nh;
  for (long hh = (long)blockIdx.x * EW_NT + threadIdx.x; hh < total; hh += (long)gridDim.x * EW_NT) {
    const int b = (int)(hh / g.nh);
    const long h = hh - (long)b * g.nh;
    const int t = st[b].final_step;
    const c2<T> *src = ((t - 1) & 1) ? b1 : b0;
    const double lamf = st[b].lam_final, eta = st[b].eta;
    int kl;
    const double lam = lam_of(kk_at(g, (int)h, kl), p.xi[b], p.q[b]);
    const double s = (h == 0) ? 0.0 : 1.0 / (1.0 + eta * (lam + lamf));
    const c2<T> v = src[hh];
    d[hh] = double2{double(v.x) * s, double(v.y) * s};
  }
}

// Non-template kernels: defined only in the library's main translation unit.
#ifdef LB_MAIN_TU
// ---------------------------------------------------------------------------
// Random feasible initial point for nearly hard subproblems
// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC'11), a counter-based
// generator: ten rounds, each multiplying words 0 and 2 by fixed constants and
// mixing the high/low halves with words 1, 3 and the key, which is bumped by
// Weyl constants between rounds.
struct Philox4 {
  uint64_t w[4];
};
__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}
__host__ __device__ inline Philox4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                              uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = mulhi64(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = mulhi64(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  return Philox4{{c0, c1, c2, c3}};
}
// uniform in (0, 1) from the top 53 bits
__host__ __device__ inline double unit_open(uint64_t w) { return ((double)(w >> 11) + 0.5) * 0x1p-53; }

// z_x standard normal (Box-Muller on counter (x, 0, 0, 0), key (seed, draw));
// per-workgroup partials [sum z, sum z^2] at partial[2 block + q]
__global__ __launch_bounds__(EW_NT) void k_ball_normals(long N, uint64_t seed, uint64_t draw, double *__restrict__ z,
                                                        double *partial) {
  __shared__ double scratch[32];
  double a = 0.0, b = 0.0;
  for (long i = (long)blockIdx.x * EW_NT + threadIdx.x; i < N; i += (long)gridDim.x * EW_NT) {
    const Philox4 w = philox4x64((uint64_t)i, 0, 0, 0, seed, draw);
    const double v = sqrt(-2.0 * log(unit_open(w.w[0]))) * cos(6.283185307179586476925286766559 * unit_open(w.w[1]));
    z[i] = v;
    a += v;
    b += v * v;
  }
  const double sa = block_sum<EW_NT>(a, scratch);
  const double sb = block_sum<EW_NT>(b, scratch + 16);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sa;
    partial[2 * blockIdx.x + 1] = sb;
  }
}
// f = [r u^(1/(N-1)) / rms(z - mean z), mean z] with u from counter (0, 1, 0, 0)
__global__ void k_ball_factor(long N, double r, uint64_t seed, uint64_t draw, const double *sums, double *f) {
  if (threadIdx.x != 0) return;
  const double zbar = sums[0] / (double)N;
  const double var = sums[1] / (double)N - zbar * zbar;
  const double u = unit_open(philox4x64(0, 1, 0, 0, seed, draw).w[0]);
  f[0] = r * pow(u, 1.0 / (double)(N - 1)) / sqrt(var);
  f[1] = zbar;
}
__global__ __launch_bounds__(EW_NT) void k_ball_scale(long N, const double *__restrict__ f, double *z) {
  const double c = f[0], zbar = f[1];
  for (long i = (long)blockIdx.x * EW_NT + threadIdx.x; i < N; i += (long)gridDim.x * EW_NT) z[i] = c * (z[i] - zbar);
}

// Per-workgroup partial sums [psi^2, psi^3, w psi, w psi^2] over instance b's
// N points (w nullable: zeros); partial[(b * bpi + block) * 4 + q]
__global__ __launch_bounds__(EW_NT) void k_field_moments(long N, int bpi, const double *__restrict__ psi,
                                                         const double *__restrict__ w, double *partial) {
  __shared__ double scratch[64];
  const int b = blockIdx.x / bpi;
  const long lb = blockIdx.x % bpi;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (long i = lb * EW_NT + threadIdx.x; i < N; i += (long)bpi * EW_NT) {
    const double x = psi[(long)b * N + i], x2 = x * x;
    a[0] += x2;
    a[1] += x2 * x;
    if (w) {
      const double y = w[(long)b * N + i];
      a[2] += y * x;
      a[3] += y * x2;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double s = block_sum<EW_NT>(a[q], scratch + 16 * q);
    if (threadIdx.x == 0) partial[((long)blockIdx.x) * 4 + q] = s;
  }
}

// out[b * nq + q] = scale * sums[b * nq + q]
__global__ void k_scale_out(const double *sums, int count, double scale, double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = scale * sums[i];
}

// Sum `nq` interleaved per-workgroup partials over the `bpi` workgroups of
// each instance in a fixed order; q listed in `is_max` use max instead.
// One workgroup per instance; out[b * nq + q].
__global__ __launch_bounds__(256) void k_finalize(const double *__restrict__ partial, int bpi, int nq,
                                                  unsigned is_max, double *__restrict__ out) {
  __shared__ double scratch[64];
  const int b = blockIdx.x;
  for (int q = 0; q < nq; ++q) {
    const bool mx = (is_max >> q) & 1u;
    double a = 0.0;
    for (int i = threadIdx.x; i < bpi; i += 256) {
      const double v = partial[((long)b * bpi + i) * nq + q];
      a = mx ? fmax(a, v) : a + v;
    }
    const double s = mx ? block_max<256>(a, scratch) : block_sum<256>(a, scratch);
    if (threadIdx.x == 0) out[b * nq + q] = s;
  }
}

// energy from the finalised sums: E_b = G_b + F_b / N
__global__ void k_energy_out(const double *sumG, int strideG, const double *sumF, int strideF, double invN, int batch,
                             double *energy) {
  const int b = threadIdx.x;
  if (b < batch) energy[b] = sumG[b * strideG] + sumF[b * strideF] * invN;
}

// real arrays: y = y + a * x
__global__ __launch_bounds__(EW_NT) void k_axpy_real(long n, double a, const double *__restrict__ x, double *y) {
  for (long i = (long)blockIdx.x * EW_NT + threadIdx.x; i < n; i += (long)gridDim.x * EW_NT) y[i] += a * x[i];
}

// The stop test of step t and the multiplier lambda_{t+1} (one workgroup):
//   resid_t = sqrt(sum of the residual partials); done if t >= 1 and
//   resid_t < tol (converged) or t >= max_inner (cap); otherwise
//   lambda_{t+1} = 0 if phi(0) <= r^2, else the root of phi(lambda) = r^2 by
//   Newton's method, applied either to phi(lambda) - r^2 from lambda = 0
//   (newton_phi, as printed) or to the equivalent 1/sqrt(phi(lambda)) - 1/r
//   from lambda_t. The latter is concave and increasing in lambda (phi is the
//   squared norm of a diagonal shifted solve), so its first step lands at or
//   below the root and the iterates then rise monotonically to it; both stop
//   by the same test. All threads run the scalar iteration on identical
//   values, so its control flow is uniform.
constexpr int NW_NT = 1024;
__device__ __forceinline__ void block_sum2_all(double &a, double &b, double *scratch /* >= 2 * 16 */) {
  const int w = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) {
    scratch[w] = a;
    scratch[16 + w] = b;
  }
  __syncthreads();
  a = b = 0.0;
#pragma unroll
  for (int i = 0; i < NW_NT / 64; ++i) {
    a += scratch[i];
    b += scratch[16 + i];
  }
  __syncthreads();
}

template <typename T, bool GEN>
__global__ __launch_bounds__(NW_NT) void k_newton(Geo g, Prm p, const double *__restrict__ mom, int nmb, long mstride,
                                                  const double *__restrict__ rpart, int rbpi,
                                                  const c2<T> *__restrict__ b0, const c2<T> *__restrict__ b1, int cpi,
                                                  SubState *st) {
  __shared__ double M[MOM_NV + 1];
  __shared__ double scratch[32];
  // one workgroup per instance of the batch: its nmb update workgroups' moment
  // partials at mom[j * mstride + inst * nmb + i], residual partials at
  // rpart[inst * rbpi + i]
  const int inst = blockIdx.x;
  st += inst;
  mom += (long)inst * nmb;
  rpart += (long)inst * rbpi;
  b0 += (long)inst * g.nh;
  b1 += (long)inst * g.nh;
  // wave w sums values w and w + 16 (value MOM_NV: the residual partials)
  // over the workgroups of the update pass. Both values' loads, KU per lane
  // each (up to 64 KU workgroups), go out before the first add waits, and
  // the step's state is read after them, so the two round trips overlap.
  constexpr int WV = NW_NT / 64, KU = 9;
  static_assert(2 * WV > MOM_NV, "two values per wave");
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int va = wv, vb = wv + WV;
  const bool hb = vb <= MOM_NV;  // uniform in the wave
  const double *sa = va < MOM_NV ? mom + (long)va * mstride : rpart;
  const double *sb = !hb ? sa : (vb < MOM_NV ? mom + (long)vb * mstride : rpart);  // !hb: loaded, not added
  const int ca = va < MOM_NV ? nmb : rbpi, cb = !hb ? 0 : (vb < MOM_NV ? nmb : rbpi);
  double xa[KU], xb[KU];
#pragma unroll
  for (int k = 0; k < KU; ++k) {  // unconditional (past the end: index 0, not added)
    const int i = lane + 64 * k;
    xa[k] = sa[i < ca ? i : 0];
    xb[k] = sb[i < cb ? i : 0];
  }
  __builtin_amdgcn_sched_barrier(0);
  // the state of this step, read before anything here writes it
  const SubState s0 = *st;
  __builtin_amdgcn_sched_barrier(0);
  {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int k = 0; k < KU; ++k) {
      const int i = lane + 64 * k;
      if (i < ca) a += xa[k];
      if (i < cb) b += xb[k];
    }
    for (int i0 = 64 * KU; i0 < ca || i0 < cb; i0 += 64 * KU) {  // more than 64 KU workgroups
#pragma unroll
      for (int k = 0; k < KU; ++k) {
        const int i = i0 + lane + 64 * k;
        xa[k] = sa[i < ca ? i : 0];
        xb[k] = sb[i < cb ? i : 0];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < KU; ++k) {
        const int i = i0 + lane + 64 * k;
        if (i < ca) a += xa[k];
        if (i < cb) b += xb[k];
      }
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
      M[va] = a;
      if (hb) M[vb] = b;
    }
  }
  __syncthreads();
  if (s0.done) return;
  const int t = s0.step;  // written by the previous step's Newton kernel
  const double resid = sqrt(M[MOM_NV]);
  const bool bad = !(resid == resid) || resid > 1e300;
  const double lam_prev = (t & 1) ? s0.lam[1] : s0.lam[0];
  if ((t >= 1 && resid < s0.tol) || t >= s0.max_inner || bad) {
    if (threadIdx.x == 0) {
      st->resid = resid;
      st->done = (resid < s0.tol) ? 1 : 2;
      if (bad) st->nonfinite = 1;
      st->final_step = t;
      st->lam_final = lam_prev;
    }
    return;
  }
  const double eta = s0.eta;
  NewtonPar np{eta, s0.r2, lam_prev, s0.newton_rtol, s0.newton_steptol, s0.max_newton, s0.newton_phi,
               s0.newton_direct_only};
  // direct sum of phi over the spectrum: the pair entries form rows e = |k0|
  // of cpi columns. Each thread owns two columns at a time (|Bk|^2 of the
  // column part formed once) and walks the rows in batches of DU with all
  // 2 DU loads of a batch issued before the first is used (rows past the end
  // re-read the last row and add nothing).
  auto direct = [&](double lam, double &phi, double &dphi) {
    constexpr int DU = 4;
    const c2<T> *bt = (t & 1) ? b1 : b0;  // b_t, written by this step's update pass
    const double xi = p.xi[inst], q = p.q[inst];
    const double e2 = eta * lam;
    const int n0 = g.n0, nrow = n0 / 2 + 1;
    double a = 0.0, b = 0.0;
    for (int ml0 = 0; ml0 < cpi; ml0 += 2 * NW_NT) {
      int mls[2];
      bool okc[2];
      double kkc[2], wc[2], lin[2], linq[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int ml = ml0 + c * NW_NT + (int)threadIdx.x;
        okc[c] = ml < cpi;
        mls[c] = okc[c] ? ml : 0;
        const ColInfo ci = col_info<GEN>(g, mls[c]);
        kkc[c] = ci.kkc;
        wc[c] = ci.w;
        lin[c] = ci.lin;
        linq[c] = ci.lin_nyq;
      }
      for (int e0 = 0; e0 < nrow; e0 += DU) {
        // entries k0 and -k0 (rows e and n0 - e of column ml, at e cpi + ml)
        c2<T> xp[2][DU], xm[2][DU];
#pragma unroll
        for (int u = 0; u < DU; ++u) {
          const int e = e0 + u < nrow ? e0 + u : nrow - 1;
          const int em = (e == 0 || 2 * e == n0) ? e : n0 - e;
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            xp[c][u] = bt[(long)e * cpi + mls[c]];
            xm[c][u] = bt[(long)em * cpi + mls[c]];
          }
        }
        double wp[2][DU], wm[2][DU];
#pragma unroll
        for (int u = 0; u < DU; ++u) {
          const int e = e0 + u < nrow ? e0 + u : nrow - 1;
          const bool paired = !(e == 0 || 2 * e == n0);
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const double px = double(xp[c][u].x), py = double(xp[c][u].y);
            const double mx = double(xm[c][u].x), my = double(xm[c][u].y);
            wp[c][u] = wc[c] * (px * px + py * py);
            wm[c][u] = paired ? wc[c] * (mx * mx + my * my) : 0.0;
          }
        }
#pragma unroll
        for (int u = 0; u < DU; ++u) {
          const int e = e0 + u;
          if (e >= nrow) break;
          const double kk0 = kk0_of(g, e);
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            if (!okc[c] || (e == 0 && mls[c] == 0)) continue;
            if constexpr (!GEN) {  // +-k0 share Lambda
              const double w = wp[c][u] + wm[c][u];
              const double r = rcp64(1.0 + eta * lam_of(kk0 + kkc[c], xi, q) + e2);
              const double r2i = r * r;
              a = fma(w, r2i, a);
              b = fma(w, r2i * r, b);
            } else {
              const int em = (e == 0 || 2 * e == n0) ? e : n0 - e;
              const double rp = rcp64(1.0 + eta * lam_of(kk_elem(g, e, kkc[c], lin[c], linq[c]), xi, q) + e2);
              const double rm = rcp64(1.0 + eta * lam_of(kk_elem(g, em, kkc[c], lin[c], linq[c]), xi, q) + e2);
              a = fma(wp[c][u], rp * rp, a);
              b = fma(wp[c][u], rp * rp * rp, b);
              a = fma(wm[c][u], rm * rm, a);
              b = fma(wm[c][u], rm * rm * rm, b);
            }
          }
        }
      }
    }
    block_sum2_all(a, b, scratch);
    phi = a;
    dphi = -2.0 * eta * b;
  };
  // Newton on the series alone in one wave: the other waves would only repeat
  // its dependent FP64 chain on the same SIMDs. An evaluation that needs the
  // sum over the spectrum ends that run (a stub returns phi = r^2), and then
  // every thread runs the iteration again with the block-collective sum.
  __shared__ double lam_w;
  __shared__ int it_w, nd_w;
  if (threadIdx.x < 64) {
    auto stub = [&](double, double &phi, double &dphi) {
      phi = np.r2;
      dphi = -1.0;
    };
    int it1 = 0, nd1 = 0;
    const double l1 = multiplier_newton(M, np, stub, it1, nd1);
    if (threadIdx.x == 0) {
      lam_w = l1;
      it_w = it1;
      nd_w = nd1;
    }
  }
  __syncthreads();
  int it = it_w, ndirect = 0;
  double lam = lam_w;
  if (nd_w != 0) {  // uniform
    it = 0;
    lam = multiplier_newton(M, np, direct, it, ndirect);
  }
  if (threadIdx.x == 0) {
    st->resid = resid;
    st->lam[(t + 1) & 1] = lam;
    st->newton_total = s0.newton_total + it;  // stores only: no read-modify-write round trip
    st->newton_direct = s0.newton_direct + ndirect;
    st->step = t + 1;
  }
}

#endif  // LB_MAIN_TU

}  // namespace lbk
