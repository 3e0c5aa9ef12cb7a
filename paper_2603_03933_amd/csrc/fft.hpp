// fft.hpp - mixed-radix Stockham FFT core for gfx950 (radices 8, 4, 2, 3).
//
// One length-N complex transform is carried out by TPF = N / R0 threads (R0 the
// first radix); a workgroup runs C such transforms side by side. Data moves
// between passes through LDS; the first pass reads its inputs and the last
// pass hands its outputs to caller-supplied functors, both at element index
// j + r * (N / R) (Stockham's autosort places pass inputs and final outputs in
// the same pattern), so a caller can stream straight from and to global
// memory with coalesced accesses.
//
// Forward transforms compute X_p = sum_e x_e exp(-2 pi i p e / N) (no
// normalisation); inverse ones use the opposite sign. Twiddles come from a
// table W[m] = exp(-2 pi i m / N), m in [0, N), computed on the host in
// extended precision and rounded once.
#pragma once
#include <hip/hip_runtime.h>

namespace lbfft {

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };
template <typename T> using c2 = typename Vec2<T>::type;

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C mul_mi(C a) {
  if constexpr (INV) return C{-a.y, a.x};
  else return C{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// Radix plan: greedy 8s, then 4s, then 2s, then 3s (N = 2^a 3^b).
// ---------------------------------------------------------------------------
constexpr int radix_at(int N, int p) {
  int n = N, i = 0;
  const int rs[3] = {8, 4, 2};
  for (int q = 0; q < 3; ++q) {
    while (n % rs[q] == 0 && n > 1) {
      if (i == p) return rs[q];
      n /= rs[q];
      ++i;
    }
  }
  while (n % 3 == 0 && n > 1) {
    if (i == p) return 3;
    n /= 3;
    ++i;
  }
  return 0;
}
constexpr int num_passes(int N) {
  int p = 0;
  while (radix_at(N, p) != 0) ++p;
  return p;
}
constexpr int span_before(int N, int p) {  // product of the radices of passes < p
  int s = 1;
  for (int i = 0; i < p; ++i) s *= radix_at(N, i);
  return s;
}
// Radix plan 2: radix 4 while 4 divides what is left, then 2s and 3s (more,
// shorter passes: N = 128 as 4, 4, 4, 2 with 32 threads per transform).
constexpr int radix_at4(int N, int p) {
  int n = N, i = 0;
  while (n % 4 == 0) {
    if (i == p) return 4;
    n /= 4;
    ++i;
  }
  while (n % 2 == 0) {
    if (i == p) return 2;
    n /= 2;
    ++i;
  }
  while (n % 3 == 0) {
    if (i == p) return 3;
    n /= 3;
    ++i;
  }
  return 0;
}
// Radix plan 1: a first pass of radix 16 when 16 divides N, then plan 0
// (two passes for N = 128 instead of three; used where data lives in LDS).
template <int PLAN> constexpr int radix_p(int N, int p) {
  if constexpr (PLAN == 0) {
    return radix_at(N, p);
  } else if constexpr (PLAN == 2) {
    return radix_at4(N, p);
  } else {
    if (N % 16 == 0 && N > 16) return p == 0 ? 16 : radix_at(N / 16, p - 1);
    return radix_at(N, p);
  }
}
template <int PLAN> constexpr int npass_p(int N) {
  int p = 0;
  while (radix_p<PLAN>(N, p) != 0) ++p;
  return p;
}
template <int PLAN> constexpr int span_p(int N, int p) {
  int s = 1;
  for (int i = 0; i < p; ++i) s *= radix_p<PLAN>(N, i);
  return s;
}
constexpr bool supported_length(int N) {
  if (N < 2) return false;
  int n = N;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}
template <int N> struct Shape {
  static_assert(supported_length(N), "FFT length must be 2^a 3^b");
  static constexpr int R0 = radix_at(N, 0);
  static constexpr int TPF = N / R0;  // threads per transform
  static constexpr int NP = num_passes(N);
};

// ---------------------------------------------------------------------------
// Small DFT kernels, in place on v[0..R)
// ---------------------------------------------------------------------------
template <typename T, bool INV> __device__ __forceinline__ void dft2(c2<T> *v) {
  c2<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T, bool INV> __device__ __forceinline__ void dft4(c2<T> *v) {
  c2<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  c2<T> t2 = cadd(v[1], v[3]), t3 = mul_mi<INV>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <typename T, bool INV> __device__ __forceinline__ void dft8(c2<T> *v) {
  // X_p = E_p + w^p O_p, X_{p+4} = E_p - w^p O_p with E, O the 4-point DFTs of
  // the even and odd samples and w = exp(-+ i pi / 4).
  c2<T> e[4] = {v[0], v[2], v[4], v[6]};
  c2<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
  const T h = T(0.70710678118654752440084436210484904);
  // w^1 o1, w^2 o2, w^3 o3
  c2<T> w1, w2, w3;
  if constexpr (!INV) {
    w1 = c2<T>{h * (o[1].x + o[1].y), h * (o[1].y - o[1].x)};
    w2 = c2<T>{o[2].y, -o[2].x};
    w3 = c2<T>{h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y)};
  } else {
    w1 = c2<T>{h * (o[1].x - o[1].y), h * (o[1].y + o[1].x)};
    w2 = c2<T>{-o[2].y, o[2].x};
    w3 = c2<T>{-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y)};
  }
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], w1);
  v[5] = csub(e[1], w1);
  v[2] = cadd(e[2], w2);
  v[6] = csub(e[2], w2);
  v[3] = cadd(e[3], w3);
  v[7] = csub(e[3], w3);
}

template <typename T, bool INV> __device__ __forceinline__ void dft3(c2<T> *v) {
  const T s3 = T(0.86602540378443864676372317075293618);  // sqrt(3)/2
  c2<T> t = cadd(v[1], v[2]);
  c2<T> u = csub(v[1], v[2]);
  c2<T> m = c2<T>{v[0].x - T(0.5) * t.x, v[0].y - T(0.5) * t.y};
  // forward: X1 = m - i s3 u, X2 = m + i s3 u
  c2<T> iu = INV ? c2<T>{-s3 * u.y, s3 * u.x} : c2<T>{s3 * u.y, -s3 * u.x};
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, iu);
  v[2] = csub(m, iu);
}

// 16 points as 4 x 4: length-4 DFTs over the samples n2 + 4 n1 (index k1),
// twiddles w^(n2 k1) with w = exp(-+ 2 pi i / 16), then length-4 DFTs over n2
// giving X_{k1 + 4 k2}.
template <typename T, bool INV> __device__ __forceinline__ void dft16(c2<T> *v) {
  c2<T> y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    y[n2][0] = v[n2];
    y[n2][1] = v[n2 + 4];
    y[n2][2] = v[n2 + 8];
    y[n2][3] = v[n2 + 12];
    dft4<T, INV>(y[n2]);
  }
  const T c = T(0.92387953251128675612818318939678829);  // cos(pi / 8)
  const T s = T(0.38268343236508977172845998403039887);  // sin(pi / 8)
  const T h = T(0.70710678118654752440084436210484904);
  const T sg = INV ? T(1) : T(-1);  // sign of the imaginary parts of w^m
  // w^m for m = n2 k1 in {1, 2, 3, 4, 6, 9}
  const c2<T> w1{c, sg * s}, w2{h, sg * h}, w3{s, sg * c}, w6{-h, sg * h}, w9{-c, -sg * s};
  y[1][1] = cmul(y[1][1], w1);
  y[1][2] = cmul(y[1][2], w2);
  y[1][3] = cmul(y[1][3], w3);
  y[2][1] = cmul(y[2][1], w2);
  y[2][2] = mul_mi<INV>(y[2][2]);  // w^4
  y[2][3] = cmul(y[2][3], w6);
  y[3][1] = cmul(y[3][1], w3);
  y[3][2] = cmul(y[3][2], w6);
  y[3][3] = cmul(y[3][3], w9);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    c2<T> b[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
    dft4<T, INV>(b);
    v[k1] = b[0];
    v[k1 + 4] = b[1];
    v[k1 + 8] = b[2];
    v[k1 + 12] = b[3];
  }
}

template <typename T, int R, bool INV> __device__ __forceinline__ void dft(c2<T> *v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 3) dft3<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else dft16<T, INV>(v);
}

// ---------------------------------------------------------------------------
// The pass loop (radix plan PLAN, TPF = N / its first radix threads per
// transform). `t` in [0, TPF) is this thread's lane within the transform,
// `c` the transform's slot in the workgroup, `lds` the workgroup's buffer and
// lidx(c, e) the LDS position of element e of slot c. load(e) supplies the
// first pass's inputs. For the last pass, fetch(e) is called for every output
// element before the butterflies (so that a caller's extra loads are all in
// flight while the pass computes) and store(e, v, aux) receives the output
// with what fetch returned. Every thread of the workgroup must call this (it
// contains barriers); threads of slots without data pass zeros through.
// ---------------------------------------------------------------------------
struct NoAux {};
struct NoFetch {
  __device__ NoAux operator()(int) const { return NoAux{}; }
};
struct NoPre {
  __device__ void operator()() const {}
};

// pre() runs once, in the first pass after its loads are issued and before its
// first barrier (callers use it to fill an LDS twiddle table that later passes
// read through `tw`: the first pass reads no twiddles)
template <typename T, int N, bool INV, int P = 0, int PLAN = 0, class LIdx, class Load, class Fetch, class Store,
          class Pre = NoPre>
__device__ __forceinline__ void fft_run(int t, int c, c2<T> *lds, const LIdx &lidx, const c2<T> *__restrict__ tw,
                                        const Load &load, const Fetch &fetch, const Store &store,
                                        const Pre &pre = Pre{}) {
  using C = c2<T>;
  constexpr int NP = npass_p<PLAN>(N);
  constexpr int R = radix_p<PLAN>(N, P);
  constexpr int NS = span_p<PLAN>(N, P);
  constexpr int TPF = N / radix_p<PLAN>(N, 0);
  constexpr int NB = N / R;                // butterflies in this pass
  constexpr int S = (NB + TPF - 1) / TPF;  // butterflies per thread
  constexpr bool EXACT = (S * TPF == NB);
  C v[S][R];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int j = t + s * TPF;
    if (EXACT || j < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = j + r * NB;
        if constexpr (P == 0) v[s][r] = load(e);
        else v[s][r] = lds[lidx(c, e)];
      }
    }
  }
  // this pass's twiddles, loaded with its data (before the barrier, which a
  // global load cannot cross)
  C w[S][R];
  if constexpr (NS > 1) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int j = t + s * TPF;
      if (EXACT || j < NB) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          w[s][r] = tw[r * k * (N / (NS * R))];
          if constexpr (INV) w[s][r].y = -w[s][r].y;
        }
      }
    }
  }
  if constexpr (P == NP - 1) {
    using Aux = decltype(fetch(0));
    Aux aux[S][R];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int j = t + s * TPF;
      if (EXACT || j < NB) {
#pragma unroll
        for (int r = 0; r < R; ++r) aux[s][r] = fetch(j + r * NB);
      }
    }
    if constexpr (P == 0) pre();
    __syncthreads();  // all reads of the buffer finish before it is rewritten
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int j = t + s * TPF;
      if (EXACT || j < NB) {
        if constexpr (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) v[s][r] = cmul(v[s][r], w[s][r]);
        }
        dft<T, R, INV>(v[s]);
      }
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int j = t + s * TPF;
      if (EXACT || j < NB) {
#pragma unroll
        for (int r = 0; r < R; ++r) store(j + r * NB, v[s][r], aux[s][r]);
      }
    }
  } else {
    if constexpr (P == 0) pre();
    __syncthreads();  // all reads of the buffer finish before it is rewritten
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int j = t + s * TPF;
      if (EXACT || j < NB) {
        const int k = j % NS;
        if constexpr (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) v[s][r] = cmul(v[s][r], w[s][r]);
        }
        dft<T, R, INV>(v[s]);
        const int base = (j / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lidx(c, base + r * NS)] = v[s][r];
      }
    }
    __syncthreads();
    fft_run<T, N, INV, P + 1, PLAN>(t, c, lds, lidx, tw, load, fetch, store);
  }
}

// LDS-to-LDS transform of slot c (rows kernels): no extra loads
template <typename T, int N, bool INV, class LIdx>
__device__ __forceinline__ void fft_lds(int t, int c, c2<T> *lds, const LIdx &lidx, const c2<T> *__restrict__ tw) {
  fft_run<T, N, INV>(
      t, c, lds, lidx, tw, [&](int e) -> c2<T> { return lds[lidx(c, e)]; }, NoFetch{},
      [&](int e, c2<T> v, NoAux) { lds[lidx(c, e)] = v; });
}

}  // namespace lbfft
