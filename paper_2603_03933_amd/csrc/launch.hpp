// launch.hpp - per-length launch table. Each supported FFT length N is compiled
// in its own translation unit (inst.hip with -DLB_N=N) into an NFuncs table
// for FP64 and FP32; the library picks tables by axis length at run time.
#pragma once
#include <hip/hip_ext.h>

#include "kernels.hpp"

namespace lb {
// Start/stop events of the enclosing timed scope (null when none). The next
// LB_LAUNCH consumes them: the runtime then records the kernel's own start and
// end, so the measured interval excludes launch gaps.
extern thread_local hipEvent_t kt_ev[2];
}  // namespace lb

#define LB_LAUNCH(K, G, B, SH, S, ...)                                \
  do {                                                                \
    hipEvent_t lb_e0_ = ::lb::kt_ev[0], lb_e1_ = ::lb::kt_ev[1];     \
    ::lb::kt_ev[0] = ::lb::kt_ev[1] = nullptr;                        \
    hipExtLaunchKernelGGL(K, G, B, SH, S, lb_e0_, lb_e1_, 0, __VA_ARGS__); \
  } while (0)

namespace lb {
using lbk::ColGeo;
using lbk::Geo;
using lbk::Prm;
using lbk::RowGeo;
using lbk::SubState;

struct PassArgs {
  hipStream_t stream = nullptr;
  int nblocks = 0;
  Geo g{};
  Prm p{};
  ColGeo cg{};
  RowGeo rg{};
  const void *tw = nullptr;
  const void *tw1 = nullptr;  // axis-1 twiddles (pair-split inverse pass)
  const void *in = nullptr;
  void *out = nullptr;
  void *out2 = nullptr;
  const double *psi = nullptr;
  const double *v = nullptr;
  const double *mpart = nullptr;
  int mbpi = 0;
  double *partial = nullptr;
  double *mom = nullptr;
  void *b0 = nullptr;
  void *b1 = nullptr;
  const void *gh = nullptr;
  SubState *st = nullptr;
  const void *gp = nullptr;
  double *gp64 = nullptr;
  float *gp32 = nullptr;
  double scale = 1.0, inv_n = 1.0, shift = 0.0;
  int zero_dc = 0;
  int keep_dc = 0;  // Hessian product: keep Lambda_0 (no projection)
  int step = 0;     // subproblem step index
  int fuse_t = -1;  // >= 1: the axis-0 inverse pass of step fuse_t first takes the multiplier step of fuse_t - 1
  long mstride = 0;  // stride between the moment partials' values (workgroups per instance x batch)
  int colv = 0;     // column-pass variant of the inner iteration's axis-0 passes (lbk::Cfg V)
};

struct NFuncs {
  int C = 0, NT = 0;  // transforms and threads per workgroup
  int colv_built = 1;  // bit V: the inner iteration's axis-0 passes built in column variant V
  int C3 = 0;          // columns per workgroup of column variant 3 (0: not built)
  void (*cols_plain)(const PassArgs &, bool inv) = nullptr;
  void (*cols_inv_scale_d)(const PassArgs &) = nullptr;
  void (*cols_fwd_update)(const PassArgs &) = nullptr;
  void (*cols_fwd_hess)(const PassArgs &) = nullptr;
  void (*cols_fwd_mul_inv)(const PassArgs &) = nullptr;
  void (*rows_r2c)(const PassArgs &, int mode) = nullptr;
  void (*rows_c2r)(const PassArgs &, int mode) = nullptr;
  void (*rows_inner)(const PassArgs &) = nullptr;
  void (*rows_energy)(const PassArgs &) = nullptr;  // FP64 tables only
  // plane passes for n1 = n_last = N (null when the plane does not fit in LDS)
  void (*plane_inner)(const PassArgs &, int n0) = nullptr;
  // the same pass with 256, 512 and 1024 threads (autotuner candidates; null where not built)
  void (*plane_inner_nt[3])(const PassArgs &, int n0) = {nullptr, nullptr, nullptr};
  // the split-plane pass (split order with 2 or 4 parts: index 0, 1) with
  // 256, 512 and 1024 threads, and the built-in thread count (null / -1
  // where it does not apply)
  void (*plane_split_nt[2][3])(const PassArgs &, int n0) = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  int plane_split_default[2] = {-1, -1};
  int plane_nt_default = 0;  // threads of plane_inner
  void (*plane_fwd_phys)(const PassArgs &, int n0) = nullptr;  // v -> out (+ Gamma' v partials)
  void (*plane_inv_phys)(const PassArgs &, int n0) = nullptr;  // in -> hv
  // the same two passes in the split order (2 or 4 workgroups per plane: index 0, 1)
  void (*plane_fwd_phys_split[2])(const PassArgs &, int n0) = {nullptr, nullptr};
  void (*plane_inv_phys_split[2])(const PassArgs &, int n0) = {nullptr, nullptr};
  // whole subproblem of one square 2D instance in one workgroup (null when it does not fit)
  void (*sub2d)(const PassArgs &) = nullptr;
};

template <typename T, int N> struct Impl {
  using C2 = lbfft::c2<T>;
  static constexpr int NT = lbk::Cfg<N>::NT;

  static void cols_plain(const PassArgs &a, bool inv) {
    lbk::OpPlain<T> op{(const C2 *)a.in, (C2 *)a.out, T(a.scale), a.zero_dc, a.g.nh, a.st};
    if (inv)
      LB_LAUNCH((lbk::k_cols<T, N, true, lbk::OpPlain<T>>), dim3(a.nblocks), dim3(NT), 0, a.stream, a.cg,
                         (const C2 *)a.tw, op);
    else
      LB_LAUNCH((lbk::k_cols<T, N, false, lbk::OpPlain<T>>), dim3(a.nblocks), dim3(NT), 0, a.stream, a.cg,
                         (const C2 *)a.tw, op);
  }
  // the ops below come in two forms: orthorhombic (|Bk|^2 without cross
  // terms, the benchmark's) and general lattice; a.g.general picks one
  // (a.cg.hsplit > 0: the split forms with a.cg.kparts parts that feed and
  // follow the split-plane pass)
  // column variants beyond V = 0 are built for the lengths the 3D inner
  // iteration uses most (64 .. 256) where they fit a workgroup
  template <int V> static constexpr bool COLV = V == 0 || (N >= 64 && N <= 256 && lbk::Cfg<N, V>::ok);
  // V = 3 (twice the columns of V = 0 per workgroup, same radix plan): the
  // inner iteration's axis-0 passes in one and two parts (runs of C/2
  // columns per part: 128 B in FP32 at 256^3)
  template <bool GEN, int KS, int V, bool FUSE> static void cols_inv_scale_d_f(const PassArgs &a) {
    lbk::OpInvScaleD<T, GEN, KS, FUSE> op{};
    op.g = a.g;
    op.p = a.p;
    op.b0 = (const C2 *)a.b0;
    op.b1 = (const C2 *)a.b1;
    op.out = (C2 *)a.out;
    op.st = a.st;
    op.twn = (const C2 *)a.tw1;
    op.t = a.step;
    op.tn = a.fuse_t;
    op.mom = a.mom;
    op.rpart = a.partial;
    op.mstride = a.mstride;
    op.nmb = a.cg.bpi;
    LB_LAUNCH((lbk::k_cols<T, N, true, lbk::OpInvScaleD<T, GEN, KS, FUSE>, V>), dim3(a.nblocks),
              dim3(lbk::Cfg<N, V>::NT), 0, a.stream, a.cg, (const C2 *)a.tw, op);
  }
  // fuse_t >= 1: the variant that first takes the multiplier step of fuse_t - 1
  template <bool GEN, int KS, int V> static void cols_inv_scale_d_t(const PassArgs &a) {
    if (a.fuse_t >= 1) cols_inv_scale_d_f<GEN, KS, V, true>(a);
    else cols_inv_scale_d_f<GEN, KS, V, false>(a);
  }
  template <bool GEN, int KS> static void cols_inv_scale_d_v(const PassArgs &a) {
    if constexpr (COLV<1>) {
      if (a.colv == 1) return cols_inv_scale_d_t<GEN, KS, 1>(a);
    }
    if constexpr (COLV<2>) {
      if (a.colv == 2) return cols_inv_scale_d_t<GEN, KS, 2>(a);
    }
    if constexpr (COLV<3> && KS <= 2) {
      if (a.colv == 3) return cols_inv_scale_d_t<GEN, KS, 3>(a);
    }
    cols_inv_scale_d_t<GEN, KS, 0>(a);
  }
  // four parts need 16 columns per workgroup (groups within rows of 16 lanes)
  static constexpr bool K4 = lbk::Cfg<N>::C == 16;
  template <bool GEN> static void cols_inv_scale_d_g(const PassArgs &a) {
    if (a.cg.hsplit && a.cg.kparts == 4) {
      if constexpr (K4) cols_inv_scale_d_v<GEN, 4>(a);
    } else if (a.cg.hsplit) {
      cols_inv_scale_d_v<GEN, 2>(a);
    } else {
      cols_inv_scale_d_v<GEN, 1>(a);
    }
  }
  static void cols_inv_scale_d(const PassArgs &a) {
    if (a.g.general) cols_inv_scale_d_g<true>(a);
    else cols_inv_scale_d_g<false>(a);
  }
  template <bool GEN, int KS, int V> static void cols_fwd_update_t(const PassArgs &a) {
    lbk::OpFwdUpdate<T, GEN, KS> op{};
    op.g = a.g;
    op.p = a.p;
    op.tmp = (const C2 *)a.in;
    op.b0 = (C2 *)a.b0;
    op.b1 = (C2 *)a.b1;
    op.gh = (const C2 *)a.gh;
    op.partial = a.partial;
    op.mom = a.mom;
    op.st = a.st;
    op.inv_n = a.inv_n;
    op.cpi = a.cg.cpi;
    op.t = a.step;
    LB_LAUNCH((lbk::k_cols<T, N, false, lbk::OpFwdUpdate<T, GEN, KS>, V>), dim3(a.nblocks),
              dim3(lbk::Cfg<N, V>::NT), 0, a.stream, a.cg, (const C2 *)a.tw, op);
  }
  template <bool GEN, int KS> static void cols_fwd_update_v(const PassArgs &a) {
    if constexpr (COLV<1>) {
      if (a.colv == 1) return cols_fwd_update_t<GEN, KS, 1>(a);
    }
    if constexpr (COLV<2>) {
      if (a.colv == 2) return cols_fwd_update_t<GEN, KS, 2>(a);
    }
    if constexpr (COLV<3> && KS <= 2) {
      if (a.colv == 3) return cols_fwd_update_t<GEN, KS, 3>(a);
    }
    cols_fwd_update_t<GEN, KS, 0>(a);
  }
  template <bool GEN> static void cols_fwd_update_g(const PassArgs &a) {
    if (a.cg.hsplit && a.cg.kparts == 4) {
      if constexpr (K4) cols_fwd_update_v<GEN, 4>(a);
    } else if (a.cg.hsplit) {
      cols_fwd_update_v<GEN, 2>(a);
    } else {
      cols_fwd_update_v<GEN, 1>(a);
    }
  }
  static void cols_fwd_update(const PassArgs &a) {
    if (a.g.general) cols_fwd_update_g<true>(a);
    else cols_fwd_update_g<false>(a);
  }
  template <bool GEN> static void cols_fwd_hess_t(const PassArgs &a) {
    lbk::OpFwdHess<T, GEN> op{};
    op.g = a.g;
    op.p = a.p;
    op.tmp = (const C2 *)a.in;
    op.x = (const C2 *)a.gh;
    op.out = (C2 *)a.out;
    op.inv_n = a.inv_n;
    op.shift = a.shift;
    LB_LAUNCH((lbk::k_cols<T, N, false, lbk::OpFwdHess<T, GEN>>), dim3(a.nblocks), dim3(NT), 0, a.stream, a.cg,
              (const C2 *)a.tw, op);
  }
  static void cols_fwd_hess(const PassArgs &a) {
    if (a.g.general) cols_fwd_hess_t<true>(a);
    else cols_fwd_hess_t<false>(a);
  }
  template <bool GEN, int KS> static void cols_fwd_mul_inv_t(const PassArgs &a) {
    LB_LAUNCH((lbk::k_cols_fwd_mul_inv<T, N, GEN, KS>), dim3(a.nblocks), dim3(NT), 0, a.stream, a.cg, a.g, a.p,
              (const C2 *)a.tw, (C2 *)a.out, a.inv_n, a.keep_dc, (const C2 *)a.tw1);
  }
  template <bool GEN> static void cols_fwd_mul_inv_g(const PassArgs &a) {
    if (a.cg.hsplit && a.cg.kparts == 4) {
      if constexpr (K4) cols_fwd_mul_inv_t<GEN, 4>(a);
    } else if (a.cg.hsplit) {
      cols_fwd_mul_inv_t<GEN, 2>(a);
    } else {
      cols_fwd_mul_inv_t<GEN, 1>(a);
    }
  }
  static void cols_fwd_mul_inv(const PassArgs &a) {
    if (a.g.general) cols_fwd_mul_inv_g<true>(a);
    else cols_fwd_mul_inv_g<false>(a);
  }

  static void rows_r2c(const PassArgs &a, int mode) {
    if (mode == 1)
      LB_LAUNCH((lbk::k_rows_r2c<T, N, 1>), dim3(a.nblocks), dim3(NT), 0, a.stream, a.rg, a.g, a.p,
                         (const C2 *)a.tw, (const double *)a.in, a.psi, (C2 *)a.out, a.partial);
    else
      LB_LAUNCH((lbk::k_rows_r2c<T, N, 0>), dim3(a.nblocks), dim3(NT), 0, a.stream, a.rg, a.g, a.p,
                         (const C2 *)a.tw, (const double *)a.in, a.psi, (C2 *)a.out, a.partial);
  }
  static void rows_c2r(const PassArgs &a, int mode) {
    if (mode == 1)
      LB_LAUNCH((lbk::k_rows_c2r<T, N, 1>), dim3(a.nblocks), dim3(NT), 0, a.stream, a.rg, a.g, a.p,
                         (const C2 *)a.tw, (const C2 *)a.in, (double *)a.out, a.psi, a.v, a.mpart, a.mbpi, a.partial, a.scale);
    else if (mode == 2)
      LB_LAUNCH((lbk::k_rows_c2r<T, N, 2>), dim3(a.nblocks), dim3(NT), 0, a.stream, a.rg, a.g, a.p,
                         (const C2 *)a.tw, (const C2 *)a.in, (double *)a.out, a.psi, a.v, a.mpart, a.mbpi, a.partial, a.scale);
    else
      LB_LAUNCH((lbk::k_rows_c2r<T, N, 0>), dim3(a.nblocks), dim3(NT), 0, a.stream, a.rg, a.g, a.p,
                         (const C2 *)a.tw, (const C2 *)a.in, (double *)a.out, a.psi, a.v, a.mpart, a.mbpi, a.partial, a.scale);
  }
  static void rows_inner(const PassArgs &a) {
    LB_LAUNCH((lbk::k_rows_inner<T, N>), dim3(a.nblocks), dim3(NT), 0, a.stream, a.rg, (const C2 *)a.tw,
                       (C2 *)a.out, (const T *)a.gp, (const SubState *)a.st);
  }
  static void rows_energy(const PassArgs &a) {
    if constexpr (std::is_same<T, double>::value)
      LB_LAUNCH((lbk::k_rows_energy<N>), dim3(a.nblocks), dim3(NT), 0, a.stream, a.rg, a.g, a.p,
                         (const double2 *)a.tw, a.psi, (double2 *)a.out, (double2 *)a.out2, a.gp64, a.gp32, a.partial);
  }

  static void plane_inner(const PassArgs &a, int n0) {
    if constexpr (lbk::PlaneCfg<T, N>::fits)
      LB_LAUNCH((lbk::k_plane_inner<T, N>), dim3(n0 * a.g.batch), dim3(lbk::PlaneCfg<T, N>::NT), 0, a.stream,
                         n0, a.g.nh, a.g.N, (const C2 *)a.tw, (C2 *)a.out, (const T *)a.gp, (const SubState *)a.st);
  }

  template <int NTV> static void plane_inner_nt(const PassArgs &a, int n0) {
    if constexpr (lbk::PlaneCfg<T, N>::fits)
      LB_LAUNCH((lbk::k_plane_inner<T, N, NTV>), dim3(n0 * a.g.batch), dim3(NTV), 0, a.stream, n0, a.g.nh, a.g.N,
                (const C2 *)a.tw, (C2 *)a.out, (const T *)a.gp, (const SubState *)a.st);
  }
  template <int K, int NTV> static void plane_split_nt(const PassArgs &a, int n0) {
    if constexpr (lbk::SplitCfg<T, N, K>::fits)
      LB_LAUNCH((lbk::k_plane_inner_split<T, N, K, NTV>), dim3(K * n0 * a.g.batch), dim3(NTV), 0, a.stream, n0,
                a.g.nh, a.g.N, (const C2 *)a.tw, (C2 *)a.out, (const T *)a.gp, (const SubState *)a.st);
  }
  static void plane_fwd_phys(const PassArgs &a, int n0) {
    if constexpr (lbk::PlaneCfg<T, N>::fits)
      LB_LAUNCH((lbk::k_plane_fwd_phys<T, N>), dim3(n0 * a.g.batch), dim3(lbk::PlaneCfg<T, N>::NT), 0, a.stream, n0,
                a.g.nh, a.g.N, a.p, (const C2 *)a.tw, a.v, a.psi, (C2 *)a.out, a.partial);
  }
  template <int K> static void plane_fwd_phys_split(const PassArgs &a, int n0) {
    if constexpr (lbk::SplitCfg<T, N, K>::fits)
      LB_LAUNCH((lbk::k_plane_fwd_phys_split<T, N, K>), dim3(K * n0 * a.g.batch), dim3(lbk::SplitCfg<T, N, K>::NT), 0,
                a.stream, n0, a.g.nh, a.g.N, a.p, (const C2 *)a.tw, a.v, a.psi, (C2 *)a.out, a.partial);
  }
  template <int K> static void plane_inv_phys_split(const PassArgs &a, int n0) {
    if constexpr (lbk::SplitCfg<T, N, K>::fits)
      LB_LAUNCH((lbk::k_plane_inv_phys_split<T, N, K>), dim3(K * n0 * a.g.batch), dim3(lbk::SplitCfg<T, N, K>::NT), 0,
                a.stream, n0, a.g.nh, a.g.N, a.p, (const C2 *)a.tw, (const C2 *)a.in, a.psi, a.v, a.mpart,
                (double *)a.out, a.scale);
  }
  static void plane_inv_phys(const PassArgs &a, int n0) {
    if constexpr (lbk::PlaneCfg<T, N>::fits)
      LB_LAUNCH((lbk::k_plane_inv_phys<T, N>), dim3(n0 * a.g.batch), dim3(lbk::PlaneCfg<T, N>::NT), 0, a.stream, n0,
                a.g.nh, a.g.N, a.p, (const C2 *)a.tw, (const C2 *)a.in, a.psi, a.v, a.mpart, (double *)a.out, a.scale);
  }

  // the whole subproblem in one workgroup: up to N = 64 (beyond, the butterflies
  // and the update no longer fit in registers together, nor b, g and Gamma' in
  // LDS beside the plane)
  static constexpr bool SUB2D = lbk::PlaneCfg<T, N>::fits && lbk::Sub2dCfg<T, N>::fits;
  static void sub2d(const PassArgs &a) {
    if constexpr (SUB2D)
      LB_LAUNCH((lbk::k_sub2d<T, N>), dim3(a.g.batch), dim3(lbk::PlaneCfg<T, N>::NT), 0, a.stream, a.g, a.p, (const C2 *)a.tw,
                (C2 *)a.b0, (C2 *)a.b1, (const C2 *)a.gh, (const T *)a.gp, a.st);
  }

  // the split kernels with K parts: thread-count variants where the whole
  // plane pass has them (n <= 128), else the built-in count only
  template <int K> static void fill_split(NFuncs &f, int ki) {
    if constexpr (lbk::SplitCfg<T, N, K>::fits) {
      constexpr int D = lbk::SplitCfg<T, N, K>::NT;
      constexpr int di = D == 256 ? 0 : D == 512 ? 1 : 2;
      if constexpr (N <= 128) {
        f.plane_split_nt[ki][0] = &plane_split_nt<K, 256>;
        f.plane_split_nt[ki][1] = &plane_split_nt<K, 512>;
        f.plane_split_nt[ki][2] = &plane_split_nt<K, 1024>;
      } else {
        f.plane_split_nt[ki][di] = &plane_split_nt<K, D>;
      }
      f.plane_split_default[ki] = di;
      f.plane_fwd_phys_split[ki] = &plane_fwd_phys_split<K>;
      f.plane_inv_phys_split[ki] = &plane_inv_phys_split<K>;
    }
  }
  static NFuncs table() {
    NFuncs f;
    f.C = lbk::Cfg<N>::C;
    f.NT = NT;
    f.colv_built = 1 | (COLV<1> ? 2 : 0) | (COLV<2> ? 4 : 0) | (COLV<3> ? 8 : 0);
    f.C3 = COLV<3> ? lbk::Cfg<N, 3>::C : 0;
    f.cols_plain = &cols_plain;
    f.cols_inv_scale_d = &cols_inv_scale_d;
    f.cols_fwd_update = &cols_fwd_update;
    f.cols_fwd_hess = &cols_fwd_hess;
    f.cols_fwd_mul_inv = &cols_fwd_mul_inv;
    f.rows_r2c = &rows_r2c;
    f.rows_c2r = &rows_c2r;
    f.rows_inner = &rows_inner;
    f.rows_energy = std::is_same<T, double>::value ? &rows_energy : nullptr;
    f.plane_inner = lbk::PlaneCfg<T, N>::fits ? &plane_inner : nullptr;
    if constexpr (lbk::PlaneCfg<T, N>::fits && N >= 64) {
      f.plane_inner_nt[0] = &plane_inner_nt<256>;
      f.plane_inner_nt[1] = &plane_inner_nt<512>;
      f.plane_inner_nt[2] = &plane_inner_nt<1024>;
    }
    fill_split<2>(f, 0);
    fill_split<4>(f, 1);
    f.plane_nt_default = lbk::PlaneCfg<T, N>::fits ? lbk::PlaneCfg<T, N>::NT : 0;
    f.plane_fwd_phys = lbk::PlaneCfg<T, N>::fits ? &plane_fwd_phys : nullptr;
    f.plane_inv_phys = lbk::PlaneCfg<T, N>::fits ? &plane_inv_phys : nullptr;

    f.sub2d = SUB2D ? &sub2d : nullptr;
    return f;
  }
};

// Defined once per supported length by inst.hip; prec is LB_FP64 or LB_FP32.
#define LB_FOR_EACH_LENGTH(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)
#define LB_DECLARE_TABLE(n) const NFuncs *funcs_##n(int prec);
LB_FOR_EACH_LENGTH(LB_DECLARE_TABLE)
#undef LB_DECLARE_TABLE

}  // namespace lb
