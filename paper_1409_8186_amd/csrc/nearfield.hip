// Near field (paper sec. 4.4, by Graf's addition theorem): at a point x of the
// propagation domain, with (r_p, theta_p) the polar coordinates of x - O_p,
//   u(x) = sum_p sum_m (i sqrt(pi / 8)) F^p_m rho^p_m H_m(k r_p) e^{i m theta_p},
// F^p_m = sqrt(a_p) J_m(k a_p) for the single-layer potential; for an operator
// set by mudiff_set_operator, F = f_L sqrt(a) J_m - f_M k sqrt(a) J'_m (its
// far-field weights: single- plus double-layer potential).  The total field
// adds the incident wave: the plane wave e^{i k beta_hat . x}, or for a point
// source s (Prop. 5) G(x, s) = (i/4) H_0(k |x - s|).  Points inside a disk get 0.
//
// One thread per point, every thread walking the same disks (so the disk data
// and the coefficients are wave-uniform loads); per (point, disk): H_0, H_1 of
// k r_p (Miller + Neumann series below 25, Hankel's expansion above), H_m by
// upward recurrence (stable for the Y part that dominates), e^{i m theta} by
// recurrence, and the mode sum for up to NF_RC right-hand sides at once.
#include "bessel.h"
#include "common.h"

namespace {

constexpr int NF_THREADS = 256;
constexpr int NF_RC = 4;

// Hankel's large-argument expansion of H_0, H_1 (DLMF 10.17.5) with a fixed
// number of terms by range: the k-th term is prod_{j<=k} (4 nu^2 - (2j-1)^2) /
// (8 j x) times the first, below 3e-17 at x = 25 for k = 18, at x = 50 for
// k = 12 and at x = 100 for k = 9 (nu = 0, 1).  Same phase handling as the
// table code: e^{ix} from sincos of the exact argument.  ix = 1 / x; the
// per-term factors (4 nu^2 - (2j-1)^2) / (8 j) are compile-time constants, so
// a term costs multiplications only.
template <int K>
__device__ __forceinline__ void hankel01_series(double ixx, cplx* s0, cplx* s1) {
  cplx t0 = cmk(1.0, 0.0), t1 = cmk(1.0, 0.0);
  cplx a0 = t0, a1 = t1;
#pragma unroll
  for (int kk = 1; kk <= K; ++kk) {
    const double q = (2.0 * kk - 1.0) * (2.0 * kk - 1.0);
    constexpr double e8 = 0.125;
    const double f0 = (-q * e8 / kk) * ixx, f1 = ((4.0 - q) * e8 / kk) * ixx;
    t0 = cmk(-t0.y * f0, t0.x * f0);  // * i * f
    t1 = cmk(-t1.y * f1, t1.x * f1);
    a0 = cadd(a0, t0);
    a1 = cadd(a1, t1);
  }
  *s0 = a0;
  *s1 = a1;
}

// H_0(x), H_1(x) given x and ixx = 1 / x.
__device__ __forceinline__ void hankel01_near(double x, double ixx, cplx* H0, cplx* H1) {
  if (x < BESSEL_X_ASY) {
    hankel01(x, H0, H1);
    return;
  }
  cplx s0, s1;
  if (x >= 100.0) hankel01_series<10>(ixx, &s0, &s1);
  else if (x >= 50.0) hankel01_series<13>(ixx, &s0, &s1);
  else hankel01_series<19>(ixx, &s0, &s1);
  const double r2 = 0.70710678118654752440;
  double sn, cs;
  sincos(x, &sn, &cs);
  const double amp = sqrt(0.63661977236758134308 * ixx);  // sqrt(2 / (pi x))
  const cplx e = cmk(amp * cs, amp * sn);
  *H0 = cmul(cmul(e, cmk(r2, -r2)), s0);   // e^{-i pi/4}
  *H1 = cmul(cmul(e, cmk(-r2, -r2)), s1);  // e^{-3 i pi/4}
}

__device__ __forceinline__ void hankel01_near(double x, cplx* H0, cplx* H1) {
  hankel01_near(x, 1.0 / x, H0, H1);
}

__global__ __launch_bounds__(NF_THREADS) void k_nearfield(DevView v, int R, const cplx* __restrict__ rho,
                                                          int n_pts, const double* __restrict__ pts,
                                                          const double* __restrict__ beta,
                                                          int point, cplx* __restrict__ out) {
  // coefficients (i sqrt(pi/8)) F rho of the current disk: [2 N_p + 1][NF_RC]
  __shared__ cplx cf[(2 * MUDIFF_MAX_NP + 1) * NF_RC];
  const int P = blockIdx.x * NF_THREADS + threadIdx.x;
  const int nchunk = (R + NF_RC - 1) / NF_RC;
  const int b = blockIdx.y / nchunk;
  const int r0 = (blockIdx.y - b * nchunk) * NF_RC;
  const int nr = min(NF_RC, R - r0);
  const double x1 = P < n_pts ? pts[2 * P] : 0.0, x2 = P < n_pts ? pts[2 * P + 1] : 0.0;
  const double k = v.kd[v.idisk[b]];
  const double ik = 1.0 / k;
  const double cst = 0.62665706865775012560;  // sqrt(pi / 8): (i pi a / 2) / sqrt(2 pi a) = i sqrt(pi/8) sqrt(a)
  cplx acc[NF_RC];
#pragma unroll
  for (int c = 0; c < NF_RC; ++c) acc[c] = cmk(0.0, 0.0);
  bool inside = false;
  for (int64_t p = v.idisk[b]; p < v.idisk[b + 1]; ++p) {
    const int Np = v.N[p];
    const int n = 2 * Np + 1;
    const int64_t i0 = v.imode[b] + v.moff[p];  // unknown of mode -N_p
    __syncthreads();  // the previous disk's coefficients are no longer read
    for (int e = threadIdx.x; e < n * NF_RC; e += NF_THREADS) {
      const int mi = e / NF_RC, c = e - mi * NF_RC;
      cplx t = cmk(0.0, 0.0);
      if (c < nr) {
        const cplx F = v.op_ff ? v.op_ff[i0 + mi] : cmk(v.sJ[i0 + mi], 0.0);
        t = cmul(F, rho[col_base(v.imode, b, R, r0 + c) + v.moff[p] + mi]);
      }
      cf[e] = cmk(-cst * t.y, cst * t.x);
    }
    __syncthreads();
    const double dx = x1 - v.cx[p], dy = x2 - v.cy[p];
    const double r2 = dx * dx + dy * dy;
    const double ap = v.a[p];
    if (r2 < ap * ap) {
      inside = true;
      continue;
    }
    const double r = sqrt(r2);   // correctly rounded: the phase of e^{i k r} rests on it
    const double ir = rsqrt(r2);  // 1 / r, and 1 / (k r) below, with no division
    const double xx = k * r;
    const double ixx = ik * ir;
    const double tox = 2.0 * ixx;  // the recurrence factor 2 (m - 1) / x is (m - 1) tox
    cplx H0, H1;
    hankel01_near(xx, ixx, &H0, &H1);
    const cplx e1 = cmk(dx * ir, dy * ir);  // e^{i theta_p}
    const cplx* c0 = cf + Np * NF_RC;     // mode 0
#pragma unroll
    for (int c = 0; c < NF_RC; ++c)
      if (c < nr) cmac(acc[c], c0[c], H0);
    cplx Hm1 = H0, Hm = H1, em = e1;
    for (int m = 1; m <= Np; ++m) {
      if (m >= 2) {
        const cplx Hn = csub(cscale(Hm, (m - 1) * tox), Hm1);
        Hm1 = Hm;
        Hm = Hn;
        em = cmul(em, e1);
      }
      // H_{-m} e^{-i m theta} = (-1)^m H_m e^{-i m theta}: both modes take
      // (c_m e^{i m theta} + (-1)^m c_{-m} e^{-i m theta}) H_m
      const cplx emc = (m & 1) ? cmk(-em.x, em.y) : cconj(em);
#pragma unroll
      for (int c = 0; c < NF_RC; ++c)
        if (c < nr) {
          cplx t = cmul(c0[m * NF_RC + c], em);
          cmac(t, c0[-m * NF_RC + c], emc);
          cmac(acc[c], t, Hm);
        }
    }
  }
  if (P >= n_pts) return;
#pragma unroll
  for (int c = 0; c < NF_RC; ++c) {
    if (c >= nr) continue;
    const int col = b * R + r0 + c;
    cplx u = acc[c];
    if (beta && point) {
      const double dx = x1 - beta[2 * col], dy = x2 - beta[2 * col + 1];
      cplx H0, H1;
      hankel01_near(k * sqrt(dx * dx + dy * dy), &H0, &H1);
      u = cadd(u, cmk(-0.25 * H0.y, 0.25 * H0.x));
    } else if (beta) {
      double sb, cb;
      sincos(beta[col], &sb, &cb);
      u = cadd(u, cexpi(k * (cb * x1 + sb * x2)));
    }
    out[(int64_t)col * n_pts + P] = inside ? cmk(0.0, 0.0) : u;
  }
}

}  // namespace

extern "C" int mudiff_nearfield(mudiff_t h, int R, const void* rho, int n_pts, const double* pts,
                                const double* beta, int flags, void* out, void* stream) {
  if (!h || !rho || !pts || !out) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  if (flags & ~MUDIFF_POINT_SOURCE) return fail(MUDIFF_ERR_INVALID, "unknown flags");
  if (R < 1 || n_pts < 1) return fail(MUDIFF_ERR_INVALID, "R < 1 or n_pts < 1");
  const int nchunk = (R + NF_RC - 1) / NF_RC;
  if ((int64_t)h->B * nchunk > 65535) return fail(MUDIFF_ERR_INVALID, "too many instance x RHS columns");
  dim3 grid((unsigned)((n_pts + NF_THREADS - 1) / NF_THREADS), (unsigned)(h->B * nchunk));
  hipLaunchKernelGGL(k_nearfield, grid, dim3(NF_THREADS), 0, (hipStream_t)stream, h->dv, R,
                     (const cplx*)rho, n_pts, pts, beta, (flags & MUDIFF_POINT_SOURCE) ? 1 : 0,
                     (cplx*)out);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}
