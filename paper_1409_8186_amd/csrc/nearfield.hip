// Near field (paper sec. 4.4, by Graf's addition theorem): at a point x of the
// propagation domain, with (r_p, theta_p) the polar coordinates of x - O_p,
//   u(x) = sum_p sum_m (i sqrt(pi / 8)) F^p_m rho^p_m H_m(k r_p) e^{i m theta_p},
// F^p_m = sqrt(a_p) J_m(k a_p) for the single-layer potential; for an operator
// set by mudiff_set_operator, F = f_L sqrt(a) J_m - f_M k sqrt(a) J'_m (its
// far-field weights: single- plus double-layer potential).  The total field
// adds the incident plane wave.  Points inside a disk get 0.
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

__global__ __launch_bounds__(NF_THREADS) void k_nearfield(DevView v, int R, const cplx* __restrict__ rho,
                                                          int n_pts, const double* __restrict__ pts,
                                                          const double* __restrict__ beta,
                                                          cplx* __restrict__ out) {
  const int P = blockIdx.x * NF_THREADS + threadIdx.x;
  const int nchunk = (R + NF_RC - 1) / NF_RC;
  const int b = blockIdx.y / nchunk;
  const int r0 = (blockIdx.y - b * nchunk) * NF_RC;
  const int nr = min(NF_RC, R - r0);
  const double x1 = P < n_pts ? pts[2 * P] : 0.0, x2 = P < n_pts ? pts[2 * P + 1] : 0.0;
  const double k = v.kd[v.idisk[b]];
  const double cst = 0.62665706865775012560;  // sqrt(pi / 8): (i pi a / 2) / sqrt(2 pi a) = i sqrt(pi/8) sqrt(a)
  cplx acc[NF_RC];
#pragma unroll
  for (int c = 0; c < NF_RC; ++c) acc[c] = cmk(0.0, 0.0);
  bool inside = false;
  for (int64_t p = v.idisk[b]; p < v.idisk[b + 1]; ++p) {
    const double dx = x1 - v.cx[p], dy = x2 - v.cy[p];
    const double r2 = dx * dx + dy * dy;
    const double ap = v.a[p];
    const int Np = v.N[p];
    const int64_t i0 = v.imode[b] + v.moff[p] + Np;  // unknown of mode 0
    if (r2 < ap * ap) {
      inside = true;
      continue;
    }
    const double r = sqrt(r2);
    const double xx = k * r;
    cplx H0, H1;
    hankel01(xx, &H0, &H1);
    const cplx e1 = cmk(dx / r, dy / r);  // e^{i theta_p}
    // coefficient (i sqrt(pi/8)) F rho of mode m, column c
    auto coef = [&](int m, int c) {
      const int64_t i = i0 + m;
      const cplx F = v.op_ff ? v.op_ff[i] : cmk(v.sJ[i], 0.0);
      const cplx rv = rho[col_base(v.imode, b, R, r0 + c) + v.moff[p] + Np + m];
      const cplx t = cmul(F, rv);
      return cmk(-cst * t.y, cst * t.x);
    };
#pragma unroll
    for (int c = 0; c < NF_RC; ++c)
      if (c < nr) cmac(acc[c], coef(0, c), H0);
    cplx Hm1 = H0, Hm = H1, em = e1;
    for (int m = 1; m <= Np; ++m) {
      if (m >= 2) {
        const cplx Hn = csub(cscale(Hm, 2.0 * (m - 1) / xx), Hm1);
        Hm1 = Hm;
        Hm = Hn;
        em = cmul(em, e1);
      }
      const cplx tp = cmul(Hm, em);                       // H_m e^{i m theta}
      cplx tm = cmul(Hm, cconj(em));                      // H_{-m} e^{-i m theta} = (-1)^m H_m e^{-i m theta}
      if (m & 1) tm = cmk(-tm.x, -tm.y);
#pragma unroll
      for (int c = 0; c < NF_RC; ++c)
        if (c < nr) {
          cmac(acc[c], coef(m, c), tp);
          cmac(acc[c], coef(-m, c), tm);
        }
    }
  }
  if (P >= n_pts) return;
#pragma unroll
  for (int c = 0; c < NF_RC; ++c) {
    if (c >= nr) continue;
    const int col = b * R + r0 + c;
    cplx u = acc[c];
    if (beta) {
      double sb, cb;
      sincos(beta[col], &sb, &cb);
      u = cadd(u, cexpi(k * (cb * x1 + sb * x2)));
    }
    out[(int64_t)col * n_pts + P] = inside ? cmk(0.0, 0.0) : u;
  }
}

}  // namespace

extern "C" int mudiff_nearfield(mudiff_t h, int R, const void* rho, int n_pts, const double* pts,
                                const double* beta, void* out, void* stream) {
  if (!h || !rho || !pts || !out) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  if (R < 1 || n_pts < 1) return fail(MUDIFF_ERR_INVALID, "R < 1 or n_pts < 1");
  const int nchunk = (R + NF_RC - 1) / NF_RC;
  if ((int64_t)h->B * nchunk > 65535) return fail(MUDIFF_ERR_INVALID, "too many instance x RHS columns");
  dim3 grid((unsigned)((n_pts + NF_THREADS - 1) / NF_THREADS), (unsigned)(h->B * nchunk));
  hipLaunchKernelGGL(k_nearfield, grid, dim3(NF_THREADS), 0, (hipStream_t)stream, h->dv, R,
                     (const cplx*)rho, n_pts, pts, beta, (cplx*)out);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}
