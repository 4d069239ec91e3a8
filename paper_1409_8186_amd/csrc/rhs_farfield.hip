// Plane-wave right-hand side (paper Prop. 4) and far field (paper sec. 4.4).
//
//   U^p_m(beta) = sqrt(2 pi a_p) e^{i k beta_hat . O_p} e^{i m (pi/2 - beta)} J_m(k a_p)
//   f = -D^{-1} U = (2 i / pi) sqrt(2 pi) e^{i k beta_hat . O_p} e^{i m (pi/2 - beta)}
//                   / (sqrt(a_p) H_m(k a_p))             (J_m cancels)
//   a(theta) = sum_p sum_m g^p_m(theta) rho^p_m,
//   g^p_m(theta) = (e^{i pi/4} / (2 sqrt k)) e^{-i k theta_hat . O_p}
//                  sqrt(a_p) J_m(k a_p) e^{i m (theta - pi/2)}
//
// Point source s (Prop. 5): the same with the incident factor
//   e = (i/4) H_m(k r_p) e^{-i m theta_p}  (r_p, theta_p: polar coordinates of s - O_p)
// in place of e^{i k beta_hat . O_p} e^{i m (pi/2 - beta)}, so that
// U = sqrt(2 pi a) J_m e as for the plane wave.
#include "bessel.h"
#include "common.h"

#define PI_D 3.14159265358979323846

// (i/4) H_m(k r) e^{-i m theta} of the source at src relative to disk p; NaN if
// the source is not outside the disk (the expansion needs r > a).
__device__ cplx point_factor(const DevView& v, int p, int m, const double* src) {
  const double dx = src[0] - v.cx[p], dy = src[1] - v.cy[p];
  const double r = sqrt(dx * dx + dy * dy);
  if (!(r > v.a[p])) return cmk(__builtin_nan(""), __builtin_nan(""));
  const double x = v.kd[p] * r;
  cplx Hm1, Hm;
  hankel01(x, &Hm1, &Hm);  // H_0, H_1
  const int am = m < 0 ? -m : m;
  if (am == 0) Hm = Hm1;
  for (int n = 1; n < am; ++n) {  // upward recurrence (stable: Y_n grows)
    const cplx Hn = csub(cscale(Hm, 2.0 * n / x), Hm1);
    Hm1 = Hm;
    Hm = Hn;
  }
  if (m < 0 && (am & 1)) Hm = cscale(Hm, -1.0);  // H_{-m} = (-1)^m H_m
  const cplx t = cmul(Hm, cexpi(-m * atan2(dy, dx)));
  return cmk(-0.25 * t.y, 0.25 * t.x);
}

// one thread per unknown of every (instance, rhs) column; `point`: beta holds
// source positions [B][R][2]; precond 0: U (or an operator's b), 1: the
// preconditioned b, 2: b (-U for the single layer)
__global__ void k_rhs(DevView v, int R, const double* __restrict__ beta, cplx* __restrict__ out,
                      int precond, int point) {
  const int64_t total = (int64_t)R * v.N_all;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  // instance: R * imode[b] <= g < R * imode[b+1]
  int lo = 0, hi = v.B;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if ((int64_t)R * v.imode[mid] <= g) lo = mid; else hi = mid;
  }
  const int b = lo;
  const int64_t Nb = v.imode[b + 1] - v.imode[b];
  const int64_t rem = g - (int64_t)R * v.imode[b];
  const int r = (int)(rem / Nb);
  const int64_t il = rem - (int64_t)r * Nb;
  const int64_t i = v.imode[b] + il;
  const int p = v.udisk[i];
  const int m = (int)(il - v.moff[p]) - v.N[p];
  cplx e;
  if (point) {
    e = point_factor(v, p, m, beta + 2 * ((int64_t)b * R + r));
  } else {
    const double be = beta[b * R + r];
    const double kk = v.kd[p];
    double sb, cb;
    sincos(be, &sb, &cb);
    const cplx e1 = cexpi(kk * (cb * v.cx[p] + sb * v.cy[p]));
    const cplx e2 = cexpi(m * (0.5 * PI_D - be));
    e = cmul(e1, e2);
  }
  const double s2pi = sqrt(2.0 * PI_D);
  if (v.op_rhs) {  // operator set by mudiff_set_operator: w_U U + w_dU dU (over its diagonal)
    out[g] = cmul(e, precond == 1 ? v.op_rhsp[i] : v.op_rhs[i]);
    return;
  }
  if (precond == 2) {  // the unpreconditioned system's right-hand side -U
    out[g] = cscale(e, -s2pi * v.sJ[i]);
    return;
  }
  if (precond) {
    const cplx w = cmul(e, v.invSH[i]);
    const double c = 2.0 / PI_D * s2pi;
    out[g] = cmk(-c * w.y, c * w.x);  // (2i/pi) sqrt(2 pi) e / (sqrt(a) H)
  } else {
    out[g] = cscale(e, s2pi * v.sJ[i]);
  }
}

int launch_rhs(mudiff_ctx* h, int R, const double* beta, cplx* out, int precond, int point,
               hipStream_t s) {
  const int64_t total = (int64_t)R * h->N_all;
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, h->dv, R, beta,
                     out, precond, point);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}

extern "C" int mudiff_rhs(mudiff_t h, int R, const double* beta, void* out, int precond,
                          void* stream) {
  if (!h || !beta || !out) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  if (R < 1) return fail(MUDIFF_ERR_INVALID, "R < 1");
  return launch_rhs(h, R, beta, (cplx*)out, precond ? 1 : 0, 0, (hipStream_t)stream);
}

extern "C" int mudiff_rhs_point(mudiff_t h, int R, const double* src, void* out, int precond,
                                void* stream) {
  if (!h || !src || !out) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  if (R < 1) return fail(MUDIFF_ERR_INVALID, "R < 1");
  return launch_rhs(h, R, src, (cplx*)out, precond ? 1 : 0, 1, (hipStream_t)stream);
}

// Far field.  Workgroup = (column, tile of FF_TH angles); its FF_DG thread
// groups split the disks of the instance (thread t: angle t % FF_TH of the
// tile, disks g, g + FF_DG, ... with g = t / FF_TH), then the group sums are
// added in LDS in a fixed order.  Small tiles and many groups keep a
// one-column call (720 angles x 400 disks) spread over the chip; instances of
// few disks take wide tiles and few groups (16 x 64 or 64 x 16 threads).
template <int FF_TH, int FF_DG>
__global__ __launch_bounds__(FF_TH* FF_DG) void k_farfield(DevView v, int R,
                                                           const cplx* __restrict__ rho,
                                                           int n_theta,
                                                           const double* __restrict__ theta,
                                                           cplx* __restrict__ a_out) {
  __shared__ cplx red[FF_DG][FF_TH];
  const int col = blockIdx.y;  // b * R + r
  const int b = col / R, r = col - (col / R) * R;
  const int tj = threadIdx.x % FF_TH, dg = threadIdx.x / FF_TH;
  const int j = blockIdx.x * FF_TH + tj;
  const double th = j < n_theta ? theta[j] : 0.0;
  const double kk = v.kd[v.idisk[b]];
  const cplx* rc = rho + col_base(v.imode, b, R, r);
  double st, ct;
  sincos(th, &st, &ct);
  const cplx ephi = cexpi(th - 0.5 * PI_D);  // e^{i (theta - pi/2)}
  cplx acc = cmk(0.0, 0.0);
  for (int64_t p = v.idisk[b] + dg; p < v.idisk[b + 1]; p += FF_DG) {
    const int Np = v.N[p];
    const int64_t o = v.moff[p];
    const int64_t i0 = v.imode[b] + o;
    // sum_m sJ_m e^{i m phi} rho_m, m = -N..N, by the phase recurrence
    cplx e = cexpi(-Np * (th - 0.5 * PI_D));
    cplx sm = cmk(0.0, 0.0);
    for (int mm = 0; mm <= 2 * Np; ++mm) {
      cmac(sm, e, v.op_ff ? cmul(rc[o + mm], v.op_ff[i0 + mm]) : cscale(rc[o + mm], v.sJ[i0 + mm]));
      e = cmul(e, ephi);
    }
    const cplx ep = cexpi(-kk * (ct * v.cx[p] + st * v.cy[p]));
    cmac(acc, ep, sm);
  }
  red[dg][tj] = acc;
  __syncthreads();
  // groups 0..FF_DG-1 added in order: first eight partial runs of FF_DG / 8
  // groups, then the eight runs
  constexpr int RUN = FF_DG / 8;
  const bool summer = threadIdx.x < 8 * FF_TH;
  const int run = threadIdx.x / FF_TH;
  cplx sacc = cmk(0.0, 0.0);
  if (summer) {
    sacc = red[run * RUN][tj];
    for (int k = 1; k < RUN; ++k) sacc = cadd(sacc, red[run * RUN + k][tj]);
  }
  __syncthreads();  // every run read before any is overwritten
  if (summer) red[run][tj] = sacc;
  __syncthreads();
  if (dg == 0 && j < n_theta) {
    cplx s = red[0][tj];
    for (int k = 1; k < 8; ++k) s = cadd(s, red[k][tj]);
    // e^{i pi/4} / (2 sqrt k)
    const double c = 0.70710678118654752440 / (2.0 * sqrt(kk));
    a_out[(int64_t)col * n_theta + j] = cmul(cmk(c, c), s);
  }
}

extern "C" int mudiff_farfield(mudiff_t h, int R, const void* rho, int n_theta, const double* theta,
                               void* a_out, void* stream) {
  if (!h || !rho || !theta || !a_out) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  if (R < 1 || n_theta < 1) return fail(MUDIFF_ERR_INVALID, "R < 1 or n_theta < 1");
  if ((int64_t)h->B * R > 65535) return fail(MUDIFF_ERR_INVALID, "too many instance x RHS columns");
  int64_t mmax = 0;  // disks of the largest instance
  for (int b = 0; b < h->B; ++b) mmax = std::max<int64_t>(mmax, h->idisk[b + 1] - h->idisk[b]);
  if (mmax >= 64) {
    dim3 grid((n_theta + 15) / 16, h->B * R);
    hipLaunchKernelGGL((k_farfield<16, 64>), grid, dim3(1024), 0, (hipStream_t)stream, h->dv, R,
                       (const cplx*)rho, n_theta, theta, (cplx*)a_out);
  } else {
    dim3 grid((n_theta + 63) / 64, h->B * R);
    hipLaunchKernelGGL((k_farfield<64, 16>), grid, dim3(1024), 0, (hipStream_t)stream, h->dv, R,
                       (const cplx*)rho, n_theta, theta, (cplx*)a_out);
  }
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}
