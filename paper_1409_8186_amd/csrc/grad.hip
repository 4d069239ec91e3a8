// Adjoint gradient of the far-field misfit with respect to disk centers, radii
// and the wavenumber (truncation orders fixed), for the forward map of the
// paper (sec. 4.2 operator, Prop. 4 right-hand side, sec. 4.4 far field).
//
//   rho = L^{-1}(-U),  a_r = g_r^T rho,  e = a - target,  loss = sum |e|^2
//   c = sum_r conj(e_r) g_r,   L^T lambda = c   solved as  L nu = P c, lambda = P nu
//   (L^T = P L P, P: m -> -m inside every disk, so the adjoint reuses the forward
//   operator and its preconditioner)
//   d loss / ds = 2 Re [ sum_r conj(e_r) (dg_r/ds)^T rho - lambda^T (dL/ds rho + dU/ds) ]
//
// Off-diagonal blocks L^{pq}_{mn} = (i pi/2) s_p(m) t^{pq}_{n-m} s_q(n), s = sqrt(a) J_m(ka):
//  * through t (centers, k):  lambda^T dL rho = (i pi/2) sum_pairs sum_nu dt_nu W^{pq}_nu,
//    W^{pq}_nu = sum_beta sum_{n-m=nu} (s lambda)^p_m (s rho)^q_n   (Gram diagonal sums),
//    d t_nu / d(x_p - x_q) = (k/2)(t_{nu-1} - t_{nu+1}),
//    d t_nu / d(y_p - y_q) = (i k/2)(t_{nu-1} + t_{nu+1}),
//    d t_nu / dk = (b/2)(t_{nu-1} e^{i alpha} - t_{nu+1} e^{-i alpha});
//    t_{+-(S+1)} are recomputed (one upward recurrence step), not stored;
//  * through s (radii, k): contractions with the raw applies
//    w_rho = sum_q T^{pq} (s rho^q)  and  w~_lambda = sum_q (T^{qp})... = (-1)^n w_nu(-n),
//    w_nu the raw apply on nu.
#include <algorithm>

#include "bessel.h"
#include "common.h"

extern "C" int mudiff_gmres(mudiff_t h, int R, const double* beta, const void* rhs, void* rho,
                            int restart, double tol, int maxit, int flags, void* workspace,
                            size_t ws_bytes, int32_t* flag, double* relres, int32_t* iters,
                            double* resvec, void* stream);
extern "C" size_t mudiff_gmres_workspace_size(mudiff_t h, int R, int restart, int flags);

#define PI_D 3.14159265358979323846
#define GR_THREADS 256

// J_m(k a_p), H_m(k a_p) at any m with |m| <= N_p + 1 (reflection for m < 0).
__device__ __forceinline__ double jv_at(const DevView& v, int p, int m) {
  const int am = m < 0 ? -m : m;
  const double x = v.Jd[v.dtab[p] + am];
  return (m < 0 && (am & 1)) ? -x : x;
}
__device__ __forceinline__ cplx hv_at(const DevView& v, int p, int m) {
  const int am = m < 0 ? -m : m;
  const cplx x = v.Hd[v.dtab[p] + am];
  return (m < 0 && (am & 1)) ? cmk(-x.x, -x.y) : x;
}

// instance of a single-column unknown index
__device__ __forceinline__ int inst_of_unknown(const DevView& v, int64_t i) {
  int lo = 0, hi = v.B;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (v.imode[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// e = a - target and loss_b = sum |e|^2 over instance b (one block per instance)
__global__ void k_misfit(int R, int n_rec, const cplx* __restrict__ a, const cplx* __restrict__ tg,
                         cplx* __restrict__ e, double* __restrict__ loss) {
  __shared__ double red[GR_THREADS];
  const int b = blockIdx.x;
  const int64_t n = (int64_t)R * n_rec, o = (int64_t)b * n;
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += GR_THREADS) {
    const cplx d = csub(a[o + k], tg[o + k]);
    e[o + k] = d;
    acc += cabs2(d);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = GR_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[b] = red[0];
}

// gph[r][i] = e^{i pi/4}/(2 sqrt k) e^{-i k theta_r . O_p} e^{i m (theta_r - pi/2)}
// (the far-field row g_r = gph * s)
__global__ void k_gphase(DevView v, int n_rec, const double* __restrict__ th, cplx* __restrict__ gph) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n_rec * v.N_all) return;
  const int r = (int)(g / v.N_all);
  const int64_t i = g - (int64_t)r * v.N_all;
  const int p = v.udisk[i];
  const int b = v.inst[p];
  const int m = (int)(i - v.imode[b] - v.moff[p]) - v.N[p];
  const double k = v.kd[p];
  double st, ct;
  sincos(th[r], &st, &ct);
  const cplx ph = cexpi(-k * (ct * v.cx[p] + st * v.cy[p]) + m * (th[r] - 0.5 * PI_D));
  const double c = 0.70710678118654752440 / (2.0 * sqrt(k));
  gph[g] = cmul(cmk(c, c), ph);
}

// adjoint right-hand side: rhs[col][flip(i)] = -c_i,  c_i = s_i sum_r conj(e_r) gph_r(i)
__global__ void k_adj_rhs(DevView v, int R, int n_rec, const cplx* __restrict__ e,
                          const cplx* __restrict__ gph, cplx* __restrict__ out) {
  const int64_t total = (int64_t)R * v.N_all;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  int lo = 0, hi = v.B;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if ((int64_t)R * v.imode[mid] <= g) lo = mid; else hi = mid;
  }
  const int b = lo;
  const int64_t Nb = v.imode[b + 1] - v.imode[b];
  const int64_t rem = g - (int64_t)R * v.imode[b];
  const int rr = (int)(rem / Nb);
  const int64_t il = rem - (int64_t)rr * Nb;
  const int64_t i = v.imode[b] + il;
  const int p = v.udisk[i];
  const int m = (int)(il - v.moff[p]) - v.N[p];
  const cplx* ec = e + ((int64_t)b * R + rr) * n_rec;
  cplx acc = cmk(0.0, 0.0);
  for (int r = 0; r < n_rec; ++r) cmacc(acc, ec[r], gph[(int64_t)r * v.N_all + i]);
  const double s = v.sJ[i];
  const int64_t flip = (int64_t)R * v.imode[b] + (int64_t)rr * Nb + v.moff[p] + (v.N[p] - m);
  out[flip] = cmk(-s * acc.x, -s * acc.y);
}

// Per ordered pair (p, q): W_nu (Gram diagonal sums over all columns), then the
// contractions with d t / d(x_p - x_q), d t / d(y_p - y_q), d t / dk.
#define GB_TILE 16
#define GR_LDS 3072  // complex values of dynamic LDS per workgroup (48 KiB)
__global__ __launch_bounds__(GR_THREADS) void k_pair_grad(DevView v, int R,
                                                          const int64_t* __restrict__ opoff,
                                                          const cplx* __restrict__ rho,
                                                          const cplx* __restrict__ nu,
                                                          cplx* __restrict__ out) {
  extern __shared__ cplx sh[];
  const int64_t g = blockIdx.x;
  int b = 0;
  {
    int lo = 0, hi = v.B;
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (opoff[mid] <= g) lo = mid; else hi = mid;
    }
    b = lo;
  }
  const int64_t d0 = v.idisk[b], Mb = v.idisk[b + 1] - d0;
  const int64_t lidx = g - opoff[b];
  const int pl = (int)(lidx / (Mb - 1));
  const int ql0 = (int)(lidx - (int64_t)pl * (Mb - 1));
  const int p = (int)d0 + pl, q = (int)d0 + ql0 + (ql0 >= pl ? 1 : 0);
  const int Np = v.N[p], Nq = v.N[q], np = 2 * Np + 1, nq = 2 * Nq + 1;
  const int S = Np + Nq, NV = 2 * S + 1;
  const int G = NV <= GR_THREADS ? GR_THREADS / NV : 1;
  const int tid = threadIdx.x;
  const int gi = tid / NV;  // beta group (valid when gi < G)
  const int64_t Nb = v.imode[b + 1] - v.imode[b];
  const int64_t ip = v.imode[b] + v.moff[p], iq = v.imode[b] + v.moff[q];
  // beta tile sized to the LDS budget (GR_LDS complex values)
  const int tile = max(1, min(GB_TILE, (GR_LDS - (NV > GR_THREADS ? NV : GR_THREADS)) / (np + nq)));
  cplx* ul = sh;                       // [tile][np]
  cplx* vl = sh + tile * np;           // [tile][nq]
  cplx* Wl = sh + tile * (np + nq);    // [G][NV] reduction, then W
  // one accumulator per (nu, group); NV > threads -> loop
  const int nloop = NV <= GR_THREADS ? 1 : (NV + GR_THREADS - 1) / GR_THREADS;
  cplx acc[4];
  for (int k = 0; k < 4; ++k) acc[k] = cmk(0.0, 0.0);
  for (int b0 = 0; b0 < R; b0 += tile) {
    const int nb = min(tile, R - b0);
    __syncthreads();
    for (int e = tid; e < nb * np; e += GR_THREADS) {
      const int bb = e / np, mi = e - (e / np) * np;
      const int64_t cb = col_base(v.imode, b, R, b0 + bb);
      // lambda_{(p,m)} = nu_{(p,-m)}: index mi <-> m = mi - Np, flipped index 2 Np - mi
      const cplx lam = nu[cb + v.moff[p] + (np - 1 - mi)];
      ul[e] = cscale(lam, v.sJ[ip + mi]);
    }
    for (int e = tid; e < nb * nq; e += GR_THREADS) {
      const int bb = e / nq, ni = e - (e / nq) * nq;
      const int64_t cb = col_base(v.imode, b, R, b0 + bb);
      vl[e] = cscale(rho[cb + v.moff[q] + ni], v.sJ[iq + ni]);
    }
    __syncthreads();
    for (int l = 0; l < nloop; ++l) {
      const int t = NV <= GR_THREADS ? tid % NV : tid + l * GR_THREADS;
      if (t >= NV || (NV <= GR_THREADS && gi >= G)) continue;
      const int nuv = t - S;  // n - m
      const int mlo = max(-Np, -Nq - nuv), mhi = min(Np, Nq - nuv);
      cplx a = acc[l & 3];
      for (int bb = (NV <= GR_THREADS ? gi : 0); bb < nb; bb += (NV <= GR_THREADS ? G : 1)) {
        const cplx* ur = ul + bb * np + Np;
        const cplx* vr = vl + bb * nq + Nq + nuv;
        for (int m = mlo; m <= mhi; ++m) cmac(a, ur[m], vr[m]);
      }
      acc[l & 3] = a;
    }
  }
  // reduce the groups: W_nu
  __syncthreads();
  if (NV <= GR_THREADS) {
    if (gi < G) Wl[gi * NV + tid % NV] = acc[0];
    __syncthreads();
    if (tid < NV) {
      cplx w = Wl[tid];
      for (int k = 1; k < G; ++k) w = cadd(w, Wl[k * NV + tid]);
      Wl[tid] = w;
    }
  } else {
    for (int l = 0; l < nloop; ++l) {
      const int t = tid + l * GR_THREADS;
      if (t < NV) Wl[t] = acc[l & 3];
    }
  }
  __syncthreads();
  // symbols of the ordered pair: t^{pq}_nu = (+-1)^nu t^{lo,hi}_nu, |nu| <= S + 1
  const int lo = p < q ? p : q;
  const int hi = p < q ? q : p;
  const int64_t gp = pair_index(v.idisk, v.ipair, b, lo, hi);
  const cplx* T = v.t + v.toff[gp] + S;
  const bool rev = p > q;
  const double dx = v.cx[p] - v.cx[q], dy = v.cy[p] - v.cy[q];
  const double bpq = hypot(dx, dy), al = atan2(dy, dx);
  const double k = v.kd[p];
  // H_{S+1} of the unordered pair by one upward step from H_S, H_{S-1}
  const double alu = atan2(v.cy[lo] - v.cy[hi], v.cx[lo] - v.cx[hi]);
  cplx HS1;
  {
    const double x = k * bpq;
    const cplx HS = cmul(T[S], cexpi(-S * alu));
    const cplx HSm = (S >= 1) ? cmul(T[S - 1], cexpi(-(S - 1) * alu)) : cmk(0.0, 0.0);
    if (S >= 1) {
      HS1 = csub(cscale(HS, 2.0 * S / x), HSm);
    } else {
      cplx h0;
      hankel01(x, &h0, &HS1);
    }
  }
  auto tval = [&](int nuv) -> cplx {
    const int an = nuv < 0 ? -nuv : nuv;
    cplx t;
    if (an <= S) {
      t = T[nuv];
    } else {
      const cplx e = cexpi(an * alu);
      t = cmul(HS1, nuv > 0 ? e : cconj(e));
      if (nuv < 0 && (an & 1)) t = cmk(-t.x, -t.y);
    }
    if (rev && (an & 1)) t = cmk(-t.x, -t.y);
    return t;
  };
  cplx cx = cmk(0.0, 0.0), cy = cmk(0.0, 0.0), ck = cmk(0.0, 0.0);
  const cplx eal = cexpi(al);
  for (int t = tid; t < NV; t += GR_THREADS) {
    const int nuv = t - S;
    const cplx W = Wl[t];
    const cplx tm = tval(nuv - 1), tp = tval(nuv + 1);
    const cplx dtx = cscale(csub(tm, tp), 0.5 * k);
    const cplx sp = cadd(tm, tp);
    const cplx dty = cmk(-0.5 * k * sp.y, 0.5 * k * sp.x);
    const cplx dtk = cscale(csub(cmul(tm, eal), cmul(tp, cconj(eal))), 0.5 * bpq);
    cmac(cx, dtx, W);
    cmac(cy, dty, W);
    cmac(ck, dtk, W);
  }
  // block reduction of the three sums
  __syncthreads();
  cplx* red = sh;
  red[3 * tid] = cx;
  red[3 * tid + 1] = cy;
  red[3 * tid + 2] = ck;
  __syncthreads();
  for (int s = GR_THREADS / 2; s > 0; s >>= 1) {
    if (tid < s)
      for (int k2 = 0; k2 < 3; ++k2) red[3 * tid + k2] = cadd(red[3 * tid + k2], red[3 * (tid + s) + k2]);
    __syncthreads();
  }
  if (tid == 0) {
    out[3 * g] = red[0];
    out[3 * g + 1] = red[1];
    out[3 * g + 2] = red[2];
  }
}

// Per unknown i (summed over the columns of its instance): the terms through
// the diagonal factors s, the diagonal blocks, the right-hand side U and the
// far-field rows g.  E_x, E_y, E_a, E_k are the complex quantities whose
// 2 Re sum over a disk (instance for k) is the gradient.
__global__ void k_unknown_grad(DevView v, int R, int n_rec, const double* __restrict__ beta,
                               const double* __restrict__ th, const cplx* __restrict__ e,
                               const cplx* __restrict__ gph, const cplx* __restrict__ rho,
                               const cplx* __restrict__ nu, const cplx* __restrict__ wr,
                               const cplx* __restrict__ wn, cplx* __restrict__ Ex,
                               cplx* __restrict__ Ey, cplx* __restrict__ Ea,
                               cplx* __restrict__ Ek) {
  extern __shared__ double cs[];  // [n_rec] cos theta, [n_rec] sin theta
  for (int r = threadIdx.x; r < n_rec; r += blockDim.x) {
    double s, c;
    sincos(th[r], &s, &c);
    cs[r] = c;
    cs[n_rec + r] = s;
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.N_all) return;
  const int p = v.udisk[i];
  const int b = v.inst[p];
  const int Np = v.N[p];
  const int64_t il = i - v.imode[b];
  const int m = (int)(il - v.moff[p]) - Np;
  const double k = v.kd[p], a = v.a[p], sa = sqrt(a);
  const double X = v.cx[p], Y = v.cy[p];
  const double J = jv_at(v, p, m), Jd = 0.5 * (jv_at(v, p, m - 1) - jv_at(v, p, m + 1));
  const cplx H = hv_at(v, p, m), Hd = cscale(csub(hv_at(v, p, m - 1), hv_at(v, p, m + 1)), 0.5);
  const double s = sa * J;
  const double s_a = J / (2.0 * sa) + k * sa * Jd;
  const double s_k = sa * a * Jd;
  const double h2 = 0.5 * PI_D;
  // dD/da = (i pi/2)(J H + k a (J' H + J H')),  dD/dk = (i pi/2) a^2 (J' H + J H')
  const cplx JH = cscale(H, J), JdH_JHd = cadd(cscale(H, Jd), cscale(Hd, J));
  const cplx dDa0 = cadd(JH, cscale(JdH_JHd, k * a)), dDk0 = cscale(JdH_JHd, a * a);
  const cplx dDa = cmk(-h2 * dDa0.y, h2 * dDa0.x), dDk = cmk(-h2 * dDk0.y, h2 * dDk0.x);
  const double sgn = (m & 1) ? -1.0 : 1.0;
  const int64_t Nb = v.imode[b + 1] - v.imode[b];
  cplx ex = cmk(0.0, 0.0), ey = ex, ea = ex, ek = ex;
  for (int rr = 0; rr < R; ++rr) {
    const int64_t cb = (int64_t)R * v.imode[b] + (int64_t)rr * Nb;
    const int64_t iflip = cb + v.moff[p] + (Np - m);
    const cplx rh = rho[cb + il];
    const cplx lam = nu[iflip];
    const cplx w1 = wr[cb + il];
    const cplx w2 = cscale(wn[iflip], sgn);
    const double be = beta[b * R + rr];
    double sb, cbeta;
    sincos(be, &sb, &cbeta);
    const double bdo = cbeta * X + sb * Y;  // beta_hat . O_p
    const cplx phase = cscale(cmul(cexpi(k * bdo), cexpi(m * (0.5 * PI_D - be))), sqrt(2.0 * PI_D));
    const cplx U = cscale(phase, s);
    // far-field sums over receivers
    const cplx* ec = e + ((int64_t)b * R + rr) * n_rec;
    cplx S0 = cmk(0.0, 0.0), Sx = S0, Sy = S0, Sk = S0;
    for (int r = 0; r < n_rec; ++r) {
      cplx t = cmk(0.0, 0.0);
      cmacc(t, ec[r], gph[(int64_t)r * v.N_all + i]);  // conj(e_r) gph_r
      const double c = cs[r], sn = cs[n_rec + r];
      S0 = cadd(S0, t);
      Sx = cadd(Sx, cmk(k * c * t.y, -k * c * t.x));     // (-i k cos) t
      Sy = cadd(Sy, cmk(k * sn * t.y, -k * sn * t.x));
      const double tdo = c * X + sn * Y;
      Sk = cadd(Sk, cadd(cscale(t, -0.5 / k), cmk(tdo * t.y, -tdo * t.x)));  // (-1/2k - i th.O) t
    }
    const cplx lamU = cmul(lam, U);
    // centers
    ex = cadd(ex, cadd(cmk(k * cbeta * lamU.y, -k * cbeta * lamU.x), cscale(cmul(rh, Sx), s)));
    ey = cadd(ey, cadd(cmk(k * sb * lamU.y, -k * sb * lamU.x), cscale(cmul(rh, Sy), s)));
    // radius
    const cplx lw = cmul(lam, w1), rw = cmul(rh, w2), lr = cmul(lam, rh);
    const cplx offa = cadd(cscale(lw, s_a), cscale(rw, s_a));
    ea = csub(ea, cmk(-h2 * offa.y, h2 * offa.x));
    ea = csub(ea, cmul(lr, dDa));
    ea = csub(ea, cscale(cmul(lam, phase), s_a));
    ea = cadd(ea, cscale(cmul(rh, S0), s_a));
    // wavenumber
    const cplx offk = cadd(cscale(lw, s_k), cscale(rw, s_k));
    ek = csub(ek, cmk(-h2 * offk.y, h2 * offk.x));
    ek = csub(ek, cmul(lr, dDk));
    ek = csub(ek, cadd(cmk(-bdo * lamU.y, bdo * lamU.x), cscale(cmul(lam, phase), s_k)));
    ek = cadd(ek, cmul(rh, cadd(cscale(Sk, s), cscale(S0, s_k))));
  }
  Ex[i] = ex;
  Ey[i] = ey;
  Ea[i] = ea;
  Ek[i] = ek;
}

// Per disk: 2 Re of the per-unknown terms plus the pair terms (row pairs add,
// column pairs subtract the derivative w.r.t. O_p - O_q), times (-i pi/2).
__global__ void k_disk_grad(DevView v, const int64_t* __restrict__ opoff,
                            const cplx* __restrict__ pg, const cplx* __restrict__ Ex,
                            const cplx* __restrict__ Ey, const cplx* __restrict__ Ea,
                            double* __restrict__ dc, double* __restrict__ da) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= v.M_all) return;
  const int b = v.inst[p];
  const int64_t d0 = v.idisk[b], Mb = v.idisk[b + 1] - d0;
  const int pl = p - (int)d0;
  const int64_t i0 = v.imode[b] + v.moff[p];
  cplx x = cmk(0.0, 0.0), y = x, r = x;
  for (int j = 0; j < 2 * v.N[p] + 1; ++j) {
    x = cadd(x, Ex[i0 + j]);
    y = cadd(y, Ey[i0 + j]);
    r = cadd(r, Ea[i0 + j]);
  }
  cplx px = cmk(0.0, 0.0), py = px;
  for (int ql = 0; ql < Mb; ++ql) {
    if (ql == pl) continue;
    const int64_t grow = opoff[b] + (int64_t)pl * (Mb - 1) + (ql - (ql > pl ? 1 : 0));
    const int64_t gcol = opoff[b] + (int64_t)ql * (Mb - 1) + (pl - (pl > ql ? 1 : 0));
    px = cadd(px, csub(pg[3 * grow], pg[3 * gcol]));
    py = cadd(py, csub(pg[3 * grow + 1], pg[3 * gcol + 1]));
  }
  const double h2 = 0.5 * PI_D;  // -(i pi/2) c  has real part  (pi/2) Im c
  dc[2 * p] = 2.0 * (x.x + h2 * px.y);
  dc[2 * p + 1] = 2.0 * (y.x + h2 * py.y);
  da[p] = 2.0 * r.x;
}

// Per instance: d loss / dk (one block).
__global__ void k_inst_grad(DevView v, const int64_t* __restrict__ opoff,
                            const cplx* __restrict__ pg, const cplx* __restrict__ Ek,
                            double* __restrict__ dk) {
  __shared__ double red[GR_THREADS];
  const int b = blockIdx.x;
  double acc = 0.0;
  for (int64_t i = v.imode[b] + threadIdx.x; i < v.imode[b + 1]; i += GR_THREADS) acc += Ek[i].x;
  for (int64_t g = opoff[b] + threadIdx.x; g < opoff[b + 1]; g += GR_THREADS)
    acc += 0.5 * PI_D * pg[3 * g + 2].y;
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = GR_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) dk[b] = 2.0 * red[0];
}

// ------------------------------------------------------------------ host
namespace {
struct GradLayout {
  size_t gm, rho, nu, rhs, wr, wn, a, e, gph, Ex, Ey, Ea, Ek, pg, opoff, flag, relres, iters,
      apply, total;
  int64_t OP;
};

// Flags of mudiff_grad that its two solves take over: graph replay and the
// s-step variant with its size.
#define GRAD_SOLVE_FLAGS (MUDIFF_GRAPH | MUDIFF_SSTEP | MUDIFF_SSTEP_SIZE(0xff))

GradLayout grad_layout(mudiff_ctx* h, int R, int n_rec, int restart, int flags) {
  GradLayout L{};
  const int64_t NT = (int64_t)R * h->N_all, C = (int64_t)h->B * R;
  L.OP = 0;
  for (int b = 0; b < h->B; ++b) {
    const int64_t Mb = h->idisk[b + 1] - h->idisk[b];
    L.OP += Mb * (Mb - 1);
  }
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  L.gm = take(mudiff_gmres_workspace_size(h, R, restart, flags));
  L.rho = take(NT * 16);
  L.nu = take(NT * 16);
  L.rhs = take(NT * 16);
  L.wr = take(NT * 16);
  L.wn = take(NT * 16);
  L.a = take(C * n_rec * 16);
  L.e = take(C * n_rec * 16);
  L.gph = take((size_t)n_rec * h->N_all * 16);
  L.Ex = take(h->N_all * 16);
  L.Ey = take(h->N_all * 16);
  L.Ea = take(h->N_all * 16);
  L.Ek = take(h->N_all * 16);
  L.pg = take(std::max<int64_t>(L.OP, 1) * 3 * 16);
  L.opoff = take((h->B + 1) * 8);
  L.flag = take(C * 4);
  L.relres = take(C * 8);
  L.iters = take(C * 4);
  L.apply = take(apply_scratch_bytes(h, R));
  L.total = o;
  return L;
}
}  // namespace

extern "C" size_t mudiff_grad_workspace_size(mudiff_t h, int R, int n_rec, int restart, int flags) {
  if (!h || R < 1 || n_rec < 1 || restart < 1 || restart > MUDIFF_MAX_RESTART) return 0;
  return grad_layout(h, R, n_rec, restart, flags & GRAD_SOLVE_FLAGS).total;
}

static int solve_ok(const int32_t* dflag, int C, hipStream_t s, bool* ok) {
  std::vector<int32_t> f(C);
  HIP_TRY(hipMemcpyAsync(f.data(), dflag, C * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *ok = true;
  for (int c = 0; c < C; ++c) *ok &= f[c] == 0;
  return MUDIFF_OK;
}

extern "C" int mudiff_grad(mudiff_t h, int R, const double* beta, int n_rec, const double* theta_rec,
                           const void* target, int restart, double tol, int maxit, int flags,
                           void* workspace, size_t ws_bytes, double* loss, double* d_centers,
                           double* d_radii, double* d_k, void* stream) {
  if (!h || !beta || !theta_rec || !target || !loss || !d_centers || !d_radii || !d_k)
    return fail(MUDIFF_ERR_INVALID, "NULL argument");
  if (R < 1 || n_rec < 1) return fail(MUDIFF_ERR_INVALID, "R < 1 or n_rec < 1");
  if (restart < 1 || restart > MUDIFF_MAX_RESTART) return fail(MUDIFF_ERR_INVALID, "restart out of range");
  if (!(tol > 0.0) || maxit < 1) return fail(MUDIFF_ERR_INVALID, "tol <= 0 or maxit < 1");
  if (h->dv.op_col) return fail(MUDIFF_ERR_INVALID, "the gradient is for the single-layer EFIE; reset the operator first");
  if (flags & MUDIFF_POINT_SOURCE) return fail(MUDIFF_ERR_INVALID, "the gradient is for plane-wave incidence");
  apply_forget_upload(h);
  const int gflags = flags & GRAD_SOLVE_FLAGS;
  GradLayout L = grad_layout(h, R, n_rec, restart, gflags);
  if (!workspace) return fail(MUDIFF_ERR_INVALID, "workspace is NULL");
  if (ws_bytes < L.total) return fail(MUDIFF_ERR_NOMEM, "grad workspace needs " + std::to_string(L.total) + " bytes");
  if (((uintptr_t)workspace) & 255) return fail(MUDIFF_ERR_INVALID, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)workspace;
  const int C = h->B * R;
  const int64_t NT = (int64_t)R * h->N_all;
  cplx* rho = (cplx*)(w + L.rho);
  cplx* nu = (cplx*)(w + L.nu);
  cplx* rhs = (cplx*)(w + L.rhs);
  cplx* wr = (cplx*)(w + L.wr);
  cplx* wn = (cplx*)(w + L.wn);
  cplx* a = (cplx*)(w + L.a);
  cplx* e = (cplx*)(w + L.e);
  cplx* gph = (cplx*)(w + L.gph);
  cplx* Ex = (cplx*)(w + L.Ex);
  cplx* Ey = (cplx*)(w + L.Ey);
  cplx* Ea = (cplx*)(w + L.Ea);
  cplx* Ek = (cplx*)(w + L.Ek);
  cplx* pg = (cplx*)(w + L.pg);
  int64_t* opoff = (int64_t*)(w + L.opoff);
  int32_t* dflag = (int32_t*)(w + L.flag);
  double* drel = (double*)(w + L.relres);
  int32_t* dit = (int32_t*)(w + L.iters);
  const size_t gm_bytes = mudiff_gmres_workspace_size(h, R, restart, gflags);
  std::vector<int64_t> oo(h->B + 1, 0);
  for (int b = 0; b < h->B; ++b) {
    const int64_t Mb = h->idisk[b + 1] - h->idisk[b];
    oo[b + 1] = oo[b] + Mb * (Mb - 1);
  }
  HIP_TRY(hipMemcpyAsync(opoff, oo.data(), (h->B + 1) * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  // forward solve
  int rc = mudiff_gmres(h, R, beta, nullptr, rho, restart, tol, maxit, gflags, w + L.gm, gm_bytes,
                        dflag, drel, dit, nullptr, stream);
  if (rc != MUDIFF_OK) return rc;
  bool ok;
  if ((rc = solve_ok(dflag, C, s, &ok)) != MUDIFF_OK) return rc;
  if (!ok) return fail(MUDIFF_ERR_NOT_CONVERGED, "forward solve did not converge");
  // far field, misfit, adjoint right-hand side
  if ((rc = mudiff_farfield(h, R, rho, n_rec, theta_rec, a, stream)) != MUDIFF_OK) return rc;
  hipLaunchKernelGGL(k_misfit, dim3(h->B), dim3(GR_THREADS), 0, s, R, n_rec, a, (const cplx*)target,
                     e, loss);
  const int64_t ng = (int64_t)n_rec * h->N_all;
  hipLaunchKernelGGL(k_gphase, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, h->dv, n_rec,
                     theta_rec, gph);
  hipLaunchKernelGGL(k_adj_rhs, dim3((unsigned)((NT + 255) / 256)), dim3(256), 0, s, h->dv, R, n_rec,
                     (const cplx*)e, (const cplx*)gph, rhs);
  HIP_TRY(hipGetLastError());
  // adjoint solve: L nu = P c  (rhs = -P c)
  rc = mudiff_gmres(h, R, nullptr, rhs, nu, restart, tol, maxit, gflags, w + L.gm, gm_bytes, dflag,
                    drel, dit, nullptr, stream);
  if (rc != MUDIFF_OK) return rc;
  if ((rc = solve_ok(dflag, C, s, &ok)) != MUDIFF_OK) return rc;
  if (!ok) return fail(MUDIFF_ERR_NOT_CONVERGED, "adjoint solve did not converge");
  // raw off-diagonal contractions on rho and nu
  cplx* part = (cplx*)(w + L.apply);
  int32_t* cnt = (int32_t*)(w + L.apply + apply_scratch_bytes(h, R) - align256((size_t)R * h->M_all * 4));
  if ((rc = launch_fill_zero(cnt, (size_t)R * h->M_all * 4, s)) != MUDIFF_OK) return rc;
  if ((rc = apply_operator(h, R, rho, wr, OP_RAW_W, part, cnt, nullptr, s)) != MUDIFF_OK) return rc;
  if ((rc = apply_operator(h, R, nu, wn, OP_RAW_W, part, cnt, nullptr, s)) != MUDIFF_OK) return rc;
  // pair terms
  if (L.OP > 0) {
    hipLaunchKernelGGL(k_pair_grad, dim3((unsigned)L.OP), dim3(GR_THREADS), GR_LDS * 16, s, h->dv, R,
                       (const int64_t*)opoff, (const cplx*)rho, (const cplx*)nu, pg);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_unknown_grad, dim3((unsigned)((h->N_all + 127) / 128)), dim3(128),
                     2 * n_rec * 8, s, h->dv, R, n_rec, beta, theta_rec, (const cplx*)e,
                     (const cplx*)gph, (const cplx*)rho, (const cplx*)nu, (const cplx*)wr,
                     (const cplx*)wn, Ex, Ey, Ea, Ek);
  hipLaunchKernelGGL(k_disk_grad, dim3((unsigned)((h->M_all + 127) / 128)), dim3(128), 0, s, h->dv,
                     (const int64_t*)opoff, (const cplx*)pg, (const cplx*)Ex, (const cplx*)Ey,
                     (const cplx*)Ea, d_centers, d_radii);
  hipLaunchKernelGGL(k_inst_grad, dim3(h->B), dim3(GR_THREADS), 0, s, h->dv, (const int64_t*)opoff,
                     (const cplx*)pg, (const cplx*)Ek, d_k);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}
