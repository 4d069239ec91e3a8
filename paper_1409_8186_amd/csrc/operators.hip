// Boundary integral operators beyond the single layer (paper sec. 3
// formulations, sec. 4.2 block formulas, Prop. 4, sec. 4.4 far fields).
//
// The four operators share the separation matrix S of the single layer:
// for p != q,  X^{pq} = c_X sqrt(a_p a_q) R_X^p (S^{pq})^T C_X^q  with
//   L: c =  i pi / 2,      R = J,  C = J
//   M: c = -i k pi / 2,    R = J,  C = J'
//   N: c =  i k pi / 2,    R = J', C = J
//   D: c = -i k^2 pi / 2,  R = J', C = J'
// (J, J' diagonal matrices of J_m(k a), J'_m(k a)), and on the diagonal
//   L: (i pi a / 2) J H,  M: 1/2 - (i pi k a / 2) J' H,  N: -1/2 + (i pi k a / 2) J' H,
//   D: -(i pi k^2 a / 2) J' H'
// (the sign of the D diagonal is the one of the normal derivative of the
// double-layer potential of a mode, which also gives the off-diagonal D blocks).
// A combination w_I I + w_L L + w_M M + w_N N + w_D D whose operators with
// nonzero weight share their row factor (L, M; or N, D) or their column
// factor (L, N; or M, D) has off-diagonal blocks sqrt(a_p a_q) r^p S^T c^q
// with one row and one column factor vector: it runs on the single-layer
// kernels with the factor tables built here.  Right-hand side
// w_U U + w_dU dU (U = d J, dU = k d J', Prop. 4) and far field
// f_L a_L + f_M a_M with (a_M)^p_m = -k (J'_m / J_m) (a_L)^p_m (the sign of the
// double-layer potential's large-r form).
#include "bessel.h"
#include "common.h"

namespace {

#define OPS_PI 3.14159265358979323846

struct OpWeights {
  cplx w[5];   // I, L, M, N, D
  cplx rU, rdU;
  cplx fL, fM;
  int shared;  // 0: shared row factor, 1: shared column factor
  int kind;    // the shared factor: 0 = J, 1 = J'
};

// J_m, J'_m, H_m, H'_m of unknown i from the disk tables (orders 0..N+1;
// J_{-m} = (-1)^m J_m, same for H and the derivatives).
__device__ void mode_values(const DevView& v, int p, int m, double* J, double* Jd, cplx* H, cplx* Hd) {
  const int am = m < 0 ? -m : m;
  const double sg = (m < 0 && (am & 1)) ? -1.0 : 1.0;
  const double* Jt = v.Jd + v.dtab[p];
  const cplx* Ht = v.Hd + v.dtab[p];
  // J_{|m|-1} with J_{-1} = -J_1
  const double Jm1 = am > 0 ? Jt[am - 1] : -Jt[1];
  const cplx Hm1 = am > 0 ? Ht[am - 1] : cscale(Ht[1], -1.0);
  *J = sg * Jt[am];
  *H = cscale(Ht[am], sg);
  // d/dx of the reflected function: (-1)^m (J_{|m|-1} - J_{|m|+1}) / 2
  *Jd = sg * 0.5 * (Jm1 - Jt[am + 1]);
  *Hd = cscale(csub(Hm1, Ht[am + 1]), 0.5 * sg);
}

__global__ void k_op_tables(DevView v, OpWeights o, cplx* __restrict__ col, cplx* __restrict__ rowA,
                            cplx* __restrict__ row, cplx* __restrict__ diag, cplx* __restrict__ rhs,
                            cplx* __restrict__ rhsp, cplx* __restrict__ ff) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.N_all) return;
  const int p = v.udisk[i];
  const int b = v.inst[p];
  const int m = (int)(i - v.imode[b] - v.moff[p]) - v.N[p];
  double J, Jd;
  cplx H, Hd;
  mode_values(v, p, m, &J, &Jd, &H, &Hd);
  const double k = v.kd[p], a = v.a[p], sa = sqrt(a);
  const cplx I1 = cmk(0.0, 1.0);
  // diagonal block value
  const cplx iJH = cmul(I1, cscale(H, J)), iJdH = cmul(I1, cscale(H, Jd)), iJdHd = cmul(I1, cscale(Hd, Jd));
  cplx d = o.w[0];
  d = cadd(d, cmul(o.w[1], cscale(iJH, 0.5 * OPS_PI * a)));
  d = cadd(d, cmul(o.w[2], csub(cmk(0.5, 0.0), cscale(iJdH, 0.5 * OPS_PI * k * a))));
  d = cadd(d, cmul(o.w[3], cadd(cmk(-0.5, 0.0), cscale(iJdH, 0.5 * OPS_PI * k * a))));
  d = cadd(d, cmul(o.w[4], cscale(iJdHd, -0.5 * OPS_PI * k * k * a)));
  // off-diagonal factors: scalars c_X, row and column Bessel factors
  const cplx cX[4] = {cmk(0.0, 0.5 * OPS_PI), cmk(0.0, -0.5 * k * OPS_PI), cmk(0.0, 0.5 * k * OPS_PI),
                      cmk(0.0, -0.5 * k * k * OPS_PI)};
  const int rK[4] = {0, 0, 1, 1}, cK[4] = {0, 1, 0, 1};  // 0: J, 1: J'
  cplx r = cmk(0.0, 0.0), c = cmk(0.0, 0.0);
  if (o.shared == 0) {
    r = cmk(sa * (o.kind ? Jd : J), 0.0);
    for (int x = 0; x < 4; ++x)
      c = cadd(c, cmul(cmul(o.w[x + 1], cX[x]), cmk(sa * (cK[x] ? Jd : J), 0.0)));
  } else {
    c = cmk(sa * (o.kind ? Jd : J), 0.0);
    for (int x = 0; x < 4; ++x)
      r = cadd(r, cmul(cmul(o.w[x + 1], cX[x]), cmk(sa * (rK[x] ? Jd : J), 0.0)));
  }
  col[i] = c;
  row[i] = r;
  diag[i] = d;
  rowA[i] = cdiv(r, d);
  const double s2pa = sqrt(2.0 * OPS_PI * a);
  const cplx bq = cscale(cadd(cscale(o.rU, J), cscale(o.rdU, k * Jd)), s2pa);
  rhs[i] = bq;
  rhsp[i] = cdiv(bq, d);
  ff[i] = cadd(cscale(o.fL, sa * J), cscale(o.fM, -k * sa * Jd));
}

// Penetrable disks (sec. 7, Example II): the transmission system
//   [ L+           -L-            ] [rho+]   [ -U  ]
//   [ -I/2 + N+    -mu (I/2 + N-) ] [rho-] = [ -dU ]
// with the interior self blocks L- = (i pi a/2) J H and I/2 + N- =
// (i pi k- a/2) J' H at k-_p a_p (diagonal in m; the sign of the (2,2) block is
// the one the jump relations give).  Eliminating rho- mode by mode and
// multiplying by J_m(k- a) (which keeps every mode solvable, also where J_m(k- a)
// vanishes):
//   [J- (N+ - I/2) - mu k- J'- L+] rho+ = -J- dU + mu k- J'- U,
// one combination of N+ and L+ (shared column factor J) with per-mode row
// weights s1 = J_m(k- a), s2 = -mu k- J'_m(k- a) (any per-mode scaling of the
// two is the same equation).  The single-scattering preconditioner divides the
// row weights out again.  J_m(k- a), m = 0..N+1,
// comes from Miller's algorithm per disk.
__global__ void k_interior_j(DevView v, const double* __restrict__ k_int, double* __restrict__ Jint) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= v.M_all) return;
  double S0, S1;
  bessel_j_miller(k_int[p] * v.a[p], v.N[p] + 1, Jint + v.dtab[p], 1, &S0, &S1);
}

__global__ void k_pen_tables(DevView v, const double* __restrict__ k_int, const double* __restrict__ mu,
                             const double* __restrict__ Jint, cplx* __restrict__ col,
                             cplx* __restrict__ rowA, cplx* __restrict__ row, cplx* __restrict__ diag,
                             cplx* __restrict__ rhs, cplx* __restrict__ rhsp, cplx* __restrict__ ff) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.N_all) return;
  const int p = v.udisk[i];
  const int b = v.inst[p];
  const int m = (int)(i - v.imode[b] - v.moff[p]) - v.N[p];
  double J, Jd;
  cplx H, Hd;
  mode_values(v, p, m, &J, &Jd, &H, &Hd);
  // interior J_m, J'_m at k- a (reflection to negative orders as for the exterior)
  const int am = m < 0 ? -m : m;
  const double sg = (m < 0 && (am & 1)) ? -1.0 : 1.0;
  const double* Jt = Jint + v.dtab[p];
  const double Ji = sg * Jt[am];
  const double Jid = sg * 0.5 * ((am > 0 ? Jt[am - 1] : -Jt[1]) - Jt[am + 1]);
  const double k = v.kd[p], a = v.a[p], sa = sqrt(a), ki = k_int[p];
  // row weights, normalised so that |s1| + |s2| = 1 (J_m and J'_m of one
  // argument never vanish together; without it the rows of high orders at small
  // k- a would be tiny)
  const double mup = mu ? mu[p] : 1.0;
  double s1 = Ji, s2 = -mup * ki * Jid;
  if (!(fabs(s1) + fabs(s2) > 0.0)) {
    // both underflowed (high order, small k- a): J'_m / J_m -> |m| / (k- a)
    s1 = 1.0;
    s2 = -mup * (double)am / a;
  }
  const double nrm = 1.0 / (fabs(s1) + fabs(s2));
  s1 *= nrm;
  s2 *= nrm;
  const cplx I1 = cmk(0.0, 1.0);
  // row factor: s1 (i k pi / 2) sqrt(a) J'_m + s2 (i pi / 2) sqrt(a) J_m
  const cplx r = cmul(I1, cmk(0.5 * OPS_PI * sa * (s1 * k * Jd + s2 * J), 0.0));
  // diagonal: s1 (N+_mm - 1/2) + s2 L+_mm,  N+_mm = -1/2 + (i pi k a / 2) J' H
  const cplx iJdH = cmul(I1, cscale(H, Jd)), iJH = cmul(I1, cscale(H, J));
  const cplx d = cadd(cscale(cadd(cmk(-1.0, 0.0), cscale(iJdH, 0.5 * OPS_PI * k * a)), s1),
                      cscale(iJH, 0.5 * OPS_PI * a * s2));
  col[i] = cmk(sa * J, 0.0);
  row[i] = r;
  diag[i] = d;
  rowA[i] = cdiv(r, d);
  const cplx bq = cmk(sqrt(2.0 * OPS_PI * a) * (-s1 * k * Jd - s2 * J), 0.0);
  rhs[i] = bq;
  rhsp[i] = cdiv(bq, d);
  ff[i] = cmk(sa * J, 0.0);
}

constexpr int OP_TABLES = 7;

cplx read_c(const double* w, int k) { return cmk(w[2 * k], w[2 * k + 1]); }

// Operator workspace: 7 complex tables per unknown, then (penetrable disks)
// the interior J table and the per-disk k-, mu.
size_t op_tables_bytes(const mudiff_ctx* h) { return (size_t)OP_TABLES * align256((size_t)h->N_all * 16); }

}  // namespace

extern "C" size_t mudiff_operator_workspace_size(mudiff_t h) {
  if (!h) return 0;
  return op_tables_bytes(h) + align256((size_t)h->D_all * 8) + 2 * align256((size_t)h->M_all * 8);
}

extern "C" int mudiff_set_penetrable(mudiff_t h, const double* k_int, const double* mu,
                                     void* workspace, size_t ws_bytes, void* stream) {
  if (!h || !k_int || !workspace) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  for (int p = 0; p < h->M_all; ++p) {
    if (!(k_int[p] > 0.0) || !std::isfinite(k_int[p])) return fail(MUDIFF_ERR_INVALID, "interior wavenumbers must be > 0");
    if (mu && (!(mu[p] > 0.0) || !std::isfinite(mu[p]))) return fail(MUDIFF_ERR_INVALID, "mu must be > 0");
  }
  const size_t need = mudiff_operator_workspace_size(h);
  if (ws_bytes < need) return fail(MUDIFF_ERR_NOMEM, "operator workspace needs " + std::to_string(need) + " bytes");
  if (((uintptr_t)workspace) & 255) return fail(MUDIFF_ERR_INVALID, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  DevView& v = h->dv;
  const size_t stride = align256((size_t)h->N_all * 16);
  char* w = (char*)workspace;
  cplx* t[OP_TABLES];
  for (int k = 0; k < OP_TABLES; ++k) t[k] = (cplx*)(w + k * stride);
  double* Jint = (double*)(w + op_tables_bytes(h));
  double* dk = (double*)((char*)Jint + align256((size_t)h->D_all * 8));
  double* dmu = (double*)((char*)dk + align256((size_t)h->M_all * 8));
  HIP_TRY(hipMemcpyAsync(dk, k_int, (size_t)h->M_all * 8, hipMemcpyHostToDevice, s));
  if (mu) HIP_TRY(hipMemcpyAsync(dmu, mu, (size_t)h->M_all * 8, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_interior_j, dim3((unsigned)((h->M_all + 63) / 64)), dim3(64), 0, s, v,
                     (const double*)dk, Jint);
  hipLaunchKernelGGL(k_pen_tables, dim3((unsigned)((h->N_all + 255) / 256)), dim3(256), 0, s, v,
                     (const double*)dk, mu ? (const double*)dmu : nullptr, (const double*)Jint, t[0],
                     t[1], t[2], t[3], t[4], t[5], t[6]);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));  // the host arrays are read by the copies above
  v.op_col = t[0];
  v.op_rowA = t[1];
  v.op_row = t[2];
  v.op_diag = t[3];
  v.op_rhs = t[4];
  v.op_rhsp = t[5];
  v.op_ff = t[6];
  h->pen_k = dk;
  h->pen_J = Jint;
  return MUDIFF_OK;
}

namespace {

// c_i = (U + L rho+)_i / (sqrt(2 pi a) J_|m|(k- a)): the interior field's
// coefficients from the Dirichlet trace of the exterior total field (written
// over U).
__global__ void k_interior_coef(DevView v, int R, const double* __restrict__ Jint,
                                cplx* __restrict__ U, const cplx* __restrict__ Lr) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)R * v.N_all) return;
  int lo = 0, hi = v.B;  // instance of g: R * imode[b] <= g
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)R * v.imode[mid] <= g) lo = mid; else hi = mid;
  }
  const int b = lo;
  const int64_t Nb = v.imode[b + 1] - v.imode[b];
  const int64_t rem = g - (int64_t)R * v.imode[b];
  const int64_t il = rem - (rem / Nb) * Nb;
  const int p = v.udisk[v.imode[b] + il];
  const int m = (int)(il - v.moff[p]) - v.N[p];
  const double Ja = Jint[v.dtab[p] + (m < 0 ? -m : m)];
  // J_m(k- a) underflowed (high order, small k- a): the mode's interior field,
  // |J_m(k- r) / J_m(k- a)| <= 1 times its trace coefficient, is below rounding
  U[g] = Ja == 0.0 ? cmk(0.0, 0.0)
                   : cscale(cadd(U[g], Lr[g]), 1.0 / (sqrt(2.0 * OPS_PI * v.a[p]) * Ja));
}

// Points inside a disk: u-(x) = sum_m c_m J_|m|(k- r) e^{i m theta} (polar
// coordinates about the disk's center); other points are left as they are.
__global__ __launch_bounds__(256) void k_interior_field(DevView v, int R, const double* __restrict__ k_int,
                                                        const cplx* __restrict__ c, int n_pts,
                                                        const double* __restrict__ pts,
                                                        cplx* __restrict__ out) {
  const int P = blockIdx.x * 256 + threadIdx.x;
  if (P >= n_pts) return;
  const int col = blockIdx.y;
  const int b = col / R, r = col - b * R;
  const double x1 = pts[2 * P], x2 = pts[2 * P + 1];
  int64_t pin = -1;
  for (int64_t p = v.idisk[b]; p < v.idisk[b + 1]; ++p) {
    const double dx = x1 - v.cx[p], dy = x2 - v.cy[p];
    if (dx * dx + dy * dy < v.a[p] * v.a[p]) pin = p;
  }
  if (pin < 0) return;
  const int p = (int)pin;
  const int Np = v.N[p];
  const double dx = x1 - v.cx[p], dy = x2 - v.cy[p];
  const double rr = sqrt(dx * dx + dy * dy);
  const cplx* cp = c + col_base(v.imode, b, R, r) + v.moff[p] + Np;  // mode 0
  cplx u;
  if (rr == 0.0) {
    u = cp[0];  // J_0(0) = 1, J_m(0) = 0
  } else {
    double Jr[MUDIFF_MAX_NP + 1], S0, S1;
    bessel_j_miller(k_int[p] * rr, Np, Jr, 1, &S0, &S1);
    const cplx e1 = cmk(dx / rr, dy / rr);
    u = cscale(cp[0], Jr[0]);
    cplx em = cmk(1.0, 0.0);
    for (int m = 1; m <= Np; ++m) {
      em = cmul(em, e1);
      cmac(u, cscale(cp[m], Jr[m]), em);
      cmac(u, cscale(cp[-m], Jr[m]), cconj(em));
    }
  }
  out[(int64_t)col * n_pts + P] = u;
}

}  // namespace

extern "C" size_t mudiff_interior_workspace_size(mudiff_t h, int R) {
  if (!h || R < 1) return 0;
  return mudiff_matvec_workspace_size(h, R) + 2 * align256((size_t)R * h->N_all * 16);
}

extern "C" int mudiff_interior_field(mudiff_t h, int R, const void* rho, const double* inc, int flags,
                                     int n_pts, const double* pts, void* out, void* workspace,
                                     size_t ws_bytes, void* stream) {
  if (!h || !rho || !inc || !pts || !out || !workspace) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  if (!h->pen_J) return fail(MUDIFF_ERR_INVALID, "no penetrable disks set on this handle");
  if (R < 1 || n_pts < 1) return fail(MUDIFF_ERR_INVALID, "R < 1 or n_pts < 1");
  if (flags & ~MUDIFF_POINT_SOURCE) return fail(MUDIFF_ERR_INVALID, "unknown flags");
  if ((int64_t)h->B * R > 65535) return fail(MUDIFF_ERR_INVALID, "too many instance x RHS columns");
  const size_t need = mudiff_interior_workspace_size(h, R);
  if (ws_bytes < need) return fail(MUDIFF_ERR_NOMEM, "interior workspace needs " + std::to_string(need) + " bytes");
  if (((uintptr_t)workspace) & 255) return fail(MUDIFF_ERR_INVALID, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const size_t mv = mudiff_matvec_workspace_size(h, R);
  char* w = (char*)workspace;
  cplx* U = (cplx*)(w + mv);
  cplx* Lr = (cplx*)(w + mv + align256((size_t)R * h->N_all * 16));
  // U and L+ rho+ with the single-layer tables: the operator pointers are
  // cleared for these two launches (kernel arguments are taken at launch)
  DevView& v = h->dv;
  const DevView saved = v;
  v.op_col = v.op_rowA = v.op_row = v.op_diag = v.op_rhs = v.op_rhsp = v.op_ff = nullptr;
  int rc = launch_fill_zero(w, mv, s);
  if (rc == MUDIFF_OK) rc = launch_rhs(h, R, inc, U, 0, (flags & MUDIFF_POINT_SOURCE) ? 1 : 0, s);
  if (rc == MUDIFF_OK) rc = mudiff_matvec(h, R, rho, Lr, MUDIFF_OP_L, w, mv, stream);
  v = saved;
  if (rc != MUDIFF_OK) return rc;
  const int64_t tot = (int64_t)R * h->N_all;
  hipLaunchKernelGGL(k_interior_coef, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, v, R,
                     h->pen_J, U, (const cplx*)Lr);
  hipLaunchKernelGGL(k_interior_field, dim3((unsigned)((n_pts + 255) / 256), (unsigned)(h->B * R)), dim3(256),
                     0, s, v, R, h->pen_k, (const cplx*)U, n_pts, pts, (cplx*)out);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}

extern "C" int mudiff_set_operator(mudiff_t h, const double* op_w, const double* rhs_w,
                                   const double* ff_w, void* workspace, size_t ws_bytes,
                                   void* stream) {
  if (!h) return fail(MUDIFF_ERR_INVALID, "NULL handle");
  DevView& v = h->dv;
  if (!op_w) {  // back to the built-in single layer
    v.op_col = v.op_rowA = v.op_row = v.op_diag = v.op_rhs = v.op_rhsp = v.op_ff = nullptr;
    h->pen_k = h->pen_J = nullptr;
    return MUDIFF_OK;
  }
  if (!rhs_w || !ff_w || !workspace) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  for (int k = 0; k < 10; ++k)
    if (!std::isfinite(op_w[k])) return fail(MUDIFF_ERR_INVALID, "non-finite operator weight");
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(rhs_w[k]) || !std::isfinite(ff_w[k])) return fail(MUDIFF_ERR_INVALID, "non-finite weight");
  const size_t need = mudiff_operator_workspace_size(h);
  if (ws_bytes < need) return fail(MUDIFF_ERR_NOMEM, "operator workspace needs " + std::to_string(need) + " bytes");
  if (((uintptr_t)workspace) & 255) return fail(MUDIFF_ERR_INVALID, "workspace must be 256-byte aligned");
  OpWeights o{};
  for (int k = 0; k < 5; ++k) o.w[k] = read_c(op_w, k);
  o.rU = read_c(rhs_w, 0);
  o.rdU = read_c(rhs_w, 1);
  o.fL = read_c(ff_w, 0);
  o.fM = read_c(ff_w, 1);
  // which operators act off the diagonal; their row kinds (L, M: J; N, D: J')
  // and column kinds (L, N: J; M, D: J')
  const int rK[4] = {0, 0, 1, 1}, cK[4] = {0, 1, 0, 1};
  int rmask = 0, cmask = 0;
  for (int x = 0; x < 4; ++x)
    if (o.w[x + 1].x != 0.0 || o.w[x + 1].y != 0.0) {
      rmask |= 1 << rK[x];
      cmask |= 1 << cK[x];
    }
  if (rmask == 3 && cmask == 3)
    return fail(MUDIFF_ERR_INVALID,
                "the operators with nonzero weight share neither their row factor (L, M or N, D) "
                "nor their column factor (L, N or M, D): not one diagonal-Toeplitz-diagonal product");
  if (rmask != 3) {
    o.shared = 0;
    o.kind = rmask == 2 ? 1 : 0;
  } else {
    o.shared = 1;
    o.kind = cmask == 2 ? 1 : 0;
  }
  const size_t stride = align256((size_t)h->N_all * 16);
  char* w = (char*)workspace;
  cplx* t[OP_TABLES];
  for (int k = 0; k < OP_TABLES; ++k) t[k] = (cplx*)(w + k * stride);
  hipLaunchKernelGGL(k_op_tables, dim3((unsigned)((h->N_all + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, v, o, t[0], t[1], t[2], t[3], t[4], t[5], t[6]);
  HIP_TRY(hipGetLastError());
  v.op_col = t[0];
  v.op_rowA = t[1];
  v.op_row = t[2];
  v.op_diag = t[3];
  v.op_rhs = t[4];
  v.op_rhsp = t[5];
  v.op_ff = t[6];
  h->pen_k = h->pen_J = nullptr;
  return MUDIFF_OK;
}

// Named formulations (sec. 3): the operator, right-hand side and far-field
// weights of each, then mudiff_set_operator.  Weight order as there: operator
// I, L, M, N, D; right-hand side U, dU; far field a_L, a_M (re, im pairs).
extern "C" int mudiff_set_formulation(mudiff_t h, int kind, double alpha, double eta_re,
                                      double eta_im, void* workspace, size_t ws_bytes,
                                      void* stream) {
  if (!h) return fail(MUDIFF_ERR_INVALID, "NULL handle");
  if (!std::isfinite(alpha) || !std::isfinite(eta_re) || !std::isfinite(eta_im))
    return fail(MUDIFF_ERR_INVALID, "alpha and eta must be finite");
  double op[10] = {0}, rw[4] = {0}, fw[4] = {0};
  auto set = [](double* a, int k, double re, double im) {
    a[2 * k] = re;
    a[2 * k + 1] = im;
  };
  enum { I_ = 0, L_ = 1, M_ = 2, N_ = 3, D_ = 4 };
  switch (kind) {
    case MUDIFF_FORM_EFIE:  // L rho = -U, the built-in single layer
      return mudiff_set_operator(h, nullptr, nullptr, nullptr, nullptr, 0, stream);
    case MUDIFF_FORM_MFIE:  // (I/2 + N) rho = -dU
      set(op, I_, 0.5, 0.0);
      set(op, N_, 1.0, 0.0);
      set(rw, 1, -1.0, 0.0);
      set(fw, 0, 1.0, 0.0);
      break;
    case MUDIFF_FORM_CFIE:  // (alpha eta L + (1 - alpha)(I/2 + N)) rho = -alpha eta U - (1 - alpha) dU
      if (eta_re == 0.0 && eta_im == 0.0) return fail(MUDIFF_ERR_INVALID, "CFIE needs eta != 0");
      set(op, L_, alpha * eta_re, alpha * eta_im);
      set(op, I_, 0.5 * (1.0 - alpha), 0.0);
      set(op, N_, 1.0 - alpha, 0.0);
      set(rw, 0, -alpha * eta_re, -alpha * eta_im);
      set(rw, 1, -(1.0 - alpha), 0.0);
      set(fw, 0, 1.0, 0.0);
      break;
    case MUDIFF_FORM_BWIE:  // (I/2 - eta L - M) psi = -U, u = -(eta L + M) psi
      if (eta_re == 0.0 && eta_im == 0.0) return fail(MUDIFF_ERR_INVALID, "Brakhage-Werner needs eta != 0");
      set(op, I_, 0.5, 0.0);
      set(op, L_, -eta_re, -eta_im);
      set(op, M_, -1.0, 0.0);
      set(rw, 0, -1.0, 0.0);
      set(fw, 0, -eta_re, -eta_im);
      set(fw, 1, -1.0, 0.0);
      break;
    case MUDIFF_FORM_SOUND_HARD_SINGLE:  // (-I/2 + N) rho = -dU, u = L rho
      set(op, I_, -0.5, 0.0);
      set(op, N_, 1.0, 0.0);
      set(rw, 1, -1.0, 0.0);
      set(fw, 0, 1.0, 0.0);
      break;
    case MUDIFF_FORM_SOUND_HARD_DOUBLE:  // D lambda = -dU, u = M lambda
      set(op, D_, 1.0, 0.0);
      set(rw, 1, -1.0, 0.0);
      set(fw, 1, 1.0, 0.0);
      break;
    default:
      return fail(MUDIFF_ERR_INVALID, "unknown formulation");
  }
  return mudiff_set_operator(h, op, rw, fw, workspace, ws_bytes, stream);
}
