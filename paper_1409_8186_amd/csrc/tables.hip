// Geometry, Bessel/Hankel tables and handle management (paper sec. 4.1-4.2).
//
// Per disk p:      J_m(k a_p), H_m(k a_p), m = 0..N_p+1 (the diagonal matrices
//                  J, H of sec. 4.2, one more order for derivatives).
// Per unknown:     sqrt(a_p) J_m, 1/(sqrt(a_p) H_m), (i pi a_p/2) J_m H_m.
// Per unordered pair p<q of an instance: the separation symbols
//                  t_s = H_s(k b_pq) e^{i s alpha_pq}, s = -(N_p+N_q)..(N_p+N_q),
//                  b_pq, alpha_pq the length and angle of O_p - O_q, with
//                  H_{-s} = (-1)^s H_s.  The reverse pair uses t^{qp}_s = (-1)^s t^{pq}_s.
#include <algorithm>
#include <cstring>

#include "bessel.h"
#include "common.h"

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

extern "C" const char* mudiff_last_error(void) { return g_last_error.c_str(); }

// ------------------------------------------------------------------ kernels

// One thread per disk: Miller J (any x), Y_0/Y_1 from the Neumann series
// (x < BESSEL_X_ASY) or Hankel's expansion, then upward recurrence for Y.
__global__ void k_disk_tables(DevView v) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= v.M_all) return;
  const int nmax = v.N[p] + 1;
  const double x = v.kd[p] * v.a[p];
  double* J = v.Jd + v.dtab[p];
  cplx* H = v.Hd + v.dtab[p];
  double S0, S1;
  bessel_j_miller(x, nmax, J, 1, &S0, &S1);
  double Y0, Y1;
  if (x < BESSEL_X_ASY) {
    bessel_y01_neumann(x, J[0], J[1], S0, S1, &Y0, &Y1);
  } else {
    cplx h0, h1;
    hankel01_asym(x, &h0, &h1);
    Y0 = h0.y;
    Y1 = h1.y;
  }
  H[0] = cmk(J[0], Y0);
  if (nmax >= 1) H[1] = cmk(J[1], Y1);
  double ym1 = Y0, y = Y1;
  for (int n = 1; n < nmax; ++n) {
    double yp1 = (2.0 * n / x) * y - ym1;
    ym1 = y;
    y = yp1;
    H[n + 1] = cmk(J[n + 1], y);
  }
}

// One thread per unknown of the single-column vector: the diagonal factors.
__global__ void k_unknown_tables(DevView v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.N_all) return;
  // locate the disk: binary search on the instance, then on the disks
  int lo = 0, hi = v.B;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (v.imode[mid] <= i) lo = mid; else hi = mid;
  }
  const int b = lo;
  int64_t il = i - v.imode[b];
  int64_t d0 = v.idisk[b], d1 = v.idisk[b + 1];
  int64_t dl = d0, dh = d1;
  while (dh - dl > 1) {
    int64_t mid = (dl + dh) >> 1;
    if (v.moff[mid] <= il) dl = mid; else dh = mid;
  }
  const int p = (int)dl;
  const int Np = v.N[p];
  const int m = (int)(il - v.moff[p]) - Np;
  const int am = m < 0 ? -m : m;
  const double sg = (m < 0 && (am & 1)) ? -1.0 : 1.0;  // reflection to negative orders
  const double J = sg * v.Jd[v.dtab[p] + am];
  const cplx H = cscale(v.Hd[v.dtab[p] + am], sg);
  const double a = v.a[p];
  const double sa = sqrt(a);
  v.sJ[i] = sa * J;
  v.invSH[i] = cdiv(cmk(1.0, 0.0), cscale(H, sa));
  const double c = 0.5 * 3.14159265358979323846 * a * J;  // L^{pp} = i c H
  v.Ldiag[i] = cmk(-c * H.y, c * H.x);
  v.udisk[i] = p;
}

// One thread per unordered pair: H_s(k b) for s = 0..S, then the phases.
__global__ void k_pair_tables(DevView v, int64_t P_all) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= P_all) return;
  int lo = 0, hi = v.B;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (v.ipair[mid] <= g) lo = mid; else hi = mid;
  }
  const int b = lo;
  const int64_t M = v.idisk[b + 1] - v.idisk[b];
  const int64_t l = g - v.ipair[b];
  // row i of the strict upper triangle: first index of row i is i(2M-i-1)/2
  double disc = (2.0 * M - 1.0) * (2.0 * M - 1.0) - 8.0 * (double)l;
  int64_t i = (int64_t)floor(((2.0 * M - 1.0) - sqrt(disc > 0 ? disc : 0.0)) * 0.5);
  if (i < 0) i = 0;
  while (i > 0 && i * (2 * M - i - 1) / 2 > l) --i;
  while ((i + 1) * (2 * M - i - 2) / 2 <= l) ++i;
  const int64_t j = l - i * (2 * M - i - 1) / 2 + i + 1;
  const int p = (int)(v.idisk[b] + i), q = (int)(v.idisk[b] + j);
  const double dx = v.cx[p] - v.cx[q], dy = v.cy[p] - v.cy[q];
  const double bpq = hypot(dx, dy), alpha = atan2(dy, dx);
  const double x = v.kd[p] * bpq;
  const int S = v.N[p] + v.N[q];
  cplx* T = v.t + v.toff[g] + S;  // T[s], s = -S..S
  // H_s for s = 0..S into T[0..S]
  if (x >= BESSEL_X_ASY) {
    cplx h0, h1;
    hankel01_asym(x, &h0, &h1);
    T[0] = h0;
    if (S >= 1) T[1] = h1;
    cplx hm1 = h0, h = h1;
    for (int n = 1; n < S; ++n) {
      cplx hp1 = csub(cscale(h, 2.0 * n / x), hm1);
      hm1 = h;
      h = hp1;
      T[n + 1] = h;
    }
  } else {
    // J_0..J_S go to the real parts of the row (S = 0 needs J_1 as well:
    // use a private pair of slots then)
    double tmp[4];
    double* Jr = S >= 1 ? reinterpret_cast<double*>(T) : tmp;
    double S0, S1;
    bessel_j_miller(x, S >= 1 ? S : 1, Jr, 2, &S0, &S1);
    double Y0, Y1;
    bessel_y01_neumann(x, Jr[0], Jr[2], S0, S1, &Y0, &Y1);
    T[0].x = Jr[0];
    T[0].y = Y0;
    if (S >= 1) T[1].y = Y1;
    double ym1 = Y0, y = Y1;
    for (int n = 1; n < S; ++n) {
      double yp1 = (2.0 * n / x) * y - ym1;
      ym1 = y;
      y = yp1;
      T[n + 1].y = y;
    }
  }
  // lane-interleaved pair records for uniform N, both orders: H_0, H_1,
  // e^{i alpha} (alpha_qp = alpha_pq + pi) and 2 / (k b)
  if (v.lane_N >= 0) {
    const int64_t pc = (int64_t)LANE_CHUNK * LANE_REC;
    const cplx e = cexpi(alpha);
    const int64_t jpq = q - v.idisk[b] - 1, jqp = p - v.idisk[b];  // q > p
    cplx* A = v.lt + v.ltoff[p] + (jpq / LANE_CHUNK) * pc + (jpq % LANE_CHUNK);
    cplx* Bq = v.lt + v.ltoff[q] + (jqp / LANE_CHUNK) * pc + (jqp % LANE_CHUNK);
    const cplx r2 = cmk(2.0 / x, 0.0);
    A[0] = T[0];
    Bq[0] = T[0];
    A[LANE_CHUNK] = T[1];
    Bq[LANE_CHUNK] = T[1];
    A[2 * LANE_CHUNK] = e;
    Bq[2 * LANE_CHUNK] = cmk(-e.x, -e.y);
    A[3 * LANE_CHUNK] = r2;
    Bq[3 * LANE_CHUNK] = r2;
  }
  // phases: t_s = H_s e^{i s alpha}, t_{-s} = (-1)^s H_s e^{-i s alpha}
  for (int s = S; s >= 1; --s) {
    cplx H = T[s];
    cplx e = cexpi(s * alpha);
    T[s] = cmul(H, e);
    cplx tm = cmul(H, cconj(e));
    T[-s] = (s & 1) ? cmk(-tm.x, -tm.y) : tm;
  }
}

// ------------------------------------------------------------------ layout
size_t sched_bytes_for(int B, const int64_t* disk_off, const int32_t* n_modes);

// Lane-interleaved table of a uniform-N batch (1 <= N <= LANE_NMAX): returns
// its size in complex values (0 when N is not uniform or out of range), the
// common N, and per disk the offset of its first chunk.
int64_t lane_layout(int B, const int64_t* disk_off, const int32_t* n_modes, int* lane_N,
                    std::vector<int64_t>* ltoff) {
  const int64_t M = disk_off[B];
  *lane_N = -1;
  if (ltoff) ltoff->assign(M, 0);  // uploaded even when there is no lane table
  for (int64_t p = 1; p < M; ++p)
    if (n_modes[p] != n_modes[0]) return 0;
  const int N = n_modes[0];
  if (N < 1 || N > LANE_NMAX) return 0;
  *lane_N = N;
  const int64_t per_chunk = (int64_t)LANE_CHUNK * LANE_REC;
  int64_t o = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t Mb = disk_off[b + 1] - disk_off[b];
    const int64_t nch = (Mb - 1 + LANE_CHUNK - 1) / LANE_CHUNK;
    for (int64_t p = disk_off[b]; p < disk_off[b + 1]; ++p) {
      if (ltoff) (*ltoff)[p] = o;
      o += nch * per_chunk;
    }
  }
  return o;
}

// Embedding length of the circulant form of instance [d0, d1): 2 (N' + N'') + 1
// with N' >= N'' its two largest orders (0 for fewer than two disks).
int64_t circ_len(const int32_t* n_modes, int64_t d0, int64_t d1) {
  if (d1 - d0 < 2) return 0;
  int a = -1, c = -1;
  for (int64_t p = d0; p < d1; ++p) {
    const int n = n_modes[p];
    if (n > a) {
      c = a;
      a = n;
    } else if (n > c) {
      c = n;
    }
  }
  // any L >= 2 (N' + N'') + 1 embeds every block; the shortest 2^i 3^j at or
  // above it takes fast transforms, and is used when it adds at most a fifth
  // to the per-frequency products (whose work grows with L)
  const int64_t lmin = 2 * (int64_t)(a + c) + 1;
  int64_t best = 0;
  for (int64_t p2 = 1; p2 <= 4 * lmin; p2 *= 2)
    for (int64_t l = p2; l <= 4 * lmin; l *= 3)
      if (l >= lmin && (best == 0 || l < best)) best = l;
  return (best <= 128 && 5 * best <= 6 * lmin) ? best : lmin;
}

namespace {
struct Layout {
  size_t off_cx, off_cy, off_a, off_kd, off_N, off_inst, off_moff, off_dtab, off_idisk, off_imode,
      off_ipair, off_toff, off_t, off_Jd, off_Hd, off_sJ, off_invSH, off_Ldiag, off_udisk, off_sched,
      off_lt, off_ltoff;
  // circulant form (MUDIFF_TABLES_CIRCULANT)
  size_t off_cL = 0, off_cTo = 0, off_cZo = 0, off_cWo = 0, off_ctw = 0, off_cnear = 0, off_cT = 0;
  int64_t c_tw = 0, c_T = 0;  // twiddles, transformed symbols (complex values)
  size_t sched_bytes, total;
};

Layout make_layout(int B, const int64_t* disk_off, const int32_t* n_modes, int64_t N_all,
                   int64_t P_all, int64_t T_all, int64_t D_all, int flags) {
  Layout L{};
  const int64_t M = disk_off[B];
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  L.off_cx = take(M * 8);
  L.off_cy = take(M * 8);
  L.off_a = take(M * 8);
  L.off_kd = take(M * 8);
  L.off_N = take(M * 4);
  L.off_inst = take(M * 4);
  L.off_moff = take(M * 8);
  L.off_dtab = take(M * 8);
  L.off_idisk = take((B + 1) * 8);
  L.off_imode = take((B + 1) * 8);
  L.off_ipair = take((B + 1) * 8);
  L.off_toff = take((P_all + 1) * 8);
  L.off_t = take(T_all * 16);
  L.off_Jd = take(D_all * 8);
  L.off_Hd = take(D_all * 16);
  L.off_sJ = take(N_all * 8);
  L.off_invSH = take(N_all * 16);
  L.off_Ldiag = take(N_all * 16);
  L.off_udisk = take(N_all * 4);
  L.sched_bytes = sched_bytes_for(B, disk_off, n_modes);
  L.off_sched = take(L.sched_bytes);
  int lane_N;
  const int64_t lt = lane_layout(B, disk_off, n_modes, &lane_N, nullptr);
  L.off_lt = take(lt * 16);
  L.off_ltoff = take(M * 8);
  if (flags & MUDIFF_TABLES_CIRCULANT) {
    for (int b = 0; b < B; ++b) {
      const int64_t Lb = circ_len(n_modes, disk_off[b], disk_off[b + 1]);
      const int64_t Mb = disk_off[b + 1] - disk_off[b];
      L.c_tw += Lb;
      L.c_T += Lb * Mb * Mb;
    }
    L.off_cL = take((size_t)B * 4);
    L.off_cTo = take((size_t)B * 8);
    L.off_cZo = take((size_t)B * 8);
    L.off_cWo = take((size_t)B * 8);
    L.off_ctw = take((size_t)L.c_tw * 16);
    L.off_cnear = take((size_t)P_all);
    L.off_cT = take((size_t)L.c_T * 16);
  }

  L.total = o;
  return L;
}

bool sizes_of(int B, const int64_t* disk_off, const int32_t* n_modes, int64_t* N_all,
              int64_t* P_all, int64_t* T_all, int64_t* D_all) {
  if (B < 1 || !disk_off || !n_modes || disk_off[0] != 0) return false;
  *N_all = *P_all = *T_all = *D_all = 0;
  for (int b = 0; b < B; ++b) {
    int64_t d0 = disk_off[b], d1 = disk_off[b + 1];
    if (d1 <= d0) return false;
    for (int64_t p = d0; p < d1; ++p) {
      if (n_modes[p] < 0 || n_modes[p] > MUDIFF_MAX_NP) return false;
      *N_all += 2 * n_modes[p] + 1;
      *D_all += n_modes[p] + 2;
      for (int64_t q = p + 1; q < d1; ++q) {
        *P_all += 1;
        *T_all += 2 * (int64_t)(n_modes[p] + n_modes[q]) + 1;
      }
    }
  }
  return true;
}
}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" size_t mudiff_tables_workspace_size(int B, const int64_t* disk_off,
                                               const int32_t* n_modes, int flags) {
  int64_t N_all, P_all, T_all, D_all;
  if (flags & ~MUDIFF_TABLES_CIRCULANT) return 0;
  if (!sizes_of(B, disk_off, n_modes, &N_all, &P_all, &T_all, &D_all)) return 0;
  if (flags & MUDIFF_TABLES_CIRCULANT)
    for (int64_t p = 0; p < disk_off[B]; ++p)
      if (n_modes[p] > 31) return 0;  // the circulant form needs N_p <= 31
  return make_layout(B, disk_off, n_modes, N_all, P_all, T_all, D_all, flags).total;
}

int circ_build(mudiff_ctx* h, hipStream_t s);

extern "C" int mudiff_tables(int B, const int64_t* disk_off, const double* centers,
                             const double* radii, const int32_t* n_modes, const double* k,
                             void* workspace, size_t ws_bytes, int flags, void* stream,
                             mudiff_t* out) {
  if (!out) return fail(MUDIFF_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (flags & ~MUDIFF_TABLES_CIRCULANT) return fail(MUDIFF_ERR_INVALID, "unknown flags");
  if (B < 1 || !disk_off || !centers || !radii || !n_modes || !k)
    return fail(MUDIFF_ERR_INVALID, "B < 1 or a NULL pointer");
  if (disk_off[0] != 0) return fail(MUDIFF_ERR_INVALID, "disk_off[0] != 0");
  for (int b = 0; b < B; ++b)
    if (disk_off[b + 1] <= disk_off[b])
      return fail(MUDIFF_ERR_INVALID, "disk_off must be strictly increasing");
  const int64_t M = disk_off[B];
  if (M > (int64_t)1 << 30) return fail(MUDIFF_ERR_INVALID, "too many disks");
  for (int64_t p = 0; p < M; ++p) {
    if (!std::isfinite(centers[2 * p]) || !std::isfinite(centers[2 * p + 1]))
      return fail(MUDIFF_ERR_INVALID, "non-finite center");
    if (!(radii[p] > 0.0) || !std::isfinite(radii[p]))
      return fail(MUDIFF_ERR_INVALID, "radius must be finite and > 0");
    if (n_modes[p] < 0 || n_modes[p] > MUDIFF_MAX_NP)
      return fail(MUDIFF_ERR_INVALID, "N_p out of range [0, MUDIFF_MAX_NP]");
  }
  for (int b = 0; b < B; ++b)
    if (!(k[b] > 0.0) || !std::isfinite(k[b]))
      return fail(MUDIFF_ERR_INVALID, "k must be finite and > 0");
  if (flags & MUDIFF_TABLES_CIRCULANT)
    for (int64_t p = 0; p < M; ++p)
      if (n_modes[p] > 31) return fail(MUDIFF_ERR_INVALID, "the circulant form needs N_p <= 31");
  // disjointness (sec. 2): b_pq > a_p + a_q inside every instance
  for (int b = 0; b < B; ++b)
    for (int64_t p = disk_off[b]; p < disk_off[b + 1]; ++p)
      for (int64_t q = p + 1; q < disk_off[b + 1]; ++q) {
        double d = std::hypot(centers[2 * p] - centers[2 * q], centers[2 * p + 1] - centers[2 * q + 1]);
        if (!(d > radii[p] + radii[q]))
          return fail(MUDIFF_ERR_OVERLAP, "disks " + std::to_string(p) + " and " +
                                               std::to_string(q) + " overlap or touch");
      }
  int64_t N_all, P_all, T_all, D_all;
  if (!sizes_of(B, disk_off, n_modes, &N_all, &P_all, &T_all, &D_all))
    return fail(MUDIFF_ERR_INVALID, "bad sizes");
  Layout L = make_layout(B, disk_off, n_modes, N_all, P_all, T_all, D_all, flags);
  if (!workspace) return fail(MUDIFF_ERR_INVALID, "workspace is NULL");
  if (ws_bytes < L.total)
    return fail(MUDIFF_ERR_NOMEM, "tables workspace needs " + std::to_string(L.total) + " bytes");
  if (((uintptr_t)workspace) & 255) return fail(MUDIFF_ERR_INVALID, "workspace must be 256-byte aligned");

  mudiff_ctx* h = new mudiff_ctx();
  h->B = B;
  h->M_all = (int)M;
  h->N_all = N_all;
  h->P_all = P_all;
  h->T_all = T_all;
  h->D_all = D_all;
  h->idisk.assign(disk_off, disk_off + B + 1);
  h->imode.assign(B + 1, 0);
  h->ipair.assign(B + 1, 0);
  h->k.assign(k, k + B);
  h->N.assign(n_modes, n_modes + M);
  h->inst.resize(M);
  h->moff.resize(M);
  h->dtab.resize(M);
  h->cx.resize(M);
  h->cy.resize(M);
  h->a.assign(radii, radii + M);
  h->toff.resize(P_all + 1);
  std::vector<double> kd(M);
  int64_t dt = 0, pi = 0, to = 0;
  for (int b = 0; b < B; ++b) {
    int64_t mo = 0;
    for (int64_t p = disk_off[b]; p < disk_off[b + 1]; ++p) {
      h->inst[p] = b;
      h->moff[p] = mo;
      mo += 2 * n_modes[p] + 1;
      h->dtab[p] = dt;
      dt += n_modes[p] + 2;
      h->cx[p] = centers[2 * p];
      h->cy[p] = centers[2 * p + 1];
      kd[p] = k[b];
      h->Nmax = std::max(h->Nmax, (int)n_modes[p]);
    }
    h->imode[b + 1] = h->imode[b] + mo;
    for (int64_t p = disk_off[b]; p < disk_off[b + 1]; ++p)
      for (int64_t q = p + 1; q < disk_off[b + 1]; ++q) {
        h->toff[pi++] = to;
        to += 2 * (int64_t)(n_modes[p] + n_modes[q]) + 1;
      }
    h->ipair[b + 1] = pi;
  }
  h->toff[P_all] = to;

  char* base = (char*)workspace;
  h->ws = workspace;
  h->ws_bytes = ws_bytes;
  DevView& v = h->dv;
  v.B = B;
  v.M_all = (int)M;
  v.N_all = N_all;
  v.cx = (double*)(base + L.off_cx);
  v.cy = (double*)(base + L.off_cy);
  v.a = (double*)(base + L.off_a);
  v.kd = (double*)(base + L.off_kd);
  v.N = (int32_t*)(base + L.off_N);
  v.inst = (int32_t*)(base + L.off_inst);
  v.moff = (int64_t*)(base + L.off_moff);
  v.dtab = (int64_t*)(base + L.off_dtab);
  v.idisk = (int64_t*)(base + L.off_idisk);
  v.imode = (int64_t*)(base + L.off_imode);
  v.ipair = (int64_t*)(base + L.off_ipair);
  v.toff = (int64_t*)(base + L.off_toff);
  v.t = (cplx*)(base + L.off_t);
  v.Jd = (double*)(base + L.off_Jd);
  v.Hd = (cplx*)(base + L.off_Hd);
  v.sJ = (double*)(base + L.off_sJ);
  v.invSH = (cplx*)(base + L.off_invSH);
  v.Ldiag = (cplx*)(base + L.off_Ldiag);
  v.udisk = (int32_t*)(base + L.off_udisk);
  v.lt = (cplx*)(base + L.off_lt);
  v.ltoff = (int64_t*)(base + L.off_ltoff);
  lane_layout(B, disk_off, n_modes, &v.lane_N, &h->ltoff);
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
      h->n_cu = ncu;
  }
  h->sched_base = base + L.off_sched;
  h->sched_bytes = L.sched_bytes;
  std::vector<int64_t> cTo, cWo;
  if (flags & MUDIFF_TABLES_CIRCULANT) {
    h->circ = true;
    h->cL.assign(B, 0);
    h->cZo.assign(B, 0);
    cTo.assign(B, 0);
    cWo.assign(B, 0);
    int64_t to_ = 0, zo = 0, wo = 0;
    for (int b = 0; b < B; ++b) {
      const int64_t Lb = circ_len(n_modes, disk_off[b], disk_off[b + 1]);
      const int64_t Mb = disk_off[b + 1] - disk_off[b];
      h->cL[b] = (int32_t)Lb;
      cTo[b] = to_;
      h->cZo[b] = zo;
      cWo[b] = wo;
      to_ += Lb * Mb * Mb;
      zo += Lb * Mb;
      wo += Lb;
    }
    h->cZ_all = zo;
    v.cL = (const int32_t*)(base + L.off_cL);
    v.cTo = (const int64_t*)(base + L.off_cTo);
    v.cZo = (const int64_t*)(base + L.off_cZo);
    v.cWo = (const int64_t*)(base + L.off_cWo);
    v.ctw = (const cplx*)(base + L.off_ctw);
    v.cT = (const cplx*)(base + L.off_cT);
    // close pairs (k b_pq < N_p + N_q): direct form; the rest go through the
    // circulant form.  Decided here, once, on the host.
    h->near_off.assign(M + 1, 0);
    h->circ_nearflag.assign(P_all, 0);
    std::vector<std::vector<int32_t>> nl((size_t)M);
    int64_t g = 0;
    h->circ_on.assign(B, 0);
    for (int b = 0; b < B; ++b) {
      double far_w = 0.0, all_w = 0.0;
      for (int64_t p = disk_off[b]; p < disk_off[b + 1]; ++p)
        for (int64_t q = p + 1; q < disk_off[b + 1]; ++q, ++g) {
          const double d = std::hypot(centers[2 * p] - centers[2 * q], centers[2 * p + 1] - centers[2 * q + 1]);
          const bool nr = k[b] * d < (double)(n_modes[p] + n_modes[q]);
          const double w = 2.0 * (2.0 * n_modes[p] + 1) * (2.0 * n_modes[q] + 1);
          all_w += w;
          if (nr) {
            h->circ_nearflag[g] = 1;
            nl[p].push_back((int32_t)q);
            nl[q].push_back((int32_t)p);
            h->n_near += 2;
          } else {
            far_w += w;
            h->n_far += 2;
          }
        }
      h->circ_on[b] = (h->cL[b] > 0 && far_w >= 0.5 * all_w) ? 1 : 0;
    }
    for (int64_t p = 0; p < M; ++p) {
      std::sort(nl[p].begin(), nl[p].end());
      h->near_off[p + 1] = h->near_off[p] + (int64_t)nl[p].size();
    }
    h->near.reserve((size_t)h->near_off[M]);
    for (int64_t p = 0; p < M; ++p) h->near.insert(h->near.end(), nl[p].begin(), nl[p].end());
  }

  hipStream_t s = (hipStream_t)stream;
  auto up = [&](const void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync((void*)dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  int st = MUDIFF_OK;
  auto chk = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && st == MUDIFF_OK)
      st = fail(MUDIFF_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  };
  chk(up(v.cx, h->cx.data(), M * 8), "upload cx");
  chk(up(v.cy, h->cy.data(), M * 8), "upload cy");
  chk(up(v.a, h->a.data(), M * 8), "upload a");
  chk(up(v.kd, kd.data(), M * 8), "upload k");
  chk(up(v.N, h->N.data(), M * 4), "upload N");
  chk(up(v.inst, h->inst.data(), M * 4), "upload inst");
  chk(up(v.moff, h->moff.data(), M * 8), "upload moff");
  chk(up(v.dtab, h->dtab.data(), M * 8), "upload dtab");
  chk(up(v.idisk, h->idisk.data(), (B + 1) * 8), "upload idisk");
  chk(up(v.imode, h->imode.data(), (B + 1) * 8), "upload imode");
  chk(up(v.ipair, h->ipair.data(), (B + 1) * 8), "upload ipair");
  chk(up(v.toff, h->toff.data(), (P_all + 1) * 8), "upload toff");
  chk(up(v.ltoff, h->ltoff.data(), M * 8), "upload ltoff");
  if (h->circ) {
    chk(up(v.cL, h->cL.data(), (size_t)B * 4), "upload cL");
    chk(up(v.cTo, cTo.data(), (size_t)B * 8), "upload cTo");
    chk(up(v.cZo, h->cZo.data(), (size_t)B * 8), "upload cZo");
    chk(up(v.cWo, cWo.data(), (size_t)B * 8), "upload cWo");
    if (P_all > 0) chk(up(base + L.off_cnear, h->circ_nearflag.data(), (size_t)P_all), "upload near flags");
  }
  // the uploads read pageable host memory that this function owns only
  // until it returns: finish them before the kernels are enqueued
  chk(hipStreamSynchronize(s), "upload sync");
  if (st != MUDIFF_OK) {
    delete h;
    return st;
  }
  // operator plan of the one-lane / generic kernels, uploaded now so that no
  // later apply has to synchronise for it (a plan that does not fit the
  // generic kernel stays unbuilt: such batches apply on the matrix cores)
  if (ensure_plan(h, s) == MUDIFF_ERR_DEVICE) st = MUDIFF_ERR_DEVICE;
  hipLaunchKernelGGL(k_disk_tables, dim3((unsigned)((M + 63) / 64)), dim3(64), 0, s, v);
  chk(hipGetLastError(), "k_disk_tables");
  hipLaunchKernelGGL(k_unknown_tables, dim3((unsigned)((N_all + 255) / 256)), dim3(256), 0, s, v);
  chk(hipGetLastError(), "k_unknown_tables");
  if (P_all > 0) {
    hipLaunchKernelGGL(k_pair_tables, dim3((unsigned)((P_all + 63) / 64)), dim3(64), 0, s, v, P_all);
    chk(hipGetLastError(), "k_pair_tables");
  }
  if (st == MUDIFF_OK && h->circ) {
    h->circ_near_dev = (const uint8_t*)(base + L.off_cnear);
    const int rc = circ_build(h, s);
    if (rc != MUDIFF_OK) st = rc;
  }
  if (st != MUDIFF_OK) {
    delete h;
    return st;
  }
  *out = h;
  return MUDIFF_OK;
}

extern "C" int mudiff_destroy(mudiff_t h) {
  if (h) {
    sched_wait(h);  // no schedule upload still reads the handle's host vectors
    if (h->sched_ev) (void)hipEventDestroy(h->sched_ev);
    if (h->aux) {
      (void)hipStreamSynchronize(h->aux);
      (void)hipStreamDestroy(h->aux);
    }
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
    if (h->join_ev) (void)hipEventDestroy(h->join_ev);
    for (hipEvent_t e : h->prof_ev) (void)hipEventDestroy(e);
  }
  delete h;
  return MUDIFF_OK;
}

extern "C" int mudiff_sizes(mudiff_t h, int64_t* n_tot) {
  if (!h || !n_tot) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  for (int b = 0; b < h->B; ++b) n_tot[b] = h->imode[b + 1] - h->imode[b];
  return MUDIFF_OK;
}

extern "C" int mudiff_disk_tables(mudiff_t h, double* J, void* H, void* stream) {
  if (!h) return fail(MUDIFF_ERR_INVALID, "NULL handle");
  hipStream_t s = (hipStream_t)stream;
  if (J) HIP_TRY(hipMemcpyAsync(J, h->dv.Jd, h->D_all * 8, hipMemcpyDeviceToDevice, s));
  if (H) HIP_TRY(hipMemcpyAsync(H, h->dv.Hd, h->D_all * 16, hipMemcpyDeviceToDevice, s));
  return MUDIFF_OK;
}

extern "C" int mudiff_pair_tables(mudiff_t h, void* t, int64_t* count, void* stream) {
  if (!h || !count) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  *count = h->T_all;
  if (t && h->T_all > 0)
    HIP_TRY(hipMemcpyAsync(t, h->dv.t, h->T_all * 16, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return MUDIFF_OK;
}
