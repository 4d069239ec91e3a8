// Restarted GMRES(m) with the single-scattering preconditioner (paper sec. 5):
// A x = f, A = D^{-1} L, f = -D^{-1} U, one Krylov space per column (instance,
// right-hand side); all columns share each operator application.
//
// Orthogonalisation is classical Gram-Schmidt applied twice (CGS2), which
// keeps the basis orthogonal to working precision with two global reductions
// per step (modified Gram-Schmidt needs j).  The Hessenberg column, the Givens
// rotations and the residual estimate |g_{j+1}| / ||f|| are updated on the
// device by the last workgroup of each column, so the host only synchronises
// to test for the end of a cycle.
//
// Reductions are per column: the rows of a column are cut into chunks, every
// chunk writes its partial sums, and the last chunk to finish (atomic counter,
// reset by itself) adds them in chunk order (deterministic).
#include <algorithm>

#include "common.h"

#define GS_THREADS 256
#define GS_WAVES (GS_THREADS / 64)
#define GS_BATCH 4

enum { ST_RUN = 0, ST_CONV = 1, ST_BREAK = 2, ST_MAXIT = 3 };

struct GState {
  int C, R, m, maxit;
  double tol;
  int64_t NT;               // complex entries of one multivector
  cplx* V;                  // [(m+1)][NT]
  const cplx* f;            // [NT] preconditioned right-hand side
  cplx* x;                  // [NT] iterate (caller's rho)
  const int64_t* ck;        // [n_chunks][2]: (col | len << 32), begin
  cplx* partial;            // [n_chunks][m+1]
  int32_t* cnt;             // [C] chunk counters (zero between kernels)
  cplx* H;                  // [C][(m+1) m]
  cplx* h1;                 // [C][m+1]
  cplx* g;                  // [C][m+1]
  double* cs;               // [C][m]
  cplx* sn;                 // [C][m]
  cplx* y;                  // [C][m]
  double* normf;            // [C]
  double* red;              // [C] scalar reduction result
  double* inv;              // [C] 1 / ||v_{j+1}||
  int32_t* status;          // [C]
  int32_t* inner;           // [C] active in the current Arnoldi cycle
  int32_t* run;             // [C] running at the start of the current cycle
  int32_t* jdone;           // [C] Arnoldi steps done in the current cycle
  int32_t* iters;           // [C] inner iterations so far
  int32_t* n_inner;         // [1] columns still active in the cycle
  double* resvec;           // [C][maxit+1] or NULL
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ void decode_chunk(const GState& s, int gidx, int* col, int* len,
                                             int64_t* begin) {
  const int64_t a = s.ck[2 * gidx];
  *col = (int)(a & 0xffffffff);
  *len = (int)(a >> 32);
  *begin = s.ck[2 * gidx + 1];
}

// Last-chunk detection for column c: returns true in exactly one workgroup.
// Release in every workgroup (write back this block's partials), acquire only
// in the last one: an agent-scope acquire invalidates the XCD's L2, so it is
// kept out of the workgroups that do not read other blocks' results.
__device__ __forceinline__ bool last_chunk(const GState& s, int c, int nck, int* flag) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) {
    int old = atomicAdd(&s.cnt[c], 1);
    *flag = (old == nck - 1);
    if (*flag) atomicExch(&s.cnt[c], 0);
  }
  __syncthreads();
  if (*flag) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *flag;
}

// Arnoldi bookkeeping of column c after step j (one thread): Hessenberg column
// hl = h1 + h2 with subdiagonal hn, previous Givens rotations, the new rotation,
// the residual estimate |g_{j+1}| / ||f|| and the stopping test.  hl, csl, snl
// are the column and the rotations 0..j-1 staged in LDS: the rotation chain
// carries one value in registers, so no step waits on a global load.
__device__ void arnoldi_step(const GState& s, int c, int j, const cplx* hl, const double* csl,
                             const cplx* snl, double hn) {
  const int m1 = s.m + 1;
  cplx* hj = s.H + (int64_t)c * m1 * s.m + (int64_t)j * m1;  // column j
  cplx cur = hl[0];
  for (int i = 0; i < j; ++i) {  // previous rotations
    const cplx nxt = hl[i + 1];
    const double ci = csl[i];
    const cplx si = snl[i];
    hj[i] = cadd(cscale(cur, ci), cmul(si, nxt));
    cur = csub(cscale(nxt, ci), cmul(cconj(si), cur));
  }
  // rotation [c s; -conj(s) c] zeroing the subdiagonal hn (real, >= 0)
  const cplx aa = cur;
  double cr;
  cplx sr;
  if (hn == 0.0) {
    cr = 1.0;
    sr = cmk(0.0, 0.0);
  } else if (aa.x == 0.0 && aa.y == 0.0) {
    cr = 0.0;
    sr = cmk(1.0, 0.0);
  } else {
    const double na = sqrt(cabs2(aa));
    const double rho = hypot(na, hn);
    cr = na / rho;
    sr = cscale(aa, hn / (na * rho));  // (a/|a|) conj(b)/rho, b real
  }
  s.cs[(int64_t)c * s.m + j] = cr;
  s.sn[(int64_t)c * s.m + j] = sr;
  hj[j] = cadd(cscale(aa, cr), cscale(sr, hn));
  cplx* gc = s.g + (int64_t)c * m1;
  const cplx gj = gc[j];
  gc[j + 1] = cmul(cscale(cconj(sr), -1.0), gj);
  gc[j] = cscale(gj, cr);
  const int it = s.iters[c] + 1;
  s.iters[c] = it;
  const double rel = sqrt(cabs2(gc[j + 1])) / s.normf[c];
  if (s.resvec) s.resvec[(int64_t)c * (s.maxit + 1) + it] = rel;
  s.jdone[c] = j + 1;
  const bool finite = isfinite(rel) && isfinite(hn);
  if (!finite) s.status[c] = ST_BREAK;
  if (!finite || rel <= s.tol || hn == 0.0 || it >= s.maxit || j + 1 >= s.m) {
    s.inner[c] = 0;
    s.inv[c] = 0.0;
    atomicSub(s.n_inner, 1);
  } else {
    s.inv[c] = 1.0 / hn;
  }
}

// Classical Gram-Schmidt applied twice on w = V[j+1], three passes per step:
//   MODE 0: h1 = V^H w                                   (dots)
//   MODE 1: w1 = w - V h1;  h2 = V^H w1;  n1 = ||w1||^2   (update + dots + norm)
//           last chunk: ||w2||^2 = n1 - ||h2||^2 (w2 = w1 - V h2 is orthogonal
//           to V h2), then the Arnoldi/Givens step of the column
//   MODE 2: V[j+1] = (w1 - V h2) / ||w2||                (update + normalise)
template <int MODE>
__global__ __launch_bounds__(GS_THREADS) void k_gs(GState s, int j, const int32_t* __restrict__ ck_first,
                                                   const int32_t* __restrict__ ck_count,
                                                   cplx* __restrict__ hdst) {
  __shared__ cplx wl[1024];
  __shared__ double sred[GS_WAVES];
  __shared__ int s_flag;
  __shared__ double s_n1;
  int c, len;
  int64_t o;
  decode_chunk(s, blockIdx.x, &c, &len, &o);
  if (!s.inner[c]) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m1 = s.m + 1;
  cplx* w = s.V + (int64_t)(j + 1) * s.NT + o;
  const double scale = MODE == 2 ? s.inv[c] : 1.0;
  double nn = 0.0;
  for (int r = tid; r < len; r += GS_THREADS) {
    cplx v = w[r];
    if (MODE >= 1) {
      const cplx* hc = (MODE == 1 ? s.h1 : hdst) + (int64_t)c * m1;
      const cplx* vr = s.V + o + r;
      int i = 0;
      for (; i + 3 <= j; i += 4) {  // four independent loads in flight
        const cplx v0 = vr[(int64_t)i * s.NT], v1 = vr[(int64_t)(i + 1) * s.NT];
        const cplx v2 = vr[(int64_t)(i + 2) * s.NT], v3 = vr[(int64_t)(i + 3) * s.NT];
        v = csub(v, cmul(hc[i], v0));
        v = csub(v, cmul(hc[i + 1], v1));
        v = csub(v, cmul(hc[i + 2], v2));
        v = csub(v, cmul(hc[i + 3], v3));
      }
      for (; i <= j; ++i) v = csub(v, cmul(hc[i], vr[(int64_t)i * s.NT]));
      if (MODE == 2) {
        w[r] = cscale(v, scale);
        continue;
      }
      w[r] = v;
      nn += cabs2(v);
    }
    wl[r] = v;
  }
  if (MODE == 2) return;
  __syncthreads();
  const int nck = ck_count[c];
  cplx* part = s.partial + (int64_t)blockIdx.x * m1;
  // wave wv takes i = wv, wv + GS_WAVES, ...; GS_BATCH of them at a time so
  // that their loads are in flight together before the wave reductions
  for (int i0 = wv; i0 <= j; i0 += GS_WAVES * GS_BATCH) {
    cplx a[GS_BATCH];
#pragma unroll
    for (int u = 0; u < GS_BATCH; ++u) {
      a[u] = cmk(0.0, 0.0);
      const int i = i0 + u * GS_WAVES;
      if (i <= j) {
        const cplx* vi = s.V + (int64_t)i * s.NT + o;
        for (int r = lane; r < len; r += 64) cmacc(a[u], vi[r], wl[r]);
      }
    }
#pragma unroll
    for (int u = 0; u < GS_BATCH; ++u) {
      a[u].x = wave_sum(a[u].x);
      a[u].y = wave_sum(a[u].y);
    }
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < GS_BATCH; ++u)
        if (i0 + u * GS_WAVES <= j) part[i0 + u * GS_WAVES] = a[u];
    }
  }
  if (MODE == 1) {  // ||w1||^2 of the chunk in the last slot (never a dot slot: j < m)
    nn = wave_sum(nn);
    if (lane == 0) sred[wv] = nn;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int k = 0; k < GS_WAVES; ++k) t += sred[k];
      part[s.m] = cmk(t, 0.0);
    }
  }
  if (!last_chunk(s, c, nck, &s_flag)) return;
  // column sums of the chunk partials, in a fixed order: wave wv takes slots
  // i = wv, wv + GS_WAVES, ..., its lanes stride over the chunks.  In MODE 1
  // slot j + 1 stands for the norm slot s.m.  The sums also go to LDS (wl is
  // free now; j + 1 <= m <= 1024 entries).
  cplx* hout = (MODE == 0 ? s.h1 : hdst) + (int64_t)c * m1;
  const cplx* pbase = s.partial + (int64_t)ck_first[c] * m1;
  const int ns = MODE == 1 ? j + 2 : j + 1;
  double hsq = 0.0;
  for (int i0 = wv; i0 < ns; i0 += GS_WAVES * GS_BATCH) {
    cplx a[GS_BATCH];
#pragma unroll
    for (int u = 0; u < GS_BATCH; ++u) {
      a[u] = cmk(0.0, 0.0);
      const int i = i0 + u * GS_WAVES;
      if (i < ns) {
        const int sl = i <= j ? i : s.m;
        for (int k = lane; k < nck; k += 64) a[u] = cadd(a[u], pbase[(int64_t)k * m1 + sl]);
      }
    }
#pragma unroll
    for (int u = 0; u < GS_BATCH; ++u) {
      a[u].x = wave_sum(a[u].x);
      a[u].y = wave_sum(a[u].y);
      const int i = i0 + u * GS_WAVES;
      if (i <= j) {
        hsq += cabs2(a[u]);
        if (lane == 0) {
          hout[i] = a[u];
          wl[i] = a[u];
        }
      } else if (i < ns && lane == 0) {
        s_n1 = a[u].x;
      }
    }
  }
  if (MODE == 0) return;
  // h = h1 + h2 and, when they fit beside it in wl (j <= 409), the previous
  // rotations into LDS; ||h2||^2 over the waves
  const cplx* h1c = s.h1 + (int64_t)c * m1;
  const bool fits = 2 * j + 1 + (j + 1) / 2 <= 1024;
  const double* csl = s.cs + (int64_t)c * s.m;
  const cplx* snl = s.sn + (int64_t)c * s.m;
  __syncthreads();
  for (int i = tid; i <= j; i += GS_THREADS) {
    wl[i] = cadd(wl[i], h1c[i]);
    if (fits && i < j) {
      wl[j + 1 + i] = snl[i];
      reinterpret_cast<double*>(wl + 2 * j + 1)[i] = csl[i];
    }
  }
  if (fits) {
    snl = wl + j + 1;
    csl = reinterpret_cast<const double*>(wl + 2 * j + 1);
  }
  if (lane == 0) sred[wv] = hsq;
  __syncthreads();
  if (tid != 0) return;
  double h2n = 0.0;
  for (int k = 0; k < GS_WAVES; ++k) h2n += sred[k];
  const double hn2 = s_n1 - h2n;
  arnoldi_step(s, c, j, wl, csl, snl, sqrt(hn2 > 0.0 ? hn2 : 0.0));
}

// Chunked per-column sum of |src|^2 -> red[c]   (running columns only if
// `only_run`).  When `sub`: src = f - src first; when `copy`: src = f.
__global__ __launch_bounds__(GS_THREADS) void k_resid(GState s, int mode, int only_run,
                                                      const int32_t* __restrict__ ck_first,
                                                      const int32_t* __restrict__ ck_count,
                                                      const cplx* __restrict__ vec_in) {
  __shared__ double sred[GS_WAVES];
  __shared__ int s_flag;
  int c, len;
  int64_t o;
  decode_chunk(s, blockIdx.x, &c, &len, &o);
  if (only_run && !s.run[c]) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m1 = s.m + 1;
  double a = 0.0;
  for (int r = tid; r < len; r += GS_THREADS) {
    cplx v;
    if (mode == 0) {
      v = vec_in[o + r];                  // norm of a given vector
    } else if (mode == 1) {
      v = s.f[o + r];                     // V0 = f
      s.V[o + r] = v;
    } else {
      v = csub(s.f[o + r], s.V[o + r]);   // V0 = f - A x
      s.V[o + r] = v;
    }
    a += cabs2(v);
  }
  a = wave_sum(a);
  if (lane == 0) sred[wv] = a;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int k = 0; k < GS_WAVES; ++k) t += sred[k];
    s.partial[(int64_t)blockIdx.x * m1] = cmk(t, 0.0);
  }
  const int nck = ck_count[c];
  if (!last_chunk(s, c, nck, &s_flag)) return;
  double t = 0.0;  // fixed order: thread stride over the chunks, then the tree
  for (int k = tid; k < nck; k += GS_THREADS) t += s.partial[(int64_t)(ck_first[c] + k) * m1].x;
  t = wave_sum(t);
  if (lane == 0) sred[wv] = t;
  __syncthreads();
  if (tid != 0) return;
  t = 0.0;
  for (int k = 0; k < GS_WAVES; ++k) t += sred[k];
  s.red[c] = t;
}

// Column setup before the first cycle: ||f||, status, iteration count.
__global__ void k_setup(GState s) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= s.C) return;
  const double nf = sqrt(s.red[c]);
  s.normf[c] = nf;
  s.iters[c] = 0;
  s.status[c] = (nf == 0.0) ? ST_CONV : (isfinite(nf) ? ST_RUN : ST_BREAK);
  s.run[c] = s.status[c] == ST_RUN;
  s.inner[c] = 0;
  s.jdone[c] = 0;
}

// Start of a cycle: beta = ||V0|| decides convergence; otherwise V0 /= beta.
__global__ void k_cycle_begin(GState s) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= s.C) return;
  s.inner[c] = 0;
  s.jdone[c] = 0;
  if (!s.run[c] || s.status[c] != ST_RUN) {
    s.run[c] = 0;
    return;
  }
  const double beta = sqrt(s.red[c]);
  const double rel = beta / s.normf[c];
  if (s.resvec && s.iters[c] == 0) s.resvec[(int64_t)c * (s.maxit + 1)] = rel;
  if (!isfinite(rel)) {
    s.status[c] = ST_BREAK;
  } else if (rel <= s.tol) {
    s.status[c] = ST_CONV;
  } else if (s.iters[c] >= s.maxit) {
    s.status[c] = ST_MAXIT;
  }
  if (s.status[c] != ST_RUN) {
    s.run[c] = 0;
    return;
  }
  s.run[c] = 1;
  s.inner[c] = 1;
  s.inv[c] = 1.0 / beta;
  cplx* gc = s.g + (int64_t)c * (s.m + 1);
  gc[0] = cmk(beta, 0.0);
  atomicAdd(s.n_inner, 1);
}

// V0 *= inv for the columns that start a cycle.
__global__ void k_scale_v0(GState s, int64_t nrows_total, const int32_t* __restrict__ row_col) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nrows_total) return;
  const int c = row_col[g];
  if (!s.inner[c]) return;
  s.V[g] = cscale(s.V[g], s.inv[c]);
}

// End of a cycle: y = R^{-1} g (upper-triangular Hessenberg after rotations).
// One wavefront per column: back substitution with the column-oriented
// update g_k -= R_{k,i} y_i spread over the lanes, g held in LDS.
__global__ __launch_bounds__(64) void k_cycle_solve(GState s) {
  __shared__ cplx gl[MUDIFF_MAX_RESTART + 1];
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const int n = s.run[c] ? s.jdone[c] : 0;
  const int m1 = s.m + 1;
  const cplx* Hc = s.H + (int64_t)c * m1 * s.m;
  const cplx* gc = s.g + (int64_t)c * m1;
  cplx* yc = s.y + (int64_t)c * s.m;
  for (int k = lane; k < n; k += 64) gl[k] = gc[k];
  __syncthreads();
  for (int i = n - 1; i >= 0; --i) {
    const cplx* col = Hc + (int64_t)i * m1;  // column i of the triangular factor
    const cplx d = col[i];
    const cplx gi = gl[i];
    const cplx yi = (d.x == 0.0 && d.y == 0.0) ? cmk(0.0, 0.0) : cdiv(gi, d);
    if (lane == 0) yc[i] = yi;
    for (int k = lane; k < i; k += 64) gl[k] = csub(gl[k], cmul(col[k], yi));
    __syncthreads();
  }
}

// x += sum_i y_i V_i over the rows of every running column.
__global__ void k_update_x(GState s, int64_t nrows_total, const int32_t* __restrict__ row_col) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nrows_total) return;
  const int c = row_col[g];
  if (!s.run[c]) return;
  const int n = s.jdone[c];
  const cplx* yc = s.y + (int64_t)c * s.m;
  cplx acc = s.x[g];
  for (int i = 0; i < n; ++i) cmac(acc, yc[i], s.V[(int64_t)i * s.NT + g]);
  s.x[g] = acc;
}

__global__ void k_finish(GState s, int32_t* flag, double* relres, int32_t* iters) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= s.C) return;
  const int st = s.status[c];
  flag[c] = st == ST_CONV ? 0 : (st == ST_MAXIT ? 1 : 2);
  relres[c] = s.normf[c] == 0.0 ? 0.0 : sqrt(s.red[c]) / s.normf[c];
  iters[c] = s.iters[c];
}

// x = 0 for every column
__global__ void k_zero_c(cplx* p, int64_t n) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) p[g] = cmk(0.0, 0.0);
}

// f = scale * src / Ldiag  (general right-hand side: f = -D^{-1} U)
__global__ void k_precond_rhs(DevView v, int R, const cplx* __restrict__ src, cplx* __restrict__ f,
                              double scale) {
  const int64_t total = (int64_t)R * v.N_all;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  int lo = 0, hi = v.B;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if ((int64_t)R * v.imode[mid] <= g) lo = mid; else hi = mid;
  }
  const int64_t Nb = v.imode[lo + 1] - v.imode[lo];
  const int64_t rem = g - (int64_t)R * v.imode[lo];
  const int64_t i = v.imode[lo] + rem % Nb;
  f[g] = cscale(cdiv(src[g], v.Ldiag[i]), scale);
}

// ------------------------------------------------------------------ host driver
// Rows per reduction chunk: about 4096 chunks over all columns (enough
// workgroups to fill the chip, few partial sums to combine), 64..1024 rows
// each (1024 = the LDS row buffer of k_gs).
static int64_t chunk_rows(int64_t NT) {
  int64_t ch = ((NT + 4095) / 4096 + 63) / 64 * 64;
  return std::min<int64_t>(std::max<int64_t>(ch, 64), 1024);
}

namespace {
struct GLayout {
  size_t V, f, apply, ck, ckf, ckc, rowcol, partial, cnt, H, h1, h2, g, cs, sn, y, normf, red, inv,
      status, inner, run, jdone, iters, ninner, total;
  int64_t n_chunks, NT;
};

GLayout glayout(mudiff_ctx* h, int R, int m) {
  GLayout L{};
  const int64_t C = (int64_t)h->B * R;
  const int64_t NT = (int64_t)R * h->N_all;
  L.NT = NT;
  // chunks: at most 1024 rows, at most 64 per column
  int64_t nck = 0;
  for (int b = 0; b < h->B; ++b) {
    const int64_t Nb = h->imode[b + 1] - h->imode[b];
    const int64_t ch = chunk_rows(NT);
    nck += (int64_t)R * ((Nb + ch - 1) / ch);
  }
  L.n_chunks = nck;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  L.V = take((size_t)(m + 1) * NT * 16);
  L.f = take(NT * 16);
  L.apply = take(apply_scratch_bytes(h, R));
  L.ck = take(nck * 16);
  L.ckf = take(C * 4);
  L.ckc = take(C * 4);
  L.rowcol = take(NT * 4);
  L.partial = take(nck * (m + 1) * 16);
  L.cnt = take(C * 4);
  L.H = take(C * (m + 1) * m * 16);
  L.h1 = take(C * (m + 1) * 16);
  L.h2 = take(C * (m + 1) * 16);
  L.g = take(C * (m + 1) * 16);
  L.cs = take(C * m * 8);
  L.sn = take(C * m * 16);
  L.y = take(C * m * 16);
  L.normf = take(C * 8);
  L.red = take(C * 8);
  L.inv = take(C * 8);
  L.status = take(C * 4);
  L.inner = take(C * 4);
  L.run = take(C * 4);
  L.jdone = take(C * 4);
  L.iters = take(C * 4);
  L.ninner = take(256);
  L.total = o;
  return L;
}
}  // namespace

extern "C" size_t mudiff_gmres_workspace_size(mudiff_t h, int R, int restart, int flags) {
  (void)flags;
  if (!h || R < 1 || restart < 1 || restart > MUDIFF_MAX_RESTART) return 0;
  return glayout(h, R, restart).total;
}

// Column of every row of a packed multivector.
namespace {
__global__ void k_rowcol(int32_t* rc, int64_t NT, int R, int B, const int64_t* imode) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= NT) return;
  int lo = 0, hi = B;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if ((int64_t)R * imode[mid] <= g) lo = mid; else hi = mid;
  }
  const int64_t Nb = imode[lo + 1] - imode[lo];
  const int r = (int)((g - (int64_t)R * imode[lo]) / Nb);
  rc[g] = lo * R + r;
}
}  // namespace

struct GmresRun {
  mudiff_ctx* h;
  GState s;
  GLayout L;
  int32_t* d_ckf;
  int32_t* d_ckc;
  int32_t* d_rowcol;
  cplx* apply_part;
  int32_t* apply_cnt;
  cplx* h2;
  hipStream_t st;
};

// One restart cycle (Arnoldi steps + solution update + true residual).
static int enqueue_cycle(GmresRun& G, int check_every, bool host_checks) {
  GState& s = G.s;
  const unsigned cb = (unsigned)((s.C + 63) / 64);
  const unsigned eb = (unsigned)((s.NT + 255) / 256);
  hipLaunchKernelGGL(k_scale_v0, dim3(eb), dim3(256), 0, G.st, s, s.NT, G.d_rowcol);
  HIP_TRY(hipGetLastError());
  for (int j = 0; j < s.m; ++j) {
    int rc = apply_operator(G.h, s.R, s.V + (int64_t)j * s.NT, s.V + (int64_t)(j + 1) * s.NT,
                            MUDIFF_OP_A, G.apply_part, G.apply_cnt, s.inner, G.st);
    if (rc != MUDIFF_OK) return rc;
    const unsigned nb = (unsigned)G.L.n_chunks;
    hipLaunchKernelGGL(k_gs<0>, dim3(nb), dim3(GS_THREADS), 0, G.st, s, j, G.d_ckf, G.d_ckc, G.h2);
    hipLaunchKernelGGL(k_gs<1>, dim3(nb), dim3(GS_THREADS), 0, G.st, s, j, G.d_ckf, G.d_ckc, G.h2);
    hipLaunchKernelGGL(k_gs<2>, dim3(nb), dim3(GS_THREADS), 0, G.st, s, j, G.d_ckf, G.d_ckc, G.h2);
    HIP_TRY(hipGetLastError());
    if (host_checks && check_every > 0 && (j + 1) % check_every == 0 && j + 1 < s.m) {
      int32_t n_in = 0;
      HIP_TRY(hipMemcpyAsync(&n_in, s.n_inner, 4, hipMemcpyDeviceToHost, G.st));
      HIP_TRY(hipStreamSynchronize(G.st));
      if (n_in <= 0) break;
    }
  }
  hipLaunchKernelGGL(k_cycle_solve, dim3(s.C), dim3(64), 0, G.st, s);
  hipLaunchKernelGGL(k_update_x, dim3(eb), dim3(256), 0, G.st, s, s.NT, G.d_rowcol);
  HIP_TRY(hipGetLastError());
  int rc = apply_operator(G.h, s.R, s.x, s.V, MUDIFF_OP_A, G.apply_part, G.apply_cnt, s.run, G.st);
  if (rc != MUDIFF_OK) return rc;
  hipLaunchKernelGGL(k_resid, dim3((unsigned)G.L.n_chunks), dim3(GS_THREADS), 0, G.st, s, 2, 1,
                     G.d_ckf, G.d_ckc, (const cplx*)nullptr);
  // the true residual decides each column's next cycle
  hipLaunchKernelGGL(k_cycle_begin, dim3(cb), dim3(64), 0, G.st, s);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}

extern "C" int mudiff_gmres(mudiff_t h, int R, const double* beta, const void* rhs, void* rho,
                            int restart, double tol, int maxit, int flags, void* workspace,
                            size_t ws_bytes, int32_t* flag, double* relres, int32_t* iters,
                            double* resvec, void* stream) {
  if (!h || !rho || !flag || !relres || !iters) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  if (!beta && !rhs) return fail(MUDIFF_ERR_INVALID, "need beta or rhs");
  if (R < 1) return fail(MUDIFF_ERR_INVALID, "R < 1");
  if (restart < 1 || restart > MUDIFF_MAX_RESTART) return fail(MUDIFF_ERR_INVALID, "restart out of range");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(MUDIFF_ERR_INVALID, "tol must be > 0");
  if (maxit < 1) return fail(MUDIFF_ERR_INVALID, "maxit < 1");
  GLayout L = glayout(h, R, restart);
  if (!workspace) return fail(MUDIFF_ERR_INVALID, "workspace is NULL");
  if (ws_bytes < L.total) return fail(MUDIFF_ERR_NOMEM, "gmres workspace needs " + std::to_string(L.total) + " bytes");
  if (((uintptr_t)workspace) & 255) return fail(MUDIFF_ERR_INVALID, "workspace must be 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  int rc = prepare_apply(h, R, st);  // uploads happen outside any graph capture
  if (rc != MUDIFF_OK) return rc;
  char* w = (char*)workspace;
  GmresRun G{};
  G.h = h;
  G.st = st;
  G.L = L;
  GState& s = G.s;
  s.C = h->B * R;
  s.R = R;
  s.m = restart;
  s.maxit = maxit;
  s.tol = tol;
  s.NT = L.NT;
  s.V = (cplx*)(w + L.V);
  s.f = (cplx*)(w + L.f);
  s.x = (cplx*)rho;
  s.ck = (int64_t*)(w + L.ck);
  s.partial = (cplx*)(w + L.partial);
  s.cnt = (int32_t*)(w + L.cnt);
  s.H = (cplx*)(w + L.H);
  s.h1 = (cplx*)(w + L.h1);
  s.g = (cplx*)(w + L.g);
  s.cs = (double*)(w + L.cs);
  s.sn = (cplx*)(w + L.sn);
  s.y = (cplx*)(w + L.y);
  s.normf = (double*)(w + L.normf);
  s.red = (double*)(w + L.red);
  s.inv = (double*)(w + L.inv);
  s.status = (int32_t*)(w + L.status);
  s.inner = (int32_t*)(w + L.inner);
  s.run = (int32_t*)(w + L.run);
  s.jdone = (int32_t*)(w + L.jdone);
  s.iters = (int32_t*)(w + L.iters);
  s.n_inner = (int32_t*)(w + L.ninner);
  s.resvec = resvec;
  G.d_ckf = (int32_t*)(w + L.ckf);
  G.d_ckc = (int32_t*)(w + L.ckc);
  G.d_rowcol = (int32_t*)(w + L.rowcol);
  G.apply_part = (cplx*)(w + L.apply);
  G.apply_cnt = (int32_t*)(w + L.apply + apply_scratch_bytes(h, R) - align256((size_t)R * h->M_all * 4));
  G.h2 = (cplx*)(w + L.h2);

  // chunk table (host) -> device
  std::vector<int64_t> ck;
  std::vector<int32_t> ckf(s.C), ckc(s.C);
  ck.reserve(2 * L.n_chunks);
  int64_t idx = 0;
  for (int b = 0; b < h->B; ++b) {
    const int64_t Nb = h->imode[b + 1] - h->imode[b];
    const int64_t ch = chunk_rows(L.NT);
    for (int r = 0; r < R; ++r) {
      const int c = b * R + r;
      const int64_t base = col_base(h->imode.data(), b, R, r);
      ckf[c] = (int32_t)idx;
      int n = 0;
      for (int64_t o = 0; o < Nb; o += ch, ++n, ++idx) {
        const int64_t len = std::min<int64_t>(ch, Nb - o);
        ck.push_back((int64_t)c | (len << 32));
        ck.push_back(base + o);
      }
      ckc[c] = n;
    }
  }
  HIP_TRY(hipMemcpyAsync((void*)s.ck, ck.data(), ck.size() * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G.d_ckf, ckf.data(), s.C * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(G.d_ckc, ckc.data(), s.C * 4, hipMemcpyHostToDevice, st));
  const unsigned eb = (unsigned)((s.NT + 255) / 256);
  const unsigned cb = (unsigned)((s.C + 63) / 64);
  hipLaunchKernelGGL(k_rowcol, dim3(eb), dim3(256), 0, st, G.d_rowcol, s.NT, R, h->B, h->dv.imode);
  HIP_TRY(hipGetLastError());
  // counters start at zero
  if ((rc = launch_fill_zero(s.cnt, s.C * 4, st)) != MUDIFF_OK) return rc;
  if ((rc = launch_fill_zero(G.apply_cnt, (size_t)R * h->M_all * 4, st)) != MUDIFF_OK) return rc;
  if ((rc = launch_fill_zero(s.n_inner, 4, st)) != MUDIFF_OK) return rc;
  // right-hand side f
  if (beta) {
    if ((rc = launch_rhs(h, R, beta, (cplx*)s.f, 1, st)) != MUDIFF_OK) return rc;
  } else {
    hipLaunchKernelGGL(k_precond_rhs, dim3(eb), dim3(256), 0, st, h->dv, R, (const cplx*)rhs,
                       (cplx*)s.f, -1.0);
    HIP_TRY(hipGetLastError());
  }
  if (resvec) {
    if ((rc = launch_fill_zero(resvec, (size_t)s.C * (maxit + 1) * 8, st)) != MUDIFF_OK) return rc;
  }
  // ||f||
  hipLaunchKernelGGL(k_resid, dim3((unsigned)L.n_chunks), dim3(GS_THREADS), 0, st, s, 0, 0,
                     G.d_ckf, G.d_ckc, s.f);
  hipLaunchKernelGGL(k_setup, dim3(cb), dim3(64), 0, st, s);
  HIP_TRY(hipGetLastError());
  // initial residual V0 = f - A x0 (or f with x0 = 0)
  if (flags & MUDIFF_X0) {
    rc = apply_operator(h, R, s.x, s.V, MUDIFF_OP_A, G.apply_part, G.apply_cnt, s.run, st);
    if (rc != MUDIFF_OK) return rc;
    hipLaunchKernelGGL(k_resid, dim3((unsigned)L.n_chunks), dim3(GS_THREADS), 0, st, s, 2, 1,
                       G.d_ckf, G.d_ckc, (const cplx*)nullptr);
  } else {
    hipLaunchKernelGGL(k_zero_c, dim3(eb), dim3(256), 0, st, s.x, s.NT);
    hipLaunchKernelGGL(k_resid, dim3((unsigned)L.n_chunks), dim3(GS_THREADS), 0, st, s, 1, 1,
                       G.d_ckf, G.d_ckc, (const cplx*)nullptr);
  }
  HIP_TRY(hipGetLastError());

  hipLaunchKernelGGL(k_cycle_begin, dim3(cb), dim3(64), 0, st, s);
  HIP_TRY(hipGetLastError());

  const bool use_graph = (flags & MUDIFF_GRAPH) != 0;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  std::vector<int32_t> hstat(s.C);
  int result = MUDIFF_OK;
  // every cycle performs at least one inner iteration per running column
  for (int64_t cyc = 0; cyc <= (int64_t)maxit; ++cyc) {
    HIP_TRY(hipMemcpyAsync(hstat.data(), s.run, s.C * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    bool any = false;
    for (int c = 0; c < s.C; ++c) any |= hstat[c] != 0;
    if (!any) break;
    if (use_graph) {
      if (!exec) {
        // capture on a private stream (the caller's may be the legacy default
        // stream, which cannot be captured); the graph is launched on `st`
        hipStream_t cap = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        hipError_t be = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (be != hipSuccess) {
          (void)hipStreamDestroy(cap);
          return fail(MUDIFF_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(be));
        }
        GmresRun Gc = G;
        Gc.st = cap;
        int e = enqueue_cycle(Gc, 0, false);
        hipError_t ce = hipStreamEndCapture(cap, &graph);
        (void)hipStreamDestroy(cap);
        if (e != MUDIFF_OK || ce != hipSuccess) {
          if (graph) (void)hipGraphDestroy(graph);
          if (e != MUDIFF_OK) return e;
          return fail(MUDIFF_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
        }
        hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
          (void)hipGraphDestroy(graph);
          return fail(MUDIFF_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
        }
      }
      HIP_TRY(hipGraphLaunch(exec, st));
    } else {
      if ((result = enqueue_cycle(G, 10, true)) != MUDIFF_OK) break;
    }
  }
  if (exec) {
    (void)hipStreamSynchronize(st);
    (void)hipGraphExecDestroy(exec);
  }
  if (graph) (void)hipGraphDestroy(graph);
  if (result != MUDIFF_OK) return result;
  hipLaunchKernelGGL(k_finish, dim3(cb), dim3(64), 0, st, s, flag, relres, iters);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}
