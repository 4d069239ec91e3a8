// Restarted GMRES(m) with the single-scattering preconditioner (paper sec. 5):
// A x = f, A = D^{-1} L, f = -D^{-1} U, one Krylov space per column (instance,
// right-hand side); all columns share each operator application.
//
// Orthogonalisation is classical Gram-Schmidt with selective
// reorthogonalisation (the Daniel-Gragg-Kaufman-Stewart test): one pass
// h = V^H w, and a second pass only when ||w - V h|| < ||w|| / sqrt(2)
// (cancellation), which keeps the basis orthogonal to working precision.  A
// looser threshold (0.1) skips the second pass on cycles of 50 steps without
// changing convergence, but over a 170-step cycle of an ill-conditioned
// low-frequency cluster the one-pass basis loses orthogonality and GMRES
// stalls.  The
// Hessenberg column, the Givens rotations and the residual estimate
// |g_{j+1}| / ||f|| are updated on the device, so the host only synchronises to
// test for the end of a cycle.
//
// Reductions are per column and free of inter-workgroup synchronisation: the
// rows of a column are cut into chunks, every chunk writes its partial sums,
// and the next kernel's workgroups each add all partials of their column in
// chunk order (the same order in every workgroup, so every workgroup derives
// bit-identical sums and decisions; the kernel boundary makes the partials
// visible).  Chunk 0 of a column does the column's Arnoldi bookkeeping.
#include <algorithm>

#include "common.h"

#define GS_THREADS 256
#define GS_WAVES (GS_THREADS / 64)
#define GS_BATCH 4
#define GS_REORTH_ETA 0.70710678118654752  // 1 / sqrt(2)

enum { ST_RUN = 0, ST_CONV = 1, ST_BREAK = 2, ST_MAXIT = 3 };

struct GState {
  int C, R, m, maxit;
  double tol;
  int64_t NT;               // complex entries of one multivector
  cplx* V;                  // [(m+1)][NT]
  const cplx* f;            // [NT] preconditioned right-hand side
  cplx* x;                  // [NT] iterate (caller's rho)
  const int64_t* ck;        // [n_chunks][2]: (col | len << 32), begin
  const int32_t* ckmap;     // chunks of the still-iterating columns, or NULL: all
  const int32_t* ckf;       // [C] first chunk of each column
  const int32_t* ckc;       // [C] chunks of each column
  cplx* P1;                 // [n_chunks][m+1] first-pass partials (slot m: ||w||^2)
  cplx* P2;                 // [n_chunks][m+1] second-pass partials (slot m: ||w1||^2)
  cplx* H;                  // [C][(m+1) m]
  cplx* g;                  // [C][m+1]
  double* cs;               // [C][m]
  cplx* sn;                 // [C][m]
  cplx* y;                  // [C][m]
  double* normf;            // [C]
  double* red;              // [C] scalar reduction result
  int32_t* status;          // [C]
  int32_t* inner;           // [C] active in the current Arnoldi cycle
  int32_t* reorth;          // [C] the current step takes a second pass
  double* inv;              // [C] 1 / ||V0|| at the start of a cycle
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

// Chunk of this workgroup (through the list of chunks of still-iterating
// columns when one is set): returns the chunk index, which also indexes the
// partial-sum buffers.
__device__ __forceinline__ int decode_chunk(const GState& s, int* col, int* len, int64_t* begin) {
  const int gidx = s.ckmap ? s.ckmap[blockIdx.x] : (int)blockIdx.x;
  const int64_t a = s.ck[2 * gidx];
  *col = (int)(a & 0xffffffff);
  *len = (int)(a >> 32);
  *begin = s.ck[2 * gidx + 1];
  return gidx;
}

// Arnoldi bookkeeping of column c after step j (one thread): Hessenberg column
// hl = h1 + h2 with subdiagonal hn, previous Givens rotations, the new rotation,
// the residual estimate |g_{j+1}| / ||f|| and the stopping test.  hl, csl, snl
// are the column and the rotations 0..j-1 staged in LDS: the rotation chain
// carries one value in registers, so no step waits on a global load.
// Values of column c that the Arnoldi step reads from global memory, loaded at
// the start of the kernel so that their latency overlaps the reductions.
struct ArnoldiPre {
  cplx gj;     // g_j
  int it;      // inner iterations so far
  double nf;   // ||f||
};

__device__ __forceinline__ ArnoldiPre arnoldi_preload(const GState& s, int c, int j) {
  return ArnoldiPre{s.g[(int64_t)c * (s.m + 1) + j], s.iters[c], s.normf[c]};
}

__device__ void arnoldi_step(const GState& s, int c, int j, const cplx* hl, const double* csl,
                             const cplx* snl, double hn, const ArnoldiPre& pre) {
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
  const cplx gj = pre.gj;
  const cplx gj1 = cmul(cscale(cconj(sr), -1.0), gj);
  gc[j + 1] = gj1;
  gc[j] = cscale(gj, cr);
  const int it = pre.it + 1;
  s.iters[c] = it;
  const double rel = sqrt(cabs2(gj1)) / pre.nf;
  if (s.resvec) s.resvec[(int64_t)c * (s.maxit + 1) + it] = rel;
  s.jdone[c] = j + 1;
  const bool finite = isfinite(rel) && isfinite(hn);
  if (!finite) s.status[c] = ST_BREAK;
  if (!finite || rel <= s.tol || hn == 0.0 || it >= s.maxit || j + 1 >= s.m) {
    s.inner[c] = 0;
    atomicSub(s.n_inner, 1);
  }
}

// Sums, in chunk order, slots 0..ns-1 of the partials of the nck chunks that
// start at pbase (slot ns-1 read from slot `last` when last >= 0) into out[]
// (LDS); returns, in every thread, sum |out[i]|^2 over i < nd.  Wave w takes
// slots w, w + GS_WAVES, ...; its lanes stride over the chunks.
__device__ double column_sums(const cplx* __restrict__ pbase, int m1, int nck, int ns, int last,
                              int nd, cplx* out, double* sred) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double sq = 0.0;
  for (int i0 = wv; i0 < ns; i0 += GS_WAVES * GS_BATCH) {
    cplx a[GS_BATCH];
#pragma unroll
    for (int u = 0; u < GS_BATCH; ++u) {
      a[u] = cmk(0.0, 0.0);
      const int i = i0 + u * GS_WAVES;
      if (i < ns) {
        const int sl = (i == ns - 1 && last >= 0) ? last : i;
        for (int k = lane; k < nck; k += 64) a[u] = cadd(a[u], pbase[(int64_t)k * m1 + sl]);
      }
    }
#pragma unroll
    for (int u = 0; u < GS_BATCH; ++u) {
      a[u].x = wave_sum(a[u].x);
      a[u].y = wave_sum(a[u].y);
      const int i = i0 + u * GS_WAVES;
      if (i < ns && lane == 0) out[i] = a[u];
      if (i < nd) sq += cabs2(a[u]);
    }
  }
  if (lane == 0) sred[wv] = sq;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < GS_WAVES; ++k) t += sred[k];
  __syncthreads();  // sred reusable
  return t;
}

// Dots of the chunk's rows of wl against V_0..V_j into part[0..j] (one wave
// per vector, GS_BATCH vectors in flight).
__device__ void chunk_dots(const GState& s, int j, int64_t o, int len, const cplx* wl,
                           cplx* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i0 = wv; i0 <= j; i0 += GS_WAVES * GS_BATCH) {
    cplx a[GS_BATCH];
    const cplx* vi[GS_BATCH];
#pragma unroll
    for (int u = 0; u < GS_BATCH; ++u) {
      a[u] = cmk(0.0, 0.0);
      const int i = min(i0 + u * GS_WAVES, j);  // past j: a valid row, result unused
      vi[u] = s.V + (int64_t)i * s.NT + o;
    }
#pragma unroll 4
    for (int r = lane; r < len; r += 64) {
      const cplx wr = wl[r];
#pragma unroll
      for (int u = 0; u < GS_BATCH; ++u) cmacc(a[u], vi[u][r], wr);
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
}

// Sum over the block of a per-thread value (every thread gets the total).
__device__ double block_sum(double v, double* sred) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < GS_WAVES; ++k) t += sred[k];
  __syncthreads();
  return t;
}

// The RPT rows tid + k * GS_THREADS (k < RPT) of a chunk of len <= RPT *
// GS_THREADS rows: v[k] = w[r_k] - sum_{i <= j} h_i V_i[r_k], with 32 / RPT
// basis vectors per round, so that 32 loads are in flight per thread.
template <int RPT>
__device__ __forceinline__ void project_rows(const GState& s, int j, const cplx* __restrict__ wc,
                                             const cplx* __restrict__ vc, int len, const cplx* h,
                                             cplx (&v)[RPT]) {
  constexpr int U = 32 / RPT;
  int r[RPT];
  bool ok[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    r[k] = threadIdx.x + k * GS_THREADS;
    ok[k] = r[k] < len;
    v[k] = ok[k] ? wc[r[k]] : cmk(0.0, 0.0);
  }
  int i = 0;
  for (; i + U - 1 <= j; i += U) {
    cplx t[U][RPT];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < RPT; ++k)
        t[u][k] = ok[k] ? vc[(int64_t)(i + u) * s.NT + r[k]] : cmk(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const cplx hu = h[i + u];
#pragma unroll
      for (int k = 0; k < RPT; ++k) v[k] = csub(v[k], cmul(hu, t[u][k]));
    }
  }
  for (; i <= j; ++i) {
    const cplx hi = h[i];
#pragma unroll
    for (int k = 0; k < RPT; ++k)
      if (ok[k]) v[k] = csub(v[k], cmul(hi, vc[(int64_t)i * s.NT + r[k]]));
  }
}

// Chunk 0 of column c, at the start of the kernel: the previous rotations go
// to LDS behind the slots 0..j+1 that the column sums will fill (when they fit)
// and thread 0 loads what the Arnoldi step reads from global memory.
__device__ bool stage_rotations(const GState& s, int c, int j, cplx* hl) {
  const bool fits = 2 * j + 2 + (j + 1) / 2 <= MUDIFF_MAX_RESTART + 1;
  if (fits) {
    const double* csg = s.cs + (int64_t)c * s.m;
    const cplx* sng = s.sn + (int64_t)c * s.m;
    for (int i = threadIdx.x; i < j; i += GS_THREADS) {
      hl[j + 2 + i] = sng[i];
      reinterpret_cast<double*>(hl + 2 * j + 2)[i] = csg[i];
    }
  }
  return fits;  // visible to thread 0 after the next barrier
}

// Chunk 0 of column c: the Arnoldi/Givens step on h = hl[0..j].
__device__ void column_step(const GState& s, int c, int j, const cplx* hl, double hn, bool staged,
                            const ArnoldiPre& pre) {
  __syncthreads();  // hl and the staged rotations complete
  if (threadIdx.x != 0) return;
  const double* csl = staged ? reinterpret_cast<const double*>(hl + 2 * j + 2)
                             : s.cs + (int64_t)c * s.m;
  const cplx* snl = staged ? hl + j + 2 : s.sn + (int64_t)c * s.m;
  arnoldi_step(s, c, j, hl, csl, snl, hn, pre);
}

// Chunk partial sums of an operator apply still to be added (one-lane-per-pair
// path): w = A V[j] is completed row by row by the first Gram-Schmidt pass.
struct PendingApply {
  DevView v;
  const cplx* part;
  int64_t part_total;
  const int32_t* nchunk;
  const int64_t* partoff;
};

// Pass 1 of step j on w = V[j+1]: partial h = V^H w and ||w||^2 into P1.  With
// FIN, w is first formed from the apply's chunk partial sums and stored.
template <bool FIN>
__global__ __launch_bounds__(GS_THREADS) void k_gs_dots(GState s, int j, PendingApply pa) {
  __shared__ cplx wl[1024];
  __shared__ double sred[GS_WAVES];
  int c, len;
  int64_t o;
  const int gi = decode_chunk(s, &c, &len, &o);
  if (!s.inner[c]) return;
  const int m1 = s.m + 1;
  cplx* w = s.V + (int64_t)(j + 1) * s.NT + o;
  double nn = 0.0;
  if (FIN) {
    const int b = c / s.R, r = c - (c / s.R) * s.R;
    const int64_t i0 = pa.v.imode[b] + (o - col_base(pa.v.imode, b, s.R, r));
    const cplx* xj = s.V + (int64_t)j * s.NT + o;
    const cplx* pr = pa.part + (int64_t)r * pa.part_total;
    for (int rr = threadIdx.x; rr < len; rr += GS_THREADS) {
      const int64_t i = i0 + rr;
      const cplx v =
          finalize(pa.v, MUDIFF_OP_A, i, xj[rr], lane_chunk_sum(pa.v, pr, pa.nchunk, pa.partoff, b, i));
      w[rr] = v;
      wl[rr] = v;
      nn += cabs2(v);
    }
  } else {
    for (int r = threadIdx.x; r < len; r += GS_THREADS) {
      const cplx v = w[r];
      wl[r] = v;
      nn += cabs2(v);
    }
  }
  nn = block_sum(nn, sred);  // (its barrier also publishes wl)
  cplx* part = s.P1 + (int64_t)gi * m1;
  chunk_dots(s, j, o, len, wl, part);
  if (threadIdx.x == 0) part[s.m] = cmk(nn, 0.0);
}

// Pass 2: every workgroup of column c adds the P1 partials (h, ||w||^2) and
// takes the same decision.  Without cancellation, V[j+1] = (w - V h) / h_{j+1,j}
// with h_{j+1,j}^2 = ||w||^2 - ||h||^2, and chunk 0 does the Arnoldi step.
// Otherwise w1 = w - V h is stored in place and its partials V^H w1, ||w1||^2
// go to P2 for the second pass.
template <int RPT>
__global__ __launch_bounds__(GS_THREADS) void k_gs_update(GState s, int j) {
  __shared__ cplx hl[MUDIFF_MAX_RESTART + 1];
  __shared__ cplx wl[1024];
  __shared__ double sred[GS_WAVES];
  int c, len;
  int64_t o;
  const int gi = decode_chunk(s, &c, &len, &o);
  if (!s.inner[c]) return;
  const int m1 = s.m + 1;
  const int nck = s.ckc[c];
  const bool first_chunk = gi == s.ckf[c];
  bool staged = false;
  ArnoldiPre pre{};
  if (first_chunk) {
    staged = stage_rotations(s, c, j, hl);
    if (threadIdx.x == 0) pre = arnoldi_preload(s, c, j);
  }
  const double hsq = column_sums(s.P1 + (int64_t)s.ckf[c] * m1, m1, nck, j + 2, s.m, j + 1, hl, sred);
  const double nw = hl[j + 1].x;
  const double hn2 = nw - hsq;
  // ||w - V h||^2 <= eta^2 ||w||^2 (or not finite): second pass
  const bool second = !(hn2 > GS_REORTH_ETA * GS_REORTH_ETA * nw);
  cplx* w = s.V + (int64_t)(j + 1) * s.NT + o;
  const cplx* vr0 = s.V + o;
  cplx v[RPT];
  project_rows<RPT>(s, j, w, vr0, len, hl, v);
  if (!second) {
    const double hn = sqrt(hn2);
    const double inv = 1.0 / hn;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = threadIdx.x + k * GS_THREADS;
      if (r < len) w[r] = cscale(v[k], inv);
    }
    if (first_chunk) {
      if (threadIdx.x == 0) s.reorth[c] = 0;
      column_step(s, c, j, hl, hn, staged, pre);
    }
    return;
  }
  double nn = 0.0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = threadIdx.x + k * GS_THREADS;
    if (r < len) {
      w[r] = v[k];
      wl[r] = v[k];
      nn += cabs2(v[k]);
    }
  }
  nn = block_sum(nn, sred);
  cplx* part = s.P2 + (int64_t)gi * m1;
  chunk_dots(s, j, o, len, wl, part);
  if (threadIdx.x == 0) {
    part[s.m] = cmk(nn, 0.0);
    if (first_chunk) s.reorth[c] = 1;
  }
}

// Second pass (columns flagged by k_gs_update): h2 = sum of the P2 partials,
// V[j+1] = (w1 - V h2) / h_{j+1,j}, h_{j+1,j}^2 = ||w1||^2 - ||h2||^2; the
// Hessenberg column is h + h2 (h re-added from P1).
template <int RPT>
__global__ __launch_bounds__(GS_THREADS) void k_gs_reorth(GState s, int j) {
  __shared__ cplx hl[MUDIFF_MAX_RESTART + 1];
  __shared__ cplx h2l[MUDIFF_MAX_RESTART + 1];
  __shared__ double sred[GS_WAVES];
  int c, len;
  int64_t o;
  const int gi = decode_chunk(s, &c, &len, &o);
  if (!s.inner[c] || !s.reorth[c]) return;
  const int m1 = s.m + 1;
  const int nck = s.ckc[c];
  const bool first_chunk = gi == s.ckf[c];
  bool staged = false;
  ArnoldiPre pre{};
  if (first_chunk) {
    staged = stage_rotations(s, c, j, hl);
    if (threadIdx.x == 0) pre = arnoldi_preload(s, c, j);
    (void)column_sums(s.P1 + (int64_t)s.ckf[c] * m1, m1, nck, j + 1, -1, 0, hl, sred);
  }
  const double h2sq =
      column_sums(s.P2 + (int64_t)s.ckf[c] * m1, m1, nck, j + 2, s.m, j + 1, h2l, sred);
  const double hn2 = h2l[j + 1].x - h2sq;
  const double hn = sqrt(hn2 > 0.0 ? hn2 : 0.0);
  const double inv = 1.0 / hn;  // unused when hn == 0: the column stops
  cplx* w = s.V + (int64_t)(j + 1) * s.NT + o;
  const cplx* vr0 = s.V + o;
  cplx v[RPT];
  project_rows<RPT>(s, j, w, vr0, len, h2l, v);
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = threadIdx.x + k * GS_THREADS;
    if (r < len) w[r] = cscale(v[k], inv);
  }
  if (!first_chunk) return;
  for (int i = threadIdx.x; i <= j; i += GS_THREADS) hl[i] = cadd(hl[i], h2l[i]);
  column_step(s, c, j, hl, hn, staged, pre);
}

// Chunked per-column sum of |src|^2: partials into P1 slot 0 (running columns
// only if `only_run`), added by k_col_sum.  When mode 2: src = f - src first
// (stored back); mode 1: src = f; mode 0: src = vec_in.
__global__ __launch_bounds__(GS_THREADS) void k_resid(GState s, int mode, int only_run,
                                                      const cplx* __restrict__ vec_in) {
  __shared__ double sred[GS_WAVES];
  int c, len;
  int64_t o;
  const int gi = decode_chunk(s, &c, &len, &o);
  if (only_run && !s.run[c]) return;
  double a = 0.0;
  for (int r = threadIdx.x; r < len; r += GS_THREADS) {
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
  a = block_sum(a, sred);
  if (threadIdx.x == 0) s.P1[(int64_t)gi * (s.m + 1)] = cmk(a, 0.0);
}

// red[c] = sum of the k_resid partials of column c (one wave per column,
// chunk order fixed).
__global__ __launch_bounds__(64) void k_col_sum(GState s, int only_run) {
  const int c = blockIdx.x, lane = threadIdx.x;
  if (only_run && !s.run[c]) return;
  const int m1 = s.m + 1;
  double t = 0.0;
  for (int k = lane; k < s.ckc[c]; k += 64) t += s.P1[(int64_t)(s.ckf[c] + k) * m1].x;
  t = wave_sum(t);
  if (lane == 0) s.red[c] = t;
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
// Rows per reduction chunk: enough chunks over all columns to fill the chip
// (about 2048), few enough per column (<= 128 where possible) that every
// workgroup can add all partials of its column, and 256..1024 rows each (one
// row per thread at least; 1024 = the LDS row buffer of the Gram-Schmidt
// kernels).
static int64_t chunk_rows(int64_t NT, int64_t ncol_max) {
  auto up64 = [](int64_t v) { return (v + 63) / 64 * 64; };
  int64_t ch = std::max(up64((NT + 2047) / 2048), up64((ncol_max + 127) / 128));
  return std::min<int64_t>(std::max<int64_t>(ch, GS_THREADS), 1024);
}

static int64_t max_col_rows(const mudiff_ctx* h) {
  int64_t mx = 1;
  for (int b = 0; b < h->B; ++b) mx = std::max(mx, h->imode[b + 1] - h->imode[b]);
  return mx;
}

namespace {
struct GLayout {
  size_t V, f, apply, ck, ckmap, ckf, ckc, rowcol, P1, P2, H, g, cs, sn, y, normf, red, inv, status,
      inner, reorth, run, jdone, iters, ninner, total;
  int64_t n_chunks, NT;
};

GLayout glayout(mudiff_ctx* h, int R, int m) {
  GLayout L{};
  const int64_t C = (int64_t)h->B * R;
  const int64_t NT = (int64_t)R * h->N_all;
  L.NT = NT;
  int64_t nck = 0;
  const int64_t ch = chunk_rows(NT, max_col_rows(h));
  for (int b = 0; b < h->B; ++b) {
    const int64_t Nb = h->imode[b + 1] - h->imode[b];
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
  L.ckmap = take(nck * 4);
  L.ckf = take(C * 4);
  L.ckc = take(C * 4);
  L.rowcol = take(NT * 4);
  L.P1 = take(nck * (m + 1) * 16);
  L.P2 = take(nck * (m + 1) * 16);
  L.H = take(C * (m + 1) * m * 16);
  L.g = take(C * (m + 1) * 16);
  L.cs = take(C * m * 8);
  L.sn = take(C * m * 16);
  L.y = take(C * m * 16);
  L.normf = take(C * 8);
  L.red = take(C * 8);
  L.inv = take(C * 8);
  L.status = take(C * 4);
  L.inner = take(C * 4);
  L.reorth = take(C * 4);
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
  int32_t* d_ckmap;
  cplx* apply_part;
  int32_t* apply_cnt;
  hipStream_t st;
  std::vector<int64_t> ck;      // host copy of the chunk table
  std::vector<int32_t> ckmap;   // chunks of the running columns (straggler phase)
  int n_compact = 0;            // running columns when the list was built (0: all chunks)
  int rpt = 1;                  // chunk rows per Gram-Schmidt thread (1, 2 or 4)
};

// Straggler phase (few running columns): the Gram-Schmidt kernels run over
// the chunks of the running columns only, and the MFMA apply over the tiles
// that hold one.  Built at a cycle boundary from the running set `run` of the
// coming cycle (inner steps and the residual apply only touch those columns).
static int compact_columns(GmresRun& G, const std::vector<int32_t>& run, int n_run) {
  G.ckmap.clear();
  for (int64_t k = 0; k < G.L.n_chunks; ++k)
    if (run[(int)(G.ck[2 * k] & 0xffffffff)]) G.ckmap.push_back((int32_t)k);
  if (!G.ckmap.empty()) {
    HIP_TRY(hipMemcpyAsync(G.d_ckmap, G.ckmap.data(), G.ckmap.size() * 4, hipMemcpyHostToDevice, G.st));
    HIP_TRY(hipStreamSynchronize(G.st));
  }
  G.n_compact = n_run;
  return apply_set_tail(G.h, G.s.R, true, G.apply_part, G.st, run.data());
}

// One restart cycle (Arnoldi steps + solution update + true residual).
static int enqueue_cycle(GmresRun& G, int check_every, bool host_checks) {
  GState& s = G.s;
  const unsigned cb = (unsigned)((s.C + 63) / 64);
  const unsigned eb = (unsigned)((s.NT + 255) / 256);
  hipLaunchKernelGGL(k_scale_v0, dim3(eb), dim3(256), 0, G.st, s, s.NT, G.d_rowcol);
  HIP_TRY(hipGetLastError());
  for (int j = 0; j < s.m; ++j) {
    bool pending = false;
    int rc = apply_operator_split(G.h, s.R, s.V + (int64_t)j * s.NT,
                                  s.V + (int64_t)(j + 1) * s.NT, MUDIFF_OP_A, G.apply_part,
                                  G.apply_cnt, s.inner, G.st, &pending);
    if (rc != MUDIFF_OK) return rc;
    // Gram-Schmidt over all chunks, or the running columns' chunks only
    GState sg = s;
    unsigned nb = (unsigned)G.L.n_chunks;
    if (G.n_compact > 0) {
      sg.ckmap = G.d_ckmap;
      nb = (unsigned)G.ckmap.size();
    }
    PendingApply pa{G.h->dv, G.apply_part, G.h->plan.part_total, G.h->plan.d_nchunk,
                    G.h->plan.d_partoff};
    if (nb > 0) {
      if (pending)
        hipLaunchKernelGGL(k_gs_dots<true>, dim3(nb), dim3(GS_THREADS), 0, G.st, sg, j, pa);
      else
        hipLaunchKernelGGL(k_gs_dots<false>, dim3(nb), dim3(GS_THREADS), 0, G.st, sg, j, pa);
      switch (G.rpt) {  // chunk rows per thread
        case 1:
          hipLaunchKernelGGL(k_gs_update<1>, dim3(nb), dim3(GS_THREADS), 0, G.st, sg, j);
          hipLaunchKernelGGL(k_gs_reorth<1>, dim3(nb), dim3(GS_THREADS), 0, G.st, sg, j);
          break;
        case 2:
          hipLaunchKernelGGL(k_gs_update<2>, dim3(nb), dim3(GS_THREADS), 0, G.st, sg, j);
          hipLaunchKernelGGL(k_gs_reorth<2>, dim3(nb), dim3(GS_THREADS), 0, G.st, sg, j);
          break;
        default:
          hipLaunchKernelGGL(k_gs_update<4>, dim3(nb), dim3(GS_THREADS), 0, G.st, sg, j);
          hipLaunchKernelGGL(k_gs_reorth<4>, dim3(nb), dim3(GS_THREADS), 0, G.st, sg, j);
          break;
      }
    }
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
                     (const cplx*)nullptr);
  hipLaunchKernelGGL(k_col_sum, dim3(s.C), dim3(64), 0, G.st, s, 1);
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
  int rc = MUDIFF_OK;
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
  s.ckmap = nullptr;
  G.d_ckmap = (int32_t*)(w + L.ckmap);
  s.P1 = (cplx*)(w + L.P1);
  s.P2 = (cplx*)(w + L.P2);
  s.H = (cplx*)(w + L.H);
  s.g = (cplx*)(w + L.g);
  s.cs = (double*)(w + L.cs);
  s.sn = (cplx*)(w + L.sn);
  s.y = (cplx*)(w + L.y);
  s.normf = (double*)(w + L.normf);
  s.red = (double*)(w + L.red);
  s.inv = (double*)(w + L.inv);
  s.status = (int32_t*)(w + L.status);
  s.inner = (int32_t*)(w + L.inner);
  s.reorth = (int32_t*)(w + L.reorth);
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
  s.ckf = G.d_ckf;
  s.ckc = G.d_ckc;
  // operator schedule (MFMA: tuned on V0 = 0 -> V1 on first use of R); uploads
  // happen here, outside any graph capture
  if ((rc = launch_fill_zero(s.V, (size_t)s.NT * 16, st)) != MUDIFF_OK) return rc;
  if ((rc = apply_set_tail(h, R, false, G.apply_part, st, nullptr)) != MUDIFF_OK) return rc;
  if ((rc = prepare_apply(h, R, s.V, s.V + s.NT, G.apply_part, st)) != MUDIFF_OK) return rc;

  // chunk table (host) -> device
  std::vector<int64_t>& ck = G.ck;
  std::vector<int32_t> ckf(s.C), ckc(s.C);
  ck.reserve(2 * L.n_chunks);
  int64_t idx = 0;
  const int64_t ch = chunk_rows(L.NT, max_col_rows(h));
  G.rpt = ch <= GS_THREADS ? 1 : (ch <= 2 * GS_THREADS ? 2 : 4);
  for (int b = 0; b < h->B; ++b) {
    const int64_t Nb = h->imode[b + 1] - h->imode[b];
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
  hipLaunchKernelGGL(k_resid, dim3((unsigned)L.n_chunks), dim3(GS_THREADS), 0, st, s, 0, 0, s.f);
  hipLaunchKernelGGL(k_col_sum, dim3(s.C), dim3(64), 0, st, s, 0);
  hipLaunchKernelGGL(k_setup, dim3(cb), dim3(64), 0, st, s);
  HIP_TRY(hipGetLastError());
  // initial residual V0 = f - A x0 (or f with x0 = 0)
  if (flags & MUDIFF_X0) {
    rc = apply_operator(h, R, s.x, s.V, MUDIFF_OP_A, G.apply_part, G.apply_cnt, s.run, st);
    if (rc != MUDIFF_OK) return rc;
    hipLaunchKernelGGL(k_resid, dim3((unsigned)L.n_chunks), dim3(GS_THREADS), 0, st, s, 2, 1,
                       (const cplx*)nullptr);
  } else {
    hipLaunchKernelGGL(k_zero_c, dim3(eb), dim3(256), 0, st, s.x, s.NT);
    hipLaunchKernelGGL(k_resid, dim3((unsigned)L.n_chunks), dim3(GS_THREADS), 0, st, s, 1, 1,
                       (const cplx*)nullptr);
  }
  hipLaunchKernelGGL(k_col_sum, dim3(s.C), dim3(64), 0, st, s, 1);
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
    int n_run = 0;
    for (int c = 0; c < s.C; ++c) n_run += hstat[c] != 0;
    if (n_run == 0) break;
    if (!use_graph && s.C >= 32 && n_run * 32 <= s.C && (G.n_compact == 0 || n_run * 2 <= G.n_compact)) {
      if ((result = compact_columns(G, hstat, n_run)) != MUDIFF_OK) break;
    }
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
  return apply_set_tail(h, R, false, G.apply_part, st, nullptr);  // back to the tuned schedule
}
