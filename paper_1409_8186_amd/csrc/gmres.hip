// Restarted GMRES(m) with the single-scattering preconditioner (paper sec. 5):
// A x = f, A = D^{-1} L, f = -D^{-1} U, one Krylov space per column (instance,
// right-hand side); all columns share each operator application.
//
// Orthogonalisation is classical Gram-Schmidt applied twice with the second
// pass delayed by one step (DCGS2): step j applies the operator to the
// candidate u = V[j] (orthogonalised once), and one reduction gives both the
// reorthogonalisation coefficients of u, s = V^H u, and the projection of
// w = A u, z = V^H w.  One sweep over the basis then finalises q_j = (u - V s)
// / rho and forms the next candidate (w - V z - g_j q_j) / rho; the Hessenberg
// column j-1 receives the correction s (from A q_{j-1} = V h + u), and A q_j
// follows from A u by linearity.  So each step reads the basis twice (once for
// the dots, once for the update) and has one reduction, against four reads and
// two or three reductions for CGS2; the basis stays orthogonal to working
// precision as with CGS2.  The Givens rotations and the residual estimate
// |g_{j+1}| / ||f|| are updated on the device one step after the operator
// application (so a converging column performs one extra application); the
// host only synchronises to test for the end of a cycle.
//
// Reductions are per column and free of inter-workgroup synchronisation: the
// rows of a column are cut into chunks, every chunk writes its partial sums,
// and the next kernel's workgroups each add all partials of their column in
// chunk order (the same order in every workgroup, so every workgroup derives
// bit-identical sums and decisions; the kernel boundary makes the partials
// visible).  Chunk 0 of a column does the column's Arnoldi bookkeeping.
#include <algorithm>

#include "common.h"
#include "ritz.h"

#define GS_THREADS 256
#define GS_WAVES (GS_THREADS / 64)
#define GS_BATCH 4
// Gram-Schmidt launches with at most this many chunks split the basis (dots)
// and the rows (update) over more workgroups
#define GS_SPREAD_CHUNKS 64

enum { ST_RUN = 0, ST_CONV = 1, ST_BREAK = 2, ST_MAXIT = 3 };

struct GState {
  int C, R, m, maxit;
  int op;                   // MUDIFF_OP_A (preconditioned) or MUDIFF_OP_L
  double tol;
  int64_t NT;               // complex entries of one multivector
  cplx* V;                  // [(m+1)][NT]
  const cplx* f;            // [NT] preconditioned right-hand side
  cplx* x;                  // [NT] iterate (caller's rho)
  const int64_t* ck;        // [n_chunks][2]: (col | len << 32), begin
  const int32_t* ckmap;     // chunks of the still-iterating columns, or NULL: all
  const int32_t* ckf;       // [C] first chunk of each column
  const int32_t* ckc;       // [C] chunks of each column
  int sl;                   // partial-sum slots per chunk (2m + 2)
  cplx* P1;                 // [n_chunks][sl] partial sums
  cplx* H;                  // [C][m][m+1] Hessenberg columns after the Givens rotations
  cplx* Hraw;               // [C][m][m+1] Hessenberg columns as formed
  cplx* htent;              // [C][m+1] tentative column of the current step
  cplx* g;                  // [C][m+1]
  double* cs;               // [C][m]
  cplx* sn;                 // [C][m]
  cplx* y;                  // [C][m]
  double* normf;            // [C]
  double* red;              // [C] scalar reduction result
  int32_t* status;          // [C]
  int32_t* inner;           // [C] active in the current Arnoldi cycle
  double* inv;              // [C] 1 / ||V0|| at the start of a cycle
  int32_t* run;             // [C] running at the start of the current cycle
  int32_t* jdone;           // [C] Arnoldi steps done in the current cycle
  int32_t* iters;           // [C] inner iterations so far
  int32_t* n_inner;         // [1] columns still active in the cycle
  double* resvec;           // [C][maxit+1] or NULL
  // s-step GMRES (ss > 0)
  int ss;                   // Newton vectors per block
  int sl2;                  // partial-sum slots per chunk, (m + 1) ss
  cplx* P2;                 // [n_chunks][(m + 1) ss]
  cplx* theta;              // [ss][C] shifts
  cplx* sab;                // [ss][C][2] (1 / sigma, -theta / sigma) of each Newton step
  cplx* xprev;              // [NT] iterate at the start of the s-step cycle
  cplx* vprev;              // [NT] its residual f - A x (unscaled)
  double* rprev;            // [C] its squared norm
  int32_t* ssbad;           // [1] set when a cycle raised a column's true residual
  cplx* sC;                 // [C][2][(m + 1) ss] projections of the two passes
  cplx* sR;                 // [C][2][ss ss] Cholesky factors of the two passes
  cplx* sRi;                // [C][ss ss] inverse of the current pass's factor
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

__device__ bool arnoldi_step(const GState& s, int c, int j, const cplx* hl, const double* csl,
                             const cplx* snl, double hn, const ArnoldiPre& pre,
                             ArnoldiPre* next = nullptr, double* cs_out = nullptr,
                             cplx* sn_out = nullptr) {
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
  if (cs_out) *cs_out = cr;
  if (sn_out) *sn_out = sr;
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
  if (next) *next = ArnoldiPre{gj1, it, pre.nf};
  if (!finite || rel <= s.tol || hn == 0.0 || it >= s.maxit || j + 1 >= s.m) {
    s.inner[c] = 0;
    atomicSub(s.n_inner, 1);
    return true;
  }
  return false;
}

// ------------------------------------------------------------------ delayed CGS2
// Partial-sum slots of a chunk (stride s.sl = 2m + 2) at step j:
//   [0, j)   V_i^H u        (reorthogonalisation of the candidate u = V[j])
//   [j, 2j)  V_i^H w        (projection of w = A u)
//   2j       u^H u,   2j+1  u^H w

// Dots of the chunk's rows of ul and wl against V_ib..V_{ie-1}: part[i] = V_i^H u,
// part[j + i] = V_i^H w (when has_w).  One wave per vector, GS_BATCH vectors
// in flight, both products from one read of V_i.
__device__ __forceinline__ void chunk_dots2(const GState& s, int j, int ib, int ie, int64_t o, int len,
                                            const cplx* ul, const cplx* wl, bool has_w,
                                            cplx* __restrict__ part) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i0 = ib + wv; i0 < ie; i0 += GS_WAVES * GS_BATCH) {
    cplx au[GS_BATCH], aw[GS_BATCH];
    const cplx* vi[GS_BATCH];
#pragma unroll
    for (int u = 0; u < GS_BATCH; ++u) {
      au[u] = cmk(0.0, 0.0);
      aw[u] = cmk(0.0, 0.0);
      const int i = min(i0 + u * GS_WAVES, ie - 1);  // past ie-1: a valid row, result unused
      vi[u] = s.V + (int64_t)i * s.NT + o;
    }
#pragma unroll 4
    for (int r = lane; r < len; r += 64) {
      const cplx ur = ul[r];
      const cplx wr = has_w ? wl[r] : cmk(0.0, 0.0);
#pragma unroll
      for (int u = 0; u < GS_BATCH; ++u) {
        const cplx vv = vi[u][r];
        cmacc(au[u], vv, ur);
        cmacc(aw[u], vv, wr);
      }
    }
    // the 4 GS_BATCH sums reduce-scattered: lane l holds value l >> 2
    double val[4 * GS_BATCH];
#pragma unroll
    for (int u = 0; u < GS_BATCH; ++u) {
      val[4 * u] = au[u].x;
      val[4 * u + 1] = au[u].y;
      val[4 * u + 2] = aw[u].x;
      val[4 * u + 3] = aw[u].y;
    }
    lane_reduce_scatter<4 * GS_BATCH>(val, lane);
    if ((lane & 3) == 0) {
      const int vi = lane >> 2, u = vi >> 2, comp = vi & 3;
      const int i = i0 + u * GS_WAVES;
      if (i < ie && (comp < 2 || has_w)) {
        double* dst = reinterpret_cast<double*>(part + (comp < 2 ? i : j + i));
        dst[comp & 1] = val[0];
      }
    }
  }
}

// Sums over the block of NV per-thread values in one LDS round (every thread
// gets the totals, added in wave order).  sred holds NV * GS_WAVES doubles.
template <int NV>
__device__ void block_sums(double (&v)[NV], double* sred) {
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    v[q] = wave_sum(v[q]);
    if ((threadIdx.x & 63) == 0) sred[q * GS_WAVES + (threadIdx.x >> 6)] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double t = 0.0;
    for (int k = 0; k < GS_WAVES; ++k) t += sred[q * GS_WAVES + k];
    v[q] = t;
  }
  __syncthreads();  // sred reusable
}

__device__ double block_sum(double v, double* sred) {
  double a[1] = {v};
  block_sums<1>(a, sred);
  return a[0];
}

// Sums over the nck chunks of a column, in a fixed order, of slots 0..ns-1 of
// their partials (at pbase, stride sl; slot ns-1 read from slot `last` when
// last >= 0) into out[] (LDS); returns, in every thread, sum |out[i]|^2 over
// i < nd.  Loads run along the slots (coalesced).  Up to 8 chunks: a thread
// adds one slot over all chunks in chunk order.  More: wave g adds chunks g,
// g + GS_WAVES, ... (16 loads in flight) for 64 slots at a time, and the wave
// sums are added in wave order through tmp[GS_WAVES * 64].  Every workgroup
// of a column so derives the same values.
__device__ double column_sums(const cplx* __restrict__ pbase, int sl, int nck, int ns, int last,
                              int nd, cplx* out, cplx* tmp, double* sred) {
  const int tid = threadIdx.x;
  double sq = 0.0;
  if (nck <= 8) {
    for (int i = tid; i < ns; i += GS_THREADS) {
      const cplx* p = pbase + ((i == ns - 1 && last >= 0) ? last : i);
      cplx t[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) t[k] = k < nck ? p[(int64_t)k * sl] : cmk(0.0, 0.0);
      cplx a = t[0];
#pragma unroll
      for (int k = 1; k < 8; ++k)
        if (k < nck) a = cadd(a, t[k]);
      out[i] = a;
      if (i < nd) sq += cabs2(a);
    }
  } else {
    const int lane = tid & 63, g = tid >> 6;
    for (int i0 = 0; i0 < ns; i0 += 64) {
      const int i = i0 + lane;
      cplx a = cmk(0.0, 0.0);
      if (i < ns) {
        const cplx* p = pbase + ((i == ns - 1 && last >= 0) ? last : i);
        for (int k0 = g; k0 < nck; k0 += 16 * GS_WAVES) {
          cplx t[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int k = k0 + u * GS_WAVES;
            t[u] = k < nck ? p[(int64_t)k * sl] : cmk(0.0, 0.0);
          }
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (k0 + u * GS_WAVES < nck) a = cadd(a, t[u]);
        }
      }
      tmp[g * 64 + lane] = a;
      __syncthreads();
      if (g == 0 && i < ns) {
        cplx v = tmp[lane];
        for (int q = 1; q < GS_WAVES; ++q) v = cadd(v, tmp[q * 64 + lane]);
        out[i] = v;
        if (i < nd) sq += cabs2(v);
      }
      __syncthreads();
    }
  }
  return block_sum(sq, sred);  // (its barrier also publishes out[])
}

// The RPT rows tid + k * GS_THREADS (k < RPT) of a chunk of len <= RPT *
// GS_THREADS rows: a[k] = u[r_k] - sum_{i < j} sc_i V_i[r_k] and
// b[k] = w[r_k] - sum_{i < j} zc_i V_i[r_k], from one read of each V_i[r_k];
// 16 / RPT basis vectors per round, so that 16 loads are in flight per thread.
template <int RPT>
__device__ __forceinline__ void project_rows2(const GState& s, int j, const cplx* __restrict__ uc,
                                              const cplx* __restrict__ wc,
                                              const cplx* __restrict__ vc, int len,
                                              const cplx* sc, const cplx* zc, cplx (&a)[RPT],
                                              cplx (&b)[RPT]) {
  constexpr int U = 16 / RPT;
  int r[RPT];
  bool ok[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    r[k] = threadIdx.x + k * GS_THREADS;
    ok[k] = r[k] < len;
    a[k] = ok[k] ? uc[r[k]] : cmk(0.0, 0.0);
    b[k] = ok[k] ? wc[r[k]] : cmk(0.0, 0.0);
  }
  int i = 0;
  for (; i + U <= j; i += U) {
    cplx t[U][RPT];
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int k = 0; k < RPT; ++k)
        t[q][k] = ok[k] ? vc[(int64_t)(i + q) * s.NT + r[k]] : cmk(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const cplx sq = sc[i + q], zq = zc[i + q];
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        a[k] = csub(a[k], cmul(sq, t[q][k]));
        b[k] = csub(b[k], cmul(zq, t[q][k]));
      }
    }
  }
  if (i < j) {  // last, partial batch: rows past j-1 are loaded but not used
    cplx t[U][RPT];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int iq = min(i + q, j - 1);
#pragma unroll
      for (int k = 0; k < RPT; ++k) t[q][k] = ok[k] ? vc[(int64_t)iq * s.NT + r[k]] : cmk(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      if (i + q >= j) break;
      const cplx sq = sc[i + q], zq = zc[i + q];
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        a[k] = csub(a[k], cmul(sq, t[q][k]));
        b[k] = csub(b[k], cmul(zq, t[q][k]));
      }
    }
  }
}

// The rotations 0..col-1 of column c into LDS: rot[0, col) = sn,
// (double*)(rot + col)[0, col) = cs.
__device__ void stage_rotations(const GState& s, int c, int col, cplx* rot) {
  const double* csg = s.cs + (int64_t)c * s.m;
  const cplx* sng = s.sn + (int64_t)c * s.m;
  for (int i = threadIdx.x; i < col; i += GS_THREADS) {
    rot[i] = sng[i];
    reinterpret_cast<double*>(rot + col)[i] = csg[i];
  }
}

// Chunk partial sums of an operator apply still to be added (one-lane-per-pair
// path): w = A V[j] is completed row by row by the dots kernel.
struct PendingApply {
  DevView v;
  const cplx* part;
  int64_t part_total;
  const int32_t* nchunk;
  const int64_t* partoff;
};

// Step j, pass 1: the chunk's partial sums of V_i^H u, V_i^H w (i < j), u^H u
// and u^H w, u = V[j] the candidate, w = V[j+1] = A u.  grid.y splits the
// basis into groups of GS_WAVES * GS_BATCH vectors, one workgroup each (every
// group forms u, w; group 0 writes the u^H u, u^H w slots), or is 1: all j.  With FIN, w is
// first formed from the apply's chunk partial sums and stored (by group 0).
// Without has_w (the end of a cycle) only V_i^H u and u^H u.
template <bool FIN>
__global__ __launch_bounds__(GS_THREADS) void k_dg_dots(GState s, int j, PendingApply pa,
                                                        int has_w) {
  __shared__ cplx ul[1024];
  __shared__ cplx wl[1024];
  __shared__ double sred[3 * GS_WAVES];
  int c, len;
  int64_t o;
  const int gi = decode_chunk(s, &c, &len, &o);
  if (!s.inner[c]) return;
  const cplx* u = s.V + (int64_t)j * s.NT + o;
  cplx* w = s.V + (int64_t)(j + 1) * s.NT + o;
  double uu = 0.0;
  cplx uw = cmk(0.0, 0.0);
  int64_t i0 = 0;
  const cplx* pr = nullptr;
  int b = 0;
  if (FIN) {
    b = c / s.R;
    const int r = c - b * s.R;
    i0 = pa.v.imode[b] + (o - col_base(pa.v.imode, b, s.R, r));
    pr = pa.part + (int64_t)r * pa.part_total;
  }
  for (int rr = threadIdx.x; rr < len; rr += GS_THREADS) {
    const cplx uv = u[rr];
    ul[rr] = uv;
    uu += cabs2(uv);
    if (has_w) {
      cplx wv;
      if (FIN) {
        wv = finalize(pa.v, s.op, i0 + rr, uv,
                      lane_chunk_sum(pa.v, pr, pa.nchunk, pa.partoff, b, i0 + rr));
        if (blockIdx.y == 0) w[rr] = wv;
      } else {
        wv = w[rr];
      }
      wl[rr] = wv;
      cmacc(uw, uv, wv);
    }
  }
  double red3[3] = {uu, uw.x, uw.y};
  block_sums<3>(red3, sred);  // (its barriers also publish ul, wl)
  uu = red3[0];
  uw = cmk(red3[1], red3[2]);
  cplx* part = s.P1 + (int64_t)gi * s.sl;
  // basis vectors [ib, ib + per) of this workgroup: all of them when grid.y is 1
  const int per = gridDim.y == 1 ? j : GS_WAVES * GS_BATCH;
  const int ib = (int)blockIdx.y * per;
  chunk_dots2(s, j, ib, min(j, ib + per), o, len, ul, wl, has_w != 0, part);
  if (threadIdx.x == 0 && blockIdx.y == 0) {
    part[2 * j] = cmk(uu, 0.0);
    part[2 * j + 1] = uw;
  }
}

// Step j, pass 2.  Every workgroup of column c adds the partials of its column
// (same order everywhere, so identical values): s = V^H u, z = V^H w, u^H u,
// u^H w; rho = ||u - V s|| = sqrt(u^H u - ||s||^2) (s is small: u was
// orthogonalised once already, so no cancellation).  Rows:
//   V[j]   = q_j    = (u - V s) / rho                       (final)
//   V[j+1] = u_next = (w - V z - g_j q_j) / rho,  g_j = (u^H w - s^H z) / rho,
// the candidate of the next step (u_next = A q_j - [V q_j] h_j, the once
// orthogonalised vector).  RPT = 0 (few chunks, latency-bound): a workgroup
// takes 64 rows of a chunk (grid.y runs over the chunk's 64-row blocks), wave
// g sums the basis vectors g, g + 4, ... of each row (the first round of them
// loaded before the column sums) and the four wave sums are added through LDS.
// RPT = 1, 2, 4 (many chunks, bandwidth-bound): one workgroup per chunk, RPT
// rows per thread, each reading the whole basis.  Block 0 of chunk 0 finalises
// Hessenberg column j-1 (its tentative entries plus s, subdiagonal rho), takes
// the Givens step, and forms the tentative column j, h_j = ([z; g_j] - H s) / rho,
// H the unrotated Hessenberg columns 0..j-1.
// basis vectors per wave and round of the row sweep of k_dg_update
constexpr int UB = 16;

template <int RPT>
__global__ __launch_bounds__(GS_THREADS) void k_dg_update(GState s, int j) {
  __shared__ cplx cl[2 * MUDIFF_MAX_RESTART + 2];
  __shared__ cplx aux[MUDIFF_MAX_RESTART + MUDIFF_MAX_RESTART + MUDIFF_MAX_RESTART / 2];
  __shared__ cplx tmp[GS_WAVES * 64];
  __shared__ cplx pab[2][GS_WAVES][64];
  __shared__ double sred[2 * GS_WAVES];
  int c, len;
  int64_t o;
  const int gi = decode_chunk(s, &c, &len, &o);
  if (!s.inner[c]) return;
  const int rb = RPT == 0 ? (int)blockIdx.y * 64 : 0;  // this workgroup's rows of the chunk
  if (rb >= len) return;
  const int m1 = s.m + 1;
  const int nck = s.ckc[c];
  const bool first_chunk = gi == s.ckf[c] && blockIdx.y == 0;
  cplx* hcol = aux;                          // column j-1 of the Hessenberg matrix
  cplx* rot = aux + MUDIFF_MAX_RESTART;      // rotations 0..j-2
  ArnoldiPre pre{};
  if (first_chunk && j >= 1) {
    stage_rotations(s, c, j - 1, rot);
    if (threadIdx.x == 0) pre = arnoldi_preload(s, c, j - 1);
    for (int i = threadIdx.x; i < j; i += GS_THREADS) hcol[i] = s.htent[(int64_t)c * m1 + i];
  }
  const int lane = threadIdx.x & 63, wq = threadIdx.x >> 6;
  const int r = rb + lane;
  const bool ok = r < len;
  cplx* u = s.V + (int64_t)j * s.NT + o;
  cplx* w = s.V + (int64_t)(j + 1) * s.NT + o;
  cplx ur = cmk(0.0, 0.0), wr = cmk(0.0, 0.0);
  const cplx* vb = s.V + o + r;
  cplx t0[UB];
  if constexpr (RPT == 0) {
    if (wq == 0 && ok) {
      ur = u[r];
      wr = w[r];
    }
    // the first round of basis rows, loaded before the column sums
#pragma unroll
    for (int q = 0; q < UB; ++q) {
      const int i = min(wq + q * GS_WAVES, j - 1);
      t0[q] = (ok && j > 0) ? vb[(int64_t)i * s.NT] : cmk(0.0, 0.0);
    }
  }
  const double ssq = column_sums(s.P1 + (int64_t)s.ckf[c] * s.sl, s.sl, nck, 2 * j + 2, -1, j, cl,
                                 tmp, sred);
  const double alpha = cl[2 * j].x;
  const cplx beta = cl[2 * j + 1];
  const double rho2 = alpha - ssq;
  const double rho = sqrt(rho2 > 0.0 ? rho2 : 0.0);
  const double inv = 1.0 / rho;  // rho == 0: breakdown, the column stops below
  cplx sz = cmk(0.0, 0.0);       // s^H z
  for (int i = threadIdx.x; i < j; i += GS_THREADS) cmacc(sz, cl[i], cl[j + i]);
  {
    double r2[2] = {sz.x, sz.y};
    block_sums<2>(r2, sred);
    sz = cmk(r2[0], r2[1]);
  }
  const cplx gj = cscale(csub(beta, sz), inv);
  if constexpr (RPT == 0) {
    // wave wq: basis vectors wq, wq + GS_WAVES, ... of row r
    cplx pa = cmk(0.0, 0.0), pb = cmk(0.0, 0.0);
  #pragma unroll
    for (int q = 0; q < UB; ++q) {
      const int i = wq + q * GS_WAVES;
      if (i < j) {
        pa = csub(pa, cmul(cl[i], t0[q]));
        pb = csub(pb, cmul(cl[j + i], t0[q]));
      }
    }
    for (int i0 = wq + UB * GS_WAVES; i0 < j; i0 += UB * GS_WAVES) {
      cplx t[UB];
  #pragma unroll
      for (int q = 0; q < UB; ++q) {
        const int i = min(i0 + q * GS_WAVES, j - 1);
        t[q] = ok ? vb[(int64_t)i * s.NT] : cmk(0.0, 0.0);
      }
  #pragma unroll
      for (int q = 0; q < UB; ++q) {
        const int i = i0 + q * GS_WAVES;
        if (i < j) {
          pa = csub(pa, cmul(cl[i], t[q]));
          pb = csub(pb, cmul(cl[j + i], t[q]));
        }
      }
    }
    pab[0][wq][lane] = pa;
    pab[1][wq][lane] = pb;
    __syncthreads();
    if (wq == 0 && ok) {
      cplx a = ur, bb = wr;
  #pragma unroll
      for (int q = 0; q < GS_WAVES; ++q) {
        a = cadd(a, pab[0][q][lane]);
        bb = cadd(bb, pab[1][q][lane]);
      }
      const cplx qv = cscale(a, inv);
      u[r] = qv;
      w[r] = cscale(csub(bb, cmul(gj, qv)), inv);
    }
  } else {
    cplx a[RPT], bb[RPT];
    project_rows2<RPT>(s, j, u, w, s.V + o, len, cl, cl + j, a, bb);
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int rr = threadIdx.x + k * GS_THREADS;
      if (rr < len) {
        const cplx qv = cscale(a[k], inv);
        u[rr] = qv;
        w[rr] = cscale(csub(bb[k], cmul(gj, qv)), inv);
      }
    }
  }
  if (!first_chunk) return;
  cplx* Hr = s.Hraw + (int64_t)c * m1 * s.m;  // unrotated columns, [k][m+1]
  if (j >= 1) {
    for (int i = threadIdx.x; i < j; i += GS_THREADS) {
      hcol[i] = cadd(hcol[i], cl[i]);
      Hr[(int64_t)(j - 1) * m1 + i] = hcol[i];
    }
    if (threadIdx.x == 0) Hr[(int64_t)(j - 1) * m1 + j] = cmk(rho, 0.0);
    __syncthreads();  // column j-1 and the staged rotations complete
    if (threadIdx.x == 0)
      arnoldi_step(s, c, j - 1, hcol, reinterpret_cast<const double*>(rot + (j - 1)), rot, rho,
                   pre);
  }
  // tentative column j, entries h_i = (g_i - sum_k Hraw[k][i] s_k) / rho,
  // g = [z; g_j], k from i-1 (Hessenberg) to j-1: waves 1.. while thread 0 takes
  // the Givens step; four lanes per entry split the sum over k (16 loads in
  // flight each) and add their parts by shuffles.
  const int w0 = j >= 1 ? 1 : 0;
  const int wv = (int)threadIdx.x >> 6;
  if (wv < w0) return;
  const int kl = lane & 3;
  const int per_pass = (GS_WAVES - w0) * 16;
  for (int i0 = 0; i0 <= j; i0 += per_pass) {
    const int i = i0 + (wv - w0) * 16 + (lane >> 2);
    cplx hs = cmk(0.0, 0.0);
    if (i <= j) {
      for (int k = (i > 0 ? i - 1 : 0) + kl; k < j; k += 64) {
        cplx t[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int kk = min(k + 4 * u, j - 1);
          t[u] = Hr[(int64_t)kk * m1 + i];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (k + 4 * u < j) hs = cadd(hs, cmul(t[u], cl[k + 4 * u]));
      }
    }
#pragma unroll
    for (int o = 1; o < 4; o <<= 1) {
      hs.x += __shfl_xor(hs.x, o, 64);
      hs.y += __shfl_xor(hs.y, o, 64);
    }
    if (kl == 0 && i <= j) {
      const cplx g = i < j ? cl[j + i] : gj;
      s.htent[(int64_t)c * m1 + i] = cscale(csub(g, hs), inv);
    }
  }
}

// End of a cycle (after m steps): column m-1 is finalised from the last
// candidate u = V[m]: s = V^H u, rho = sqrt(u^H u - ||s||^2).  One workgroup
// per column.
__global__ __launch_bounds__(GS_THREADS) void k_dg_flush(GState s) {
  __shared__ cplx cl[MUDIFF_MAX_RESTART + 1];
  __shared__ cplx aux[MUDIFF_MAX_RESTART + MUDIFF_MAX_RESTART + MUDIFF_MAX_RESTART / 2];
  __shared__ cplx tmp[GS_WAVES * 64];
  __shared__ double sred[GS_WAVES];
  const int c = blockIdx.x;
  if (!s.inner[c]) return;
  const int j = s.m;
  const int m1 = s.m + 1;
  cplx* hcol = aux;
  cplx* rot = aux + MUDIFF_MAX_RESTART;
  stage_rotations(s, c, j - 1, rot);
  ArnoldiPre pre{};
  if (threadIdx.x == 0) pre = arnoldi_preload(s, c, j - 1);
  for (int i = threadIdx.x; i < j; i += GS_THREADS) hcol[i] = s.htent[(int64_t)c * m1 + i];
  const double ssq = column_sums(s.P1 + (int64_t)s.ckf[c] * s.sl, s.sl, s.ckc[c], j + 1, 2 * j, j,
                                 cl, tmp, sred);
  const double rho2 = cl[j].x - ssq;
  const double rho = sqrt(rho2 > 0.0 ? rho2 : 0.0);
  cplx* Hr = s.Hraw + (int64_t)c * m1 * s.m;
  for (int i = threadIdx.x; i < j; i += GS_THREADS) {
    hcol[i] = cadd(hcol[i], cl[i]);
    Hr[(int64_t)(j - 1) * m1 + i] = hcol[i];
  }
  if (threadIdx.x == 0) Hr[(int64_t)(j - 1) * m1 + j] = cmk(rho, 0.0);
  __syncthreads();
  if (threadIdx.x == 0)
    arnoldi_step(s, c, j - 1, hcol, reinterpret_cast<const double*>(rot + (j - 1)), rot, rho, pre);
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
  if (threadIdx.x == 0) s.P1[(int64_t)gi * s.sl] = cmk(a, 0.0);
}

// red[c] = sum of the k_resid partials of column c (one wave per column,
// chunk order fixed).
__global__ __launch_bounds__(64) void k_col_sum(GState s, int only_run) {
  const int c = blockIdx.x, lane = threadIdx.x;
  if (only_run && !s.run[c]) return;
  double t = 0.0;
  for (int k = lane; k < s.ckc[c]; k += 64) t += s.P1[(int64_t)(s.ckf[c] + k) * s.sl].x;
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
// One wavefront per column.  Up to 64 steps: the triangle is staged into LDS
// in one sweep (16 columns of loads in flight), lane k keeps g_k and 1 / R_kk
// in registers, and each step broadcasts g_i and 1 / R_ii from lane i and
// updates g_k -= R_ki y_i in the lanes k < i, with no barrier.  Longer cycles:
// column-oriented update with g in LDS.
#define SOLVE_SMALL 64
__device__ __forceinline__ double lane_bcast(double v, int l) {  // l wave-uniform
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

__global__ __launch_bounds__(64) void k_cycle_solve(GState s) {
  __shared__ cplx gl[MUDIFF_MAX_RESTART + 1];
  __shared__ cplx tri[SOLVE_SMALL * (SOLVE_SMALL + 1) / 2];
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const int n = s.run[c] ? s.jdone[c] : 0;
  const int m1 = s.m + 1;
  const cplx* Hc = s.H + (int64_t)c * m1 * s.m;
  const cplx* gc = s.g + (int64_t)c * m1;
  cplx* yc = s.y + (int64_t)c * s.m;
  if (n <= SOLVE_SMALL) {
    // column i, rows 0..i, at tri[i (i + 1) / 2 + k]
    for (int i0 = 0; i0 < n; i0 += 16) {
      cplx t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = min(i0 + u, n - 1);
        t[u] = lane <= i ? Hc[(int64_t)i * m1 + lane] : cmk(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = i0 + u;
        if (i < n && lane <= i) tri[i * (i + 1) / 2 + lane] = t[u];
      }
    }
    cplx g = lane < n ? gc[lane] : cmk(0.0, 0.0);
    __syncthreads();
    cplx rinv = cmk(0.0, 0.0);  // 1 / R_kk, 0 for a zero pivot
    if (lane < n) {
      const cplx d = tri[lane * (lane + 1) / 2 + lane];
      if (d.x != 0.0 || d.y != 0.0) rinv = cdiv(cmk(1.0, 0.0), d);
    }
    for (int i = n - 1; i >= 0; --i) {
      const cplx rik = lane < i ? tri[i * (i + 1) / 2 + lane] : cmk(0.0, 0.0);
      const cplx gi = cmk(lane_bcast(g.x, i), lane_bcast(g.y, i));
      const cplx yi = cmul(gi, cmk(lane_bcast(rinv.x, i), lane_bcast(rinv.y, i)));
      if (lane == 0) yc[i] = yi;
      if (lane < i) g = csub(g, cmul(rik, yi));
    }
    return;
  }
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

// f = scale * src / Ldiag  (general right-hand side: f = -D^{-1} U), or
// without the preconditioner (div = 0) f = scale * src
__global__ void k_precond_rhs(DevView v, int R, const cplx* __restrict__ src, cplx* __restrict__ f,
                              double scale, int div) {
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
  f[g] = div ? cscale(cdiv(src[g], v.op_diag ? v.op_diag[i] : v.Ldiag[i]), scale) : cscale(src[g], scale);
}

// ------------------------------------------------------------------ block GMRES
// With MUDIFF_BLOCK the R columns of an instance are split into blocks of sb
// consecutive columns, and the columns of a block share one block Krylov space
// (block Arnoldi): step j applies the operator to the sb basis vectors of
// block V_j at once, orthogonalises the result W against V_0..V_j by classical
// Gram-Schmidt applied twice, and factors W = V_{j+1} H_{j+1,j} by Cholesky QR
// applied twice (a Cholesky pivot below 1e-14 of its column's squared norm drops
// that direction: its basis vector is zero from then on).  The block
// Hessenberg matrix is reduced to triangular form by one Householder reflector
// of length sb + 1 per column as it grows, and the same reflectors applied to
// the right-hand sides E_1 B (B from the QR of the block's residual) give every
// column's residual estimate after every step.  A block stops when all its
// columns are below the tolerance (or at the end of the cycle, or at maxit);
// at a restart the columns whose true residual meets the tolerance leave the
// block (their vectors are zero in the next cycle).  The basis blocks are the
// same packed multivectors [B][R][N_b] as the lockstep basis: V_j of every
// block of every instance is one multivector, so each step is one batched
// operator apply.  Reductions over rows go through per-chunk partial sums
// added in chunk order, as in the lockstep kernels.
#define BG_SMAX 16      // largest block
#define BG_TILE 64      // rows per LDS tile
#define BG_CHUNK 1024   // rows per reduction chunk
#define BG_MAXDIM 2048  // largest restart * block size (the back substitution stages it in LDS)

struct BState {
  GState s;
  const int64_t* imode;  // [B + 1] first unknown of every instance
  int sb;                // columns per block
  int nbpi;              // blocks per instance
  int NB;                // blocks
  const int32_t* bck;    // [n_chunks][2] block, first row of every reduction chunk
  const int32_t* bckoff; // [NB + 1] first chunk of every block
  const int32_t* btile;  // [NB + 1] first 64-row tile of every block
  cplx* P;               // [n_chunks][m + 1][sb * sb] partial sums
  cplx* T;               // [NB][sb][(m + 1) sb] Gram-Schmidt coefficients, column-major
  cplx* Hb;              // [NB][m sb][(m + 1) sb] block Hessenberg (triangularised in place)
  cplx* Gb;              // [NB][sb][(m + 1) sb] right-hand sides of the least-squares problem
  cplx* Rq;              // [NB][sb][sb] factor of the first Cholesky QR pass
  cplx* Ri;              // [NB][sb][sb] inverse of the current Cholesky QR factor
  cplx* hv;              // [NB][m sb][sb + 1] Householder vectors (first entry 1)
  cplx* htau;            // [NB][m sb] Householder coefficients
  cplx* Y;               // [NB][sb][(m + 1) sb] solution of the least-squares problem
  int32_t* bin;          // [NB] block iterating in the current cycle
  int32_t* brun;         // [NB] block has a running column in the current cycle
  int32_t* bsteps;       // [NB] steps done in the current cycle
  int32_t* bact;         // [C] column takes part in the next operator apply
};

__device__ __forceinline__ int bg_ld(const BState& bs) { return (bs.s.m + 1) * bs.sb; }

// Block of a reduction chunk / of a 64-row tile (binary search in the prefix).
__device__ __forceinline__ int bg_find(const int32_t* pre, int n, int g) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Column cl of block kb: global column index (or -1 past R) and its first entry.
__device__ __forceinline__ int bg_col(const BState& bs, int kb, int cl, int64_t* base) {
  const int b = kb / bs.nbpi, r = (kb % bs.nbpi) * bs.sb + cl;
  if (cl >= bs.sb || r >= bs.s.R) return -1;
  *base = col_base(bs.imode, b, bs.s.R, r);
  return b * bs.s.R + r;
}

// P[chunk][i][a sb + c] = sum over the chunk's rows of conj(V_i[row][a]) W[row][c]
// for i < gridDim.y (V_i = Vb + i vstride), blocks with gate[kb] set; columns
// that are not running count as zero.  Thread (a, c) of each row phase adds
// every rsplit-th row of each LDS tile; the phases are added in order.
__global__ __launch_bounds__(256) void k_bdots(BState bs, const cplx* __restrict__ Vb,
                                               int64_t vstride, const cplx* __restrict__ W,
                                               const int32_t* __restrict__ gate) {
  __shared__ cplx vt[BG_TILE * BG_SMAX];
  __shared__ cplx wt[BG_TILE * BG_SMAX];
  __shared__ cplx red[256];
  const int g = blockIdx.x, i = blockIdx.y, t = threadIdx.x;
  const int kb = bs.bck[2 * g], row0 = bs.bck[2 * g + 1];
  if (!gate[kb]) return;
  const int sb = bs.sb, np = sb * sb;
  const int rsplit = max(1, 256 / np);
  const int pr = t % np, rs = t / np;
  const int a = pr / sb, c = pr % sb;
  const int b = kb / bs.nbpi;
  const int64_t Nb = bs.imode[b + 1] - bs.imode[b];
  const int rows = (int)min((int64_t)BG_CHUNK, Nb - row0);
  const cplx* Vi = Vb + (int64_t)i * vstride;
  cplx acc = cmk(0.0, 0.0);
  for (int t0 = 0; t0 < rows; t0 += BG_TILE) {
    const int tl = min(BG_TILE, rows - t0);
    __syncthreads();
    for (int e = t; e < BG_TILE * sb; e += 256) {
      const int col = e / BG_TILE, rr = e - col * BG_TILE;
      cplx v = cmk(0.0, 0.0), w = cmk(0.0, 0.0);
      int64_t base;
      const int cc = bg_col(bs, kb, col, &base);
      if (cc >= 0 && rr < tl && bs.s.run[cc]) {
        const int64_t off = base + row0 + t0 + rr;
        v = Vi[off];
        w = W[off];
      }
      vt[rr * sb + col] = v;
      wt[rr * sb + col] = w;
    }
    __syncthreads();
    if (rs < rsplit)
      for (int rr = rs; rr < tl; rr += rsplit) cmacc(acc, vt[rr * sb + a], wt[rr * sb + c]);
  }
  red[t] = acc;
  __syncthreads();
  if (t < np) {
    cplx sum = red[t];
    for (int q = 1; q < rsplit; ++q) sum = cadd(sum, red[q * np + t]);
    bs.P[((int64_t)g * (bs.s.m + 1) + i) * np + t] = sum;
  }
}

// Gram-Schmidt coefficients of step j from the chunk partials (chunk order):
// T[kb] rows i sb + a, column c; the Hessenberg block column j receives them
// (pass 0) or adds them (pass 1).
__global__ __launch_bounds__(256) void k_bsum(BState bs, int j, int pass) {
  const int kb = blockIdx.x, i = blockIdx.y, t = threadIdx.x;
  if (!bs.bin[kb]) return;
  const int sb = bs.sb, np = sb * sb, ld = bg_ld(bs);
  if (t >= np) return;
  const int a = t / sb, c = t % sb;
  cplx sum = cmk(0.0, 0.0);
  for (int g = bs.bckoff[kb]; g < bs.bckoff[kb + 1]; ++g)
    sum = cadd(sum, bs.P[((int64_t)g * (bs.s.m + 1) + i) * np + t]);
  bs.T[(int64_t)kb * ld * sb + (int64_t)c * ld + i * sb + a] = sum;
  cplx* h = bs.Hb + (int64_t)kb * ld * (bs.s.m * sb) + (int64_t)(j * sb + c) * ld + i * sb + a;
  *h = pass ? cadd(*h, sum) : sum;
}

// W[row][c] += sign * sum_{i < n_i} sum_a V_i[row][a] coef[kb][c][i sb + a] over
// the rows of every block with gate[kb] set (n_i = nsteps[kb] * ... when given,
// else ni), running columns only.  One 64-row tile per workgroup; thread
// (row, column group) keeps up to 4 columns; the basis tile and the sb x sb
// coefficients of each i are staged in LDS.
__global__ __launch_bounds__(256) void k_bupdate(BState bs, const cplx* __restrict__ Vb,
                                                 int64_t vstride, cplx* __restrict__ W,
                                                 const cplx* __restrict__ coef, int ni,
                                                 const int32_t* __restrict__ nsteps,
                                                 const int32_t* __restrict__ gate, double sign) {
  __shared__ cplx vt[BG_TILE * BG_SMAX];
  __shared__ cplx cs[BG_SMAX * BG_SMAX];
  const int t = threadIdx.x;
  const int kb = bg_find(bs.btile, bs.NB, blockIdx.x);
  if (!gate[kb]) return;
  const int sb = bs.sb, ld = bg_ld(bs);
  const int b = kb / bs.nbpi;
  const int64_t Nb = bs.imode[b + 1] - bs.imode[b];
  const int row0 = (blockIdx.x - bs.btile[kb]) * BG_TILE;
  const int tl = (int)min((int64_t)BG_TILE, Nb - row0);
  const int n_i = nsteps ? nsteps[kb] : ni;
  const int rr = t & 63, cg = t >> 6;
  cplx acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = cmk(0.0, 0.0);
  const cplx* ck = coef + (int64_t)kb * ld * sb;
  for (int i = 0; i < n_i; ++i) {
    __syncthreads();
    for (int e = t; e < sb * sb; e += 256) {
      const int a = e / sb, c = e - a * sb;
      cs[e] = ck[(int64_t)c * ld + i * sb + a];
    }
    const cplx* Vi = Vb + (int64_t)i * vstride;
    for (int e = t; e < BG_TILE * sb; e += 256) {
      const int col = e / BG_TILE, r = e - col * BG_TILE;
      cplx v = cmk(0.0, 0.0);
      int64_t base;
      const int cc = bg_col(bs, kb, col, &base);
      if (cc >= 0 && r < tl && bs.s.run[cc]) v = Vi[base + row0 + r];
      vt[r * sb + col] = v;
    }
    __syncthreads();
    for (int a = 0; a < sb; ++a) {
      const cplx v = vt[rr * sb + a];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = cg + 4 * q;
        if (c < sb) cmac(acc[q], v, cs[a * sb + c]);
      }
    }
  }
  if (rr >= tl) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = cg + 4 * q;
    int64_t base;
    const int cc = bg_col(bs, kb, c, &base);
    if (cc < 0 || !bs.s.run[cc]) continue;
    const int64_t off = base + row0 + rr;
    W[off] = cadd(W[off], cscale(acc[q], sign));
  }
}

// W = W Ri[kb] (Ri upper triangular) over the rows of every block with
// gate[kb] set; columns that are not running are set to zero.
__global__ __launch_bounds__(256) void k_bscale(BState bs, cplx* __restrict__ W,
                                                const int32_t* __restrict__ gate) {
  __shared__ cplx wt[BG_TILE * BG_SMAX];
  __shared__ cplx cs[BG_SMAX * BG_SMAX];
  const int t = threadIdx.x;
  const int kb = bg_find(bs.btile, bs.NB, blockIdx.x);
  if (!gate[kb]) return;
  const int sb = bs.sb;
  const int b = kb / bs.nbpi;
  const int64_t Nb = bs.imode[b + 1] - bs.imode[b];
  const int row0 = (blockIdx.x - bs.btile[kb]) * BG_TILE;
  const int tl = (int)min((int64_t)BG_TILE, Nb - row0);
  for (int e = t; e < sb * sb; e += 256) cs[e] = bs.Ri[(int64_t)kb * sb * sb + e];
  for (int e = t; e < BG_TILE * sb; e += 256) {
    const int col = e / BG_TILE, r = e - col * BG_TILE;
    cplx v = cmk(0.0, 0.0);
    int64_t base;
    const int cc = bg_col(bs, kb, col, &base);
    if (cc >= 0 && r < tl && bs.s.run[cc]) v = W[base + row0 + r];
    wt[r * sb + col] = v;
  }
  __syncthreads();
  const int rr = t & 63, cg = t >> 6;
  if (rr >= tl) return;
  for (int c = cg; c < sb; c += 4) {
    int64_t base;
    const int cc = bg_col(bs, kb, c, &base);
    if (cc < 0) continue;
    cplx acc = cmk(0.0, 0.0);
    if (bs.s.run[cc])
      for (int a = 0; a <= c; ++a) cmac(acc, wt[rr * sb + a], cs[a * sb + c]);
    W[base + row0 + rr] = acc;
  }
}

// Cholesky QR factor of one block: Gram matrix G = W^H W from the chunk
// partials (slot 0), G = R^H R with R upper triangular, a pivot below 1e-14 of
// its column's squared norm (or not positive) dropping that row of R, and
// Ri = the inverse of R on the kept rows (zero elsewhere), so that W Ri has
// orthonormal kept columns and zero dropped ones.  mode 0 (first pass): Rq = R.
// mode 1 (second pass): the factor of the original W is R Rq; at step j >= 0 it
// is the Hessenberg block H_{j+1,j}; at j < 0 (start of a cycle) it is the
// first block of the right-hand sides (the rest of Gb is cleared).
__global__ __launch_bounds__(256) void k_bchol(BState bs, int mode, int j,
                                               const int32_t* __restrict__ gate) {
  __shared__ cplx G[BG_SMAX * BG_SMAX];   // [a][c], becomes R
  __shared__ cplx Ii[BG_SMAX * BG_SMAX];
  __shared__ double dg[BG_SMAX];
  __shared__ double piv[BG_SMAX];
  const int kb = blockIdx.x, t = threadIdx.x;
  if (!gate[kb]) return;
  const int sb = bs.sb, np = sb * sb, ld = bg_ld(bs);
  if (t < np) {
    cplx sum = cmk(0.0, 0.0);
    for (int g = bs.bckoff[kb]; g < bs.bckoff[kb + 1]; ++g)
      sum = cadd(sum, bs.P[(int64_t)g * (bs.s.m + 1) * np + t]);
    G[t] = sum;
  }
  __syncthreads();
  if (t < sb) dg[t] = G[t * sb + t].x;
  __syncthreads();
  // right-looking Cholesky on the upper triangle
  for (int k = 0; k < sb; ++k) {
    if (t == 0) {
      const double d = G[k * sb + k].x;
      piv[k] = (d > 1e-14 * dg[k] && d > 0.0) ? sqrt(d) : 0.0;
    }
    __syncthreads();
    const double rk = piv[k];
    if (t < sb) {  // row k of R
      const int c = t;
      if (c < k) G[k * sb + c] = cmk(0.0, 0.0);
      else if (c == k) G[k * sb + k] = cmk(rk, 0.0);
      else G[k * sb + c] = rk > 0.0 ? cscale(G[k * sb + c], 1.0 / rk) : cmk(0.0, 0.0);
    }
    __syncthreads();
    if (t < np) {  // trailing update G[a][c] -= conj(R[k][a]) R[k][c], a, c > k
      const int a = t / sb, c = t % sb;
      if (a > k && c > k) {
        cplx acc = G[t];
        const cplx ra = G[k * sb + a], rc = G[k * sb + c];
        acc = csub(acc, cmul(cconj(ra), rc));
        G[t] = acc;
      }
    }
    __syncthreads();
  }
  // inverse on the kept rows: thread c solves R x = e_c by back substitution
  if (t < sb) {
    const int c = t;
    for (int a = sb - 1; a >= 0; --a) {
      cplx x = cmk(0.0, 0.0);
      if (a <= c && piv[a] > 0.0) {
        x = a == c ? cmk(1.0, 0.0) : cmk(0.0, 0.0);
        for (int k = a + 1; k <= c; ++k) x = csub(x, cmul(G[a * sb + k], Ii[k * sb + c]));
        x = cscale(x, 1.0 / piv[a]);
      }
      Ii[a * sb + c] = x;
    }
  }
  __syncthreads();
  cplx* Ri = bs.Ri + (int64_t)kb * np;
  cplx* Rq = bs.Rq + (int64_t)kb * np;
  if (t < np) Ri[t] = Ii[t];
  if (mode == 0) {
    if (t < np) Rq[t] = G[t];
    return;
  }
  // R_total = R Rq (both upper triangular): [a][c] = sum_{a <= k <= c} R[a][k] Rq[k][c]
  if (t < np) {
    const int a = t / sb, c = t % sb;
    cplx acc = cmk(0.0, 0.0);
    for (int k = a; k <= c; ++k) cmac(acc, G[a * sb + k], Rq[k * sb + c]);
    Ii[t] = acc;  // reuse: the inverse is already stored
  }
  __syncthreads();
  if (j >= 0) {
    cplx* h = bs.Hb + (int64_t)kb * ld * (bs.s.m * sb);
    if (t < np) {
      const int a = t / sb, c = t % sb;
      h[(int64_t)(j * sb + c) * ld + (j + 1) * sb + a] = Ii[t];
    }
  } else {
    cplx* gk = bs.Gb + (int64_t)kb * ld * sb;
    for (int e = t; e < ld * sb; e += 256) {
      const int c = e / ld, row = e - c * ld;
      gk[e] = row < sb ? Ii[row * sb + c] : cmk(0.0, 0.0);
    }
  }
}

// Least-squares update of step j, one workgroup of 64 sb threads per block:
// (A) wave w applies the reflectors of the earlier columns to Hessenberg
// column j sb + w, its window of sb + 1 rows held across the lanes and moved
// down one row per reflector; (B) the sb new reflectors are formed and applied
// in LDS to the new columns and to the right-hand sides; (C) each column's
// residual estimate, the stopping test and the next apply's column set.
__global__ __launch_bounds__(1024) void k_blsq(BState bs, int j) {
  __shared__ cplx Hl[2 * BG_SMAX * BG_SMAX];  // rows j sb .. (j + 2) sb - 1, [row][w]
  __shared__ cplx Gl[2 * BG_SMAX * BG_SMAX];
  __shared__ cplx vl[BG_SMAX + 1];
  __shared__ cplx taul;
  __shared__ double est[BG_SMAX];
  __shared__ int cont;
  const GState& s = bs.s;
  const int kb = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (!bs.bin[kb]) return;
  const int sb = bs.sb, ld = bg_ld(bs), m = s.m;
  const int r0 = j * sb;  // first row of the new block (and number of earlier reflectors)
  cplx* Hk = bs.Hb + (int64_t)kb * ld * (m * sb);
  cplx* Gk = bs.Gb + (int64_t)kb * ld * sb;
  cplx* hvk = bs.hv + (int64_t)kb * (m * sb) * (sb + 1);
  cplx* htk = bs.htau + (int64_t)kb * (m * sb);
  // (A)
  {
    cplx* hc = Hk + (int64_t)(r0 + w) * ld;
    cplx x = lane <= sb ? hc[lane] : cmk(0.0, 0.0);
    for (int r = 0; r < r0; ++r) {
      const cplx v = lane <= sb ? hvk[(int64_t)r * (sb + 1) + lane] : cmk(0.0, 0.0);
      const cplx tau = htk[r];
      const cplx nxt = (lane == sb) ? hc[r + 1 + sb] : cmk(0.0, 0.0);
      double dre = 0.0, dim = 0.0;
      {  // d = v^H x over the window
        const cplx p = cmul(cconj(v), x);
        dre = wave_sum(p.x);
        dim = wave_sum(p.y);
      }
      const cplx f = cmul(cconj(tau), cmk(dre, dim));
      if (lane <= sb) x = csub(x, cmul(f, v));
      if (lane == 0) hc[r] = x;
      const double sx = __shfl_down(x.x, 1, 64), sy = __shfl_down(x.y, 1, 64);
      x = lane == sb ? nxt : cmk(sx, sy);
    }
    if (lane <= sb) Hl[lane * sb + w] = x;                       // rows r0 .. r0 + sb
    if (lane > sb && lane < 2 * sb) Hl[lane * sb + w] = hc[r0 + lane];  // rows below, untouched
  }
  for (int e = t; e < 2 * sb * sb; e += 64 * sb) {
    const int row = e / sb, c = e - row * sb;
    Gl[e] = Gk[(int64_t)c * ld + r0 + row];
  }
  __syncthreads();
  // (B)
  for (int q = 0; q < sb; ++q) {
    if (w == 0) {
      const cplx xv = lane <= sb ? Hl[(q + lane) * sb + q] : cmk(0.0, 0.0);
      const double s2 = wave_sum(lane >= 1 ? cabs2(xv) : 0.0);
      const cplx alpha = cmk(__shfl(xv.x, 0, 64), __shfl(xv.y, 0, 64));
      cplx tau = cmk(0.0, 0.0), scale = cmk(0.0, 0.0);
      double beta = alpha.x;
      if (s2 > 0.0 || alpha.y != 0.0) {
        const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + s2);
        beta = alpha.x >= 0.0 ? -nrm : nrm;
        tau = cmk((beta - alpha.x) / beta, -alpha.y / beta);
        scale = cdiv(cmk(1.0, 0.0), csub(alpha, cmk(beta, 0.0)));
      }
      if (lane <= sb) {
        const cplx v = lane == 0 ? cmk(1.0, 0.0) : cmul(xv, scale);
        vl[lane] = (tau.x == 0.0 && tau.y == 0.0 && lane > 0) ? cmk(0.0, 0.0) : v;
        Hl[(q + lane) * sb + q] = lane == 0 ? cmk(beta, 0.0) : cmk(0.0, 0.0);
      }
      if (lane == 0) taul = tau;
    }
    __syncthreads();
    // y <- y - conj(tau) v (v^H y) for the columns q+1.. of Hl and every column of Gl
    const int nt = (sb - q - 1) + sb;
    if (t < nt) {
      cplx* base = t < sb - q - 1 ? Hl + (q + 1 + t) : Gl + (t - (sb - q - 1));
      cplx d = cmk(0.0, 0.0);
      for (int l = 0; l <= sb; ++l) cmacc(d, vl[l], base[(q + l) * sb]);
      const cplx f = cmul(cconj(taul), d);
      for (int l = 0; l <= sb; ++l) base[(q + l) * sb] = csub(base[(q + l) * sb], cmul(f, vl[l]));
    }
    if (t <= sb) hvk[(int64_t)(r0 + q) * (sb + 1) + t] = vl[t];
    if (t == 0) htk[r0 + q] = taul;
    __syncthreads();
  }
  // write back the new block rows and the right-hand sides
  for (int e = t; e < 2 * sb * sb; e += 64 * sb) {
    const int row = e / sb, c = e - row * sb;
    Hk[(int64_t)(r0 + c) * ld + r0 + row] = Hl[e];
    Gk[(int64_t)c * ld + r0 + row] = Gl[e];
  }
  // (C) residual estimates |G[(j+1) sb .. (j+2) sb - 1][c]| / ||f_c||
  if (t < sb) {
    double a = 0.0;
    for (int l = sb; l < 2 * sb; ++l) a += cabs2(Gl[l * sb + t]);
    est[t] = sqrt(a);
  }
  if (t == 0) cont = 0;
  __syncthreads();
  if (t < sb) {
    int64_t base;
    const int c = bg_col(bs, kb, t, &base);
    if (c >= 0 && s.run[c]) {
      const int it = s.iters[c] + 1;
      s.iters[c] = it;
      const double rel = est[t] / s.normf[c];
      if (s.resvec && it <= s.maxit) s.resvec[(int64_t)c * (s.maxit + 1) + it] = rel;
      if (!isfinite(rel)) s.status[c] = ST_BREAK;
      if (isfinite(rel) && rel > s.tol && it < s.maxit) atomicOr(&cont, 1);
    }
  }
  __syncthreads();
  const bool go = cont && j + 1 < m;
  if (t == 0) {
    bs.bsteps[kb] = j + 1;
    if (!go) {
      bs.bin[kb] = 0;
      atomicSub(s.n_inner, 1);
    }
  }
  if (!go && t < sb) {
    int64_t base;
    const int c = bg_col(bs, kb, t, &base);
    if (c >= 0) bs.bact[c] = 0;
  }
}

// End of a cycle: Y = R^{-1} G for every block that ran (R the triangularised
// Hessenberg, n = steps * sb rows; zero pivots give zero), one workgroup per
// (block, right-hand side), G's column staged in LDS.
__global__ __launch_bounds__(256) void k_bsolve(BState bs) {
  __shared__ cplx gl[BG_MAXDIM];
  __shared__ cplx yi_s;
  const int kb = blockIdx.x, c = blockIdx.y, t = threadIdx.x;
  if (!bs.brun[kb]) return;
  const int sb = bs.sb, ld = bg_ld(bs);
  const int n = bs.bsteps[kb] * sb;
  const cplx* Hk = bs.Hb + (int64_t)kb * ld * (bs.s.m * sb);
  const cplx* gc = bs.Gb + (int64_t)kb * ld * sb + (int64_t)c * ld;
  cplx* yc = bs.Y + (int64_t)kb * ld * sb + (int64_t)c * ld;
  for (int k = t; k < n; k += 256) gl[k] = gc[k];
  __syncthreads();
  for (int i = n - 1; i >= 0; --i) {
    const cplx* col = Hk + (int64_t)i * ld;
    if (t == 0) {
      const cplx d = col[i];
      const cplx y = (d.x == 0.0 && d.y == 0.0) ? cmk(0.0, 0.0) : cdiv(gl[i], d);
      yi_s = y;
      yc[i] = y;
    }
    __syncthreads();
    const cplx y = yi_s;
    for (int k = t; k < i; k += 256) gl[k] = csub(gl[k], cmul(col[k], y));
    __syncthreads();
  }
}

// Start of a cycle, per column: the true residual norm decides convergence
// (as k_cycle_begin; the residual block is normalised by its QR instead).
__global__ void k_bcycle_begin(GState s) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= s.C) return;
  if (!s.run[c] || s.status[c] != ST_RUN) {
    s.run[c] = 0;
    return;
  }
  const double rel = sqrt(s.red[c]) / s.normf[c];
  if (s.resvec && s.iters[c] == 0) s.resvec[(int64_t)c * (s.maxit + 1)] = rel;
  if (!isfinite(rel)) s.status[c] = ST_BREAK;
  else if (rel <= s.tol) s.status[c] = ST_CONV;
  else if (s.iters[c] >= s.maxit) s.status[c] = ST_MAXIT;
  s.run[c] = s.status[c] == ST_RUN;
}

// Start of a cycle, per block: it runs if one of its columns does.
__global__ void k_bblock_begin(BState bs) {
  const int kb = blockIdx.x * blockDim.x + threadIdx.x;
  if (kb >= bs.NB) return;
  int any = 0;
  for (int cl = 0; cl < bs.sb; ++cl) {
    int64_t base;
    const int c = bg_col(bs, kb, cl, &base);
    if (c >= 0) {
      bs.bact[c] = bs.s.run[c];
      any |= bs.s.run[c];
    }
  }
  bs.brun[kb] = any;
  bs.bin[kb] = any;
  bs.bsteps[kb] = 0;
  if (any) atomicAdd(bs.s.n_inner, 1);
}

__global__ void k_zero_i(int32_t* p, int n) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) p[g] = 0;
}

// ------------------------------------------------------------------ s-step GMRES
// With MUDIFF_SSTEP each restart cycle after the first builds its Krylov basis
// ss vectors at a time (s-step, or communication-avoiding, GMRES): from the
// last orthonormal basis vector q_j the operator is applied ss times back to
// back in the scaled Newton form v_i = (A - theta_i) v_{i-1} / sigma_i, with
// the shifts theta_i the Ritz values of the first cycle's Hessenberg matrix in
// Leja order and sigma_i = max_k |lambda_k - theta_i| over those Ritz values
// (so the basis stays well conditioned and its norms stay near one), and the
// block [v_1 .. v_ss] is then
// orthogonalised at once: against q_0..q_j by classical Gram-Schmidt and within
// itself by Cholesky QR, both applied twice (each pass one reduction over the
// rows and one sweep; the Gram matrix of the projected block follows from the
// unprojected one minus C^H C).  With V = [Q, Q_new] R_hat (R_hat the
// coefficients of the v_i) and A [v_0..v_{ss-1}] = [v_0..v_ss] B (theta_i on
// the diagonal of B, sigma_i below), the ss new Hessenberg columns are
//   H_new = (R_hat B - [H_old R_top; 0]) R_s^{-1},
// R_top the rows of R_hat on q_0..q_{j-1} and R_s the square block on
// q_j..q_{j+ss-1}; they then enter the Givens update one by one, with the
// residual estimate and stopping test of every column as in the one-vector
// process.  Per ss steps: ss applies, four reduction/sweep launches and one
// small per-column kernel, against 2 ss launches for delayed CGS2.
#define SS_MAX 16
// dst[e] = src(e), e < n, for the nt threads of a block: eight loads in flight
// per thread before the stores (a load-store loop would wait on every load).
template <class F>
__device__ __forceinline__ void ss_stage(cplx* dst, int n, int tid, int nt, F src) {
  for (int e0 = tid; e0 < n; e0 += 8 * nt) {
    cplx v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * nt;
      v[u] = e < n ? src(e) : cmk(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * nt;
      if (e < n) dst[e] = v[u];
    }
  }
}
#define SS_MREST 64    // longest restart of an s-step solve (LDS of the per-column kernels)
#define SS_CL ((SS_MREST + 1) * SS_MAX)

// P2[chunk][l ss + k] = sum over the chunk's rows of conj(V_l) V_{j0+1+k},
// l < j0 + 1 + sb, k < sb: the projections on the basis and the block's Gram
// matrix.  One wave per left vector l, lanes along the rows, the sb sums
// reduce-scattered over the lanes.
__global__ __launch_bounds__(GS_THREADS) void k_ss_dots(GState s, int j0, int sb) {
  int c, len;
  int64_t o;
  const int gi = decode_chunk(s, &c, &len, &o);
  if (!s.inner[c]) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nl = j0 + 1 + sb;
  const cplx* wb = s.V + (int64_t)(j0 + 1) * s.NT + o;
  for (int l = blockIdx.y * GS_WAVES + wv; l < nl; l += gridDim.y * GS_WAVES) {
    cplx acc[SS_MAX];
#pragma unroll
    for (int k = 0; k < SS_MAX; ++k) acc[k] = cmk(0.0, 0.0);
    const cplx* vl = s.V + (int64_t)l * s.NT + o;
    for (int r = lane; r < len; r += 64) {
      const cplx a = vl[r];
#pragma unroll
      for (int k = 0; k < SS_MAX; ++k)
        if (k < sb) cmacc(acc[k], a, wb[(int64_t)k * s.NT + r]);
    }
    double val[2 * SS_MAX];
#pragma unroll
    for (int k = 0; k < SS_MAX; ++k) {
      val[2 * k] = acc[k].x;
      val[2 * k + 1] = acc[k].y;
    }
    lane_reduce_scatter<2 * SS_MAX>(val, lane);
    const int vi = lane >> 1;
    if ((lane & 1) == 0 && vi < 2 * sb) {
      double* dst = reinterpret_cast<double*>(s.P2 + (int64_t)gi * s.sl2 + l * s.ss + (vi >> 1));
      dst[vi & 1] = val[0];
    }
  }
}

// Per column: the chunk partials added in chunk order give C = Q^H W
// ((j0 + 1) x sb) and G = W^H W, stored for k_ss_chol; one thread per slot,
// sixteen chunk loads in flight.
__global__ __launch_bounds__(GS_THREADS) void k_ss_red(GState s, int j0, int sb, int pass) {
  const int c = blockIdx.x;
  if (!s.inner[c]) return;
  const int e = blockIdx.y * GS_THREADS + threadIdx.x;
  const int nl = j0 + 1 + sb, ss = s.ss;
  if (e >= nl * sb) return;
  const int l = e / sb, k = e - (e / sb) * sb;
  const int k0 = s.ckf[c], nck = s.ckc[c];
  const cplx* src = s.P2 + (int64_t)k0 * s.sl2 + l * ss + k;
  cplx a = cmk(0.0, 0.0);
  for (int q = 0; q < nck; q += 16) {
    cplx v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = q + u < nck ? src[(int64_t)(q + u) * s.sl2] : cmk(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (q + u < nck) a = cadd(a, v[u]);
  }
  // slots l <= j0: C (this pass); l > j0: the Gram matrix, kept in the R slot
  if (l <= j0) s.sC[((int64_t)c * 2 + pass) * s.sl2 + l * ss + k] = a;
  else s.sR[((int64_t)c * 2 + pass) * ss * ss + (l - j0 - 1) * ss + k] = a;
}

// Per column, one wavefront: R = chol(G - C^H C) (a pivot below 1e-14 of its
// diagonal entry, or not positive, drops that row) and its inverse on the kept
// rows, R over the Gram matrix in the R slot of this pass.
__global__ __launch_bounds__(64) void k_ss_chol(GState s, int j0, int sb, int pass) {
  __shared__ cplx Cl[SS_CL];
  __shared__ cplx G[SS_MAX * SS_MAX];
  __shared__ cplx Ii[SS_MAX * SS_MAX];
  __shared__ double dg[SS_MAX], piv[SS_MAX];
  const int c = blockIdx.x, t = threadIdx.x;
  if (!s.inner[c]) return;
  const int ss = s.ss;
  const cplx* Cg = s.sC + ((int64_t)c * 2 + pass) * s.sl2;
  cplx* Rg = s.sR + ((int64_t)c * 2 + pass) * ss * ss;
  ss_stage(Cl, (j0 + 1) * sb, t, 64, [&](int e) { return Cg[(e / sb) * ss + e % sb]; });
  ss_stage(Ii, sb * sb, t, 64, [&](int e) { return Rg[(e / sb) * ss + e % sb]; });
  __syncthreads();
  for (int e = t; e < sb * sb; e += 64) G[(e / sb) * SS_MAX + e % sb] = Ii[e];
  __syncthreads();
  for (int e = t; e < sb * sb; e += 64) {  // G - C^H C
    const int a = e / sb, k = e - (e / sb) * sb;
    cplx g = G[a * SS_MAX + k];
    for (int l = 0; l <= j0; ++l) g = csub(g, cmul(cconj(Cl[l * sb + a]), Cl[l * sb + k]));
    Ii[a * SS_MAX + k] = g;
  }
  __syncthreads();
  for (int e = t; e < sb * sb; e += 64) G[(e / sb) * SS_MAX + e % sb] = Ii[(e / sb) * SS_MAX + e % sb];
  if (t < sb) dg[t] = Ii[t * SS_MAX + t].x;
  __syncthreads();
  for (int k = 0; k < sb; ++k) {
    if (t == 0) {
      const double d = G[k * SS_MAX + k].x;
      piv[k] = (d > 1e-14 * dg[k] && d > 0.0) ? sqrt(d) : 0.0;
    }
    __syncthreads();
    const double rk = piv[k];
    if (t < sb) {
      if (t < k) G[k * SS_MAX + t] = cmk(0.0, 0.0);
      else if (t == k) G[k * SS_MAX + k] = cmk(rk, 0.0);
      else G[k * SS_MAX + t] = rk > 0.0 ? cscale(G[k * SS_MAX + t], 1.0 / rk) : cmk(0.0, 0.0);
    }
    __syncthreads();
    for (int e = t; e < sb * sb; e += 64) {
      const int a = e / sb, cc = e - (e / sb) * sb;
      if (a > k && cc > k) G[a * SS_MAX + cc] = csub(G[a * SS_MAX + cc], cmul(cconj(G[k * SS_MAX + a]), G[k * SS_MAX + cc]));
    }
    __syncthreads();
  }
  if (t < sb) {  // column t of R^{-1} on the kept rows
    for (int a = sb - 1; a >= 0; --a) {
      cplx x = cmk(0.0, 0.0);
      if (a <= t && piv[a] > 0.0) {
        x = a == t ? cmk(1.0, 0.0) : cmk(0.0, 0.0);
        for (int k = a + 1; k <= t; ++k) x = csub(x, cmul(G[a * SS_MAX + k], Ii[k * SS_MAX + t]));
        x = cscale(x, 1.0 / piv[a]);
      }
      Ii[a * SS_MAX + t] = x;
    }
  }
  __syncthreads();
  cplx* Rig = s.sRi + (int64_t)c * ss * ss;
  for (int e = t; e < sb * sb; e += 64) {
    const int a = e / sb, k = e - (e / sb) * sb;
    Rg[a * ss + k] = G[a * SS_MAX + k];
    Rig[a * ss + k] = Ii[a * SS_MAX + k];
  }
}

// Rows of the block: W_k <- (W_k - sum_{l <= j0} V_l C[l][k]) R^{-1} with the
// current pass's C and R^{-1} staged in LDS.  64 rows per workgroup, four
// threads per row splitting the basis vectors (l = g, g + 4, ...; eight loads
// in flight), their sums added in LDS in a fixed order.
#define SS_UR 64
__global__ __launch_bounds__(GS_THREADS) void k_ss_update(GState s, int j0, int sb, int pass) {
  __shared__ cplx Cl[SS_CL];
  __shared__ cplx Ri[SS_MAX * SS_MAX];
  __shared__ cplx part[3 * SS_UR * SS_MAX];
  int c, len;
  int64_t o;
  decode_chunk(s, &c, &len, &o);
  if (!s.inner[c]) return;
  const int t = threadIdx.x, ss = s.ss;
  const cplx* Cg = s.sC + ((int64_t)c * 2 + pass) * s.sl2;
  ss_stage(Cl, (j0 + 1) * sb, t, GS_THREADS, [&](int e) { return Cg[(e / sb) * ss + e % sb]; });
  const cplx* Rig = s.sRi + (int64_t)c * ss * ss;
  ss_stage(Ri, sb * sb, t, GS_THREADS, [&](int e) { return Rig[(e / sb) * ss + e % sb]; });
  __syncthreads();
  const int rl = t & (SS_UR - 1), g = t / SS_UR;
  const int r = blockIdx.y * SS_UR + rl;
  const bool in = r < len;
  cplx acc[SS_MAX];
#pragma unroll
  for (int k = 0; k < SS_MAX; ++k) acc[k] = cmk(0.0, 0.0);
  if (in) {
    const cplx* vr = s.V + o + r;
    for (int l0 = g; l0 <= j0; l0 += 32) {
      cplx v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int l = l0 + 4 * u;
        v[u] = l <= j0 ? vr[(int64_t)l * s.NT] : cmk(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int l = l0 + 4 * u;
        if (l > j0) break;
#pragma unroll
        for (int k = 0; k < SS_MAX; ++k)
          if (k < sb) cmac(acc[k], v[u], Cl[l * sb + k]);
      }
    }
  }
  if (g > 0) {
#pragma unroll
    for (int k = 0; k < SS_MAX; ++k)
      if (k < sb) part[((g - 1) * SS_UR + rl) * SS_MAX + k] = acc[k];
  }
  __syncthreads();
  if (g != 0 || !in) return;
  cplx w[SS_MAX];
  cplx* wb = s.V + (int64_t)(j0 + 1) * s.NT + o + r;
#pragma unroll
  for (int k = 0; k < SS_MAX; ++k) w[k] = k < sb ? wb[(int64_t)k * s.NT] : cmk(0.0, 0.0);
#pragma unroll
  for (int k = 0; k < SS_MAX; ++k) {
    cplx a = acc[k];
#pragma unroll
    for (int q = 0; q < 3; ++q) a = cadd(a, part[(q * SS_UR + rl) * SS_MAX + k]);
    w[k] = csub(w[k], a);
  }
#pragma unroll
  for (int k = 0; k < SS_MAX; ++k) {
    cplx a = cmk(0.0, 0.0);
#pragma unroll
    for (int q = 0; q <= k; ++q)
      if (k < sb) cmac(a, w[q], Ri[q * sb + k]);
    if (k < sb) wb[(int64_t)k * s.NT] = a;
  }
}

// Wide variants of the two sweeps, for many chunks (many right-hand sides):
// there the sweeps are bound by HBM bandwidth, and k_ss_dots, which re-reads
// the block's new vectors once per basis vector, moves (j0 + 1 + sb) sb
// vectors through L2 per pass.  k_ss_dots_w stages a tile of SSW_TR rows of
// all nl = j0 + 1 + sb vectors in LDS (rows padded to SSW_TR + 1 against bank
// conflicts); each thread accumulates a block of 2 basis vectors x 4 new
// vectors over every ks-th row of the tile (ks row groups fill the
// workgroup), and the row groups' sums are added in group order at the end:
// every vector is read once from HBM.  k_ss_update_w: one thread per row
// (SSW_RB rows per workgroup), the whole sweep of that row in registers.
#define SSW_TR 32
#define SSW_RB 1024
#define SSW_MIN_CHUNKS 256  // chunks from which the wide variants run

__global__ __launch_bounds__(GS_THREADS) void k_ss_dots_w(GState s, int j0, int sb) {
  extern __shared__ cplx tile[];  // [nl][SSW_TR + 1], then the row groups' sums
  int c, len;
  int64_t o;
  const int gi = decode_chunk(s, &c, &len, &o);
  if (!s.inner[c]) return;
  const int t = threadIdx.x, ld = SSW_TR + 1;
  const int nl = j0 + 1 + sb;
  const int nkb = (sb + 3) >> 2, nblk = ((nl + 1) >> 1) * nkb;  // <= 40 * 4 blocks
  const int ks = max(1, GS_THREADS / nblk);
  const int blk = t % nblk, g = t / nblk;
  const bool act = g < ks;
  const int l0 = 2 * (blk / nkb), k0 = 4 * (blk - (blk / nkb) * nkb);
  cplx acc[2][4];
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = cmk(0.0, 0.0);
  const cplx* vb = s.V + o;
  for (int r0 = 0; r0 < len; r0 += SSW_TR) {
    const int tr = min(SSW_TR, len - r0);
    __syncthreads();  // the previous tile is consumed
    for (int e0 = t; e0 < nl * SSW_TR; e0 += 8 * GS_THREADS) {
      cplx v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * GS_THREADS, l = e / SSW_TR, r = e - l * SSW_TR;
        v[u] = (l < nl && r < tr) ? vb[(int64_t)l * s.NT + r0 + r] : cmk(0.0, 0.0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * GS_THREADS, l = e / SSW_TR, r = e - l * SSW_TR;
        if (l < nl) tile[l * ld + r] = v[u];
      }
    }
    __syncthreads();
    if (act) {
      for (int r = g; r < tr; r += ks) {
        cplx a[2], b[4];
#pragma unroll
        for (int u = 0; u < 2; ++u) a[u] = l0 + u < nl ? tile[(l0 + u) * ld + r] : cmk(0.0, 0.0);
#pragma unroll
        for (int v = 0; v < 4; ++v) b[v] = k0 + v < sb ? tile[(j0 + 1 + k0 + v) * ld + r] : cmk(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) cmacc(acc[u][v], a[u], b[v]);
      }
    }
  }
  __syncthreads();  // the tile buffer now holds the row groups' sums [g][blk][8]
  if (act) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) tile[(g * nblk + blk) * 8 + u * 4 + v] = acc[u][v];
  }
  __syncthreads();
  cplx* part = s.P2 + (int64_t)gi * s.sl2;
  for (int e = t; e < nblk * 8; e += GS_THREADS) {
    const int bq = e >> 3, q = e & 7;
    const int l = 2 * (bq / nkb) + (q >> 2), k = 4 * (bq - (bq / nkb) * nkb) + (q & 3);
    if (l >= nl || k >= sb) continue;
    cplx a = cmk(0.0, 0.0);
    for (int gg = 0; gg < ks; ++gg) a = cadd(a, tile[(gg * nblk + bq) * 8 + q]);
    part[l * s.ss + k] = a;
  }
}

__global__ __launch_bounds__(GS_THREADS) void k_ss_update_w(GState s, int j0, int sb, int pass) {
  __shared__ cplx Cl[SS_CL];
  __shared__ cplx Ri[SS_MAX * SS_MAX];
  int c, len;
  int64_t o;
  decode_chunk(s, &c, &len, &o);
  if (!s.inner[c]) return;
  const int t = threadIdx.x, ss = s.ss;
  const int rb = (int)blockIdx.y * SSW_RB;
  if (rb >= len) return;
  const cplx* Cg = s.sC + ((int64_t)c * 2 + pass) * s.sl2;
  ss_stage(Cl, (j0 + 1) * sb, t, GS_THREADS, [&](int e) { return Cg[(e / sb) * ss + e % sb]; });
  const cplx* Rig = s.sRi + (int64_t)c * ss * ss;
  ss_stage(Ri, sb * sb, t, GS_THREADS, [&](int e) { return Rig[(e / sb) * ss + e % sb]; });
  __syncthreads();
  const int re = min(len, rb + SSW_RB);
  for (int r = rb + t; r < re; r += GS_THREADS) {
    cplx acc[SS_MAX];
#pragma unroll
    for (int k = 0; k < SS_MAX; ++k) acc[k] = cmk(0.0, 0.0);
    const cplx* vr = s.V + o + r;
    for (int l0 = 0; l0 <= j0; l0 += 8) {
      cplx v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = l0 + u <= j0 ? vr[(int64_t)(l0 + u) * s.NT] : cmk(0.0, 0.0);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (l0 + u > j0) break;
#pragma unroll
        for (int k = 0; k < SS_MAX; ++k)
          if (k < sb) cmac(acc[k], v[u], Cl[(l0 + u) * sb + k]);
      }
    }
    cplx w[SS_MAX];
    cplx* wb = s.V + (int64_t)(j0 + 1) * s.NT + o + r;
#pragma unroll
    for (int k = 0; k < SS_MAX; ++k) w[k] = k < sb ? csub(wb[(int64_t)k * s.NT], acc[k]) : cmk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < SS_MAX; ++k) {
      cplx a = cmk(0.0, 0.0);
#pragma unroll
      for (int q = 0; q <= k; ++q)
        if (k < sb) cmac(a, w[q], Ri[q * sb + k]);
      if (k < sb) wb[(int64_t)k * s.NT] = a;
    }
  }
}

// Per column, after the second pass: the coefficients of the Newton vectors
// (C = C1 + C2 R1, R = R2 R1), the new Hessenberg columns (all sb, or up to the
// first dropped pivot of R and one more), written raw, then each through the
// Givens update (arnoldi_step) until the column stops.
#define SS_HT 256
__global__ __launch_bounds__(SS_HT) void k_ss_hess(GState s, int j0, int sb) {
  __shared__ cplx Cm[SS_CL];                                // C  [l][k], l <= j0
  __shared__ cplx Rm[SS_MAX * SS_MAX];                      // R  [a][k]
  __shared__ cplx X[(SS_MREST + SS_MAX + 1) * SS_MAX];      // new columns [row][k]
  __shared__ cplx Ho[(SS_MREST + 1) * SS_MREST];            // earlier raw columns [q][row], rows <= j0
  __shared__ cplx hl[SS_MREST + 1];
  __shared__ double csl[SS_MREST];
  __shared__ cplx snl[SS_MREST];
  __shared__ int nuse;
  const int c = blockIdx.x, t = threadIdx.x;
  if (!s.inner[c]) return;
  const int ss = s.ss, m1 = s.m + 1;
  const cplx* C1 = s.sC + (int64_t)c * 2 * s.sl2;
  const cplx* C2 = C1 + s.sl2;
  const cplx* R1 = s.sR + (int64_t)c * 2 * ss * ss;
  const cplx* R2 = R1 + ss * ss;
  // stage C1 in Cm, C2 in X, R1 in Rm, R2 in Ho (scratch until used below)
  ss_stage(Cm, (j0 + 1) * sb, t, SS_HT, [&](int e) { return C1[(e / sb) * ss + e % sb]; });
  ss_stage(X, (j0 + 1) * sb, t, SS_HT, [&](int e) { return C2[(e / sb) * ss + e % sb]; });
  ss_stage(Rm, sb * sb, t, SS_HT, [&](int e) { return R1[(e / sb) * ss + e % sb]; });
  ss_stage(Ho, sb * sb, t, SS_HT, [&](int e) { return R2[(e / sb) * ss + e % sb]; });
  __syncthreads();
  for (int e = t; e < (j0 + 1) * sb; e += SS_HT) {  // C = C1 + C2 R1 (in place: own entry)
    const int l = e / sb, k = e - (e / sb) * sb;
    cplx a = Cm[e];
    for (int q = 0; q <= k; ++q) cmac(a, X[l * sb + q], Rm[q * sb + k]);
    Cm[e] = a;
  }
  for (int e = t; e < sb * sb; e += SS_HT) {  // R = R2 R1, into the tail of Ho
    const int a = e / sb, k = e - (e / sb) * sb;
    cplx rr = cmk(0.0, 0.0);
    for (int q = a; q <= k; ++q) cmac(rr, Ho[a * sb + q], Rm[q * sb + k]);
    Ho[SS_MAX * SS_MAX + e] = rr;
  }
  __syncthreads();
  for (int e = t; e < sb * sb; e += SS_HT) Rm[e] = Ho[SS_MAX * SS_MAX + e];
  __syncthreads();
  if (t == 0) {
    int u = 0;
    while (u < sb && (Rm[u * sb + u].x != 0.0 || Rm[u * sb + u].y != 0.0)) ++u;
    nuse = u;
  }
  __syncthreads();
  // columns: the su Newton vectors with kept pivots give su columns; past a
  // dropped one (v_{su+1} in the span of the basis) one more column follows
  // exactly, with a zero subdiagonal (the Krylov space is invariant there)
  const int su = nuse < sb ? nuse + 1 : sb;
  const int nrow = j0 + su + 1;
  // R_hat column i (i = 0..sb) at row r: e_{j0} for i = 0; C[r][i-1] for r <= j0;
  // R[r-j0-1][i-1] for j0 < r
  auto rhat = [&](int r, int i) -> cplx {
    if (i == 0) return r == j0 ? cmk(1.0, 0.0) : cmk(0.0, 0.0);
    if (r <= j0) return Cm[r * sb + (i - 1)];
    const int a = r - j0 - 1;
    return a < sb && a <= i - 1 ? Rm[a * sb + (i - 1)] : cmk(0.0, 0.0);
  };
  const cplx* Hr = s.Hraw + (int64_t)c * m1 * s.m;  // column j at Hr + j m1, rows 0..j+1
  const cplx* th = s.theta;
  ss_stage(Ho, j0 * (j0 + 1), t, SS_HT, [&](int e) {  // H_old columns 0..j0-1, rows 0..j0
    const int q = e / (j0 + 1), r = e - (e / (j0 + 1)) * (j0 + 1);
    return r <= q + 1 ? Hr[(int64_t)q * m1 + r] : cmk(0.0, 0.0);
  });
  __syncthreads();
  // Y = R_hat B - [H_old R_top; 0] on rows 0..j0+su, columns 0..su-1 (R_top:
  // rows q < j0 of R_hat, zero in column 0)
  for (int e = t; e < nrow * su; e += SS_HT) {
    const int r = e / su, i = e - (e / su) * su;
    const double sg = 1.0 / s.sab[2 * ((int64_t)i * s.C + c)].x;  // sigma_i
    cplx y = cadd(cmul(th[(int64_t)i * s.C + c], rhat(r, i)), cscale(rhat(r, i + 1), sg));
    if (r <= j0 && i >= 1) {
      cplx acc = cmk(0.0, 0.0);
      for (int q = max(0, r - 1); q < j0; ++q) cmac(acc, Ho[q * (j0 + 1) + r], Cm[q * sb + (i - 1)]);
      y = csub(y, acc);
    }
    X[r * SS_MAX + i] = y;
  }
  __syncthreads();
  // X <- Y R_s^{-1}, R_s[a][i] = R_hat[j0 + a][i] (upper triangular): column by column
  for (int i = 0; i < su; ++i) {
    const cplx d = rhat(j0 + i, i);
    for (int r = t; r < nrow; r += SS_HT) {
      cplx y = X[r * SS_MAX + i];
      for (int q = 0; q < i; ++q) y = csub(y, cmul(X[r * SS_MAX + q], rhat(j0 + q, i)));
      X[r * SS_MAX + i] = cdiv(y, d);
    }
    __syncthreads();
  }
  // the new columns j0..j0+su-1: raw storage, then the Givens update (the
  // rotations of the earlier columns staged once; thread 0 appends its own)
  for (int q = t; q < j0; q += SS_HT) {
    csl[q] = s.cs[(int64_t)c * s.m + q];
    snl[q] = s.sn[(int64_t)c * s.m + q];
  }
  // raw columns: all at once (rows 0..j+1 of column j0 + i)
  for (int e = t; e < su * (nrow); e += SS_HT) {
    const int i = e / nrow, r = e - (e / nrow) * nrow;
    if (r <= j0 + i + 1) s.Hraw[(int64_t)c * m1 * s.m + (int64_t)(j0 + i) * m1 + r] = X[r * SS_MAX + i];
  }
  __syncthreads();  // csl, snl staged
  // Givens update of the block: thread i applies the rotations of the earlier
  // columns to new column i (all columns at once), then the su new rotations
  // follow one by one, each formed by thread 0 and applied by the threads of
  // the later columns; the bookkeeping of every column is that of
  // arnoldi_step (residual estimate, stopping test), and the first column that
  // stops ends the block.
  __shared__ double crs[SS_MAX];
  __shared__ cplx srs[SS_MAX];
  __shared__ int nstop;
  if (t < su) {
    cplx cur = X[t];
    for (int q = 0; q < j0; ++q) {
      const cplx nx = X[(q + 1) * SS_MAX + t];
      const double ci = csl[q];
      const cplx si = snl[q];
      X[q * SS_MAX + t] = cadd(cscale(cur, ci), cmul(si, nx));
      cur = csub(cscale(nx, ci), cmul(cconj(si), cur));
    }
    X[j0 * SS_MAX + t] = cur;
  }
  if (t == 0) nstop = su;
  __syncthreads();
  const int m = s.m;
  cplx* Hc = s.H + (int64_t)c * m1 * m;
  cplx* gc = s.g + (int64_t)c * m1;
  cplx gcur = cmk(0.0, 0.0);  // thread 0: g_j, iterations, ||f|| carried in registers
  int itc = 0;
  double nf = 1.0;
  if (t == 0) {
    gcur = gc[j0];
    itc = s.iters[c];
    nf = s.normf[c];
  }
  for (int k = 0; k < su; ++k) {
    const int j = j0 + k;
    if (t == 0) {
      const cplx aa = X[j * SS_MAX + k];
      const double hn = X[(j + 1) * SS_MAX + k].x;  // real by construction
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
        sr = cscale(aa, hn / (na * rho));
      }
      crs[k] = cr;
      srs[k] = sr;
      s.cs[(int64_t)c * m + j] = cr;
      s.sn[(int64_t)c * m + j] = sr;
      X[j * SS_MAX + k] = cadd(cscale(aa, cr), cscale(sr, hn));
      const cplx gj = gcur;
      const cplx gj1 = cmul(cscale(cconj(sr), -1.0), gj);
      gc[j + 1] = gj1;
      gc[j] = cscale(gj, cr);
      gcur = gj1;
      const int it = ++itc;
      s.iters[c] = it;
      const double rel = sqrt(cabs2(gj1)) / nf;
      if (s.resvec) s.resvec[(int64_t)c * (s.maxit + 1) + it] = rel;
      s.jdone[c] = j + 1;
      const bool finite = isfinite(rel) && isfinite(hn);
      if (!finite) s.status[c] = ST_BREAK;
      if (!finite || rel <= s.tol || hn == 0.0 || it >= s.maxit || j + 1 >= m) {
        s.inner[c] = 0;
        atomicSub(s.n_inner, 1);
        nstop = k + 1;
      }
    }
    __syncthreads();
    if (k + 1 >= nstop) break;
    if (t > k && t < su) {  // rotation k on rows j, j+1 of the later new columns
      const double ci = crs[k];
      const cplx si = srs[k];
      const cplx u = X[j * SS_MAX + t], v = X[(j + 1) * SS_MAX + t];
      X[j * SS_MAX + t] = cadd(cscale(u, ci), cmul(si, v));
      X[(j + 1) * SS_MAX + t] = csub(cscale(v, ci), cmul(cconj(si), u));
    }
    __syncthreads();
  }
  // the rotated columns (rows 0..j) of the processed columns
  for (int e = t; e < nstop * nrow; e += SS_HT) {
    const int i = e / nrow, r = e - (e / nrow) * nrow;
    if (r <= j0 + i) Hc[(int64_t)(j0 + i) * m1 + r] = X[r * SS_MAX + i];
  }
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
  size_t V, f, apply, ck, ckmap, ckf, ckc, rowcol, P1, H, Hraw, htent, g, cs, sn, y, normf, red,
      inv, status, inner, run, jdone, iters, ninner, total;
  int64_t n_chunks, NT;
  // block GMRES (sb > 0)
  int sb = 0, nbpi = 0, NB = 0;
  int64_t n_bck = 0, n_btile = 0;
  size_t bck, bckoff, btile, bP, bT, bH, bG, bRq, bRi, bhv, btau, bY, bin, brun, bsteps, bact;
  // s-step GMRES (ss > 0)
  int ss = 0;
  size_t sP2, stheta, ssab, sxprev, svprev, srprev, ssbad, sC, sR, sRi;
};

// Block geometry of block GMRES: reduction chunks and 64-row tiles of every
// block (optional host outputs).
void block_geometry(const mudiff_ctx* h, int R, int sb, int64_t* n_bck, int64_t* n_btile,
                    std::vector<int32_t>* bck, std::vector<int32_t>* bckoff,
                    std::vector<int32_t>* btile) {
  const int nbpi = (R + sb - 1) / sb;
  int64_t nc = 0, nt = 0;
  for (int b = 0; b < h->B; ++b) {
    const int64_t Nb = h->imode[b + 1] - h->imode[b];
    for (int k = 0; k < nbpi; ++k) {
      const int kb = b * nbpi + k;
      if (bckoff) bckoff->push_back((int32_t)nc);
      if (btile) btile->push_back((int32_t)nt);
      for (int64_t r = 0; r < Nb; r += BG_CHUNK, ++nc)
        if (bck) {
          bck->push_back(kb);
          bck->push_back((int32_t)r);
        }
      nt += (Nb + BG_TILE - 1) / BG_TILE;
    }
  }
  if (bckoff) bckoff->push_back((int32_t)nc);
  if (btile) btile->push_back((int32_t)nt);
  *n_bck = nc;
  *n_btile = nt;
}

GLayout glayout(mudiff_ctx* h, int R, int m, int sb = 0, int ss = 0) {
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
  L.P1 = take(nck * (2 * m + 2) * 16);
  L.H = take(C * (m + 1) * m * 16);
  L.Hraw = take(C * (m + 1) * m * 16);
  L.htent = take(C * (m + 1) * 16);
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
  if (sb > 0) {
    L.sb = sb;
    L.nbpi = (R + sb - 1) / sb;
    L.NB = h->B * L.nbpi;
    block_geometry(h, R, sb, &L.n_bck, &L.n_btile, nullptr, nullptr, nullptr);
    const size_t NB = (size_t)L.NB, ld = (size_t)(m + 1) * sb, np = (size_t)sb * sb;
    L.bck = take(L.n_bck * 8);
    L.bckoff = take((NB + 1) * 4);
    L.btile = take((NB + 1) * 4);
    L.bP = take((size_t)L.n_bck * (m + 1) * np * 16);
    L.bT = take(NB * ld * sb * 16);
    L.bH = take(NB * ld * m * sb * 16);
    L.bG = take(NB * ld * sb * 16);
    L.bRq = take(NB * np * 16);
    L.bRi = take(NB * np * 16);
    L.bhv = take(NB * m * sb * (sb + 1) * 16);
    L.btau = take(NB * m * sb * 16);
    L.bY = take(NB * ld * sb * 16);
    L.bin = take(NB * 4);
    L.brun = take(NB * 4);
    L.bsteps = take(NB * 4);
    L.bact = take(C * 4);
  }
  if (ss > 0) {
    L.ss = ss;
    L.sP2 = take((size_t)nck * (m + 1) * ss * 16);
    L.stheta = take((size_t)ss * C * 16);
    L.ssab = take((size_t)ss * C * 32);
    L.sxprev = take((size_t)NT * 16);
    L.svprev = take((size_t)NT * 16);
    L.srprev = take((size_t)C * 8);
    L.ssbad = take(4);
    L.sC = take((size_t)C * 2 * (m + 1) * ss * 16);
    L.sR = take((size_t)C * 2 * ss * ss * 16);
    L.sRi = take((size_t)C * ss * ss * 16);
  }
  L.total = o;
  return L;
}
}  // namespace

// Columns per block of a MUDIFF_BLOCK solve (0: not a block solve; -1: invalid).
static int block_size_of(int flags, int R, int restart) {
  if (!(flags & MUDIFF_BLOCK)) return (flags & 0xff00) ? -1 : 0;
  int sb = (flags >> 8) & 0xff;
  if (sb == 0) sb = 8;
  if (sb > BG_SMAX) return -1;
  sb = std::min(sb, R);
  if ((int64_t)restart * sb > BG_MAXDIM) return -1;
  return sb;
}

// Newton vectors per block of a MUDIFF_SSTEP solve (0: not s-step; -1: invalid).
static int sstep_size_of(int flags, int restart) {
  if (!(flags & MUDIFF_SSTEP)) return (flags & 0xff0000) ? -1 : 0;
  if (flags & MUDIFF_BLOCK) return -1;
  int ss = (flags >> 16) & 0xff;
  if (ss == 0) ss = 8;
  if (ss < 2 || ss > SS_MAX || restart > SS_MREST) return -1;
  return std::min(ss, restart);
}

static bool known_gmres_flags(int flags) {
  return (flags & ~(MUDIFF_X0 | MUDIFF_GRAPH | MUDIFF_POINT_SOURCE | MUDIFF_NO_PRECOND |
                    MUDIFF_BLOCK | MUDIFF_SSTEP | 0xff00 | 0xff0000)) == 0;
}

extern "C" size_t mudiff_gmres_workspace_size(mudiff_t h, int R, int restart, int flags) {
  if (!h || R < 1 || restart < 1 || restart > MUDIFF_MAX_RESTART) return 0;
  if (!known_gmres_flags(flags)) return 0;
  const int sb = block_size_of(flags, R, restart);
  const int ss = sstep_size_of(flags, restart);
  if (sb < 0 || ss < 0) return 0;
  return glayout(h, R, restart, sb, ss).total;
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
  int64_t ch = 256;             // rows per Gram-Schmidt chunk
  BState bs{};                  // block GMRES (L.sb > 0)
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
                                  s.V + (int64_t)(j + 1) * s.NT, s.op, G.apply_part,
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
      // few chunks (latency-bound): the basis split over workgroups; many
      // chunks (bandwidth-bound): one workgroup per chunk
      const bool spread = nb <= GS_SPREAD_CHUNKS;
      const unsigned vg = spread ? (unsigned)std::max(1, (j + GS_WAVES * GS_BATCH - 1) / (GS_WAVES * GS_BATCH)) : 1u;
      if (pending)
        hipLaunchKernelGGL(k_dg_dots<true>, dim3(nb, vg), dim3(GS_THREADS), 0, G.st, sg, j, pa, 1);
      else
        hipLaunchKernelGGL(k_dg_dots<false>, dim3(nb, vg), dim3(GS_THREADS), 0, G.st, sg, j, pa, 1);
      if (spread)
        hipLaunchKernelGGL(k_dg_update<0>, dim3(nb, (unsigned)(G.ch / 64)), dim3(GS_THREADS), 0, G.st, sg, j);
      else if (G.ch <= GS_THREADS)
        hipLaunchKernelGGL(k_dg_update<1>, dim3(nb), dim3(GS_THREADS), 0, G.st, sg, j);
      else if (G.ch <= 2 * GS_THREADS)
        hipLaunchKernelGGL(k_dg_update<2>, dim3(nb), dim3(GS_THREADS), 0, G.st, sg, j);
      else
        hipLaunchKernelGGL(k_dg_update<4>, dim3(nb), dim3(GS_THREADS), 0, G.st, sg, j);
    }
    HIP_TRY(hipGetLastError());
    if (host_checks && check_every > 0 && (j + 1) % check_every == 0 && j + 1 < s.m) {
      int32_t n_in = 0;
      HIP_TRY(hipMemcpyAsync(&n_in, s.n_inner, 4, hipMemcpyDeviceToHost, G.st));
      HIP_TRY(hipStreamSynchronize(G.st));
      if (n_in <= 0) break;
    }
  }
  {  // columns that ran all m steps: Hessenberg column m-1 from the last candidate V[m]
    GState sg = s;
    unsigned nb = (unsigned)G.L.n_chunks;
    if (G.n_compact > 0) {
      sg.ckmap = G.d_ckmap;
      nb = (unsigned)G.ckmap.size();
    }
    PendingApply pa{};
    if (nb > 0)
      hipLaunchKernelGGL(k_dg_dots<false>,
                         dim3(nb, nb <= GS_SPREAD_CHUNKS ? (unsigned)((s.m + GS_WAVES * GS_BATCH - 1) / (GS_WAVES * GS_BATCH)) : 1u),
                         dim3(GS_THREADS), 0, G.st, sg, s.m, pa, 0);
    hipLaunchKernelGGL(k_dg_flush, dim3(s.C), dim3(GS_THREADS), 0, G.st, s);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_cycle_solve, dim3(s.C), dim3(64), 0, G.st, s);
  hipLaunchKernelGGL(k_update_x, dim3(eb), dim3(256), 0, G.st, s, s.NT, G.d_rowcol);
  HIP_TRY(hipGetLastError());
  int rc = apply_operator(G.h, s.R, s.x, s.V, s.op, G.apply_part, G.apply_cnt, s.run, G.st);
  if (rc != MUDIFF_OK) return rc;
  hipLaunchKernelGGL(k_resid, dim3((unsigned)G.L.n_chunks), dim3(GS_THREADS), 0, G.st, s, 2, 1,
                     (const cplx*)nullptr);
  hipLaunchKernelGGL(k_col_sum, dim3(s.C), dim3(64), 0, G.st, s, 1);
  // the true residual decides each column's next cycle
  hipLaunchKernelGGL(k_cycle_begin, dim3(cb), dim3(64), 0, G.st, s);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}

// One restart cycle of block GMRES: QR of the residual block, up to m block
// Arnoldi steps with the least-squares update after each, the solution update
// and the true residual that decides each column's next cycle.
static int enqueue_bcycle(GmresRun& G, int check_every, bool host_checks) {
  BState& bs = G.bs;
  const GState& s = bs.s;
  hipStream_t st = G.st;
  const unsigned nbk = (unsigned)G.L.n_bck, ntl = (unsigned)G.L.n_btile, NB = (unsigned)G.L.NB;
  const int64_t NT = s.NT;
  auto cholqr = [&](cplx* W, int j, const int32_t* gate) {
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(k_bdots, dim3(nbk, 1), dim3(256), 0, st, bs, (const cplx*)W, NT,
                         (const cplx*)W, gate);
      hipLaunchKernelGGL(k_bchol, dim3(NB), dim3(256), 0, st, bs, pass, j, gate);
      hipLaunchKernelGGL(k_bscale, dim3(ntl), dim3(256), 0, st, bs, W, gate);
    }
  };
  cholqr(s.V, -1, bs.brun);
  HIP_TRY(hipGetLastError());
  for (int j = 0; j < s.m; ++j) {
    cplx* W = s.V + (int64_t)(j + 1) * NT;
    int rc = apply_operator(G.h, s.R, s.V + (int64_t)j * NT, W, s.op, G.apply_part, G.apply_cnt,
                            bs.bact, st);
    if (rc != MUDIFF_OK) return rc;
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(k_bdots, dim3(nbk, (unsigned)(j + 1)), dim3(256), 0, st, bs,
                         (const cplx*)s.V, NT, (const cplx*)W, (const int32_t*)bs.bin);
      hipLaunchKernelGGL(k_bsum, dim3(NB, (unsigned)(j + 1)), dim3(256), 0, st, bs, j, pass);
      hipLaunchKernelGGL(k_bupdate, dim3(ntl), dim3(256), 0, st, bs, (const cplx*)s.V, NT, W,
                         (const cplx*)bs.T, j + 1, (const int32_t*)nullptr,
                         (const int32_t*)bs.bin, -1.0);
    }
    cholqr(W, j, bs.bin);
    hipLaunchKernelGGL(k_blsq, dim3(NB), dim3(64 * bs.sb), 0, st, bs, j);
    HIP_TRY(hipGetLastError());
    if (host_checks && check_every > 0 && (j + 1) % check_every == 0 && j + 1 < s.m) {
      int32_t n_in = 0;
      HIP_TRY(hipMemcpyAsync(&n_in, s.n_inner, 4, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (n_in <= 0) break;
    }
  }
  hipLaunchKernelGGL(k_bsolve, dim3(NB, (unsigned)bs.sb), dim3(256), 0, st, bs);
  hipLaunchKernelGGL(k_bupdate, dim3(ntl), dim3(256), 0, st, bs, (const cplx*)s.V, NT, s.x,
                     (const cplx*)bs.Y, 0, (const int32_t*)bs.bsteps, (const int32_t*)bs.brun, 1.0);
  HIP_TRY(hipGetLastError());
  int rc = apply_operator(G.h, s.R, s.x, s.V, s.op, G.apply_part, G.apply_cnt, s.run, st);
  if (rc != MUDIFF_OK) return rc;
  hipLaunchKernelGGL(k_resid, dim3((unsigned)G.L.n_chunks), dim3(GS_THREADS), 0, st, s, 2, 1,
                     (const cplx*)nullptr);
  hipLaunchKernelGGL(k_col_sum, dim3(s.C), dim3(64), 0, st, s, 1);
  hipLaunchKernelGGL(k_bcycle_begin, dim3((unsigned)((s.C + 63) / 64)), dim3(64), 0, st, s);
  hipLaunchKernelGGL(k_zero_i, dim3(1), dim3(64), 0, st, s.n_inner, 1);
  hipLaunchKernelGGL(k_bblock_begin, dim3((NB + 63) / 64), dim3(64), 0, st, bs);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}

// Guard of an s-step cycle.  Restarted GMRES never raises a column's true
// residual (the update minimises over a space that contains zero), but a
// Newton basis built from poor shifts can lose orthogonality so far that the
// computed update does.  Before the cycle: the iterate, its residual and the
// squared norm of every column that runs are saved.  After it: a column whose
// true residual grew (by more than 1e-10 relative, far above rounding) gets
// them back, and the flag is raised; the solve then continues with the
// one-vector process, which cannot do that.
__global__ void k_ss_save(GState s, int64_t nrows_total, const int32_t* __restrict__ row_col) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < s.C) s.rprev[g] = s.red[g];
  if (g >= nrows_total) return;
  if (!s.inner[row_col[g]]) return;
  s.xprev[g] = s.x[g];
  s.vprev[g] = s.V[g];
}

__device__ __forceinline__ bool ss_cycle_failed(const GState& s, int c) {
  return s.run[c] && s.red[c] > s.rprev[c] * (1.0 + 1e-10);
}

__global__ void k_ss_guard_rows(GState s, int64_t nrows_total, const int32_t* __restrict__ row_col) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nrows_total) return;
  if (!ss_cycle_failed(s, row_col[g])) return;
  s.x[g] = s.xprev[g];
  s.V[g] = s.vprev[g];
}

__global__ void k_ss_guard_cols(GState s) {  // after k_ss_guard_rows
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= s.C || !ss_cycle_failed(s, c)) return;
  s.red[c] = s.rprev[c];
  atomicExch(s.ssbad, 1);
}

// One restart cycle of s-step GMRES (after the first cycle has given the
// shifts): blocks of ss Newton vectors, each orthogonalised by two
// reduction/sweep passes and folded into the Hessenberg matrix, then the
// solution update and the true residual as in enqueue_cycle.
static int enqueue_sscycle(GmresRun& G, bool host_checks) {
  GState& s = G.s;
  hipStream_t st = G.st;
  const unsigned eb = (unsigned)((s.NT + 255) / 256);
  const unsigned cb = (unsigned)((s.C + 63) / 64);
  const unsigned nb = (unsigned)G.L.n_chunks;
  const unsigned ry = (unsigned)((G.ch + SS_UR - 1) / SS_UR);
  const bool wide = nb >= SSW_MIN_CHUNKS;  // bandwidth-bound sweeps (many right-hand sides)
  const unsigned ryw = (unsigned)((G.ch + SSW_RB - 1) / SSW_RB);
  const unsigned sb_rows = (unsigned)((std::max<int64_t>(s.NT, s.C) + 255) / 256);
  hipLaunchKernelGGL(k_ss_save, dim3(sb_rows), dim3(256), 0, st, s, s.NT, G.d_rowcol);
  hipLaunchKernelGGL(k_scale_v0, dim3(eb), dim3(256), 0, st, s, s.NT, G.d_rowcol);
  HIP_TRY(hipGetLastError());
  for (int j0 = 0; j0 < s.m; j0 += s.ss) {
    const int sb = std::min(s.ss, s.m - j0);
    for (int i = 0; i < sb; ++i) {
      int rc = apply_operator(G.h, s.R, s.V + (int64_t)(j0 + i) * s.NT, s.V + (int64_t)(j0 + i + 1) * s.NT,
                              s.op, G.apply_part, G.apply_cnt, s.inner, st, s.sab + 2 * (int64_t)i * s.C);
      if (rc != MUDIFF_OK) return rc;
    }
    const unsigned nvg = (unsigned)((j0 + 1 + sb + GS_WAVES - 1) / GS_WAVES);
    for (int pass = 0; pass < 2; ++pass) {
      if (wide) {
        const int nl = j0 + 1 + sb;
        const size_t lds = (size_t)std::max(nl * (SSW_TR + 1), GS_THREADS * 8) * 16;
        hipLaunchKernelGGL(k_ss_dots_w, dim3(nb), dim3(GS_THREADS), lds, st, s, j0, sb);
      } else {
        hipLaunchKernelGGL(k_ss_dots, dim3(nb, nvg), dim3(GS_THREADS), 0, st, s, j0, sb);
      }
      hipLaunchKernelGGL(k_ss_red, dim3((unsigned)s.C, (unsigned)(((j0 + 1 + sb) * sb + GS_THREADS - 1) / GS_THREADS)),
                         dim3(GS_THREADS), 0, st, s, j0, sb, pass);
      hipLaunchKernelGGL(k_ss_chol, dim3((unsigned)s.C), dim3(64), 0, st, s, j0, sb, pass);
      if (wide)
        hipLaunchKernelGGL(k_ss_update_w, dim3(nb, ryw), dim3(GS_THREADS), 0, st, s, j0, sb, pass);
      else
        hipLaunchKernelGGL(k_ss_update, dim3(nb, ry), dim3(GS_THREADS), 0, st, s, j0, sb, pass);
    }
    hipLaunchKernelGGL(k_ss_hess, dim3((unsigned)s.C), dim3(SS_HT), 0, st, s, j0, sb);
    HIP_TRY(hipGetLastError());
    if (host_checks && j0 + sb < s.m) {
      int32_t n_in = 0;
      HIP_TRY(hipMemcpyAsync(&n_in, s.n_inner, 4, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (n_in <= 0) break;
    }
  }
  hipLaunchKernelGGL(k_cycle_solve, dim3(s.C), dim3(64), 0, st, s);
  hipLaunchKernelGGL(k_update_x, dim3(eb), dim3(256), 0, st, s, s.NT, G.d_rowcol);
  HIP_TRY(hipGetLastError());
  int rc = apply_operator(G.h, s.R, s.x, s.V, s.op, G.apply_part, G.apply_cnt, s.run, st);
  if (rc != MUDIFF_OK) return rc;
  hipLaunchKernelGGL(k_resid, dim3(nb), dim3(GS_THREADS), 0, st, s, 2, 1, (const cplx*)nullptr);
  hipLaunchKernelGGL(k_col_sum, dim3(s.C), dim3(64), 0, st, s, 1);
  hipLaunchKernelGGL(k_ss_guard_rows, dim3(eb), dim3(256), 0, st, s, s.NT, G.d_rowcol);
  hipLaunchKernelGGL(k_ss_guard_cols, dim3(cb), dim3(64), 0, st, s);
  hipLaunchKernelGGL(k_cycle_begin, dim3(cb), dim3(64), 0, st, s);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}

// Shifts of the s-step cycles from the first cycle: per running column, the
// Ritz values (eigenvalues of the square Hessenberg matrix of its jdone steps)
// in Leja order, ss of them (columns that stopped get zeros).
static int sstep_shifts(GmresRun& G) {
  GState& s = G.s;
  const int m = s.m, m1 = m + 1, C = s.C, ss = s.ss;
  std::vector<cplx> Hr((size_t)C * m1 * m);
  std::vector<int32_t> run(C), jd(C);
  HIP_TRY(hipMemcpyAsync(Hr.data(), s.Hraw, Hr.size() * 16, hipMemcpyDeviceToHost, G.st));
  HIP_TRY(hipMemcpyAsync(run.data(), s.run, (size_t)C * 4, hipMemcpyDeviceToHost, G.st));
  HIP_TRY(hipMemcpyAsync(jd.data(), s.jdone, (size_t)C * 4, hipMemcpyDeviceToHost, G.st));
  HIP_TRY(hipStreamSynchronize(G.st));
  std::vector<cplx> th((size_t)ss * C, cmk(0.0, 0.0));
  std::vector<cplx> ab((size_t)2 * ss * C);  // (1 / sigma, -theta / sigma)
  for (size_t e = 0; e < (size_t)ss * C; ++e) {
    ab[2 * e] = cmk(1.0, 0.0);
    ab[2 * e + 1] = cmk(0.0, 0.0);
  }
  std::vector<ritz::cd> Hc, ev;
  for (int c = 0; c < C; ++c) {
    const int n = jd[c];
    if (!run[c] || n < 1) continue;
    Hc.assign((size_t)n * n, ritz::cd(0.0));
    for (int j = 0; j < n; ++j)
      for (int r = 0; r <= std::min(j + 1, n - 1); ++r) {
        const cplx v = Hr[(size_t)c * m1 * m + (size_t)j * m1 + r];
        Hc[(size_t)j * n + r] = ritz::cd(v.x, v.y);
      }
    ritz::hessenberg_eigenvalues(n, Hc.data(), n, ev);
    const std::vector<ritz::cd> lj = ritz::leja(ev, ss);
    const std::vector<double> sg = ritz::newton_scales(ev, lj);
    for (int i = 0; i < (int)lj.size(); ++i) {
      const size_t e = (size_t)i * C + c;
      th[e] = cmk(lj[i].real(), lj[i].imag());
      ab[2 * e] = cmk(1.0 / sg[i], 0.0);
      ab[2 * e + 1] = cmk(-lj[i].real() / sg[i], -lj[i].imag() / sg[i]);
    }
  }
  HIP_TRY(hipMemcpyAsync(s.theta, th.data(), th.size() * 16, hipMemcpyHostToDevice, G.st));
  HIP_TRY(hipMemcpyAsync(s.sab, ab.data(), ab.size() * 16, hipMemcpyHostToDevice, G.st));
  HIP_TRY(hipStreamSynchronize(G.st));
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
  if (!known_gmres_flags(flags)) return fail(MUDIFF_ERR_INVALID, "unknown flags");
  const int sb = block_size_of(flags, R, restart);
  if (sb < 0)
    return fail(MUDIFF_ERR_INVALID, "block size must be 1.." + std::to_string(BG_SMAX) +
                                        " with restart * block size <= " + std::to_string(BG_MAXDIM));
  int ss = sstep_size_of(flags, restart);  // 0 from a fallback to one-vector cycles on
  if (ss < 0)
    return fail(MUDIFF_ERR_INVALID, "s-step size must be 2.." + std::to_string(SS_MAX) +
                                        " with restart <= " + std::to_string(SS_MREST) +
                                        ", not with MUDIFF_BLOCK");
  GLayout L = glayout(h, R, restart, sb, ss);
  if (!workspace) return fail(MUDIFF_ERR_INVALID, "workspace is NULL");
  apply_forget_upload(h);
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
  s.op = (flags & MUDIFF_NO_PRECOND) ? MUDIFF_OP_L : MUDIFF_OP_A;
  s.maxit = maxit;
  s.tol = tol;
  s.NT = L.NT;
  s.V = (cplx*)(w + L.V);
  s.f = (cplx*)(w + L.f);
  s.x = (cplx*)rho;
  s.ck = (int64_t*)(w + L.ck);
  s.ckmap = nullptr;
  G.d_ckmap = (int32_t*)(w + L.ckmap);
  s.sl = 2 * restart + 2;
  s.P1 = (cplx*)(w + L.P1);
  s.H = (cplx*)(w + L.H);
  s.Hraw = (cplx*)(w + L.Hraw);
  s.htent = (cplx*)(w + L.htent);
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
  s.ss = ss;
  s.sl2 = (restart + 1) * ss;
  s.P2 = ss ? (cplx*)(w + L.sP2) : nullptr;
  s.theta = ss ? (cplx*)(w + L.stheta) : nullptr;
  s.sab = ss ? (cplx*)(w + L.ssab) : nullptr;
  s.xprev = ss ? (cplx*)(w + L.sxprev) : nullptr;
  s.vprev = ss ? (cplx*)(w + L.svprev) : nullptr;
  s.rprev = ss ? (double*)(w + L.srprev) : nullptr;
  s.ssbad = ss ? (int32_t*)(w + L.ssbad) : nullptr;
  s.sC = ss ? (cplx*)(w + L.sC) : nullptr;
  s.sR = ss ? (cplx*)(w + L.sR) : nullptr;
  s.sRi = ss ? (cplx*)(w + L.sRi) : nullptr;
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
  G.ch = ch;
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
    if ((rc = launch_rhs(h, R, beta, (cplx*)s.f, s.op == MUDIFF_OP_A ? 1 : 2,
                         (flags & MUDIFF_POINT_SOURCE) ? 1 : 0, st)) != MUDIFF_OK)
      return rc;
  } else {
    hipLaunchKernelGGL(k_precond_rhs, dim3(eb), dim3(256), 0, st, h->dv, R, (const cplx*)rhs,
                       (cplx*)s.f, -1.0, s.op == MUDIFF_OP_A ? 1 : 0);
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
    rc = apply_operator(h, R, s.x, s.V, s.op, G.apply_part, G.apply_cnt, s.run, st);
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

  if (sb > 0) {  // block GMRES: block tables, then the first cycle's column and block state
    BState& bs = G.bs;
    bs.s = s;
    bs.imode = h->dv.imode;
    bs.sb = sb;
    bs.nbpi = L.nbpi;
    bs.NB = L.NB;
    std::vector<int32_t> bck, bckoff, btile;
    int64_t n_bck = 0, n_btile = 0;
    block_geometry(h, R, sb, &n_bck, &n_btile, &bck, &bckoff, &btile);
    bs.bck = (const int32_t*)(w + L.bck);
    bs.bckoff = (const int32_t*)(w + L.bckoff);
    bs.btile = (const int32_t*)(w + L.btile);
    bs.P = (cplx*)(w + L.bP);
    bs.T = (cplx*)(w + L.bT);
    bs.Hb = (cplx*)(w + L.bH);
    bs.Gb = (cplx*)(w + L.bG);
    bs.Rq = (cplx*)(w + L.bRq);
    bs.Ri = (cplx*)(w + L.bRi);
    bs.hv = (cplx*)(w + L.bhv);
    bs.htau = (cplx*)(w + L.btau);
    bs.Y = (cplx*)(w + L.bY);
    bs.bin = (int32_t*)(w + L.bin);
    bs.brun = (int32_t*)(w + L.brun);
    bs.bsteps = (int32_t*)(w + L.bsteps);
    bs.bact = (int32_t*)(w + L.bact);
    HIP_TRY(hipMemcpyAsync((void*)bs.bck, bck.data(), bck.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync((void*)bs.bckoff, bckoff.data(), bckoff.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync((void*)bs.btile, btile.data(), btile.size() * 4, hipMemcpyHostToDevice, st));
    // the host vectors go out of scope: wait for the copies
    HIP_TRY(hipStreamSynchronize(st));
    hipLaunchKernelGGL(k_bcycle_begin, dim3(cb), dim3(64), 0, st, s);
    hipLaunchKernelGGL(k_zero_i, dim3(1), dim3(64), 0, st, s.n_inner, 1);
    hipLaunchKernelGGL(k_bblock_begin, dim3((unsigned)((L.NB + 63) / 64)), dim3(64), 0, st, bs);
  } else {
    hipLaunchKernelGGL(k_cycle_begin, dim3(cb), dim3(64), 0, st, s);
  }
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
    if (ss > 0) {  // s-step: the first cycle by delayed CGS2 gives the shifts
      if (cyc == 0) {
        if ((result = enqueue_cycle(G, 10, true)) != MUDIFF_OK) break;
        if ((result = sstep_shifts(G)) != MUDIFF_OK) break;
        hipLaunchKernelGGL(k_zero_i, dim3(1), dim3(64), 0, st, s.ssbad, 1);
        continue;
      }
      int32_t bad = 0;  // a cycle raised a true residual: one-vector cycles from here on
      HIP_TRY(hipMemcpyAsync(&bad, s.ssbad, 4, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (bad) {
        ss = 0;
        if (exec) {
          (void)hipGraphExecDestroy(exec);
          exec = nullptr;
        }
        if (graph) {
          (void)hipGraphDestroy(graph);
          graph = nullptr;
        }
      }
    }
    if (sb == 0 && ss == 0 && s.C >= 32 && n_run * 32 <= s.C &&
        (G.n_compact == 0 || n_run * 2 <= G.n_compact)) {
      if ((result = compact_columns(G, hstat, n_run)) != MUDIFF_OK) break;
      // the captured cycle launches the full apply and sweeps: capture it again
      // on the running columns (the stream is idle since the status copy)
      if (exec) {
        (void)hipGraphExecDestroy(exec);
        exec = nullptr;
      }
      if (graph) {
        (void)hipGraphDestroy(graph);
        graph = nullptr;
      }
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
        int e = sb > 0 ? enqueue_bcycle(Gc, 0, false)
                       : (ss > 0 ? enqueue_sscycle(Gc, false) : enqueue_cycle(Gc, 0, false));
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
      if ((result = sb > 0 ? enqueue_bcycle(G, 10, true)
                           : (ss > 0 ? enqueue_sscycle(G, true) : enqueue_cycle(G, 10, true))) != MUDIFF_OK)
        break;
    }
  }
  if (exec) {
    (void)hipStreamSynchronize(st);
    (void)hipGraphExecDestroy(exec);
  }
  if (graph) (void)hipGraphDestroy(graph);
  if (result != MUDIFF_OK) {
    // later applies on the handle must not keep the straggler schedule
    (void)apply_set_tail(h, R, false, G.apply_part, st, nullptr);
    return result;
  }
  hipLaunchKernelGGL(k_finish, dim3(cb), dim3(64), 0, st, s, flag, relres, iters);
  HIP_TRY(hipGetLastError());
  return apply_set_tail(h, R, false, G.apply_part, st, nullptr);  // back to the tuned schedule
}
