// Time reversal with a far-field mirror (paper sec. 7, Example III): the
// time-reversal matrix T = conj(F)^T F of the mirror's far-field matrix F, the
// eigen-decomposition of T, and the Herglotz waves its eigenvectors define.
//
// Layout: X[j][i] = F[i][j] = a(theta_i; alpha_j), i.e. row j of X is the far
// field of incidence j at the receivers (mudiff_farfield's output for one
// instance with R = n incidences), so the columns of F are contiguous rows.
#include <algorithm>

#include "common.h"

namespace {

typedef double dort_d4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ T = F^H F
// T[a][b] = sum_i conj(X[a][i]) X[b][i]:
//   Re T = Xr Xr^T + Xi Xi^T,   Im T = Xr Xi^T - Xi Xr^T,
// four real 16x4-by-4x16 products per step of four receivers on the FP64
// matrix cores (v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16],
// B[l/16][l%16] and D[4v + l/16][l%16]).  One wave per 16x16 tile of T.
__global__ __launch_bounds__(64) void k_tro(int n, int m, const cplx* __restrict__ X,
                                            cplx* __restrict__ T) {
  const int a0 = blockIdx.x * 16, b0 = blockIdx.y * 16;
  const int lane = threadIdx.x, r = lane & 15, kk = lane >> 4;
  const int ra = a0 + r, rb = b0 + r;
  dort_d4 accr = {0.0, 0.0, 0.0, 0.0}, acci = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = 0; i0 < m; i0 += 4) {
    const int i = i0 + kk;
    const cplx xa = (ra < n && i < m) ? X[(int64_t)ra * m + i] : cmk(0.0, 0.0);
    const cplx xb = (rb < n && i < m) ? X[(int64_t)rb * m + i] : cmk(0.0, 0.0);
    accr = __builtin_amdgcn_mfma_f64_16x16x4f64(xa.x, xb.x, accr, 0, 0, 0);
    accr = __builtin_amdgcn_mfma_f64_16x16x4f64(xa.y, xb.y, accr, 0, 0, 0);
    acci = __builtin_amdgcn_mfma_f64_16x16x4f64(xa.x, xb.y, acci, 0, 0, 0);
    acci = __builtin_amdgcn_mfma_f64_16x16x4f64(-xa.y, xb.x, acci, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int a = a0 + 4 * v + kk, b = b0 + r;
    if (a < n && b < n) T[(int64_t)a * n + b] = cmk(accr[v], acci[v]);
  }
}

// ------------------------------------------------------------------ one-sided Jacobi
// The eigenpairs of T = F^H F follow from orthogonalising the columns of F by
// plane rotations (Hestenes): F J_1 J_2 ... = F V with orthogonal columns, so
// V^H T V = diag(|F v_j|^2).  A sweep pairs every two columns once, in rounds
// of n'/2 disjoint pairs (circle method over n' = n rounded up to even; the
// pairs with the padding index are skipped), one workgroup per pair and one
// launch per round: the pairs of a round touch disjoint columns, so no
// synchronisation between workgroups is needed.
constexpr int JAC_THREADS = 256;

__device__ __forceinline__ void round_pair(int r, int k, int np, int* p, int* q) {
  if (k == 0) {
    *p = r;
    *q = np - 1;
  } else {
    *p = (r + k) % (np - 1);
    *q = (r - k + np - 1) % (np - 1);
  }
  if (*p > *q) {
    const int t = *p;
    *p = *q;
    *q = t;
  }
}

// Sum over the block of four per-thread values, in a fixed order.
__device__ void block_sum4(double (&v)[4], double* sred) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[c] += __shfl_xor(v[c], o, 64);
    if (lane == 0) sred[c * (JAC_THREADS / 64) + wv] = v[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double t = 0.0;
    for (int k = 0; k < JAC_THREADS / 64; ++k) t += sred[c * (JAC_THREADS / 64) + k];
    v[c] = t;
  }
}

// Rotation of columns p, q of F (rows p, q of X) and of V (rows p, q of Vt)
// that zeroes gamma = f_p^H f_q: with zeta = (beta - alpha) / (2 |gamma|),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), cs = 1 / sqrt(1 + t^2),
// s = t cs gamma / |gamma|:  [f_p, f_q] <- [f_p, f_q] [[cs, s], [-conj(s), cs]].
// A pair counts as orthogonal when |gamma| <= tol sqrt(alpha beta), or when
// |gamma| <= eps |F|_F^2, below the rounding level of the entries of T.  The
// four rows are loaded into registers at once (EPT elements per thread; EPT = 0:
// rows longer than 8 * JAC_THREADS, streamed twice).  n_rot counts the
// rotations of the sweep.  These rounds serve rows longer than 1024 entries;
// shorter ones take the block rounds below.
template <int EPT>
__global__ __launch_bounds__(JAC_THREADS) void k_jacobi_round(int n, int m, int np, int r,
                                                              cplx* __restrict__ X,
                                                              cplx* __restrict__ Vt, double tol,
                                                              const double* __restrict__ fro2,
                                                              int32_t* __restrict__ n_rot) {
  __shared__ double sred[4 * (JAC_THREADS / 64)];
  int p, q;
  round_pair(r, blockIdx.x, np, &p, &q);
  if (q >= n) return;  // pair with the padding index
  cplx* fp = X + (int64_t)p * m;
  cplx* fq = X + (int64_t)q * m;
  cplx* vp = Vt + (int64_t)p * n;
  cplx* vq = Vt + (int64_t)q * n;
  constexpr int E = EPT > 0 ? EPT : 1;
  cplx ra[E], rb[E], va[E], vb[E];
  double v[4] = {0.0, 0.0, 0.0, 0.0};  // alpha, beta, Re gamma, Im gamma
  auto gram = [&](cplx a, cplx b) {
    v[0] += cabs2(a);
    v[1] += cabs2(b);
    v[2] = fma(a.x, b.x, fma(a.y, b.y, v[2]));
    v[3] = fma(a.x, b.y, fma(-a.y, b.x, v[3]));
  };
  if constexpr (EPT > 0) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int i = threadIdx.x + e * JAC_THREADS;
      ra[e] = i < m ? fp[i] : cmk(0.0, 0.0);
      rb[e] = i < m ? fq[i] : cmk(0.0, 0.0);
      va[e] = i < n ? vp[i] : cmk(0.0, 0.0);
      vb[e] = i < n ? vq[i] : cmk(0.0, 0.0);
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) gram(ra[e], rb[e]);
  } else {
    for (int i = threadIdx.x; i < m; i += JAC_THREADS) gram(fp[i], fq[i]);
  }
  block_sum4(v, sred);
  const double al = v[0], be = v[1];
  const double g = sqrt(v[2] * v[2] + v[3] * v[3]);
  if (!(g > tol * sqrt(al * be)) || !(g > 2.220446049250313e-16 * fro2[0])) return;
  const double zeta = (be - al) / (2.0 * g);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double cs = 1.0 / sqrt(1.0 + t * t);
  const cplx s = cmk(t * cs * v[2] / g, t * cs * v[3] / g);
  const cplx sc = cconj(s);
  if constexpr (EPT > 0) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int i = threadIdx.x + e * JAC_THREADS;
      if (i < m) {
        fp[i] = csub(cscale(ra[e], cs), cmul(sc, rb[e]));
        fq[i] = cadd(cmul(s, ra[e]), cscale(rb[e], cs));
      }
      if (i < n) {
        vp[i] = csub(cscale(va[e], cs), cmul(sc, vb[e]));
        vq[i] = cadd(cmul(s, va[e]), cscale(vb[e], cs));
      }
    }
  } else {
    for (int i = threadIdx.x; i < m; i += JAC_THREADS) {
      const cplx a = fp[i], b = fq[i];
      fp[i] = csub(cscale(a, cs), cmul(sc, b));
      fq[i] = cadd(cmul(s, a), cscale(b, cs));
    }
    for (int i = threadIdx.x; i < n; i += JAC_THREADS) {
      const cplx a = vp[i], b = vq[i];
      vp[i] = csub(cscale(a, cs), cmul(sc, b));
      vq[i] = cadd(cmul(s, a), cscale(b, cs));
    }
  }
  if (threadIdx.x == 0) atomicAdd(n_rot, 1);
}

// Block rounds, for rows of X and Vt of at most EPT * NT entries (NT threads
// per workgroup).  The columns are grouped in nb = ceil(n / 4) blocks of JB = 4,
// block P holding columns P, P + nb, P + 2 nb, P + 3 nb (neighbouring columns of
// a far-field matrix are nearly parallel; spread over different blocks they
// take fewer sweeps), and a round pairs the blocks (circle method over nb
// rounded up to even, nb').  The workgroup of blocks (P, Q) rotates the 16
// pairs (p_i, q_j) in four steps of the four disjoint pairs
// (p_i, q_{(i+s) mod 4}); in the first round of a sweep it first rotates the 6
// pairs inside each of its two blocks, in three steps.  Every pair of columns
// is rotated once per sweep, as in the rounds above, in nb' launches instead of
// n' - 1 (V follows one launch behind F, see the kernel).  The 8 columns of F
// stay in registers for the round; the 16 sums of a step (alpha, beta, gamma of each pair) share one block
// reduction: a reduce-scatter across the wave (lane swaps and DPP) leaves sum c
// on lanes 4c..4c+3, then the waves' partial sums are added from LDS in a fixed
// order by lane k (mod 4) for pair k, which also computes that pair's rotation,
// handed to the wave by readlane: one copy of the rotation arithmetic per step.
// Slots past column n - 1 and those of the padding block read as zero and are
// never rotated or stored.  Blocks of 8 (63 launches a sweep at n = 512) were
// slower: they put the sweep's arithmetic on half as many compute units.

// The value of x on lane l, for the whole wave.
__device__ __forceinline__ double wave_bcast(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __hiloint2double(hi, lo);
}

constexpr int JB = 4;

// Rotation records: rec[parity of the round][workgroup][step][pair] = (cs,
// Re s, Im s, 1 if rotated else 0), at most 7 steps a round.
constexpr int JSTEPS = 7;

__device__ __forceinline__ double* jac_rec(double* rec, int rr, int nwg, int wg, int st, int k) {
  return rec + 4 * ((((int64_t)(rr & 1) * nwg + wg) * JSTEPS + st) * JB + k);
}

// The steps of round rr in order, each as its four pairs (a[k], b[k]) of slots.
template <typename StepFn>
__device__ __forceinline__ void jac_steps(int rr, StepFn&& step) {
  if (rr == 0) {
    // inside the blocks: (0,1)(2,3), (0,2)(1,3), (0,3)(1,2) in P and in Q (this
    // order took 8 sweeps on a 512-cell far-field matrix, the circle order 11)
    step(0, {0, 2, 4, 6}, {1, 3, 5, 7});
    step(1, {0, 1, 4, 5}, {2, 3, 6, 7});
    step(2, {0, 1, 4, 5}, {3, 2, 7, 6});
  }
  const int s0 = rr == 0 ? 3 : 0;
  step(s0, {0, 1, 2, 3}, {4, 5, 6, 7});
  step(s0 + 1, {0, 1, 2, 3}, {5, 6, 7, 4});
  step(s0 + 2, {0, 1, 2, 3}, {6, 7, 4, 5});
  step(s0 + 3, {0, 1, 2, 3}, {7, 4, 5, 6});
}

// One launch: workgroups [0, nf) take round r on the columns of F and record
// each rotation; workgroups [nf, nf + nv) apply the rotations recorded in round
// rv = r - 1 (the previous launch) to the columns of V, on other compute units
// and off the path of F's reductions.  r = -1: V only (the last round of a
// sweep); rv = -1: F only (the first).
template <int EPT, int NT>
__global__ __launch_bounds__(NT) void k_jacobi_block_round(int n, int m, int nbp, int r, int rv,
                                                            cplx* __restrict__ X,
                                                            cplx* __restrict__ Vt, double tol,
                                                            const double* __restrict__ fro2,
                                                            double* __restrict__ rec,
                                                            int32_t* __restrict__ n_rot) {
  constexpr int NW = NT / 64, NS = 4 * JB, LPV = 64 / NS;
  __shared__ double sred[2][NS][NW + 1];  // padded: the lanes of different pairs hit different banks
  const int nwg = nbp / 2, nf = r >= 0 ? nwg : 0;
  const bool frole = (int)blockIdx.x < nf;
  const int rr = frole ? r : rv, wg = frole ? (int)blockIdx.x : (int)blockIdx.x - nf;
  int P, Q;
  round_pair(rr, wg, nbp, &P, &Q);
  const int nb = (n + JB - 1) / JB;
  if (Q >= nb && rr > 0) return;  // the padding block: nothing inside a block left to do
  int col[2 * JB];  // column of each slot, -1 for none
#pragma unroll
  for (int j = 0; j < 2 * JB; ++j) {
    const int B = j < JB ? P : Q;
    const int c = B + nb * (j & (JB - 1));
    col[j] = (B < nb && c < n) ? c : -1;
  }
  unsigned touched = 0u;
  if (!frole) {
    // V: replay the round's rotations on the rows of Vt
    cplx v[2 * JB][EPT];
#pragma unroll
    for (int j = 0; j < 2 * JB; ++j)
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int i = threadIdx.x + e * NT;
        v[j][e] = (col[j] >= 0 && i < n) ? Vt[(int64_t)col[j] * n + i] : cmk(0.0, 0.0);
      }
    jac_steps(rr, [&](int st, const int (&a)[JB], const int (&b)[JB]) {
#pragma unroll
      for (int k = 0; k < JB; ++k) {
        const double* q = jac_rec(rec, rr, nwg, wg, st, k);
        if (q[3] == 0.0) continue;
        const double c = q[0];
        const cplx sn = cmk(q[1], q[2]);
        const cplx sc = cconj(sn);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
          const cplx x = v[a[k]][e], y = v[b[k]][e];
          v[a[k]][e] = csub(cscale(x, c), cmul(sc, y));
          v[b[k]][e] = cadd(cmul(sn, x), cscale(y, c));
        }
        touched |= (1u << a[k]) | (1u << b[k]);
      }
    });
#pragma unroll
    for (int j = 0; j < 2 * JB; ++j) {
      if (!((touched >> j) & 1u) || col[j] < 0) continue;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int i = threadIdx.x + e * NT;
        if (i < n) Vt[(int64_t)col[j] * n + i] = v[j][e];
      }
    }
    return;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double eps_f = 2.220446049250313e-16 * fro2[0];
  cplx f[2 * JB][EPT];
#pragma unroll
  for (int j = 0; j < 2 * JB; ++j)
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int i = threadIdx.x + e * NT;
      f[j][e] = (col[j] >= 0 && i < m) ? X[(int64_t)col[j] * m + i] : cmk(0.0, 0.0);
    }
  int buf = 0, cnt = 0;
  // One step: the JB disjoint pairs (a[k], b[k]).
  jac_steps(rr, [&](int st, const int (&a)[JB], const int (&b)[JB]) {
    double s[NS];
#pragma unroll
    for (int k = 0; k < JB; ++k) {
      double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const cplx x = f[a[k]][e], y = f[b[k]][e];
        al += cabs2(x);
        be += cabs2(y);
        gr = fma(x.x, y.x, fma(x.y, y.y, gr));
        gi = fma(x.x, y.y, fma(-x.y, y.x, gi));
      }
      s[4 * k] = al;
      s[4 * k + 1] = be;
      s[4 * k + 2] = gr;
      s[4 * k + 3] = gi;
    }
    lane_reduce_scatter<NS>(s, lane);  // lanes LPV c .. LPV c + LPV - 1: the wave's sum c
    if ((lane & (LPV - 1)) == 0) sred[buf][lane / LPV][wv] = s[0];
    __syncthreads();
    double q4[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double u = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) u += sred[buf][4 * (lane & (JB - 1)) + c][w];
      q4[c] = u;
    }
    buf ^= 1;
    // the rotation of the rounds above, with the same correctly rounded square
    // roots and quotients (an rsqrt form of it, a few ulp less orthogonal, took
    // 11 sweeps instead of 8 on a 512-cell far-field matrix)
    double cs = 1.0, snr = 0.0, sni = 0.0;
    const double g = sqrt(q4[2] * q4[2] + q4[3] * q4[3]);
    const bool rot = (g > tol * sqrt(q4[0] * q4[1])) && (g > eps_f);
    if (rot) {
      const double zeta = (q4[1] - q4[0]) / (2.0 * g);
      const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      cs = 1.0 / sqrt(1.0 + tt * tt);
      snr = tt * cs * q4[2] / g;
      sni = tt * cs * q4[3] / g;
    }
    if (threadIdx.x < JB) {  // the record for V (vector stores, lanes 0..3)
      double* q = jac_rec(rec, rr, nwg, wg, st, threadIdx.x);
      q[0] = cs;
      q[1] = snr;
      q[2] = sni;
      q[3] = rot ? 1.0 : 0.0;
    }
#pragma unroll
    for (int k = 0; k < JB; ++k) {
      if (!__builtin_amdgcn_readlane((int)rot, k)) continue;
      const double c = wave_bcast(cs, k);
      const cplx sn = cmk(wave_bcast(snr, k), wave_bcast(sni, k));
      const cplx sc = cconj(sn);
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const cplx x = f[a[k]][e], y = f[b[k]][e];
        f[a[k]][e] = csub(cscale(x, c), cmul(sc, y));
        f[b[k]][e] = cadd(cmul(sn, x), cscale(y, c));
      }
      ++cnt;
      touched |= (1u << a[k]) | (1u << b[k]);
    }
  });
#pragma unroll
  for (int j = 0; j < 2 * JB; ++j) {
    if (!((touched >> j) & 1u) || col[j] < 0) continue;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      const int i = threadIdx.x + e * NT;
      if (i < m) X[(int64_t)col[j] * m + i] = f[j][e];
    }
  }
  if (threadIdx.x == 0 && cnt > 0) atomicAdd(n_rot, cnt);
}

// Vt = I.
__global__ void k_eye(int n, cplx* __restrict__ Vt) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n * n) return;
  Vt[g] = cmk((g / n) == (g % n) ? 1.0 : 0.0, 0.0);
}

// Squared norm of every row of X, one workgroup per row.
__global__ __launch_bounds__(JAC_THREADS) void k_row_norms(int m, const cplx* __restrict__ X,
                                                           double* __restrict__ out) {
  __shared__ double sred[4 * (JAC_THREADS / 64)];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const cplx* x = X + (int64_t)blockIdx.x * m;
  for (int i = threadIdx.x; i < m; i += JAC_THREADS) v[0] += cabs2(x[i]);
  block_sum4(v, sred);
  if (threadIdx.x == 0) out[blockIdx.x] = v[0];
}

// out[0] = sum of in[0..n) (one workgroup, fixed order).
__global__ __launch_bounds__(JAC_THREADS) void k_sum(int n, const double* __restrict__ in,
                                                     double* __restrict__ out) {
  __shared__ double sred[4 * (JAC_THREADS / 64)];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < n; i += JAC_THREADS) v[0] += in[i];
  block_sum4(v, sred);
  if (threadIdx.x == 0) out[0] = v[0];
}

// Eigenvalues in decreasing order (ties by index) and the matching rows of Vt:
// one workgroup per eigenpair computes its rank and copies its row.
__global__ __launch_bounds__(JAC_THREADS) void k_rank_sort(int n, const double* __restrict__ wr,
                                                           const cplx* __restrict__ Vt,
                                                           double* __restrict__ w,
                                                           cplx* __restrict__ evec) {
  __shared__ int cnt[JAC_THREADS / 64];
  const int j = blockIdx.x;
  const double wj = wr[j];
  int c = 0;
  for (int i = threadIdx.x; i < n; i += JAC_THREADS) c += (wr[i] > wj || (wr[i] == wj && i < j));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = c;
  __syncthreads();
  int rank = 0;
  for (int k = 0; k < JAC_THREADS / 64; ++k) rank += cnt[k];
  if (threadIdx.x == 0) w[rank] = wj;
  for (int i = threadIdx.x; i < n; i += JAC_THREADS) evec[(int64_t)rank * n + i] = Vt[(int64_t)j * n + i];
}

// ------------------------------------------------------------------ Herglotz waves
// u[t][x] = sum_j h f[t][j] exp(i k (x_1 cos alpha_j + x_2 sin alpha_j)), one
// thread per point, up to HG_F parameter vectors per pass sharing each
// exponential; (cos, sin) of the angles staged in LDS in blocks.
constexpr int HG_THREADS = 256;
constexpr int HG_F = 4;
constexpr int HG_ANG = 512;

__global__ __launch_bounds__(HG_THREADS) void k_herglotz(int n_alpha, const double* __restrict__ alpha,
                                                         int n_f, const cplx* __restrict__ f, double k,
                                                         double h, int n_pts,
                                                         const double* __restrict__ pts,
                                                         cplx* __restrict__ u) {
  __shared__ double cs[HG_ANG], sn[HG_ANG];
  const int P = blockIdx.x * HG_THREADS + threadIdx.x;
  const int t0 = blockIdx.y * HG_F;
  const int nf = min(HG_F, n_f - t0);
  const double x1 = P < n_pts ? pts[2 * P] : 0.0, x2 = P < n_pts ? pts[2 * P + 1] : 0.0;
  cplx acc[HG_F];
#pragma unroll
  for (int t = 0; t < HG_F; ++t) acc[t] = cmk(0.0, 0.0);
  for (int j0 = 0; j0 < n_alpha; j0 += HG_ANG) {
    const int nj = min(HG_ANG, n_alpha - j0);
    __syncthreads();
    for (int j = threadIdx.x; j < nj; j += HG_THREADS) sincos(alpha[j0 + j], &sn[j], &cs[j]);
    __syncthreads();
    for (int j = 0; j < nj; ++j) {
      const cplx e = cexpi(k * (x1 * cs[j] + x2 * sn[j]));
#pragma unroll
      for (int t = 0; t < HG_F; ++t)
        if (t < nf) cmac(acc[t], f[(int64_t)(t0 + t) * n_alpha + j0 + j], e);
    }
  }
  if (P < n_pts) {
#pragma unroll
    for (int t = 0; t < HG_F; ++t)
      if (t < nf) u[(int64_t)(t0 + t) * n_pts + P] = cscale(acc[t], h);
  }
}

}  // namespace

extern "C" int mudiff_tro(int n, int m, const void* X, void* T, void* stream) {
  if (n < 1 || m < 1) return fail(MUDIFF_ERR_INVALID, "n, m must be >= 1");
  if (!X || !T) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  const unsigned g = (unsigned)((n + 15) / 16);
  hipLaunchKernelGGL(k_tro, dim3(g, g), dim3(64), 0, (hipStream_t)stream, n, m, (const cplx*)X,
                     (cplx*)T);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}

// Rotation records of the block rounds: two rounds of nb'/2 workgroups.
static size_t jac_rec_bytes(int n) {
  const int nb = (n + JB - 1) / JB, nbp = nb + (nb & 1);
  return align256((size_t)2 * (nbp / 2) * JSTEPS * JB * 4 * sizeof(double));
}

extern "C" size_t mudiff_tro_eigh_workspace_size(int n, int m) {
  if (n < 1 || m < 1) return 0;
  return align256((size_t)n * n * 16) + align256((size_t)n * 8) + 256 + 256 + jac_rec_bytes(n);
}

extern "C" int mudiff_tro_eigh(int n, int m, void* X, double* w, void* evec, int max_sweeps,
                               double tol, void* workspace, size_t ws_bytes, int32_t* sweeps,
                               void* stream) {
  if (n < 1 || m < 1) return fail(MUDIFF_ERR_INVALID, "n, m must be >= 1");
  if (!X || !w || !evec || !workspace || !sweeps) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  if (max_sweeps < 1) return fail(MUDIFF_ERR_INVALID, "max_sweeps < 1");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(MUDIFF_ERR_INVALID, "tol must be > 0");
  const size_t need = mudiff_tro_eigh_workspace_size(n, m);
  if (ws_bytes < need) return fail(MUDIFF_ERR_NOMEM, "tro_eigh workspace needs " + std::to_string(need) + " bytes");
  if (((uintptr_t)workspace) & 255) return fail(MUDIFF_ERR_INVALID, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  char* wsp = (char*)workspace;
  cplx* Vt = (cplx*)wsp;
  double* wr = (double*)(wsp + align256((size_t)n * n * 16));
  double* fro2 = (double*)(wsp + align256((size_t)n * n * 16) + align256((size_t)n * 8));
  int32_t* n_rot = (int32_t*)((char*)fro2 + 256);
  double* rec = (double*)((char*)n_rot + 256);
  cplx* Xc = (cplx*)X;
  const int np = n + (n & 1);
  hipLaunchKernelGGL(k_eye, dim3((unsigned)(((int64_t)n * n + 255) / 256)), dim3(256), 0, s, n, Vt);
  hipLaunchKernelGGL(k_row_norms, dim3((unsigned)n), dim3(JAC_THREADS), 0, s, m, (const cplx*)Xc, wr);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(JAC_THREADS), 0, s, n, (const double*)wr, fro2);
  HIP_TRY(hipGetLastError());
  int used = -1;
  for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
    int rc = launch_fill_zero(n_rot, 4, s);
    if (rc != MUDIFF_OK) return rc;
    const int len = std::max(n, m);
    // rows of at most 1024 entries: blocks of JB columns; launch r takes round r
    // on F and round r - 1 on V, a last launch round nb' - 2 on V
    const int nb = (n + JB - 1) / JB, nbp = nb + (nb & 1), nwg = nbp / 2;
    for (int r = 0; len <= 1024 && r <= nbp - 1; ++r) {
      const int rf = r < nbp - 1 ? r : -1, rv = r - 1;
      const dim3 g((unsigned)((rf >= 0 ? nwg : 0) + (rv >= 0 ? nwg : 0)));
      if (len <= 256)
        hipLaunchKernelGGL((k_jacobi_block_round<1, 256>), g, dim3(256), 0, s, n, m, nbp, rf, rv, Xc, Vt, tol, (const double*)fro2, rec, n_rot);
      else if (len <= 512)
        hipLaunchKernelGGL((k_jacobi_block_round<2, 256>), g, dim3(256), 0, s, n, m, nbp, rf, rv, Xc, Vt, tol, (const double*)fro2, rec, n_rot);
      else
        hipLaunchKernelGGL((k_jacobi_block_round<2, 512>), g, dim3(512), 0, s, n, m, nbp, rf, rv, Xc, Vt, tol, (const double*)fro2, rec, n_rot);
    }
    for (int r = 0; len > 1024 && r < np - 1; ++r) {
      const dim3 g((unsigned)(np / 2)), b(JAC_THREADS);
      if (len <= 8 * JAC_THREADS)
        hipLaunchKernelGGL(k_jacobi_round<8>, g, b, 0, s, n, m, np, r, Xc, Vt, tol, (const double*)fro2, n_rot);
      else
        hipLaunchKernelGGL(k_jacobi_round<0>, g, b, 0, s, n, m, np, r, Xc, Vt, tol, (const double*)fro2, n_rot);
    }
    HIP_TRY(hipGetLastError());
    int32_t h_rot = 0;
    HIP_TRY(hipMemcpyAsync(&h_rot, n_rot, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (h_rot == 0) {
      used = sweep;
      break;
    }
  }
  hipLaunchKernelGGL(k_row_norms, dim3((unsigned)n), dim3(JAC_THREADS), 0, s, m, (const cplx*)Xc, wr);
  hipLaunchKernelGGL(k_rank_sort, dim3((unsigned)n), dim3(JAC_THREADS), 0, s, n, (const double*)wr,
                     (const cplx*)Vt, w, (cplx*)evec);
  HIP_TRY(hipGetLastError());
  *sweeps = used;
  return MUDIFF_OK;
}

extern "C" int mudiff_herglotz(int n_alpha, const double* alpha, int n_f, const void* f, double k,
                               double h, int n_pts, const double* pts, void* u, void* stream) {
  if (n_alpha < 1 || n_f < 1 || n_pts < 0) return fail(MUDIFF_ERR_INVALID, "bad sizes");
  if (!(k > 0.0) || !std::isfinite(k) || !std::isfinite(h)) return fail(MUDIFF_ERR_INVALID, "k must be > 0, h finite");
  if (!alpha || !f || (n_pts > 0 && (!pts || !u))) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  if (n_pts == 0) return MUDIFF_OK;
  dim3 grid((unsigned)((n_pts + HG_THREADS - 1) / HG_THREADS), (unsigned)((n_f + HG_F - 1) / HG_F));
  hipLaunchKernelGGL(k_herglotz, grid, dim3(HG_THREADS), 0, (hipStream_t)stream, n_alpha, alpha, n_f,
                     (const cplx*)f, k, h, n_pts, pts, (cplx*)u);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}
