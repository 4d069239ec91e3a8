// Circulant-embedded form of the well-separated off-diagonal blocks (paper
// sec. 5: the block-Toeplitz matrix-vector products are done with FFTs).
//
// A block (p, q) acts as w_m = sum_n t^{pq}_{n-m} z_n (m = -N_p..N_p,
// n = -N_q..N_q).  Embedded in a circulant of length L >= n_p + n_q - 1 it is
// diagonalised by the discrete Fourier transform.  With one length L_b for
// every pair of an instance and indices k = n + N_q, j = m + N_p:
//   Z_f = sum_k w^{-f k} z_k,   w = e^{2 pi i / L_b},
//   T_f[p][q] = (1/L_b) sum_s t^{pq}_s w^{f (s + N_q - N_p)},
//   w^p_j = sum_f w^{f j} sum_q T_f[p][q] Z^q_f.
// The middle step is, for each frequency f, one dense complex product of the
// M_b x M_b matrix T_f with the M_b x R panel of transformed inputs: it runs
// on the FP64 matrix cores (k_circ_gemm), the transforms of the inputs and
// outputs are small dense sums (k_circ_fwd on the vector units, and the
// output pass k_circ_finish_mfma on the matrix cores).  T_f is zero on the diagonal and for close pairs (k b_pq < N_p + N_q):
// their symbols grow by orders of magnitude with the order, and a transform
// would spread that rounding over every mode, so they stay in the direct form.
#include "common.h"

// Instances whose length L_b is 2^a 3^b take mixed radix-2/3 fast transforms
// (k_circ_fwd_fft, k_circ_finish_fft) instead of the direct sums; the tables
// pick such a length where it costs little (see circ_len).
#define CF_LMAX 128
__host__ __device__ __forceinline__ bool circ_fft_len(int L) {
  if (L < 2 || L > CF_LMAX) return false;
  while (L % 3 == 0) L /= 3;
  return (L & (L - 1)) == 0;
}

// Twiddles w^j = e^{2 pi i j / L_b}, j < L_b, of every instance.
__global__ void k_circ_twiddles(DevView v, cplx* tw) {
  const int b = blockIdx.y;
  const int Lb = v.cL[b];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Lb) return;
  double s, c;
  sincospi(2.0 * (double)j / (double)Lb, &s, &c);
  tw[v.cWo[b] + j] = cmk(c, s);
}

// T_f[p][q] for one row disk p and 16 column disks, every f: the symbol rows
// (sign of the reverse pair applied, zero for close pairs and p = q) are
// staged in LDS, thread (q, f-lane) sums its row against the twiddles.
#define CS_Q 16
__global__ __launch_bounds__(256) void k_circ_symbols(DevView v, const uint8_t* __restrict__ nearf,
                                                      cplx* __restrict__ cT, int ts) {
  extern __shared__ cplx lds[];
  cplx* rows = lds;                   // [CS_Q][ts]
  cplx* tw = lds + CS_Q * ts;         // [L_b]
  const int p = blockIdx.x, tid = threadIdx.x;
  const int b = v.inst[p];
  const int Lb = v.cL[b];
  if (Lb == 0) return;
  const int64_t d0 = v.idisk[b], Mb = v.idisk[b + 1] - d0;
  const int64_t q0 = (int64_t)blockIdx.y * CS_Q;
  if (q0 >= Mb) return;
  const int Np = v.N[p];
  for (int e = tid; e < CS_Q * ts; e += 256) {
    const int kq = e / ts, u = e - (e / ts) * ts;
    const int64_t ql = q0 + kq;
    cplx val = cmk(0.0, 0.0);
    if (ql < Mb) {
      const int q = (int)(d0 + ql);
      if (q != p) {
        const int64_t g = pair_index(v.idisk, v.ipair, b, p, q);
        const int S = Np + v.N[q];
        if (!nearf[g] && u <= 2 * S) {
          val = v.t[v.toff[g] + u];                                   // s = u - S
          if (p > q && ((u - S) & 1)) val = cmk(-val.x, -val.y);       // t^{pq}_s = (-1)^s t^{qp}_s
        }
      }
    }
    rows[e] = val;
  }
  for (int e = tid; e < Lb; e += 256) tw[e] = v.ctw[v.cWo[b] + e];
  __syncthreads();
  const int kq = tid & (CS_Q - 1);
  const int64_t ql = q0 + kq;
  if (ql >= Mb) return;
  const int q = (int)(d0 + ql);
  const int S = Np + v.N[q];
  const int sh = v.N[q] - Np;
  const double inv = 1.0 / (double)Lb;
  cplx* out = cT + v.cTo[b] + (int64_t)(p - d0) * Mb + ql;
  const cplx* row = rows + kq * ts;
  for (int f = tid / CS_Q; f < Lb; f += 256 / CS_Q) {
    cplx acc = cmk(0.0, 0.0);
    int idx = (int)(((int64_t)f * (sh - S)) % Lb);  // f (s + N_q - N_p) mod L_b at s = -S
    if (idx < 0) idx += Lb;
    for (int u = 0; u <= 2 * S; ++u) {
      cmac(acc, row[u], tw[idx]);
      idx += f;
      if (idx >= Lb) idx -= Lb;
    }
    out[(int64_t)f * Mb * Mb] = cscale(acc, inv);
  }
}

// Transformed inputs Z_f[q][r] = sum_k w^{-f k} z^q_k for one column disk q and
// 32 right-hand sides: the panel z (already scaled by its column factor) is
// staged in LDS as [k][r], thread (f-lane, r) runs over the frequencies.
#define CF_R 32
__global__ __launch_bounds__(256) void k_circ_fwd(DevView v, int R, const cplx* __restrict__ z,
                                                  cplx* __restrict__ zh,
                                                  const int32_t* __restrict__ con,
                                                  const int32_t* __restrict__ active) {
  __shared__ cplx zs[64 * CF_R];
  __shared__ cplx tw[128];
  const int q = blockIdx.x, tid = threadIdx.x;
  const int b = v.inst[q];
  if (!con[b] || circ_fft_len(v.cL[b])) return;  // 2^a 3^b: k_circ_fwd_fft
  // columns per workgroup: 32, or 16 / 8 for fewer right-hand sides (the
  // frequencies then spread over more threads)
  const int cw = R >= CF_R ? CF_R : (R > 8 ? 16 : 8);
  const int r0 = blockIdx.y * cw;
  if (r0 >= R) return;
  if (active) {
    bool any = false;
    for (int r = r0; r < min(R, r0 + cw); ++r) any |= active[b * R + r] != 0;
    if (!any) return;
  }
  const int Lb = v.cL[b];
  const int nq = 2 * v.N[q] + 1;
  const int64_t d0 = v.idisk[b], Mb = v.idisk[b + 1] - d0;
  const int64_t mq = v.moff[q];
  for (int e = tid; e < cw * nq; e += 256) {
    const int r = e / nq, k = e - (e / nq) * nq;
    cplx val = cmk(0.0, 0.0);
    if (r0 + r < R) val = z[col_base(v.imode, b, R, r0 + r) + mq + k];
    zs[k * cw + r] = val;
  }
  for (int e = tid; e < Lb; e += 256) tw[e] = v.ctw[v.cWo[b] + e];
  __syncthreads();
  const int r = tid % cw;
  if (r0 + r >= R) return;
  cplx* out = zh + (int64_t)R * v.cZo[b] + (q - d0) * R + r0 + r;
  for (int f = tid / cw; f < Lb; f += 256 / cw) {
    cplx acc = cmk(0.0, 0.0);
    int idx = 0;
    for (int k = 0; k < nq; ++k) {
      cmacc(acc, tw[idx], zs[k * cw + r]);  // conj(w^{f k}) z_k
      idx += f;
      if (idx >= Lb) idx -= Lb;
    }
    out[(int64_t)f * Mb * R] = acc;
  }
}

// Lengths L_b = 3^P take radix-3 fast transforms instead of the direct sums
// (Stockham order, so no digit reversal): stage s splits each sub-transform of
// length n = L / 3^s into three of length n / 3 with the butterfly
//   y_{3j}   = a + b + c,
//   y_{3j+1} = (a + b zeta + c conj(zeta)) w^j,
//   y_{3j+2} = (a + b conj(zeta) + c zeta) w^{2j},
// a, b, c the entries j, j + n/3, j + 2n/3 of the sub-transform, w = e^{-+2 pi i / n}
// and zeta = e^{-+2 pi i / 3} (sign - forward, + inverse), all read from the
// instance's twiddle table.  The columns of a workgroup run side by side in LDS.

// In-place (ping-pong) transform of the L x CR block x[k][c] in LDS; returns
// the buffer holding the result in natural order.  Stockham stages: radix 3
// while 3 divides the remaining length, then radix 4, then at most one radix
// 2; a stage of radix p maps x[(j + s m) stride + k], s < p, to
// y[(p j + r) stride + k] (the p-point DFT times the twiddle w^{r j stride}),
// m = n / p, then stride *= p.
template <int CR>
__device__ cplx* fft3_only_lds(cplx* x, cplx* y, const cplx* tw, int L, bool inverse) {
  const int tid = threadIdx.x;
  const cplx zt = tw[L / 3];
  const double sgn = inverse ? zt.y : -zt.y;  // Im(zeta)
  int stride = 1;
  for (int n = L; n > 1; n /= 3) {
    const int m = n / 3;
    for (int e = tid; e < m * stride * CR; e += blockDim.x) {
      const int c = e % CR, t = e / CR;
      const int k = t % stride, j = t / stride;
      const cplx a = x[((j)*stride + k) * CR + c];
      const cplx bb = x[((j + m) * stride + k) * CR + c];
      const cplx cc = x[((j + 2 * m) * stride + k) * CR + c];
      const cplx sm = cadd(bb, cc), df = csub(bb, cc);
      const cplx tt = csub(a, cscale(sm, 0.5));
      const cplx id = cmk(-sgn * df.y, sgn * df.x);  // i Im(zeta) (b - c)
      cplx w1 = tw[j * stride], w2 = tw[2 * j * stride];
      if (!inverse) {
        w1 = cconj(w1);
        w2 = cconj(w2);
      }
      y[((3 * j) * stride + k) * CR + c] = cadd(a, sm);
      y[((3 * j + 1) * stride + k) * CR + c] = cmul(cadd(tt, id), w1);
      y[((3 * j + 2) * stride + k) * CR + c] = cmul(csub(tt, id), w2);
    }
    __syncthreads();
    cplx* sw = x;
    x = y;
    y = sw;
    stride *= 3;
  }
  return x;
}

template <int CR>
__device__ cplx* fft23_lds(cplx* x, cplx* y, const cplx* tw, int L, bool inverse) {
  int p3 = L;
  while (p3 % 3 == 0) p3 /= 3;
  if (p3 == 1) return fft3_only_lds<CR>(x, y, tw, L, inverse);  // powers of 3: one stage kind
  const int tid = threadIdx.x;
  int stride = 1;
  for (int n = L; n > 1;) {
    if (n % 3 == 0) {
      const cplx zt = tw[L / 3];
      const double sgn = inverse ? zt.y : -zt.y;  // Im(zeta)
      const int m = n / 3;
      for (int e = tid; e < m * stride * CR; e += blockDim.x) {
        const int c = e % CR, t = e / CR;
        const int k = t % stride, j = t / stride;
        const cplx a = x[((j)*stride + k) * CR + c];
        const cplx bb = x[((j + m) * stride + k) * CR + c];
        const cplx cc = x[((j + 2 * m) * stride + k) * CR + c];
        const cplx sm = cadd(bb, cc), df = csub(bb, cc);
        const cplx tt = csub(a, cscale(sm, 0.5));
        const cplx id = cmk(-sgn * df.y, sgn * df.x);  // i Im(zeta) (b - c)
        cplx w1 = tw[j * stride], w2 = tw[2 * j * stride];
        if (!inverse) {
          w1 = cconj(w1);
          w2 = cconj(w2);
        }
        y[((3 * j) * stride + k) * CR + c] = cadd(a, sm);
        y[((3 * j + 1) * stride + k) * CR + c] = cmul(cadd(tt, id), w1);
        y[((3 * j + 2) * stride + k) * CR + c] = cmul(csub(tt, id), w2);
      }
      n = m;
      stride *= 3;
    } else if (n % 4 == 0) {
      const int m = n / 4;
      for (int e = tid; e < m * stride * CR; e += blockDim.x) {
        const int c = e % CR, t = e / CR;
        const int k = t % stride, j = t / stride;
        const cplx a0 = x[((j)*stride + k) * CR + c];
        const cplx a1 = x[((j + m) * stride + k) * CR + c];
        const cplx a2 = x[((j + 2 * m) * stride + k) * CR + c];
        const cplx a3 = x[((j + 3 * m) * stride + k) * CR + c];
        const cplx t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), d = csub(a1, a3);
        const cplx t3 = inverse ? cmk(-d.y, d.x) : cmk(d.y, -d.x);  // zeta (a1 - a3), zeta = -+i
        cplx w1 = tw[j * stride], w2 = tw[2 * j * stride], w3 = tw[3 * j * stride];
        if (!inverse) {
          w1 = cconj(w1);
          w2 = cconj(w2);
          w3 = cconj(w3);
        }
        y[((4 * j) * stride + k) * CR + c] = cadd(t0, t2);
        y[((4 * j + 1) * stride + k) * CR + c] = cmul(cadd(t1, t3), w1);
        y[((4 * j + 2) * stride + k) * CR + c] = cmul(csub(t0, t2), w2);
        y[((4 * j + 3) * stride + k) * CR + c] = cmul(csub(t1, t3), w3);
      }
      n = m;
      stride *= 4;
    } else {
      const int m = n / 2;
      for (int e = tid; e < m * stride * CR; e += blockDim.x) {
        const int c = e % CR, t = e / CR;
        const int k = t % stride, j = t / stride;
        const cplx a = x[((j)*stride + k) * CR + c];
        const cplx bb = x[((j + m) * stride + k) * CR + c];
        cplx w = tw[j * stride];
        if (!inverse) w = cconj(w);
        y[((2 * j) * stride + k) * CR + c] = cadd(a, bb);
        y[((2 * j + 1) * stride + k) * CR + c] = cmul(csub(a, bb), w);
      }
      n = m;
      stride *= 2;
    }
    __syncthreads();
    cplx* sw = x;
    x = y;
    y = sw;
  }
  return x;
}

// Forward transforms of the scaled input panels of one column disk q and CR
// right-hand sides, for instances with L_b = 2^a 3^b <= LM.
template <int CR, int LM>
__global__ __launch_bounds__(256) void k_circ_fwd_fft(DevView v, int R, const cplx* __restrict__ z,
                                                      cplx* __restrict__ zh,
                                                      const int32_t* __restrict__ con,
                                                      const int32_t* __restrict__ active) {
  __shared__ cplx buf[2 * LM * CR];
  __shared__ cplx tw[LM];
  const int q = blockIdx.x, tid = threadIdx.x;
  const int b = v.inst[q];
  if (!con[b]) return;
  const int Lb = v.cL[b];
  if (!circ_fft_len(Lb) || Lb > LM || Lb <= (LM > 81 ? 81 : 0)) return;  // this launch's length class
  const int r0 = blockIdx.y * CR;
  if (r0 >= R) return;
  if (active) {
    bool any = false;
    for (int r = r0; r < min(R, r0 + CR); ++r) any |= active[b * R + r] != 0;
    if (!any) return;
  }
  const int nq = 2 * v.N[q] + 1;
  const int64_t d0 = v.idisk[b], Mb = v.idisk[b + 1] - d0;
  for (int e = tid; e < Lb * CR; e += 256) {  // along the modes of a column: coalesced
    const int c = e / Lb, k = e - (e / Lb) * Lb;
    cplx val = cmk(0.0, 0.0);
    if (k < nq && r0 + c < R) val = z[col_base(v.imode, b, R, r0 + c) + v.moff[q] + k];
    buf[k * CR + c] = val;
  }
  for (int e = tid; e < Lb; e += 256) tw[e] = v.ctw[v.cWo[b] + e];
  __syncthreads();
  const cplx* res = fft23_lds<CR>(buf, buf + LM * CR, tw, Lb, false);
  cplx* out = zh + (int64_t)R * v.cZo[b] + (q - d0) * R + r0;
  for (int e = tid; e < Lb * CR; e += 256) {
    const int f = e / CR, c = e - (e / CR) * CR;
    if (r0 + c < R) out[(int64_t)f * Mb * R + c] = res[e];
  }
}

// W_f = T_f Z_f for every frequency of the instances using the form: a dense
// complex product per (instance, frequency) on v_mfma_f64_16x16x4f64.  Work
// item: (instance, frequency, row tile, column tile).  Workgroup: 4 waves as
// WR x WC, each wave WM x WN tiles of 16 rows x 8 complex columns; a complex
// product is two real MFMAs against [Re Z | Im Z] (lane l holds A[l % 16][l / 16],
// B[l / 16][l % 16], D[4 v + l / 16][l % 16]).  K steps of BK column disks are
// staged in LDS, the next one loaded into registers while the current one is
// on the matrix cores; with DB the step goes to a second LDS buffer, so that
// one barrier per step separates the buffers.  Consecutive items (the tiles of
// one frequency) are placed on one XCD, whose L2 then serves the rows of T_f
// and the panel Z_f to all of them.
typedef double cg_d4 __attribute__((ext_vector_type(4)));

// PF2: two register sets for the staged K steps, so that step kc + 2 is
// loaded while step kc is on the matrix cores (two steps of latency hiding).
// G3: Gauss's three-product form of the complex product.  A wave tile is then
// 16 rows x 16 complex columns, and per k-step of 4 it issues three real MFMAs
// instead of four:
//   P1 = Re T Re Z,  P2 = Im T Im Z,  P3 = (Re T + Im T)(Re Z + Im Z),
//   Re W = P1 - P2,  Im W = P3 - P1 - P2,
// with B[k][j] the j-th complex column itself (no [Re | Im] split), so every
// lane holds whole output elements and the epilogue needs no lane exchange.
// The rounding error of Im W is bounded by a small multiple of eps times
// sum |T| |Z| over the contraction (N. J. Higham, "Stability of a method for
// multiplying complex matrices with three real matrix multiplications", SIAM
// J. Matrix Anal. Appl. 13, 1992): normwise as accurate as the four-product form.
template <int WR, int WC, int WM, int WN, int BK, bool DB, bool PF2, bool G3 = false>
__global__ __launch_bounds__(WR * WC * 64) void k_circ_gemm(DevView v, int R, const cplx* __restrict__ zh,
                                                   cplx* __restrict__ wh,
                                                   const int32_t* __restrict__ items, int n_items,
                                                   const int32_t* __restrict__ active) {
  constexpr int NT = WR * WC * 64;
  constexpr int CW = G3 ? 16 : 8;  // complex columns of a wave's MFMA tile
  constexpr int BM = WR * 16 * WM, BN = WC * CW * WN;
  constexpr int AS = BK + 1, BS = BN + 1;  // LDS row strides (complex)
  constexpr int NA = BM * BK / NT, NB = (BK * BN + NT - 1) / NT;
  constexpr int ASZ = BM * AS, BSZ = BK * BS;
  static_assert(!PF2 || DB, "two register sets need two LDS buffers");
  __shared__ cplx As[(DB ? 2 : 1) * ASZ];
  __shared__ cplx Bs[(DB ? 2 : 1) * BSZ];
  const int i = blockIdx.x;
  const int xc = i & 7, slot = i >> 3;
  const int it = xc * (n_items >> 3) + min(xc, n_items & 7) + slot;
  const int32_t* rec = items + 4 * (int64_t)it;
  const int b = rec[0], f = rec[1];
  const int64_t row0 = (int64_t)rec[2] * BM;
  const int col0 = rec[3] * BN;
  if (active) {
    bool any = false;
    for (int c = col0; c < min(R, col0 + BN); ++c) any |= active[b * R + c] != 0;
    if (!any) return;
  }
  const int64_t Mb = v.idisk[b + 1] - v.idisk[b];
  const cplx* __restrict__ A = v.cT + v.cTo[b] + (int64_t)f * Mb * Mb;
  const int64_t zo = (int64_t)R * v.cZo[b] + (int64_t)f * Mb * R;
  const cplx* __restrict__ Bm = zh + zo;
  cplx* __restrict__ C = wh + zo;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int j = lane & 15, kq = lane >> 4;
  const int wr = wave / WC, wc = wave - (wave / WC) * WC;
  cplx ra[2][NA], rb[2][NB];
  auto load = [&](int64_t k0, cplx (&xa)[NA], cplx (&xb)[NB]) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + u * NT;
      const int r = e / BK, c = e - (e / BK) * BK;
      const int64_t gr = row0 + r, gc = k0 + c;
      xa[u] = (gr < Mb && gc < Mb) ? A[gr * Mb + gc] : cmk(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + u * NT;
      const int r = e / BN, c = e - (e / BN) * BN;
      const int64_t gr = k0 + r;
      const int gc = col0 + c;
      xb[u] = (e < BK * BN && gr < Mb && gc < R) ? Bm[gr * R + gc] : cmk(0.0, 0.0);
    }
  };
  auto store = [&](int buf, const cplx (&xa)[NA], const cplx (&xb)[NB]) {
    cplx* as = As + buf * ASZ;
    cplx* bs = Bs + buf * BSZ;
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + u * NT;
      as[(e / BK) * AS + (e % BK)] = xa[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + u * NT;
      if (e < BK * BN) bs[(e / BN) * BS + (e % BN)] = xb[u];
    }
  };
  // four-product form: acc1 = Re T [Re Z | Im Z], acc2 = Im T [Re Z | Im Z];
  // G3: acc1 = P1, acc2 = P2, acc3 = P3
  cg_d4 acc1[WM][WN], acc2[WM][WN], acc3[G3 ? WM : 1][G3 ? WN : 1];
#pragma unroll
  for (int mt = 0; mt < WM; ++mt)
#pragma unroll
    for (int nt = 0; nt < WN; ++nt) {
      acc1[mt][nt] = cg_d4{0.0, 0.0, 0.0, 0.0};
      acc2[mt][nt] = cg_d4{0.0, 0.0, 0.0, 0.0};
      if constexpr (G3) acc3[mt][nt] = cg_d4{0.0, 0.0, 0.0, 0.0};
    }
  auto compute = [&](int buf) {
    const cplx* as = As + buf * ASZ;
    const cplx* bs = Bs + buf * BSZ;
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      cplx a[WM];
#pragma unroll
      for (int mt = 0; mt < WM; ++mt) a[mt] = as[(wr * 16 * WM + 16 * mt + j) * AS + 4 * kk + kq];
      if constexpr (G3) {
        cplx bz[WN];
#pragma unroll
        for (int nt = 0; nt < WN; ++nt) bz[nt] = bs[(4 * kk + kq) * BS + wc * 16 * WN + 16 * nt + j];
#pragma unroll
        for (int mt = 0; mt < WM; ++mt) {
          const double asum = a[mt].x + a[mt].y;
#pragma unroll
          for (int nt = 0; nt < WN; ++nt) {
            const double bsum = bz[nt].x + bz[nt].y;
            acc1[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mt].x, bz[nt].x, acc1[mt][nt], 0, 0, 0);
            acc2[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mt].y, bz[nt].y, acc2[mt][nt], 0, 0, 0);
            acc3[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(asum, bsum, acc3[mt][nt], 0, 0, 0);
          }
        }
      } else {
        double bv[WN];
#pragma unroll
        for (int nt = 0; nt < WN; ++nt) {
          const cplx zz = bs[(4 * kk + kq) * BS + wc * 8 * WN + 8 * nt + (j & 7)];
          bv[nt] = j < 8 ? zz.x : zz.y;
        }
#pragma unroll
        for (int mt = 0; mt < WM; ++mt)
#pragma unroll
          for (int nt = 0; nt < WN; ++nt) {
            acc1[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mt].x, bv[nt], acc1[mt][nt], 0, 0, 0);
            acc2[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[mt].y, bv[nt], acc2[mt][nt], 0, 0, 0);
          }
      }
    }
  };
  const int64_t nk = (Mb + BK - 1) / BK;
  if constexpr (PF2) {
    // register set s holds the steps kc with kc % 2 == s
    load(0, ra[0], rb[0]);
    if (nk > 1) load(BK, ra[1], rb[1]);
    store(0, ra[0], rb[0]);
    __syncthreads();
    for (int64_t kc = 0; kc < nk; kc += 2) {
      // even step kc: buffer 0; set 0 is free for step kc + 2
      if (kc + 2 < nk) load((kc + 2) * BK, ra[0], rb[0]);
      compute(0);
      if (kc + 1 < nk) store(1, ra[1], rb[1]);
      __syncthreads();
      if (kc + 1 >= nk) break;
      // odd step kc + 1: buffer 1; set 1 is free for step kc + 3
      if (kc + 3 < nk) load((kc + 3) * BK, ra[1], rb[1]);
      compute(1);
      if (kc + 2 < nk) store(0, ra[0], rb[0]);
      __syncthreads();
    }
  } else if constexpr (DB) {
    load(0, ra[0], rb[0]);
    store(0, ra[0], rb[0]);
    __syncthreads();
    for (int64_t kc = 0; kc < nk; ++kc) {
      const int cur = (int)(kc & 1);
      if (kc + 1 < nk) load((kc + 1) * BK, ra[0], rb[0]);  // in flight during the MFMAs
      compute(cur);
      if (kc + 1 < nk) store(cur ^ 1, ra[0], rb[0]);       // its readers passed the last barrier
      __syncthreads();
    }
  } else {
    load(0, ra[0], rb[0]);
    for (int64_t kc = 0; kc < nk; ++kc) {
      __syncthreads();  // previous step done with LDS
      store(0, ra[0], rb[0]);
      __syncthreads();
      if (kc + 1 < nk) load((kc + 1) * BK, ra[0], rb[0]);  // in flight during the MFMAs
      compute(0);
    }
  }
#pragma unroll
  for (int mt = 0; mt < WM; ++mt)
#pragma unroll
    for (int nt = 0; nt < WN; ++nt)
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const int64_t row = row0 + wr * 16 * WM + 16 * mt + 4 * vv + kq;
        if constexpr (G3) {
          const double p1 = acc1[mt][nt][vv], p2 = acc2[mt][nt][vv];
          const int col = col0 + wc * 16 * WN + 16 * nt + j;
          if (row < Mb && col < R) C[row * R + col] = cmk(p1 - p2, acc3[mt][nt][vv] - p1 - p2);
        } else {
          const double a1 = acc1[mt][nt][vv], a2 = acc2[mt][nt][vv];
          const double other = __shfl_xor(a2, 8, 64);
          const double val = j < 8 ? a1 - other : a1 + other;  // Re W (j < 8), Im W (j >= 8)
          const double im = __shfl_xor(val, 8, 64);
          const int col = col0 + wc * 8 * WN + 8 * nt + (j & 7);
          if (j < 8 && row < Mb && col < R) C[row * R + col] = cmk(val, im);
        }
      }
}

// The inverse transform as a small dense product on the matrix cores (the
// same complex-as-two-real-MFMAs scheme as k_circ_gemm, lane l holding
// A[l % 16][l / 16], B[l / 16][l % 16], D[4 v + l / 16][l % 16]): per row disk p,
//   w^p [n_p x R] = G [n_p x L] W^p [L x R],  G[j][f] = w^{f j};
// the panel W^p is staged in LDS as [f][32 columns], each wave computing one
// tile of 8 right-hand sides over all rows.  (The forward transform, n_q <= 63
// terms per frequency, runs faster on the vector units: k_circ_fwd.)
typedef double ct_d4 __attribute__((ext_vector_type(4)));
#define CT_R 32       // right-hand sides per workgroup

template <int TF>
__device__ __forceinline__ void ct_product(const cplx* __restrict__ tw, int Lb, int nrow, int nk,
                                           const cplx* __restrict__ panel, int c, int j, int kq,
                                           int t0, int ts, ct_d4 (&acc1)[TF], ct_d4 (&acc2)[TF]) {
  // acc[t] += A[row][k] panel[k][c] for the row tile 16 (t0 + ts t), A[row][k] = w^{row k},
  // rows < nrow, k < nk.  Lane (j, kq) holds A[row][k] for its k = k0 + kq in
  // registers and advances it by the factor w^{4 row} per K step (both read
  // exactly from the twiddle table; a few steps of rounding per entry).
  cplx a[TF], st[TF];
#pragma unroll
  for (int t = 0; t < TF; ++t) {
    const int row = 16 * (t0 + ts * t) + j;
    a[t] = cmk(0.0, 0.0);
    st[t] = cmk(0.0, 0.0);
    if (row < nrow) {
      a[t] = tw[(row * kq) % Lb];
      st[t] = tw[(4 * row) % Lb];
    }
  }
  for (int k0 = 0; k0 < nk; k0 += 4) {
    const int k = k0 + kq;
    const bool in = k < nk;
    const cplx zz = in ? panel[k * CT_R + c] : cmk(0.0, 0.0);
    const double bv = j < 8 ? zz.x : zz.y;
#pragma unroll
    for (int t = 0; t < TF; ++t) {
      if (16 * (t0 + ts * t) >= nrow) continue;  // wave-uniform
      acc1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(in ? a[t].x : 0.0, bv, acc1[t], 0, 0, 0);
      acc2[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(in ? a[t].y : 0.0, bv, acc2[t], 0, 0, 0);
      a[t] = cmul(a[t], st[t]);
    }
  }
}

// Output pass with the inverse transforms on the matrix cores: one workgroup
// per (row disk p, 8 nct right-hand sides, nct = 4 / wpc column tiles).  For an
// instance in the form, the rows f of W^p are staged in LDS, and the wpc waves
// of column tile w / wpc form w^p_j for its 8 right-hand sides, row tiles
// w % wpc, w % wpc + wpc, ..., leaving them in LDS; then, coalesced over the
// modes, the close-pair partial sums are added and the epilogue applied.
// Workgroups whose right-hand sides have all stopped iterating do nothing.
template <int TM>
__global__ __launch_bounds__(256) void k_circ_finish_mfma(
    DevView v, int R, const cplx* __restrict__ x, cplx* __restrict__ y, int op,
    const cplx* __restrict__ part, int64_t blk, int npad, int RC, const int32_t* __restrict__ dgrp,
    const int32_t* __restrict__ drow, const int32_t* __restrict__ gnseg,
    const int64_t* __restrict__ gbase, const int32_t* __restrict__ active,
    const cplx* __restrict__ wh, const int32_t* __restrict__ con, const cplx* __restrict__ shift,
    int wpc) {
  extern __shared__ cplx lds[];
  cplx* tw = lds;                          // [L_b]
  cplx* ws = lds + 128;                    // W^p rows [f][r], then the results [r][j]
  const int p = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int j = lane & 15, kq = lane >> 4;
  const int b = v.inst[p];
  const int ncol = 8 * (4 / wpc);          // right-hand sides of this workgroup
  const int r0 = blockIdx.y * ncol;
  if (r0 >= R) return;
  if (active) {
    bool any = false;
    for (int r = r0; r < min(R, r0 + ncol); ++r) any |= active[b * R + r] != 0;
    if (!any) return;
  }
  const int np = 2 * v.N[p] + 1;
  const int64_t d0 = v.idisk[b], Mb = v.idisk[b + 1] - d0;
  const bool circ = con[b] != 0;
  if (circ && circ_fft_len(v.cL[b])) return;  // k_circ_finish_fft
  const int ldw = np + 1;
  if (circ) {
    const int Lb = v.cL[b];
    const cplx* src = wh + (int64_t)R * v.cZo[b] + (p - d0) * R + r0;
    for (int e = tid; e < Lb * CT_R; e += 256) {
      const int f = e / CT_R, rr = e - (e / CT_R) * CT_R;
      ws[e] = rr < ncol && r0 + rr < R ? src[(int64_t)f * Mb * R + rr] : cmk(0.0, 0.0);
    }
    for (int e = tid; e < Lb; e += 256) tw[e] = v.ctw[v.cWo[b] + e];
    __syncthreads();
    ct_d4 acc1[TM], acc2[TM];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      acc1[t] = ct_d4{0.0, 0.0, 0.0, 0.0};
      acc2[t] = ct_d4{0.0, 0.0, 0.0, 0.0};
    }
    const int ct = wave / wpc, t0 = wave - (wave / wpc) * wpc;
    ct_product<TM>(tw, Lb, np, Lb, ws, 8 * ct + (j & 7), j, kq, t0, wpc, acc1, acc2);
    __syncthreads();  // every wave is done reading W^p: reuse ws for the results
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const double a1 = acc1[t][vv], a2 = acc2[t][vv];
        const double other = __shfl_xor(a2, 8, 64);
        const double val = j < 8 ? a1 - other : a1 + other;
        const double im = __shfl_xor(val, 8, 64);
        const int m = 16 * (t0 + wpc * t) + 4 * vv + kq;
        if (j < 8 && m < np) ws[(8 * ct + (j & 7)) * ldw + m] = cmk(val, im);
      }
    __syncthreads();
  }
  const int gr = dgrp[p];
  const int ns = gnseg[gr];
  const int64_t ip = v.imode[b] + v.moff[p];
  for (int e = tid; e < ncol * np; e += 256) {
    const int rr = e / np, m = e - (e / np) * np;
    const int r = r0 + rr;
    if (r >= R || (active && active[b * R + r] == 0)) continue;
    const int t = r / RC, rc = r - (r / RC) * RC;
    const cplx* pr = part + (gbase[gr] + (int64_t)t * ns) * blk + ((int64_t)drow[p] * npad + m) * RC + rc;
    cplx w = circ ? ws[rr * ldw + m] : cmk(0.0, 0.0);
    for (int sg = 0; sg < ns; ++sg) w = cadd(w, pr[(int64_t)sg * blk]);
    const int64_t g = col_base(v.imode, b, R, r) + v.moff[p] + m;
    cplx o = finalize(v, op, ip + m, x[g], w);
    if (shift) o = affine(shift, b * R + r, o, x[g]);
    y[g] = o;
  }
}

// Output pass for instances in the form with L_b = 2^a 3^b <= LM: inverse
// transform of the rows f of W^p for CR right-hand sides (only the n_p modes
// are kept), then, as in k_circ_finish_mfma, the close pairs' partial sums and
// the epilogue, coalesced over the modes.
template <int CR, int LM>
__global__ __launch_bounds__(256) void k_circ_finish_fft(
    DevView v, int R, const cplx* __restrict__ x, cplx* __restrict__ y, int op,
    const cplx* __restrict__ part, int64_t blk, int npad, int RC, const int32_t* __restrict__ dgrp,
    const int32_t* __restrict__ drow, const int32_t* __restrict__ gnseg,
    const int64_t* __restrict__ gbase, const int32_t* __restrict__ active,
    const cplx* __restrict__ wh, const int32_t* __restrict__ con,
    const cplx* __restrict__ shift) {
  __shared__ cplx buf[2 * LM * CR];
  __shared__ cplx tw[LM];
  const int p = blockIdx.x, tid = threadIdx.x;
  const int b = v.inst[p];
  if (!con[b]) return;
  const int Lb = v.cL[b];
  if (!circ_fft_len(Lb) || Lb > LM || Lb <= (LM > 81 ? 81 : 0)) return;  // this launch's length class
  const int r0 = blockIdx.y * CR;
  if (r0 >= R) return;
  if (active) {
    bool any = false;
    for (int r = r0; r < min(R, r0 + CR); ++r) any |= active[b * R + r] != 0;
    if (!any) return;
  }
  const int np = 2 * v.N[p] + 1;
  const int64_t d0 = v.idisk[b], Mb = v.idisk[b + 1] - d0;
  const cplx* src = wh + (int64_t)R * v.cZo[b] + (p - d0) * R + r0;
  for (int e = tid; e < Lb * CR; e += 256) {
    const int f = e / CR, c = e - (e / CR) * CR;
    buf[e] = r0 + c < R ? src[(int64_t)f * Mb * R + c] : cmk(0.0, 0.0);
  }
  for (int e = tid; e < Lb; e += 256) tw[e] = v.ctw[v.cWo[b] + e];
  __syncthreads();
  const cplx* res = fft23_lds<CR>(buf, buf + LM * CR, tw, Lb, true);
  const int gr = dgrp[p];
  const int ns = gnseg[gr];
  const int64_t ip = v.imode[b] + v.moff[p];
  for (int e = tid; e < CR * np; e += 256) {
    const int rr = e / np, m = e - (e / np) * np;
    const int r = r0 + rr;
    if (r >= R || (active && active[b * R + r] == 0)) continue;
    const int t = r / RC, rc = r - (r / RC) * RC;
    const cplx* pr = part + (gbase[gr] + (int64_t)t * ns) * blk + ((int64_t)drow[p] * npad + m) * RC + rc;
    cplx w = res[m * CR + rr];
    for (int sg = 0; sg < ns; ++sg) w = cadd(w, pr[(int64_t)sg * blk]);
    const int64_t g = col_base(v.imode, b, R, r) + v.moff[p] + m;
    cplx o = finalize(v, op, ip + m, x[g], w);
    if (shift) o = affine(shift, b * R + r, o, x[g]);
    y[g] = o;
  }
}

// Product variants: tile (rows, complex columns), K step, LDS buffers
// (3: two buffers and two register sets), workgroup size, real products per
// complex product (4, or 3 in Gauss's form).
struct CircVariant {
  int bm, bn, bk, db, nt, mult;
  void (*fn)(DevView, int, const cplx*, cplx*, const int32_t*, int, const int32_t*);
};
static const CircVariant kCircVar[] = {
    {64, 64, 16, 1, 256, 4, k_circ_gemm<2, 2, 2, 4, 16, false, false>},
    {64, 64, 16, 2, 256, 4, k_circ_gemm<2, 2, 2, 4, 16, true, false>},
    {64, 32, 16, 2, 256, 4, k_circ_gemm<2, 2, 2, 2, 16, true, false>},
    {64, 32, 32, 2, 256, 4, k_circ_gemm<2, 2, 2, 2, 32, true, false>},
    {128, 32, 16, 2, 256, 4, k_circ_gemm<2, 2, 4, 2, 16, true, false>},
    {128, 16, 16, 2, 256, 4, k_circ_gemm<4, 1, 2, 2, 16, true, false>},
    {128, 8, 16, 2, 256, 4, k_circ_gemm<4, 1, 2, 1, 16, true, false>},
    {64, 8, 16, 2, 256, 4, k_circ_gemm<4, 1, 1, 1, 16, true, false>},
    {64, 32, 16, 3, 256, 4, k_circ_gemm<2, 2, 2, 2, 16, true, true>},
    {128, 32, 16, 2, 512, 4, k_circ_gemm<4, 2, 2, 2, 16, true, false>},
    {128, 32, 16, 3, 512, 4, k_circ_gemm<4, 2, 2, 2, 16, true, true>},
    {128, 16, 16, 3, 256, 4, k_circ_gemm<4, 1, 2, 2, 16, true, true>},
    {128, 32, 8, 3, 512, 4, k_circ_gemm<4, 2, 2, 2, 8, true, true>},
    {128, 32, 8, 2, 512, 4, k_circ_gemm<4, 2, 2, 2, 8, true, false>},
    {64, 32, 8, 3, 256, 4, k_circ_gemm<2, 2, 2, 2, 8, true, true>},
    {128, 64, 8, 3, 512, 4, k_circ_gemm<4, 2, 2, 4, 8, true, true>},
    {128, 64, 16, 3, 512, 4, k_circ_gemm<4, 2, 2, 4, 16, true, true>},
    {128, 32, 4, 2, 512, 4, k_circ_gemm<4, 2, 2, 2, 4, true, false>},
    {128, 32, 8, 2, 1024, 4, k_circ_gemm<8, 2, 1, 2, 8, true, false>},
    {64, 32, 8, 2, 256, 4, k_circ_gemm<2, 2, 2, 2, 8, true, false>},
    {128, 16, 8, 2, 256, 4, k_circ_gemm<4, 1, 2, 2, 8, true, false>},
    {128, 8, 8, 2, 256, 4, k_circ_gemm<4, 1, 2, 1, 8, true, false>},
    {256, 32, 8, 2, 512, 4, k_circ_gemm<4, 2, 4, 2, 8, true, false>},
    // Gauss's three-product form (16-column wave tiles)
    {128, 32, 8, 2, 512, 3, k_circ_gemm<4, 2, 2, 1, 8, true, false, true>},
    {128, 32, 16, 2, 512, 3, k_circ_gemm<4, 2, 2, 1, 16, true, false, true>},
    {128, 32, 8, 3, 512, 3, k_circ_gemm<4, 2, 2, 1, 8, true, true, true>},
    {128, 64, 8, 2, 512, 3, k_circ_gemm<4, 2, 2, 2, 8, true, false, true>},
    {256, 32, 8, 2, 512, 3, k_circ_gemm<4, 2, 4, 1, 8, true, false, true>},
    {64, 32, 8, 2, 256, 3, k_circ_gemm<2, 2, 2, 1, 8, true, false, true>},
    {128, 16, 8, 2, 256, 3, k_circ_gemm<4, 1, 2, 1, 8, true, false, true>},
    {128, 16, 16, 2, 256, 3, k_circ_gemm<4, 1, 2, 1, 16, true, false, true>},
};
#define N_CIRC_VAR ((int)(sizeof(kCircVar) / sizeof(kCircVar[0])))

// Default product variant for R columns, and the variants worth timing.
int circ_variant(int R) { return R >= 48 ? 2 : (R >= 24 ? 2 : (R >= 12 ? 5 : 6)); }
std::vector<int> circ_variants(int R) {
  if (R >= 48) return {2, 8, 9, 10, 12, 13, 14, 15, 16, 17, 18, 19, 22, 23, 24, 25, 26, 27, 28};
  if (R >= 24) return {2, 3, 4, 8, 9, 10, 12, 13, 14, 19, 23, 24, 28};
  if (R >= 12) return {5, 6, 11, 20, 29, 30};
  return {6, 7, 21};
}
void circ_tile(int var, int* bm, int* bn) {
  *bm = kCircVar[var].bm;
  *bn = kCircVar[var].bn;
}
void circ_var_dims(int var, int* bm, int* bn, int* bk, int* db, int* nt, int* mult) {
  *bm = kCircVar[var].bm;
  *bn = kCircVar[var].bn;
  *bk = kCircVar[var].bk;
  *db = kCircVar[var].db;
  *nt = kCircVar[var].nt;
  *mult = kCircVar[var].mult;
}

// Enqueue the transforms of the inputs and the per-frequency products.
// z: inputs scaled by their column factors [B][R][N_b]; zh, wh: [sum_b L_b M_b][R].
// Which transform kernels a launch needs: instances in the form with L_b =
// 2^a 3^b (fast transforms, 8 right-hand sides per workgroup, in two length
// classes with their own LDS size: *fft for L_b <= 81, *fft_wide for longer
// ones) and with other lengths (direct sums).
static void circ_kinds(const mudiff_ctx* h, const int32_t* con_h, bool* fft, bool* dft,
                       bool* fft_wide) {
  *fft = *dft = *fft_wide = false;
  for (int b = 0; b < h->B; ++b) {
    if (!con_h[b]) continue;
    if (!circ_fft_len(h->cL[b])) *dft = true;
    else if (h->cL[b] > 81) *fft_wide = true;
    else *fft = true;
  }
}

int circ_launch(mudiff_ctx* h, int R, const cplx* z, cplx* zh, cplx* wh, const int32_t* citems,
                int n_citems, int var, const int32_t* con, const int32_t* con_h,
                const int32_t* active, hipStream_t s) {
  bool fft, dft, wide;
  circ_kinds(h, con_h, &fft, &dft, &wide);
  const int cw = R >= CF_R ? CF_R : (R > 8 ? 16 : 8);
  if (dft)
    hipLaunchKernelGGL(k_circ_fwd, dim3((unsigned)h->M_all, (unsigned)((R + cw - 1) / cw)), dim3(256), 0,
                       s, h->dv, R, z, zh, con, active);
  if (fft)
    hipLaunchKernelGGL((k_circ_fwd_fft<8, 81>), dim3((unsigned)h->M_all, (unsigned)((R + 7) / 8)),
                       dim3(256), 0, s, h->dv, R, z, zh, con, active);
  if (wide)
    hipLaunchKernelGGL((k_circ_fwd_fft<8, CF_LMAX>), dim3((unsigned)h->M_all, (unsigned)((R + 7) / 8)),
                       dim3(256), 0, s, h->dv, R, z, zh, con, active);
  HIP_TRY(hipGetLastError());
  prof_mark(h, s, 2);
  if (n_citems > 0) {
    hipLaunchKernelGGL(kCircVar[var].fn, dim3((unsigned)n_citems), dim3(kCircVar[var].nt), 0, s, h->dv, R,
                       (const cplx*)zh, wh, citems, n_citems, active);
    HIP_TRY(hipGetLastError());
  }
  prof_mark(h, s, 3);
  return MUDIFF_OK;
}

int circ_finish(mudiff_ctx* h, int R, const cplx* x, cplx* y, int op, const cplx* part, int64_t blk,
                int npad, int RC, const int32_t* dgrp, const int32_t* drow, const int32_t* gnseg,
                const int64_t* gbase, const int32_t* active, const cplx* wh, const int32_t* con,
                const int32_t* con_h, const cplx* shift, hipStream_t s) {
  bool fft, dft, wide;
  circ_kinds(h, con_h, &fft, &dft, &wide);
  if (fft)
    hipLaunchKernelGGL((k_circ_finish_fft<8, 81>), dim3((unsigned)h->M_all, (unsigned)((R + 7) / 8)),
                       dim3(256), 0, s, h->dv, R, x, y, op, part, blk, npad, RC, dgrp, drow, gnseg,
                       gbase, active, wh, con, shift);
  if (wide)
    hipLaunchKernelGGL((k_circ_finish_fft<8, CF_LMAX>), dim3((unsigned)h->M_all, (unsigned)((R + 7) / 8)),
                       dim3(256), 0, s, h->dv, R, x, y, op, part, blk, npad, RC, dgrp, drow, gnseg,
                       gbase, active, wh, con, shift);
  HIP_TRY(hipGetLastError());
  bool direct = dft;  // instances outside the form: partial sums only, in the MFMA finish
  for (int b = 0; b < h->B && !direct; ++b) direct = con_h[b] == 0;
  if (!direct) return MUDIFF_OK;
  int Lmax = 0;
  for (int32_t l : h->cL) Lmax = std::max(Lmax, (int)l);
  const int tm = (2 * h->Nmax + 1 + 15) / 16;  // row tiles: n_p <= 63 (N_p <= 31), L_b <= 125
  // waves per 8-column tile: few right-hand sides spread the row tiles instead
  const int wpc = R >= 32 ? 1 : (R > 8 ? 2 : 4);
  const int tmw = (tm + wpc - 1) / wpc;
  typedef void (*fn_t)(DevView, int, const cplx*, cplx*, int, const cplx*, int64_t, int, int,
                       const int32_t*, const int32_t*, const int32_t*, const int64_t*, const int32_t*,
                       const cplx*, const int32_t*, const cplx*, int);
  static const fn_t fin[5] = {nullptr, k_circ_finish_mfma<1>, k_circ_finish_mfma<2>, k_circ_finish_mfma<3>,
                              k_circ_finish_mfma<4>};
  if (tm < 1 || tm > 4 || Lmax > 128) return fail(MUDIFF_ERR_INVALID, "circulant form: orders out of range");
  const size_t lds = (128 + (size_t)CT_R * std::max(Lmax, 2 * h->Nmax + 2)) * 16;
  const int ncol = 8 * (4 / wpc);
  hipLaunchKernelGGL(fin[tmw], dim3((unsigned)h->M_all, (unsigned)((R + ncol - 1) / ncol)), dim3(256), lds, s,
                     h->dv, R, x, y, op, part, blk, npad, RC, dgrp, drow, gnseg, gbase, active, wh, con, shift,
                     wpc);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}

// Twiddles and transformed symbols of a handle built with the circulant flag
// (enqueued on s after the pair tables).
int circ_build(mudiff_ctx* h, hipStream_t s) {
  int Lmax = 0;
  int64_t Mmax = 0;
  for (int b = 0; b < h->B; ++b) {
    Lmax = std::max(Lmax, h->cL[b]);
    Mmax = std::max(Mmax, h->idisk[b + 1] - h->idisk[b]);
  }
  if (Lmax == 0) return MUDIFF_OK;
  cplx* tw = const_cast<cplx*>(h->dv.ctw);
  hipLaunchKernelGGL(k_circ_twiddles, dim3((unsigned)((Lmax + 255) / 256), (unsigned)h->B), dim3(256), 0, s,
                     h->dv, tw);
  HIP_TRY(hipGetLastError());
  const int ts = 4 * h->Nmax + 1;  // longest symbol row
  const size_t lds = ((size_t)CS_Q * ts + Lmax) * 16;
  hipLaunchKernelGGL(k_circ_symbols, dim3((unsigned)h->M_all, (unsigned)((Mmax + CS_Q - 1) / CS_Q)),
                     dim3(256), lds, s, h->dv, h->circ_near_dev, const_cast<cplx*>(h->dv.cT), ts);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}

extern "C" int mudiff_circulant_info(mudiff_t h, int64_t* far_pairs, int64_t* near_pairs, int* L_max) {
  if (!h) return fail(MUDIFF_ERR_INVALID, "NULL handle");
  int lm = 0;
  for (int32_t l : h->cL) lm = std::max(lm, (int)l);
  if (far_pairs) *far_pairs = h->circ ? h->n_far : 0;
  if (near_pairs) *near_pairs = h->circ ? h->n_near : 0;
  if (L_max) *L_max = lm;
  return MUDIFF_OK;
}
