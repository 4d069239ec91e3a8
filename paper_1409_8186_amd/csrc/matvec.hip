// Operator apply y = L x or y = D^{-1} L x (paper sec. 4.2 block formulas,
// sec. 5 single-scattering preconditioner).
//
// Off-diagonal block (p, q):  (L^{pq} x^q)_m = (i pi/2) s_m sum_n t^{pq}_{n-m} z^q_n,
//   s_m = sqrt(a_p) J_m(k a_p),  z^q_n = sqrt(a_q) J_n(k a_q) x^q_n,
// a Toeplitz product in the mode difference n - m.  The preconditioned form
// divides row m of disk p by L^{pp}_{mm}: (A x)_m = x_m + w_m / (sqrt(a_p) H_m(k a_p)),
// w_m = sum_{q != p} sum_n t^{pq}_{n-m} z^q_n (J_m(k a_p) cancels exactly).
//
// Work decomposition: an item is (row disk p, chunk of column disks).  A
// 256-thread workgroup stages, for a pass of PP column disks, the symbol rows
// t^{pq} and the scaled inputs z^q in LDS (coalesced global loads), then each
// thread accumulates BT consecutive outputs m of one pair over all n.  Chunk
// partial sums go to scratch; the last workgroup of a row (atomic counter)
// adds them in chunk order, so the result does not depend on scheduling.
#include "common.h"

#include <mutex>


#define APPLY_THREADS 256
#define APPLY_NPASS 2

__global__ void k_fill_zero(uint32_t* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0u;
}

int launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  size_t n = bytes / 4;
  if (n == 0) return MUDIFF_OK;
  unsigned g = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_zero, dim3(g), dim3(256), 0, s, (uint32_t*)p, n);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}

// acc[b] += sum_n tb[n - b] z[n],  tb = trow + (LB - 1) - m0
template <int BT, int NQ>
__device__ __forceinline__ void toeplitz_block(const cplx* __restrict__ zrow,
                                               const cplx* __restrict__ tb, int nq_pad,
                                               cplx (&acc)[BT]) {
  if constexpr (NQ > 0) {
#pragma unroll
    for (int n = 0; n < NQ; ++n) {
      const cplx z = zrow[n];
#pragma unroll
      for (int b = 0; b < BT; ++b) cmac(acc[b], tb[n - b], z);
    }
  } else {
    for (int n0 = 0; n0 < nq_pad; n0 += BT) {
#pragma unroll
      for (int d = 0; d < BT; ++d) {
        const cplx z = zrow[n0 + d];
#pragma unroll
        for (int b = 0; b < BT; ++b) cmac(acc[b], tb[n0 + d - b], z);
      }
    }
  }
}

// Output of row unknown i from x_i and the off-diagonal contraction w_i.

// NSPEC >= 0: every disk of the launch has N_p = NSPEC (exact loop bounds).
template <int BT, int NSPEC>
__global__ __launch_bounds__(APPLY_THREADS) void k_apply(
    DevView v, int R, const cplx* __restrict__ x, cplx* __restrict__ y, int op,
    cplx* __restrict__ part, int64_t part_total, int32_t* __restrict__ counters,
    const int32_t* __restrict__ items, const int32_t* __restrict__ nchunk,
    const int64_t* __restrict__ partoff, const int32_t* __restrict__ active, int zs, int ts,
    int ppcap, const cplx* __restrict__ shift) {
  extern __shared__ cplx lds[];
  __shared__ int s_last;
  const int it = blockIdx.x, r = blockIdx.y;
  const int p = items[4 * it], c = items[4 * it + 1], jb = items[4 * it + 2], je = items[4 * it + 3];
  const int b = v.inst[p];
  if (active && active[b * R + r] == 0) return;
  const int Np = NSPEC >= 0 ? NSPEC : v.N[p];
  const int np = 2 * Np + 1;
  const int L = (np + BT - 1) / BT;
  const int LB = L * BT;
  const int PP = min(APPLY_THREADS / L, ppcap);
  const int64_t d0 = v.idisk[b];
  const int64_t i0 = v.imode[b];
  const int64_t cb = col_base(v.imode, b, R, r);
  const cplx* __restrict__ xc = x + cb;
  const int tid = threadIdx.x;
  const int slot = tid / L, mb = tid - (tid / L) * L;
  const int m0 = mb * BT;
  cplx* zl = lds;                 // [PP][zs]
  cplx* tl = lds + PP * zs;       // [PP][ts]

  cplx acc[BT];
#pragma unroll
  for (int k = 0; k < BT; ++k) acc[k] = cmk(0.0, 0.0);

  for (int j0 = jb; j0 < je; j0 += PP) {
    const int nslot = min(PP, je - j0);
    __syncthreads();
    // stage z^q = sqrt(a_q) J_n(k a_q) x^q_n
    for (int e = tid; e < PP * zs; e += APPLY_THREADS) {
      const int k = e / zs, n = e - (e / zs) * zs;
      cplx z = cmk(0.0, 0.0);
      if (k < nslot) {
        const int q = (int)(d0 + j0 + k + ((d0 + j0 + k) >= p ? 1 : 0));
        const int nq = 2 * (NSPEC >= 0 ? NSPEC : v.N[q]) + 1;
        if (n < nq) {
          const int64_t iq = v.moff[q] + n;
          z = col_scale(v, i0 + iq, xc[iq]);
        }
      }
      zl[e] = z;
    }
    // stage symbol rows: u = n - m + LB - 1  <->  s = u - (LB - 1) - N_q + N_p
    for (int e = tid; e < PP * ts; e += APPLY_THREADS) {
      const int k = e / ts, u = e - (e / ts) * ts;
      cplx t = cmk(0.0, 0.0);
      if (k < nslot) {
        const int q = (int)(d0 + j0 + k + ((d0 + j0 + k) >= p ? 1 : 0));
        const int Nq = NSPEC >= 0 ? NSPEC : v.N[q];
        const int S = Np + Nq;
        const int s = u - (LB - 1) - Nq + Np;
        if (s >= -S && s <= S) {
          const int64_t g = pair_index(v.idisk, v.ipair, b, p, q);
          t = v.t[v.toff[g] + S + s];
          if (p > q && (s & 1)) t = cmk(-t.x, -t.y);  // t^{qp}_s = (-1)^s t^{pq}_s
        }
      }
      tl[e] = t;
    }
    __syncthreads();
    if (slot < nslot) {
      const cplx* tb = tl + slot * ts + (LB - 1) - m0;
      if constexpr (NSPEC >= 0)
        toeplitz_block<BT, 2 * NSPEC + 1>(zl + slot * zs, tb, 0, acc);
      else
        toeplitz_block<BT, 0>(zl + slot * zs, tb, zs, acc);
    }
  }
  // reduce over pair slots
  __syncthreads();
  cplx* red = lds;  // [PP][LB]
  if (slot < PP) {
#pragma unroll
    for (int k = 0; k < BT; ++k) red[slot * LB + m0 + k] = acc[k];
  }
  __syncthreads();
  const int nch = nchunk[p];
  const int64_t ip = i0 + v.moff[p];  // unknown index (single column) of mode -N_p
  cplx* yc = y + cb + v.moff[p];
  const cplx* xp = xc + v.moff[p];
  const int nslot_max = min(PP, je - jb);
  if (nch == 1) {
    for (int m = tid; m < np; m += APPLY_THREADS) {
      cplx w = cmk(0.0, 0.0);
      for (int k = 0; k < nslot_max; ++k) w = cadd(w, red[k * LB + m]);
      cplx o = finalize(v, op, ip + m, xp[m], w);
      if (shift) o = affine(shift, b * R + r, o, xp[m]);
      yc[m] = o;
    }
    return;
  }
  cplx* pr = part + (int64_t)r * part_total + partoff[p];
  for (int m = tid; m < np; m += APPLY_THREADS) {
    cplx w = cmk(0.0, 0.0);
    for (int k = 0; k < nslot_max; ++k) w = cadd(w, red[k * LB + m]);
    pr[(int64_t)c * np + m] = w;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // publish this chunk
  __syncthreads();
  if (tid == 0) {
    int32_t* cnt = counters + (int64_t)r * v.M_all + p;
    int old = atomicAdd(cnt, 1);
    s_last = (old == nch - 1);
    if (s_last) atomicExch(cnt, 0);
  }
  __syncthreads();
  if (!s_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // see the other chunks
  for (int m = tid; m < np; m += APPLY_THREADS) {
    cplx w = cmk(0.0, 0.0);
    for (int k = 0; k < nch; ++k) {
      w = cadd(w, pr[(int64_t)k * np + m]);  // visible after the fence above
    }
    cplx o = finalize(v, op, ip + m, xp[m], w);
    if (shift) o = affine(shift, b * R + r, o, xp[m]);
    yc[m] = o;
  }
}

// ------------------------------------------------------------------ one lane per pair
// Uniform N_p = N (<= 12), few right-hand sides.  A work item is one wave: row
// disk p, one right-hand side and a chunk of up to 64 column disks q, one
// lane per ordered pair (p, q), with all n = 2N+1 outputs of the pair in
// registers.  Each pair is read as one lane-interleaved record (H_0, H_1,
// e^{i alpha_pq}, 2 / (k b_pq)): the orders H_nu(k b_pq), nu <= 2N, follow by
// the upward recurrence H_{nu+1} = (2 nu / x) H_nu - H_{nu-1}, whose rounding
// error stays at the level of eps |H_nu| (the growing Y part dominates |H_nu|
// wherever the J part decays), and the phase e^{i nu alpha} by recurrence;
// t_{+nu} = H_nu e^{i nu alpha}, t_{-nu} = (-1)^nu H_nu e^{-i nu alpha}.  The
// product runs diagonal by diagonal (w_m += t_s z_{m+s}) with the scaled
// inputs z in registers.  The 2n real outputs are summed over the lanes by a
// reduce-scatter butterfly (lane l ends with the sum of value l >> sh) and
// stored as the chunk's partial sum; k_apply_finish adds the chunks of each
// row in order.  Single-wave items keep every SIMD busy to the end of the
// launch (rows of unequal cost or rows fewer than the compute units would
// leave whole workgroups idle), and the two launches need no counters or
// memory fences.
template <int N, bool OPC>
__global__ __launch_bounds__(64) void k_apply_lane(
    DevView v, int R, const cplx* __restrict__ x, cplx* __restrict__ part, int64_t part_total,
    const int32_t* __restrict__ items, const int32_t* __restrict__ active) {
  constexpr int n = 2 * N + 1, S = 2 * N;
  constexpr int NV = 2 * n <= 8 ? 8 : (2 * n <= 16 ? 16 : (2 * n <= 32 ? 32 : 64));
  constexpr int SH = NV == 8 ? 3 : (NV == 16 ? 2 : (NV == 32 ? 1 : 0));  // 6 - log2 NV
  const int r = blockIdx.y;
  const int32_t* itp = items + (int64_t)LANE_ITEM_INTS * blockIdx.x;
  const int p = itp[0], jb = itp[2], je = itp[3], b = itp[4];
  if (active && active[b * R + r] == 0) return;
  const int lane = threadIdx.x;
  const int64_t d0 = itp[5];
  const int64_t i0 = *reinterpret_cast<const int64_t*>(itp + 6);
  const int64_t cb = (int64_t)R * i0 + (int64_t)r * *reinterpret_cast<const int64_t*>(itp + 8);
  const int64_t recb = *reinterpret_cast<const int64_t*>(itp + 10);
  const int64_t pb = *reinterpret_cast<const int64_t*>(itp + 12);
  const int j = jb + lane;
  cplx acc[n];
#pragma unroll
  for (int m = 0; m < n; ++m) acc[m] = cmk(0.0, 0.0);
  if (j < je) {
    const int q = (int)(d0 + j + ((d0 + j) >= p ? 1 : 0));
    const cplx* __restrict__ rec = v.lt + recb + lane;
    const int64_t iq = (int64_t)(q - d0) * n;  // uniform N: moff[q] = (q - d0) n
    const cplx h0 = rec[0];
    cplx H = rec[LANE_CHUNK];
    const cplx E = rec[2 * LANE_CHUNK];
    const double r2 = rec[3 * LANE_CHUNK].x;
    cplx z[n];
#pragma unroll
    for (int k = 0; k < n; ++k)
      z[k] = OPC ? cmul(x[cb + iq + k], v.op_col[i0 + iq + k]) : cscale(x[cb + iq + k], v.sJ[i0 + iq + k]);
#pragma unroll
    for (int m = 0; m < n; ++m) cmac(acc[m], h0, z[m]);
    cplx Hm = h0;
    cplx P = E;
#pragma unroll
    for (int nu = 1; nu <= S; ++nu) {
      if (nu > 1) {
        const cplx Hn = csub(cscale(H, (nu - 1) * r2), Hm);  // H_nu from H_{nu-1}, H_{nu-2}
        Hm = H;
        H = Hn;
        P = cmul(P, E);
      }
      const cplx tp = cmul(H, P);
      cplx tm = cmul(H, cconj(P));
      if (nu & 1) tm = cmk(-tm.x, -tm.y);
#pragma unroll
      for (int m = 0; m < n - nu; ++m) cmac(acc[m], tp, z[m + nu]);
#pragma unroll
      for (int m = nu; m < n; ++m) cmac(acc[m], tm, z[m - nu]);
    }
  }
  double val[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) val[k] = k < 2 * n ? ((k & 1) ? acc[k >> 1].y : acc[k >> 1].x) : 0.0;
  lane_reduce_scatter<NV>(val, lane);
  const int vi = lane >> SH;
  if ((lane & ((1 << SH) - 1)) == 0 && vi < 2 * n) {
    double* pr = reinterpret_cast<double*>(part + (int64_t)r * part_total + pb);
    pr[vi] = val[0];
  }
}

// y = finalize(sum over the chunks of row p of the partial sums), one thread
// per output row, chunks added in order.
__global__ void k_apply_finish(DevView v, int R, const cplx* __restrict__ x, cplx* __restrict__ y,
                               int op, const cplx* __restrict__ part, int64_t part_total,
                               const int32_t* __restrict__ nchunk,
                               const int64_t* __restrict__ partoff,
                               const int32_t* __restrict__ active,
                               const cplx* __restrict__ shift) {
  const int64_t total = (int64_t)R * v.N_all;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  // column (b, r) and unknown i of the packed row g
  int lo = 0, hi = v.B;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)R * v.imode[mid] <= g) lo = mid; else hi = mid;
  }
  const int b = lo;
  const int64_t Nb = v.imode[b + 1] - v.imode[b];
  const int64_t rem = g - (int64_t)R * v.imode[b];
  const int r = (int)(rem / Nb);
  if (active && active[b * R + r] == 0) return;
  const int64_t i = v.imode[b] + (rem - (int64_t)r * Nb);
  const cplx w = lane_chunk_sum(v, part + (int64_t)r * part_total, nchunk, partoff, b, i);
  cplx o = finalize(v, op, i, x[g], w);
  if (shift) o = affine(shift, b * R + r, o, x[g]);
  y[g] = o;
}

// ------------------------------------------------------------------ multi-RHS (MFMA)
// For R right-hand sides the block product T^{pq} Z^q (n_p x n_q times n_q x R)
// is a dense contraction: it runs on FP64 MFMA (v_mfma_f64_16x16x4f64,
// D[16x16] += A[16x4] B[4x16]).  A complex product is two real MFMAs: the B
// panel holds [Re Z | Im Z] for 8 right-hand sides side by side, so
//   acc1 = Re(T) [Re Z | Im Z],  acc2 = Im(T) [Re Z | Im Z],
//   Re W = acc1[:, :8] - acc2[:, 8:],  Im W = acc1[:, 8:] + acc2[:, :8].
// Lane layout (checked on the device): lane l holds A[l % 16][l / 16],
// B[l / 16][l % 16] and D[4 v + l / 16][l % 16], v < 4.
//
// Work item: a group of rp <= RP row disks of one instance (disks of equal row
// tile count grouped together, so that the waves of a workgroup issue equal
// numbers of MFMAs between barriers), a tile of 8 CT right-hand sides and a
// segment [q0, q1) of its column disks.  Wave w of the workgroup computes row
// w / CT and right-hand-side sub-tile w % CT.  The input panel
// Z^q = sqrt(a_q) J_n(k a_q) x^q_n is formed once per apply for all columns
// (k_apply_mfma_scale); per column disk q its panel and the symbol rows of the
// item's row disks are staged in LDS once for all waves, and the next disk's
// values are gathered into registers while the current one is on the matrix
// cores.  The workgroups are persistent: each takes items from a queue
// (one atomic counter, items sorted by decreasing cost), so instances of very
// different sizes share one launch and the launch ends evenly.  Each item's
// sums go to its own partial block; k_apply_mfma_finish adds the segments of
// every row in order (no inter-workgroup synchronisation).  The tile shape
// (RP, CT), the segment length and the workgroup size are chosen per handle
// and R by timing the candidates on the real data (mfma_autotune).
typedef double mf_d4 __attribute__((ext_vector_type(4)));

#define MF_REC 7       // item record: row group, rp, tile, q0, q1, partial block, list flag

// Column of element (n, c) of the staged input panel [4 ktmax][RC] in LDS:
// c XOR a function of the row n, so that a staging store (consecutive rows, one
// column) spreads over 16 bank groups and an MFMA B read (rows n..n+3, eight
// columns) puts even and odd rows in different halves of the banks.
__device__ __forceinline__ int mf_zcol(int n, int c, int RC) {
  const int f = ((n & 1) << 3) | ((n >> 1) & 7);
  return c ^ (f & (RC >= 16 ? 15 : RC - 1));
}

// K row tiles of one wave against one staged column disk: KT k-steps of 4,
// two real MFMAs per tile and step (Re T, Im T against [Re Z | Im Z]); zl is
// the staged panel and zc this lane's panel column.
template <int K, int MT>
__device__ __forceinline__ void mf_tiles(const cplx* trow, const cplx* zl, int zc, int RC, int j,
                                         int kq, int KT, mf_d4* acc1, mf_d4* acc2) {
  for (int kk = 0; kk < KT; ++kk) {
    const int n = 4 * kk + kq;
    const cplx zz = zl[n * RC + mf_zcol(n, zc, RC)];
    const double bv = j < 8 ? zz.x : zz.y;
#pragma unroll
    for (int mt = 0; mt < K; ++mt) {
      const cplx t = trow[n - (16 * mt + j) + 16 * MT - 1];  // A[i = lane % 16][k = kq]
      acc1[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(t.x, bv, acc1[mt], 0, 0, 0);
      acc2[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(t.y, bv, acc2[mt], 0, 0, 0);
    }
  }
}

// MT row tiles of 16 (n_p <= 16 MT); ZK / TK staged input / symbol values per
// thread, sized on the host for the batch (4 ktmax RC <= ZK THREADS and
// RP TL <= TK THREADS), which keeps the register footprint of the staging to
// what the batch needs.
// An item with its list flag set takes its column disks from qlist[q0..q1):
// entry (q << 8) | mask, mask bit r set when row r of the item's group is a
// close pair with q (the circulant form covers the other pairs).
template <int MT, int THREADS, int ZK, int TK>
__global__ __launch_bounds__(THREADS) void k_apply_mfma(
    DevView v, int R, const cplx* __restrict__ x, const int32_t* __restrict__ active,
    const int32_t* __restrict__ items, int n_items, int32_t* __restrict__ head,
    cplx* __restrict__ part, int64_t blk, int npad, int ktmax, int RP, int CT,
    const int32_t* __restrict__ grow, const int32_t* __restrict__ qlist) {
  extern __shared__ cplx lds[];
  __shared__ int s_item;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int j = lane & 15, kq = lane >> 4;
  const int RC = 8 * CT;
  const int row = wave / CT, ctile = wave - (wave / CT) * CT;
  const int TL = 4 * ktmax + 16 * MT - 1;  // symbol row length in LDS
  const int zrows = 4 * ktmax;
  cplx* zl = lds;                          // [4 ktmax][RC]
  cplx* tl = lds + zrows * RC;             // [RP][TL]
  // this thread's staging slots: input panel element (column zc, row zn),
  // symbol element (row trr, position tru)
  int zc[ZK], zn[ZK], trr[TK], tru[TK];
#pragma unroll
  for (int k = 0; k < ZK; ++k) {
    const int e = tid + k * THREADS;
    zc[k] = e / zrows;
    zn[k] = e - zc[k] * zrows;
  }
#pragma unroll
  for (int k = 0; k < TK; ++k) {
    const int e = tid + k * THREADS;
    trr[k] = e / TL;
    tru[k] = e - trr[k] * TL;
  }
  for (;;) {
    __syncthreads();  // the previous item is done with s_item and LDS
    if (tid == 0) s_item = atomicAdd(head, 1);
    __syncthreads();
    const int it = s_item;
    if (it >= n_items) break;
    const int32_t* rec = items + (int64_t)MF_REC * it;
    const int rp = rec[1], tile = rec[2], qb = rec[3], qe = rec[4];
    const int32_t* __restrict__ ql = rec[6] ? qlist : nullptr;
    // column disk and row mask of list position i (qb <= i < qe)
    auto qat = [&](int i) { return ql ? (ql[i] >> 8) : i; };
    auto mat = [&](int i) { return ql ? (ql[i] & 0xff) : 0xff; };
    const int32_t* grp = grow + (int64_t)rec[0] * RP;  // the item's row disks
    const int64_t pb = rec[5];
    const int c0 = tile * RC;
    const int b = v.inst[grp[0]];
    bool any = false;  // converged columns: the whole tile may be skipped
    for (int r = c0; r < min(R, c0 + RC); ++r)
      if (!active || active[b * R + r]) any = true;
    if (!any) continue;
    const int64_t i0 = v.imode[b];
    const bool row_ok = row < rp;
    const int p = row_ok ? grp[row] : -1;
    const int mtp = row_ok ? (2 * v.N[p] + 1 + 15) >> 4 : 0;  // row tiles of this row disk
    bool wave_active = row_ok;
    if (wave_active) {
      wave_active = false;
      for (int c = 0; c < 8; ++c) {
        const int r = c0 + ctile * 8 + c;
        if (r < R && (!active || active[b * R + r])) wave_active = true;
      }
    }
    mf_d4 acc1[MT], acc2[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      acc1[t] = mf_d4{0.0, 0.0, 0.0, 0.0};
      acc2[t] = mf_d4{0.0, 0.0, 0.0, 0.0};
    }
    // Gathered values of the next column disk, loaded while the current one is
    // on the matrix cores: nothing in the gather consumes a load (the input
    // arrives scaled by its column factor, the symbol sign is applied when
    // staging), so the gather does not hold up the MFMAs behind it.  N and the
    // mode offset of the disks are read one disk ahead of their gather, N of
    // the item's row disks once.
    cplx zr[ZK], tr[TK];
    double tsg[TK];
    int32_t tof[TK];  // symbol offsets (the MFMA path requires T_all < 2^31)
    int npr[TK], prw[TK];  // N and index of this thread's symbol-row disks
#pragma unroll
    for (int k = 0; k < TK; ++k) {
      prw[k] = trr[k] < rp ? grp[trr[k]] : -1;
      npr[k] = prw[k] >= 0 ? v.N[prw[k]] : 0;
    }
    auto gather = [&](int q, int qmask, int Nq, int64_t mq) {
      const int nq = 2 * Nq + 1;
#pragma unroll
      for (int k = 0; k < ZK; ++k) {
        const int c = zc[k], n = zn[k];
        cplx z = cmk(0.0, 0.0);
        if (c < RC && n < nq && c0 + c < R) z = x[col_base(v.imode, b, R, c0 + c) + mq + n];
        zr[k] = z;
      }
#pragma unroll
      for (int k = 0; k < TK; ++k) {
        const int rr = trr[k], u = tru[k];
        cplx t = cmk(0.0, 0.0);
        double sg = 1.0;
        const int pr = prw[k];
        if (rr < rp && pr != q && ((qmask >> rr) & 1)) {
          const int Npr = npr[k];
          const int S = Npr + Nq;
          const int s = u - (16 * MT - 1) - Nq + Npr;
          if (s >= -S && s <= S) {
            t = v.t[tof[k] + S + s];
            if (pr > q && (s & 1)) sg = -1.0;
          }
        }
        tr[k] = t;
        tsg[k] = sg;
      }
    };
    // symbol-row offsets of column disk q, loaded one disk ahead of gather(q)
    // so that gathering the symbols is a single dependent load
    auto load_toff = [&](int q, int qmask) {
#pragma unroll
      for (int k = 0; k < TK; ++k) {
        const int pr = prw[k];
        tof[k] = (q >= 0 && trr[k] < rp && pr != q && ((qmask >> trr[k]) & 1))
                     ? (int32_t)v.toff[pair_index(v.idisk, v.ipair, b, pr, q)] : 0;
      }
    };
    // disk, row mask, N and mode offset of list positions i (0), i + 1 (1)
    // and i + 2 (2)
    int qd0 = -1, qd1 = -1, qd2 = -1, qm0 = 0, qm1 = 0, qm2 = 0;
    int Nq0 = 0, Nq1 = 0, Nq2 = 0;
    int64_t mq0 = 0, mq1 = 0, mq2 = 0;
    if (qb < qe) {
      qd0 = qat(qb);
      qm0 = mat(qb);
      Nq0 = v.N[qd0];
      mq0 = v.moff[qd0];
    }
    if (qb + 1 < qe) {
      qd1 = qat(qb + 1);
      qm1 = mat(qb + 1);
      Nq1 = v.N[qd1];
      mq1 = v.moff[qd1];
    }
    if (qb < qe) {
      load_toff(qd0, qm0);
      gather(qd0, qm0, Nq0, mq0);
      load_toff(qd1, qm1);
    }
    for (int qi = qb; qi < qe; ++qi) {
      const int q = qd0;
      const int nq = 2 * Nq0 + 1, KT = (nq + 3) >> 2;
      __syncthreads();  // previous column disk done with LDS
#pragma unroll
      for (int k = 0; k < ZK; ++k)
        if (zc[k] < RC) zl[zn[k] * RC + mf_zcol(zn[k], zc[k], RC)] = zr[k];
#pragma unroll
      for (int k = 0; k < TK; ++k)
        if (trr[k] < RP) tl[trr[k] * TL + tru[k]] = cscale(tr[k], tsg[k]);
      __syncthreads();
      qd2 = -1;
      qm2 = 0;
      if (qi + 2 < qe) {  // used by the next iteration's gather
        qd2 = qat(qi + 2);
        qm2 = mat(qi + 2);
        Nq2 = v.N[qd2];
        mq2 = v.moff[qd2];
      }
      if (qi + 1 < qe) {  // in flight during the MFMAs
        gather(qd1, qm1, Nq1, mq1);
        load_toff(qd2, qm2);
      }
      if (wave_active && q != p && ((qm0 >> row) & 1)) {
        const cplx* trow = tl + row * TL;
        const int zcl = ctile * 8 + (j & 7);
        // only the row tiles of this row disk (wave-uniform count)
        if (mtp >= MT) mf_tiles<MT, MT>(trow, zl, zcl, RC, j, kq, KT, acc1, acc2);
        else if constexpr (MT >= 2) {
          if (mtp == MT - 1) mf_tiles<MT - 1, MT>(trow, zl, zcl, RC, j, kq, KT, acc1, acc2);
          else if constexpr (MT >= 3) {
            if (mtp == MT - 2) mf_tiles<MT - 2, MT>(trow, zl, zcl, RC, j, kq, KT, acc1, acc2);
            else if constexpr (MT >= 4) mf_tiles<MT - 3, MT>(trow, zl, zcl, RC, j, kq, KT, acc1, acc2);
          }
        }
      }
      qd0 = qd1;
      qm0 = qm1;
      Nq0 = Nq1;
      mq0 = mq1;
      qd1 = qd2;
      qm1 = qm2;
      Nq1 = Nq2;
      mq1 = mq2;
    }
    if (!wave_active) continue;
    // partial block [RP][npad][RC]: row r of the item, mode row m, RHS column
    cplx* pbk = part + pb * blk + (int64_t)row * npad * RC + ctile * 8 + (j & 7);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) {
        const double a1 = acc1[mt][vv], a2 = acc2[mt][vv];
        const double other = __shfl_xor(a2, 8, 64);
        const double val = j < 8 ? a1 - other : a1 + other;  // Re W (j < 8), Im W (j >= 8)
        const double im = __shfl_xor(val, 8, 64);
        const int m = 16 * mt + 4 * vv + kq;  // D row 4 v + lane / 16
        if (j < 8) pbk[(int64_t)m * RC] = cmk(val, im);
      }
    }
  }
}

// Close pairs of the instances in the circulant form with 8-column tiles (few
// right-hand sides): one wave per (row disk p, tile of 8 columns, group of row
// tiles), no LDS and no barriers.  The wave walks p's close list; per column disk q and k step it
// loads the input panel element of its lane (B[k][j]: Re or Im of column j & 7
// at mode 4 kt + k) and per row tile the symbol value of its lane (A[i][k]:
// t_{(n - N_q) - (m - N_p)}, m = 16 mt + i), straight into the operand layout
// of v_mfma_f64_16x16x4f64 (two MFMAs per complex product, as k_apply_mfma),
// and accumulates the whole row in registers; the sum goes to segment 0 of the
// row's group, which the output pass adds.  In the work queue the same pairs
// cost two barriers and an LDS staging round per listed column disk, with only
// the few waves whose row is close to it on the matrix cores.  The kernel is
// bound by load latency, so the row tiles of a row disk are split over waves
// (MTW tiles each, blockIdx.z the group): with the accumulators of two tiles
// the register budget is held to eight waves per SIMD, at one more input load
// per k step.
template <int MT, int MTW>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8))) void k_apply_close(
    DevView v, int R, const cplx* __restrict__ z, cplx* __restrict__ part, int64_t blk, int npad,
    const int32_t* __restrict__ dgrp, const int32_t* __restrict__ drow,
    const int64_t* __restrict__ gbase, const int32_t* __restrict__ nptr,
    const int32_t* __restrict__ nql, const int32_t* __restrict__ con,
    const int32_t* __restrict__ active, const int32_t* __restrict__ rord) {
  // rows by decreasing work, so that the longest lists do not end the launch
  const int p = rord[blockIdx.x], t = blockIdx.y, lane = threadIdx.x;
  const int mt0 = MTW * (int)blockIdx.z;  // first row tile of this wave
  const int b = v.inst[p];
  if (!con[b]) return;
  const int c0 = 8 * t;
  if (c0 >= R) return;
  const int Np = v.N[p], np_ = 2 * Np + 1, mtp = (np_ + 15) >> 4;
  // tiles from 16 mtp on hold no mode of p and are never read
  if (mt0 >= mtp) return;
  if (active) {
    bool any = false;
    for (int r = c0; r < min(R, c0 + 8); ++r) any |= active[b * R + r] != 0;
    if (!any) return;
  }
  const int j = lane & 15, kq = lane >> 4;
  mf_d4 acc1[MTW], acc2[MTW];
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    acc1[i] = mf_d4{0.0, 0.0, 0.0, 0.0};
    acc2[i] = mf_d4{0.0, 0.0, 0.0, 0.0};
  }
  const int col = c0 + (j & 7);
  const bool colok = col < R;
  const int64_t cb = colok ? col_base(v.imode, b, R, col) : 0;
  for (int e = nptr[p]; e < nptr[p + 1]; ++e) {
    const int q = nql[e];
    const int Nq = v.N[q], nq_ = 2 * Nq + 1, S = Np + Nq, KT = (nq_ + 3) >> 2;
    const cplx* __restrict__ trow = v.t + v.toff[pair_index(v.idisk, v.ipair, b, p, q)] + S;
    const bool flip = p > q;  // t^{pq}_s = (-1)^s t^{qp}_s
    const cplx* __restrict__ zq = z + cb + v.moff[q];
    for (int kt = 0; kt < KT; ++kt) {
      const int n = 4 * kt + kq;
      double bv = 0.0;
      if (colok && n < nq_) {
        const cplx zz = zq[n];
        bv = j < 8 ? zz.x : zz.y;
      }
#pragma unroll
      for (int i = 0; i < MTW; ++i) {
        const int mt = mt0 + i;
        if (mt < mtp) {  // wave-uniform
          const int m = 16 * mt + j;
          cplx a = cmk(0.0, 0.0);
          if (m < np_ && n < nq_) {
            const int sv = (n - Nq) - (m - Np);
            a = trow[sv];
            if (flip && (sv & 1)) a = cmk(-a.x, -a.y);
          }
          acc1[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, bv, acc1[i], 0, 0, 0);
          acc2[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, bv, acc2[i], 0, 0, 0);
        }
      }
    }
  }
  // segment 0 of the group's tile t: [RP][npad][8]
  cplx* pbk = part + (gbase[dgrp[p]] + t) * blk + (int64_t)drow[p] * npad * 8 + (j & 7);
#pragma unroll
  for (int i = 0; i < MTW; ++i) {
    const int mt = mt0 + i;
    if (mt >= MT) break;
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) {
      const double a1 = acc1[i][vv], a2 = acc2[i][vv];
      const double other = __shfl_xor(a2, 8, 64);
      const double val = j < 8 ? a1 - other : a1 + other;  // Re W (j < 8), Im W (j >= 8)
      const double im = __shfl_xor(val, 8, 64);
      const int m = 16 * mt + 4 * vv + kq;
      if (j < 8) pbk[(int64_t)m * 8] = cmk(val, im);
    }
  }
}

// z = x scaled by the column factor of its unknown (sqrt(a) J_n, or the
// operator's column table), once per apply: the MFMA gathers then load one
// value per panel element.
__global__ void k_apply_mfma_scale(DevView v, int R, const cplx* __restrict__ x, cplx* __restrict__ z,
                                   const int32_t* __restrict__ active) {
  // blockIdx.x: column (b, r); blockIdx.y: 256-unknown slice of that column
  const int col = blockIdx.x, b = col / R;
  if (active && active[col] == 0) return;  // columns that no longer iterate
  const int64_t Nb = v.imode[b + 1] - v.imode[b];
  const int64_t k = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (k >= Nb) return;
  const int64_t g = (int64_t)R * v.imode[b] + (int64_t)(col - b * R) * Nb + k;
  z[g] = col_scale(v, v.imode[b] + k, x[g]);
}

// y = finalize(sum over the segments of the MFMA partial blocks), one thread
// per output row, segments added in order.
__global__ void k_apply_mfma_finish(DevView v, int R, const cplx* __restrict__ x,
                                    cplx* __restrict__ y, int op, const cplx* __restrict__ part,
                                    int64_t blk, int npad, int RC, const int32_t* __restrict__ dgrp,
                                    const int32_t* __restrict__ drow,
                                    const int32_t* __restrict__ gnseg,
                                    const int64_t* __restrict__ gbase,
                                    const int32_t* __restrict__ active,
                                    const cplx* __restrict__ wh,
                                    const int32_t* __restrict__ con,
                                    const cplx* __restrict__ shift) {
  const int64_t total = (int64_t)R * v.N_all;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  int lo = 0, hi = v.B;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)R * v.imode[mid] <= g) lo = mid; else hi = mid;
  }
  const int b = lo;
  const int64_t Nb = v.imode[b + 1] - v.imode[b];
  const int64_t rem = g - (int64_t)R * v.imode[b];
  const int r = (int)(rem / Nb);
  if (active && active[b * R + r] == 0) return;
  const int64_t i = v.imode[b] + (rem - (int64_t)r * Nb);
  const int p = v.udisk[i];
  const int64_t m = i - v.imode[b] - v.moff[p];
  const int gr = dgrp[p];
  const int t = r / RC, rc = r - (r / RC) * RC;
  const int ns = gnseg[gr];
  const cplx* pr = part + (gbase[gr] + (int64_t)t * ns) * blk +
                   ((int64_t)drow[p] * npad + m) * RC + rc;
  cplx w = cmk(0.0, 0.0);
  for (int s = 0; s < ns; ++s) w = cadd(w, pr[(int64_t)s * blk]);
  if (wh && con[b]) {  // well-separated pairs: w_j += sum_f w^{f j} W_f[p][r]
    const int Lb = v.cL[b];
    const int64_t d0 = v.idisk[b], Mb = v.idisk[b + 1] - d0;
    const cplx* __restrict__ wf = wh + (int64_t)R * v.cZo[b] + (p - d0) * R + r;
    const cplx* __restrict__ tw = v.ctw + v.cWo[b];
    const int jm = (int)m;
    int idx = 0;
    cplx acc = cmk(0.0, 0.0);
    for (int f = 0; f < Lb; ++f) {
      cmac(acc, tw[idx], wf[(int64_t)f * Mb * R]);
      idx += jm;
      if (idx >= Lb) idx -= Lb;
    }
    w = cadd(w, acc);
  }
  cplx o = finalize(v, op, i, x[g], w);
  if (shift) o = affine(shift, b * R + r, o, x[g]);
  y[g] = o;
}

// R at and above which the MFMA kernel applies the operator (N_p <= 31).
#define MFMA_MIN_R 8
// Column-disk segment length once few columns are still iterating: short
// segments spread a large straggler instance over many workgroups.
#define MFMA_TAIL_QS 16

static bool use_mfma(const mudiff_ctx* h, int R) {
  return R >= MFMA_MIN_R && h->Nmax <= 31 && h->mfma_enabled && h->T_all < ((int64_t)1 << 31);
}

int circ_variant(int R);
std::vector<int> circ_variants(int R);
void circ_tile(int var, int* bm, int* bn);
void circ_var_dims(int var, int* bm, int* bn, int* bk, int* db, int* nt, int* mult);
int circ_finish(mudiff_ctx* h, int R, const cplx* x, cplx* y, int op, const cplx* part, int64_t blk,
                int npad, int RC, const int32_t* dgrp, const int32_t* drow, const int32_t* gnseg,
                const int64_t* gbase, const int32_t* active, const cplx* wh, const int32_t* con,
                const int32_t* con_h, const cplx* shift, hipStream_t s);
int circ_launch(mudiff_ctx* h, int R, const cplx* z, cplx* zh, cplx* wh, const int32_t* citems,
                int n_citems, int var, const int32_t* con, const int32_t* con_h,
                const int32_t* active, hipStream_t s);

// Host schedule of the MFMA apply for one tile choice.  With c.circ, the
// instances marked circ_on keep only their close pairs in the MFMA items
// (column lists) and get per-frequency product items instead.
static void mfma_build(const mudiff_ctx* h, int R, const MfmaChoice& c, MfmaSched& S,
                       const std::vector<int32_t>& cols = {}) {
  S.R = R;
  S.c = c;
  S.dev_base = nullptr;
  const int RC = 8 * c.CT;
  S.ntile = (R + RC - 1) / RC;
  const int mt = (2 * h->Nmax + 1 + 15) / 16;
  S.npad = 16 * mt;
  S.blk = (int64_t)c.RP * S.npad * RC;
  S.items.clear();
  S.grow.clear();
  S.gnseg.clear();
  S.gbase.clear();
  S.qlist.clear();
  S.citems.clear();
  S.nptr.clear();
  S.nq.clear();
  S.rord.clear();
  S.close_rows = c.circ && h->circ && c.CT == 1;
  S.con.assign(h->B, 0);
  S.dgrp.assign(h->M_all, 0);
  S.drow.assign(h->M_all, 0);
  S.cvar = c.cvar >= 0 ? c.cvar : circ_variant(R);
  int cbm = 0, cbn = 0;
  circ_tile(S.cvar, &cbm, &cbn);
  struct It {
    double cost;
    int32_t r[MF_REC];
  };
  std::vector<It> its;
  auto tile_runs = [&](int b, int r0, int r1) {  // straggler schedule: a running column in [r0, r1)
    if (cols.empty()) return true;
    for (int r = r0; r < std::min(R, r1); ++r)
      if (cols[(size_t)b * R + r] != 0) return true;
    return false;
  };
  int64_t pb = 0;
  for (int b = 0; b < h->B; ++b) {
    const int64_t d0 = h->idisk[b], d1 = h->idisk[b + 1], Mb = d1 - d0;
    const bool circ = c.circ && h->circ && h->circ_on[b];
    S.con[b] = circ ? 1 : 0;
    const int64_t qs = c.QS > 0 ? c.QS : Mb;
    // row disks ordered by their number of 16-row tiles (stable), in groups of
    // RP; for the column lists of the circulant form, by a Z-order (Morton)
    // code of their centers within each tile class, so that a group's rows are
    // neighbours and share most of their close column disks
    std::vector<int32_t> ord((size_t)Mb);
    for (int64_t k = 0; k < Mb; ++k) ord[(size_t)k] = (int32_t)(d0 + k);
    std::vector<uint32_t> zc;
    if (circ) {
      double x0 = h->cx[d0], x1 = x0, y0 = h->cy[d0], y1 = y0;
      for (int64_t q = d0; q < d1; ++q) {
        x0 = std::min(x0, h->cx[q]);
        x1 = std::max(x1, h->cx[q]);
        y0 = std::min(y0, h->cy[q]);
        y1 = std::max(y1, h->cy[q]);
      }
      const double sc = 65535.0 / std::max(std::max(x1 - x0, y1 - y0), 1e-300);
      zc.resize((size_t)Mb);
      for (int64_t k = 0; k < Mb; ++k) {
        const uint32_t ix = (uint32_t)((h->cx[d0 + k] - x0) * sc), iy = (uint32_t)((h->cy[d0 + k] - y0) * sc);
        uint32_t z = 0;
        for (int bit = 0; bit < 16; ++bit)
          z |= (((ix >> bit) & 1u) << (2 * bit)) | (((iy >> bit) & 1u) << (2 * bit + 1));
        zc[(size_t)k] = z;
      }
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t u, int32_t w) {
      const int tu = (2 * h->N[u] + 16) / 16, tw = (2 * h->N[w] + 16) / 16;
      if (tu != tw) return tu > tw;
      return circ && zc[(size_t)(u - d0)] < zc[(size_t)(w - d0)];
    });
    for (int64_t o = 0; o < Mb; o += c.RP) {
      const int rp = (int)std::min<int64_t>(c.RP, Mb - o);
      const int gi = (int)S.gnseg.size();
      for (int k = 0; k < c.RP; ++k) {
        const int32_t pk = k < rp ? ord[(size_t)(o + k)] : -1;
        S.grow.push_back(pk);
        if (pk >= 0) {
          S.dgrp[pk] = gi;
          S.drow[pk] = k;
        }
      }
      double rows = 0.0;
      for (int k = 0; k < rp; ++k) rows += 2 * h->N[ord[(size_t)(o + k)]] + 1;
      // column disks of the group: a contiguous range, or the list of the
      // close pairs of its rows (with the mask of the rows close to each)
      int64_t ncol = Mb, lbase = 0;
      std::vector<double> lw;  // column widths of the list entries
      if (circ && S.close_rows) {
        ncol = 0;  // k_apply_close writes segment 0 of every tile
      } else if (circ) {
        std::map<int32_t, int> mask;
        for (int k = 0; k < rp; ++k) {
          const int32_t pk = ord[(size_t)(o + k)];
          for (int64_t e = h->near_off[pk]; e < h->near_off[pk + 1]; ++e) mask[h->near[(size_t)e]] |= 1 << k;
        }
        lbase = (int64_t)S.qlist.size();
        for (const auto& kv : mask) {
          S.qlist.push_back((kv.first << 8) | kv.second);
          lw.push_back(2.0 * h->N[kv.first] + 1);
        }
        ncol = (int64_t)mask.size();
      }
      const int64_t qsg = circ ? (c.QS > 0 ? c.QS : std::max<int64_t>(ncol, 1)) : qs;
      const int nseg = (circ && S.close_rows) ? 1 : (int)((ncol + qsg - 1) / qsg);
      S.gnseg.push_back(nseg);
      S.gbase.push_back(pb);
      for (int t = 0; t < S.ntile; ++t) {
        if (!tile_runs(b, t * RC, (t + 1) * RC)) continue;
        for (int sg = 0; sg < (circ && S.close_rows ? 0 : nseg); ++sg) {
          const int64_t i0 = sg * qsg, i1 = std::min<int64_t>(ncol, i0 + qsg);
          double cw = 0.0;
          for (int64_t i = i0; i < i1; ++i) cw += circ ? lw[(size_t)i] : 2.0 * h->N[d0 + i] + 1;
          It e;
          e.cost = rows * cw + 64.0 * (double)(i1 - i0);  // MACs + per-disk staging
          e.r[0] = gi;
          e.r[1] = rp;
          e.r[2] = t;
          e.r[3] = (int32_t)((circ ? lbase : d0) + i0);
          e.r[4] = (int32_t)((circ ? lbase : d0) + i1);
          e.r[5] = (int32_t)(pb + (int64_t)t * nseg + sg);
          e.r[6] = circ ? 1 : 0;
          its.push_back(e);
        }
      }
      pb += (int64_t)S.ntile * nseg;
    }
    if (circ) {  // per-frequency products: (instance, frequency, row tile, column tile)
      const int Lb = h->cL[b];
      const int nrt = (int)((Mb + cbm - 1) / cbm), nct = (R + cbn - 1) / cbn;
      for (int f = 0; f < Lb; ++f)
        for (int rt = 0; rt < nrt; ++rt)
          for (int ct = 0; ct < nct; ++ct) {
            if (!tile_runs(b, ct * cbn, (ct + 1) * cbn)) continue;
            S.citems.push_back(b);
            S.citems.push_back(f);
            S.citems.push_back(rt);
            S.citems.push_back(ct);
          }
    }
  }
  S.n_pb = pb;
  if (S.close_rows) {
    S.nptr.assign((size_t)h->M_all + 1, 0);
    std::vector<int64_t> work((size_t)h->M_all, 0);  // k steps x row tiles of each row's list
    for (int p = 0; p < h->M_all; ++p) {
      if (S.con[(size_t)h->inst[p]])
        for (int64_t e = h->near_off[p]; e < h->near_off[p + 1]; ++e) {
          const int32_t q = h->near[(size_t)e];
          S.nq.push_back(q);
          work[(size_t)p] += (int64_t)((2 * h->N[q] + 4) / 4) * ((2 * h->N[p] + 16) / 16);
        }
      S.nptr[(size_t)p + 1] = (int32_t)S.nq.size();
    }
    S.rord.resize((size_t)h->M_all);
    for (int p = 0; p < h->M_all; ++p) S.rord[(size_t)p] = p;
    std::stable_sort(S.rord.begin(), S.rord.end(),
                     [&](int32_t u, int32_t w) { return work[(size_t)u] > work[(size_t)w]; });
  }
  std::stable_sort(its.begin(), its.end(), [](const It& a, const It& b) { return a.cost > b.cost; });
  S.items.resize(its.size() * MF_REC);
  for (size_t k = 0; k < its.size(); ++k)
    for (int f = 0; f < MF_REC; ++f) S.items[k * MF_REC + f] = its[k].r[f];
  S.n_items = (int)its.size();
  S.n_citems = (int)(S.citems.size() / 4);
}

// Byte layout of the MFMA schedule inside the apply scratch:
// [head][items][dgrp][grow][gnseg][gbase][partial blocks][scaled input][drow]
// [qlist][product items][con][transformed inputs][transformed outputs]
#define MF_NOFF 17
static size_t mfma_scratch_layout(const mudiff_ctx* h, const MfmaSched& S, size_t* off) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  off[0] = take(4);
  off[1] = take(S.items.size() * 4);
  off[2] = take((size_t)h->M_all * 4);
  off[3] = take(S.grow.size() * 4);
  off[4] = take(S.gnseg.size() * 4);
  off[5] = take(S.gbase.size() * 8);
  off[6] = take((size_t)S.n_pb * S.blk * 16);
  off[7] = take((size_t)S.R * h->N_all * 16);  // the input with its column scale applied
  off[8] = take((size_t)h->M_all * 4);
  off[9] = take(S.qlist.size() * 4);
  off[10] = take(S.citems.size() * 4);
  off[11] = take((size_t)h->B * 4);
  const size_t zw = S.c.circ ? (size_t)S.R * h->cZ_all * 16 : 0;
  off[12] = take(zw);
  off[13] = take(zw);
  off[14] = take(S.nptr.size() * 4);  // close lists of the 8-column tiles
  off[15] = take(S.nq.size() * 4);
  off[16] = take(S.rord.size() * 4);
  return o;
}

// Candidate tile choices for R right-hand sides (RP * CT waves of 64 lanes).
static std::vector<MfmaChoice> mfma_candidates(int R) {
  std::vector<MfmaChoice> out;
  const int ctmax = std::max(1, std::min(4, (R + 7) / 8));
  for (int waves : {4, 8})
    for (int ct : {1, 2, 4}) {
      if (ct > ctmax && ct > 1) continue;
      const int rp = waves / ct;
      if (rp < 1 || rp > 8) continue;
      for (int qs : {0, 32}) out.push_back(MfmaChoice{ct, rp, qs, 64 * waves, false});
    }
  return out;
}

// The circulant form is a candidate when the tables hold it and some
// instance is worth it (and the caller has not switched it off for R).
static bool circ_usable(const mudiff_ctx* h, int R) {
  if (!h->circ || h->M_all >= (1 << 23)) return false;  // column lists hold q << 8
  auto f = h->circ_modes.find(R);
  if (f != h->circ_modes.end() && f->second == 0) return false;
  for (uint8_t c : h->circ_on)
    if (c) return true;
  return false;
}

static MfmaChoice mfma_default(int R) {
  const int ct0 = std::min(4, (R + 7) / 8);
  const int ct = ct0 == 3 ? 4 : ct0;
  return MfmaChoice{ct, 4 / ct, 0, 256, false};
}

void sched_wait(mudiff_ctx* h) {
  if (h->sched_pending) {
    (void)hipEventSynchronize(h->sched_ev);
    h->sched_pending = false;
  }
}

// Upload schedule S into the apply scratch at `base`, asynchronously: the
// host vectors of S stay untouched until sched_wait (S = the handle's
// schedule) or a synchronisation of the stream (a local S).  Not for use under
// graph capture.
static int mfma_upload(mudiff_ctx* h, MfmaSched& S, char* base, hipStream_t s) {
  size_t off[MF_NOFF];
  mfma_scratch_layout(h, S, off);
  if (!S.qlist.empty())
    HIP_TRY(hipMemcpyAsync(base + off[9], S.qlist.data(), S.qlist.size() * 4, hipMemcpyHostToDevice, s));
  if (!S.citems.empty())
    HIP_TRY(hipMemcpyAsync(base + off[10], S.citems.data(), S.citems.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + off[11], S.con.data(), (size_t)h->B * 4, hipMemcpyHostToDevice, s));
  if (!S.nptr.empty())
    HIP_TRY(hipMemcpyAsync(base + off[14], S.nptr.data(), S.nptr.size() * 4, hipMemcpyHostToDevice, s));
  if (!S.nq.empty())
    HIP_TRY(hipMemcpyAsync(base + off[15], S.nq.data(), S.nq.size() * 4, hipMemcpyHostToDevice, s));
  if (!S.rord.empty())
    HIP_TRY(hipMemcpyAsync(base + off[16], S.rord.data(), S.rord.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + off[1], S.items.data(), S.items.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + off[2], S.dgrp.data(), (size_t)h->M_all * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + off[3], S.grow.data(), S.grow.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + off[8], S.drow.data(), (size_t)h->M_all * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + off[4], S.gnseg.data(), S.gnseg.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + off[5], S.gbase.data(), S.gbase.size() * 8, hipMemcpyHostToDevice, s));
  if (!h->sched_ev) HIP_TRY(hipEventCreateWithFlags(&h->sched_ev, hipEventDisableTiming));
  if (S.c.circ && !h->aux) {
    HIP_TRY(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming));
  }
  HIP_TRY(hipEventRecord(h->sched_ev, s));
  h->sched_pending = true;
  S.dev_base = base;
  return MUDIFF_OK;
}

// Enqueue one MFMA apply with schedule S already uploaded at S.dev_base.
typedef void (*mf_fn)(DevView, int, const cplx*, const int32_t*, const int32_t*, int, int32_t*,
                      cplx*, int64_t, int, int, int, int, const int32_t*, const int32_t*);

#define MF_TK3(MT, TH, ZK)                                 \
  if (zk == ZK) {                                          \
    if (tk == 1) return k_apply_mfma<MT, TH, ZK, 1>;       \
    if (tk == 2) return k_apply_mfma<MT, TH, ZK, 2>;       \
    if (TH == 256 && tk == 4) return k_apply_mfma<MT, TH, ZK, 4>; \
  }
#define MF_MT(MT)                                                                   \
  if (mt == MT) {                                                                   \
    if (th == 512) { MF_TK3(MT, 512, 1) MF_TK3(MT, 512, 2) MF_TK3(MT, 512, 4) }     \
    if (th == 256) { MF_TK3(MT, 256, 1) MF_TK3(MT, 256, 2) MF_TK3(MT, 256, 4)       \
                     MF_TK3(MT, 256, 8) }                                           \
  }

// Kernel variant for MT row tiles, workgroup size th and staging sizes zk, tk
// (powers of two; at 512 threads zk <= 4, tk <= 2, at 256 zk <= 8, tk <= 4).
static mf_fn mf_select(int mt, int th, int zk, int tk) {
  MF_MT(1) MF_MT(2) MF_MT(3) MF_MT(4)
  return nullptr;
}
#undef MF_MT
#undef MF_TK3

static int mfma_launch(mudiff_ctx* h, const MfmaSched& S, const cplx* x, cplx* y, int op,
                       const int32_t* active, hipStream_t s, const cplx* shift = nullptr) {
  size_t off[MF_NOFF];
  mfma_scratch_layout(h, S, off);
  char* base = (char*)S.dev_base;
  int32_t* head = (int32_t*)(base + off[0]);
  cplx* part = (cplx*)(base + off[6]);
  const int mt = S.npad / 16;
  const int kt = (2 * h->Nmax + 1 + 3) / 4;
  const int RC = 8 * S.c.CT;
  const size_t lds = ((size_t)4 * kt * RC + (size_t)S.c.RP * (4 * kt + 16 * mt - 1)) * 16;
  prof_open(h, s);
  int rc = launch_fill_zero(head, 4, s);
  if (rc != MUDIFF_OK) return rc;
  cplx* z = (cplx*)(base + off[7]);
  int64_t nbmax = 0;  // longest instance vector
  for (int b = 0; b < h->B; ++b) nbmax = std::max(nbmax, h->imode[b + 1] - h->imode[b]);
  if ((nbmax + 255) / 256 > 65535) return fail(MUDIFF_ERR_INVALID, "instance too large for the input scaling grid");
  hipLaunchKernelGGL(k_apply_mfma_scale, dim3((unsigned)(h->B * S.R), (unsigned)((nbmax + 255) / 256)), dim3(256),
                     0, s, h->dv, S.R, x, z, active);
  HIP_TRY(hipGetLastError());
  prof_mark(h, s, 1);
  cplx* wh = nullptr;
  const int32_t* con = (const int32_t*)(base + off[11]);
  // direct-form work (the work queue and the close-pair rows): in the straggler
  // phase of a solve with the circulant form it runs on the second stream,
  // beside the transforms and products, which share none of its outputs (there
  // every launch is small and latency-bound; on a full batch the close-pair
  // waves would crowd the products and transforms out of the compute units)
  mf_fn fn = nullptr;  // checked before the fork, so that every error leaves the streams joined
  if (S.n_items > 0) {
    const int TL = 4 * kt + 16 * mt - 1;
    auto pow2 = [](int v) { int r = 1; while (r < v) r <<= 1; return r; };
    const int zk = pow2((4 * kt * RC + S.c.threads - 1) / S.c.threads);
    const int tk = pow2((S.c.RP * TL + S.c.threads - 1) / S.c.threads);
    fn = mf_select(mt, S.c.threads, zk, tk);
    if (!fn) return fail(MUDIFF_ERR_INVALID, "no MFMA apply variant for this tile");
  }
  if (S.close_rows && (mt < 1 || mt > 4)) return fail(MUDIFF_ERR_INVALID, "close pairs: orders out of range");
  hipStream_t cs = s;
  const bool fork = h->mfma_tail && S.c.circ && (S.n_items > 0 || S.close_rows) && h->aux;
  if (fork) {
    HIP_TRY(hipEventRecord(h->fork_ev, s));
    HIP_TRY(hipStreamWaitEvent(h->aux, h->fork_ev, 0));
    cs = h->aux;
  }
  auto launch_direct = [&]() -> int {
    if (S.n_items > 0) {
      const int32_t* it = (const int32_t*)(base + off[1]);
      // persistent grid: as many workgroups as are resident at once
      int per_cu = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, S.c.threads, lds) !=
              hipSuccess || per_cu < 1)
        per_cu = 1;
      const int grid = std::max(1, std::min(S.n_items, per_cu * h->n_cu));
      hipLaunchKernelGGL(fn, dim3(grid), dim3(S.c.threads), lds, cs, h->dv, S.R, (const cplx*)z, active, it,
                         S.n_items, head, part, S.blk, S.npad, kt, S.c.RP, S.c.CT,
                         (const int32_t*)(base + off[3]), (const int32_t*)(base + off[9]));
      HIP_TRY(hipGetLastError());
    }
    if (S.close_rows) {  // every row of the form writes its segment (zeros without close pairs)
      typedef void (*close_fn)(DevView, int, const cplx*, cplx*, int64_t, int, const int32_t*,
                               const int32_t*, const int64_t*, const int32_t*, const int32_t*,
                               const int32_t*, const int32_t*, const int32_t*);
      static const close_fn kClose[5] = {nullptr, k_apply_close<1, 1>, k_apply_close<2, 2>,
                                         k_apply_close<3, 2>, k_apply_close<4, 2>};
      const unsigned zg = mt > 2 ? 2u : 1u;  // groups of two row tiles
      hipLaunchKernelGGL(kClose[mt], dim3((unsigned)h->M_all, (unsigned)S.ntile, zg), dim3(64), 0, cs, h->dv,
                         S.R, (const cplx*)z, part, S.blk, S.npad, (const int32_t*)(base + off[2]),
                         (const int32_t*)(base + off[8]), (const int64_t*)(base + off[5]),
                         (const int32_t*)(base + off[14]), (const int32_t*)(base + off[15]), con, active,
                         (const int32_t*)(base + off[16]));
      HIP_TRY(hipGetLastError());
    }
    return MUDIFF_OK;
  };
  if (fork) {
    if ((rc = launch_direct()) != MUDIFF_OK) return rc;
    HIP_TRY(hipEventRecord(h->join_ev, cs));
  }
  if (S.c.circ) {  // well-separated pairs of the marked instances
    cplx* zh = (cplx*)(base + off[12]);
    wh = (cplx*)(base + off[13]);
    rc = circ_launch(h, S.R, z, zh, wh, (const int32_t*)(base + off[10]), S.n_citems, S.cvar, con,
                     S.con.data(), active, s);
    if (rc != MUDIFF_OK) return rc;
  } else {
    prof_mark(h, s, 2);
    prof_mark(h, s, 3);
  }
  if (fork) HIP_TRY(hipStreamWaitEvent(s, h->join_ev, 0));
  else if ((rc = launch_direct()) != MUDIFF_OK) return rc;
  prof_mark(h, s, 4);
  if (S.c.circ) {
    rc = circ_finish(h, S.R, x, y, op, (const cplx*)part, S.blk, S.npad, RC,
                     (const int32_t*)(base + off[2]), (const int32_t*)(base + off[8]),
                     (const int32_t*)(base + off[4]), (const int64_t*)(base + off[5]), active,
                     (const cplx*)wh, con, S.con.data(), shift, s);
    prof_mark(h, s, 5);
    return rc;
  }
  const int64_t total = (int64_t)S.R * h->N_all;
  hipLaunchKernelGGL(k_apply_mfma_finish, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     h->dv, S.R, x, y, op, (const cplx*)part, S.blk, S.npad, RC,
                     (const int32_t*)(base + off[2]), (const int32_t*)(base + off[8]),
                     (const int32_t*)(base + off[4]), (const int64_t*)(base + off[5]), active,
                     (const cplx*)wh, con, shift);
  HIP_TRY(hipGetLastError());
  prof_mark(h, s, 5);
  return MUDIFF_OK;
}

// Largest apply scratch any candidate choice needs for R.
static size_t mfma_scratch_bytes(mudiff_ctx* h, int R) {
  auto f = h->mfma_bytes.find(R);
  if (f != h->mfma_bytes.end()) return f->second;
  size_t mx = 0;
  for (MfmaChoice c : mfma_candidates(R)) {
    for (int circ = 0; circ < (h->circ ? 2 : 1); ++circ)
      for (int qs : {c.QS, MFMA_TAIL_QS}) {  // also the short-segment form used for stragglers
        c.QS = qs;
        c.circ = circ != 0;
        std::vector<int> vars = circ ? circ_variants(R) : std::vector<int>{-1};
        for (int cv : vars) {
          c.cvar = cv;
          MfmaSched S;
          mfma_build(h, R, c, S);
          size_t off[MF_NOFF];
          mx = std::max(mx, mfma_scratch_layout(h, S, off));
        }
      }
  }
  h->mfma_bytes[R] = mx;
  return mx;
}

// Pick the tile choice for R by timing every candidate on x -> y (outputs
// are overwritten; the inputs only need to be finite), then leave the chosen
// schedule uploaded at `scratch`.  Segmented candidates are skipped when no
// instance has more disks than a segment: their schedule is the unsegmented one.
static int mfma_autotune(mudiff_ctx* h, int R, const cplx* x, cplx* y, char* scratch,
                         hipStream_t s) {
  int64_t mmax = 0;
  for (int b = 0; b < h->B; ++b) mmax = std::max(mmax, h->idisk[b + 1] - h->idisk[b]);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best = 0.0f;
  MfmaChoice bc = mfma_default(R);
  int rc = MUDIFF_OK;
  std::vector<MfmaChoice> cands;
  auto fc = h->circ_modes.find(R);
  const int cmode = fc != h->circ_modes.end() ? fc->second : -1;
  const bool cu = circ_usable(h, R);
  if (cu)  // the circulant form first: it usually sets the bar the direct tiles then fail
    for (MfmaChoice c : mfma_candidates(R)) {
      c.circ = true;
      cands.push_back(c);
    }
  if (cmode != 1 || !cu)
    for (const MfmaChoice& c : mfma_candidates(R)) cands.push_back(c);
  // The direct form's work (8 flops per complex multiply-add over every
  // ordered pair) at the FP64 matrix-core peak, 78.6 TFLOP/s: no direct tile
  // beats it, so once a candidate's pair of applies is faster than twice that,
  // the direct tiles are not timed.
  double dflops = 0.0;
  for (int b = 0; b < h->B; ++b) {
    double sn = 0.0, sn2 = 0.0;
    for (int64_t p = h->idisk[b]; p < h->idisk[b + 1]; ++p) {
      const double n = 2.0 * h->N[(size_t)p] + 1.0;
      sn += n;
      sn2 += n * n;
    }
    dflops += 8.0 * R * (sn * sn - sn2);
  }
  const float direct_floor_ms = (float)(2.0 * dflops / 78.6e12 * 1e3);
  // one warm-up and two timed applies of candidate c; keeps the fastest (and
  // returns the time, 0 when skipped or failed)
  auto time_one = [&](const MfmaChoice& c) -> float {
    MfmaSched S;
    mfma_build(h, R, c, S);
    struct Drain {  // the local schedule's copies finish before it is released
      hipStream_t st;
      ~Drain() { (void)hipStreamSynchronize(st); }
    } drain{s};
    if ((rc = mfma_upload(h, S, scratch, s)) != MUDIFF_OK) return 0.0f;
    (void)hipEventRecord(e0, s);
    if ((rc = mfma_launch(h, S, x, y, MUDIFF_OP_A, nullptr, s)) != MUDIFF_OK) return 0.0f;  // warm-up
    (void)hipEventRecord(e1, s);
    if (best > 0.0f) {  // a warm-up already twice as slow as the best pair of applies: no contender
      float w = 0.0f;
      if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&w, e0, e1) == hipSuccess &&
          w > best)
        return 0.0f;
    }
    (void)hipEventRecord(e0, s);
    for (int k = 0; k < 2 && rc == MUDIFF_OK; ++k) rc = mfma_launch(h, S, x, y, MUDIFF_OP_A, nullptr, s);
    (void)hipEventRecord(e1, s);
    if (rc != MUDIFF_OK) return 0.0f;
    if (hipEventSynchronize(e1) != hipSuccess) {
      rc = fail(MUDIFF_ERR_DEVICE, "autotune: event synchronisation failed");
      return 0.0f;
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (best == 0.0f || ms < best) {
      best = ms;
      bc = c;
    }
    return ms;
  };
  for (const MfmaChoice& c : cands) {
    if (c.QS > 0 && mmax <= c.QS) continue;
    if (!c.circ && best > 0.0f && direct_floor_ms > best) continue;
    time_one(c);
    if (rc != MUDIFF_OK) break;
  }
  if (rc == MUDIFF_OK && bc.circ) {  // then the per-frequency product variants on that tile
    const MfmaChoice base = bc;
    std::vector<std::pair<float, MfmaChoice>> seen{{best, base}};
    for (int cv : circ_variants(R)) {
      if (cv == circ_variant(R)) continue;
      MfmaChoice c = base;
      c.cvar = cv;
      const float ms = time_one(c);
      if (rc != MUDIFF_OK) break;
      if (ms > 0.0f) seen.push_back({ms, c});
    }
    // variants a few percent apart swap places from one timing to the next:
    // the three fastest are timed three times more and ranked by their mean
    if (rc == MUDIFF_OK && seen.size() > 1) {
      std::stable_sort(seen.begin(), seen.end(),
                       [](const std::pair<float, MfmaChoice>& a, const std::pair<float, MfmaChoice>& b) {
                         return a.first < b.first;
                       });
      seen.resize(std::min<size_t>(seen.size(), 3));
      float bmean = 0.0f;
      MfmaChoice bbest = bc;
      for (const auto& sc : seen) {
        float sum = 0.0f;
        for (int rep = 0; rep < 3 && rc == MUDIFF_OK; ++rep) {
          best = 0.0f;  // time every repetition in full
          sum += time_one(sc.second);
        }
        if (rc != MUDIFF_OK) break;
        if (bmean == 0.0f || sum / 3.0f < bmean) {
          bmean = sum / 3.0f;
          bbest = sc.second;
        }
      }
      if (rc == MUDIFF_OK) {
        bc = bbest;
        best = bmean;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != MUDIFF_OK) return rc;
  h->mfma_choice[R] = bc;
  h->mfma_time_ms[R] = best / 2.0f;
  sched_wait(h);
  mfma_build(h, R, bc, h->mfma_sched);
  return mfma_upload(h, h->mfma_sched, scratch, s);
}

// Make the schedule for R current and uploaded at `scratch` (autotuning on
// first use of R when x, y are given, else the default choice).
static int mfma_prepare(mudiff_ctx* h, int R, const cplx* x, cplx* y, char* scratch,
                        hipStream_t s) {
  auto f = h->mfma_choice.find(R);
  if (f == h->mfma_choice.end()) {
    if (x && y && h->mfma_tune) return mfma_autotune(h, R, x, y, scratch, s);
    MfmaChoice d = mfma_default(R);
    d.circ = circ_usable(h, R);
    h->mfma_choice[R] = d;
    f = h->mfma_choice.find(R);
  }
  MfmaChoice c = f->second;
  if (h->mfma_tail) c.QS = MFMA_TAIL_QS;
  if (h->mfma_sched.R != R || !(h->mfma_sched.c == c)) {
    sched_wait(h);
    mfma_build(h, R, c, h->mfma_sched, h->mfma_tail ? h->mfma_tail_cols : std::vector<int32_t>{});
  }
  if (h->mfma_sched.dev_base != scratch) return mfma_upload(h, h->mfma_sched, scratch, s);
  return MUDIFF_OK;
}

int apply_set_tail(mudiff_ctx* h, int R, bool tail, cplx* scratch, hipStream_t s,
                   const int32_t* cols) {
  if (!use_mfma(h, R)) return MUDIFF_OK;
  if (!tail && !h->mfma_tail) return MUDIFF_OK;
  h->mfma_tail = tail;
  if (tail && cols) h->mfma_tail_cols.assign(cols, cols + (size_t)h->B * R);
  else h->mfma_tail_cols.clear();
  h->mfma_sched.R = 0;  // rebuild
  return mfma_prepare(h, R, nullptr, nullptr, (char*)scratch, s);
}

// ------------------------------------------------------------------ planning
namespace {
typedef void (*apply_fn)(DevView, int, const cplx*, cplx*, int, cplx*, int64_t, int32_t*,
                         const int32_t*, const int32_t*, const int64_t*, const int32_t*, int, int, int,
                         const cplx*);
typedef void (*lane_fn)(DevView, int, const cplx*, cplx*, int64_t, const int32_t*,
                        const int32_t*);

struct Variant {
  int bt, nspec;
  apply_fn fn;
};

// LDS-staged kernels: generic (nspec = -1) and uniform-N specialisations
const Variant kVariants[] = {
    {4, -1, k_apply<4, -1>}, {5, -1, k_apply<5, -1>}, {6, -1, k_apply<6, -1>},
    {8, -1, k_apply<8, -1>}, {5, 12, k_apply<5, 12>}, {4, 15, k_apply<4, 15>},
};

const Variant* find_variant(int bt, int nspec) {
  for (const Variant& v : kVariants)
    if (v.bt == bt && v.nspec == nspec) return &v;
  return nullptr;
}

struct LaneVariant {
  int n;
  lane_fn fn;     // single-layer column factors (real)
  lane_fn fn_op;  // column factors of an operator set by mudiff_set_operator
};

// one-lane-per-pair kernels (uniform N)
const LaneVariant kLane[] = {
    {1, k_apply_lane<1, false>, k_apply_lane<1, true>},
    {2, k_apply_lane<2, false>, k_apply_lane<2, true>},
    {3, k_apply_lane<3, false>, k_apply_lane<3, true>},
    {4, k_apply_lane<4, false>, k_apply_lane<4, true>},
    {5, k_apply_lane<5, false>, k_apply_lane<5, true>},
    {6, k_apply_lane<6, false>, k_apply_lane<6, true>},
    {7, k_apply_lane<7, false>, k_apply_lane<7, true>},
    {8, k_apply_lane<8, false>, k_apply_lane<8, true>},
    {9, k_apply_lane<9, false>, k_apply_lane<9, true>},
    {10, k_apply_lane<10, false>, k_apply_lane<10, true>},
    {11, k_apply_lane<11, false>, k_apply_lane<11, true>},
    {12, k_apply_lane<12, false>, k_apply_lane<12, true>},
};

const LaneVariant* find_lane(int n) {
  for (const LaneVariant& v : kLane)
    if (v.n == n) return &v;
  return nullptr;
}
}  // namespace

// Host plan of the operator apply: kernel variant, work items and partial-sum
// layout, from the batch description alone (also used to size workspaces).
struct PlanHost {
  int lane = 0;  // 1: one-lane-per-pair kernel (uniform N = nspec)
  int item_ints = 4;
  int waves = 1;
  int bt = 4, nspec = -1, zs = 0, ts = 0, ppcap = 1;
  size_t lds = 0;
  int64_t part = 0;
  std::vector<int32_t> items, nch;
  std::vector<int64_t> poff;
};

// The uniform-N specialisation when every disk has the same N and one is
// compiled, else the generic kernel with BT = 4.
static void choose_variant(int M, const int32_t* N, int* bt, int* nspec) {
  bool uniform = true;
  for (int p = 1; p < M; ++p)
    if (N[p] != N[0]) uniform = false;
  if (uniform) {
    for (const Variant& v : kVariants)
      if (v.nspec == N[0]) {
        *bt = v.bt;
        *nspec = v.nspec;
        return;
      }
  }
  *bt = 4;
  *nspec = -1;
}

#define APPLY_LDS_BUDGET (64 * 1024)

void make_plan(int B, const int64_t* idisk, const int32_t* N, PlanHost& P) {
  const int M = (int)idisk[B];
  P.items.clear();
  P.nch.assign(M, 0);
  P.poff.assign(M, 0);
  P.part = 0;
  P.lds = 0;
  bool uniform = true;
  for (int p = 1; p < M; ++p)
    if (N[p] != N[0]) uniform = false;
  if (uniform && N[0] <= LANE_NMAX && find_lane(N[0])) {
    P.lane = 1;
    P.item_ints = LANE_ITEM_INTS;
    P.nspec = N[0];
    const int np = 2 * N[0] + 1;
    int lane_N = -1;
    std::vector<int64_t> ltoff;
    lane_layout(B, idisk, N, &lane_N, &ltoff);
    auto push64 = [&](int64_t v) {
      P.items.push_back((int32_t)(v & 0xffffffff));
      P.items.push_back((int32_t)(v >> 32));
    };
    int64_t i0 = 0;  // first unknown of instance b
    for (int b = 0; b < B; ++b) {
      const int64_t d0 = idisk[b], Mb = idisk[b + 1] - d0;
      const int64_t n = (Mb - 1 + LANE_CHUNK - 1) / LANE_CHUNK;  // 0 for M = 1
      for (int64_t p = d0; p < d0 + Mb; ++p) {
        P.nch[p] = (int32_t)n;
        P.poff[p] = P.part;
        P.part += std::max<int64_t>(n, 1) * np;
        for (int64_t c = 0; c < n; ++c) {
          const int64_t jb = c * LANE_CHUNK, je = std::min<int64_t>(jb + LANE_CHUNK, Mb - 1);
          P.items.push_back((int32_t)p);
          P.items.push_back((int32_t)c);
          P.items.push_back((int32_t)jb);
          P.items.push_back((int32_t)je);
          P.items.push_back(b);
          P.items.push_back((int32_t)d0);
          push64(i0);
          push64(Mb * np);
          push64(ltoff[p] + c * (int64_t)(LANE_CHUNK * LANE_REC));
          push64(P.poff[p] + c * np);
          push64(0);
        }
      }
      i0 += Mb * np;
    }
    return;
  }
  P.lane = 0;
  choose_variant(M, N, &P.bt, &P.nspec);
  const int bt = P.bt;
  int nmax = 0;
  for (int p = 0; p < M; ++p) nmax = std::max(nmax, (int)N[p]);
  // LDS rows: z stride zs (padded to BT), symbol rows ts = zs + LB_max - 1
  P.zs = ((2 * nmax + 1) + bt - 1) / bt * bt;
  P.ts = P.zs + P.zs - 1;
  P.ppcap = std::max(1, (int)(APPLY_LDS_BUDGET / ((size_t)(P.zs + P.ts) * 16)));
  for (int b = 0; b < B; ++b) {
    const int64_t d0 = idisk[b], Mb = idisk[b + 1] - d0;
    for (int64_t p = d0; p < d0 + Mb; ++p) {
      const int np = 2 * N[p] + 1;
      const int L = (np + bt - 1) / bt;
      const int pp = std::max(1, std::min(APPLY_THREADS / L, P.ppcap));
      const int64_t qc = (int64_t)pp * APPLY_NPASS;
      const int64_t n = std::max<int64_t>(1, (Mb - 1 + qc - 1) / qc);
      P.nch[p] = (int32_t)n;
      P.poff[p] = P.part;
      P.part += n * np;
      for (int64_t c = 0; c < n; ++c) {
        int64_t jb = c * qc, je = std::min<int64_t>(jb + qc, Mb - 1);
        P.items.push_back((int32_t)p);
        P.items.push_back((int32_t)c);
        P.items.push_back((int32_t)jb);
        P.items.push_back((int32_t)je);
      }
      P.lds = std::max(P.lds, (size_t)pp * (P.zs + P.ts) * 16);
      P.lds = std::max(P.lds, (size_t)pp * L * bt * 16);
    }
  }
}

size_t plan_sched_bytes(const PlanHost& P, int M) {
  return align256(P.items.size() * 4) + align256((size_t)M * 4) + align256((size_t)M * 8) + 256;
}

size_t sched_bytes_for(int B, const int64_t* disk_off, const int32_t* n_modes) {
  PlanHost H;
  make_plan(B, disk_off, n_modes, H);
  return plan_sched_bytes(H, (int)disk_off[B]);
}

int ensure_plan(mudiff_ctx* h, hipStream_t s) {
  if (h->plan.ready) return MUDIFF_OK;
  PlanHost H;
  make_plan(h->B, h->idisk.data(), h->N.data(), H);
  if (H.lds > 64 * 1024) return fail(MUDIFF_ERR_INVALID, "operator rows too long for LDS");
  if (plan_sched_bytes(H, h->M_all) > h->sched_bytes)
    return fail(MUDIFF_ERR_INVALID, "schedule area too small");
  MatvecPlan& P = h->plan;
  P.d_items = (int32_t*)h->sched_base;
  P.d_nchunk = (int32_t*)(h->sched_base + align256(H.items.size() * 4));
  P.d_partoff = (int64_t*)((char*)P.d_nchunk + align256(h->M_all * 4));
  if (!H.items.empty())
    HIP_TRY(hipMemcpyAsync(P.d_items, H.items.data(), H.items.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(P.d_nchunk, H.nch.data(), h->M_all * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(P.d_partoff, H.poff.data(), h->M_all * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));  // the host vectors are released on return
  P.lane = H.lane;
  P.Bt = H.bt;
  P.spec_N = H.nspec;
  P.zs = H.zs;
  P.ts = H.ts;
  P.ppcap = H.ppcap;
  P.part_total = H.part;
  P.lds_bytes = H.lds;
  P.n_items = (int)(H.items.size() / H.item_ints);
  P.waves = H.waves;
  P.ready = true;
  return MUDIFF_OK;
}

// Apply scratch: the partial sums (or the MFMA schedule and partial blocks),
// then R * M_all counters of the generic kernel.
size_t apply_scratch_bytes(mudiff_ctx* h, int R) {
  const size_t counters = align256((size_t)R * h->M_all * 4);
  if (use_mfma(h, R)) return align256(mfma_scratch_bytes(h, R)) + counters;
  if (h->plan_part < 0) {
    PlanHost H;
    make_plan(h->B, h->idisk.data(), h->N.data(), H);
    h->plan_part = H.part;
  }
  return align256((size_t)R * h->plan_part * 16) + counters;
}

void apply_forget_upload(mudiff_ctx* h) { h->mfma_sched.dev_base = nullptr; }

int prepare_apply(mudiff_ctx* h, int R, const cplx* x, cplx* y, cplx* scratch, hipStream_t s) {
  if (use_mfma(h, R)) return mfma_prepare(h, R, x, y, (char*)scratch, s);
  return ensure_plan(h, s);
}

int apply_operator_split(mudiff_ctx* h, int R, const cplx* x, cplx* y, int op, cplx* part,
                         int32_t* counters, const int32_t* active, hipStream_t s,
                         bool* pending) {
  *pending = false;
  if (use_mfma(h, R)) return apply_operator(h, R, x, y, op, part, counters, active, s);
  int st = ensure_plan(h, s);
  if (st != MUDIFF_OK) return st;
  const MatvecPlan& P = h->plan;
  if (P.lane) {
    const LaneVariant* lv = find_lane(P.spec_N);
    if (!lv) return fail(MUDIFF_ERR_INVALID, "no operator kernel variant");
    if (P.n_items > 0) {
      hipLaunchKernelGGL(h->dv.op_col ? lv->fn_op : lv->fn, dim3(P.n_items, R), dim3(64), 0, s,
                         h->dv, R, x, part, P.part_total, P.d_items, active);
      HIP_TRY(hipGetLastError());
    }
    *pending = true;  // the chunk sums still have to be added and finalised
    return MUDIFF_OK;
  }
  return apply_operator(h, R, x, y, op, part, counters, active, s);
}

int apply_operator(mudiff_ctx* h, int R, const cplx* x, cplx* y, int op, cplx* part,
                   int32_t* counters, const int32_t* active, hipStream_t s, const cplx* shift) {
  if (use_mfma(h, R)) {
    int st = mfma_prepare(h, R, nullptr, nullptr, (char*)part, s);  // no-op when current
    if (st != MUDIFF_OK) return st;
    return mfma_launch(h, h->mfma_sched, x, y, op, active, s, shift);
  }
  int st = ensure_plan(h, s);
  if (st != MUDIFF_OK) return st;
  const MatvecPlan& P = h->plan;
  prof_open(h, s);
  prof_mark(h, s, 1);
  prof_mark(h, s, 2);
  prof_mark(h, s, 3);
  if (P.lane) {
    const LaneVariant* lv = find_lane(P.spec_N);
    if (!lv) return fail(MUDIFF_ERR_INVALID, "no operator kernel variant");
    if (P.n_items > 0) {
      hipLaunchKernelGGL(h->dv.op_col ? lv->fn_op : lv->fn, dim3(P.n_items, R), dim3(64), 0, s,
                         h->dv, R, x, part, P.part_total, P.d_items, active);
      HIP_TRY(hipGetLastError());
    }
    prof_mark(h, s, 4);
    const int64_t total = (int64_t)R * h->N_all;
    hipLaunchKernelGGL(k_apply_finish, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       h->dv, R, x, y, op, (const cplx*)part, P.part_total, P.d_nchunk,
                       P.d_partoff, active, shift);
    HIP_TRY(hipGetLastError());
    prof_mark(h, s, 5);
    return MUDIFF_OK;
  }
  const Variant* var = find_variant(P.Bt, P.spec_N);
  if (!var) return fail(MUDIFF_ERR_INVALID, "no operator kernel variant");
  hipLaunchKernelGGL(var->fn, dim3(P.n_items, R), dim3(APPLY_THREADS), P.lds_bytes, s, h->dv, R, x,
                     y, op, part, P.part_total, counters, P.d_items, P.d_nchunk, P.d_partoff, active,
                     P.zs, P.ts, P.ppcap, shift);
  HIP_TRY(hipGetLastError());
  prof_mark(h, s, 4);
  prof_mark(h, s, 5);
  return MUDIFF_OK;
}

namespace {
// Mode flip P (x^p_m -> x^p_{-m} in every disk) of R columns: out = P in, or
// in place when out == in (one thread per pair m > 0 then).  L^T = P L P.
__global__ void k_flip_modes(DevView v, int R, const cplx* in, cplx* out) {
  const int64_t total = (int64_t)R * v.N_all;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  int lo = 0, hi = v.B;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)R * v.imode[mid] <= g) lo = mid; else hi = mid;
  }
  const int64_t Nb = v.imode[lo + 1] - v.imode[lo];
  const int64_t rem = g - (int64_t)R * v.imode[lo];
  const int64_t il = rem - (rem / Nb) * Nb;
  const int p = v.udisk[v.imode[lo] + il];
  const int64_t m = il - v.moff[p] - v.N[p];
  const int64_t g2 = g - 2 * m;  // mode -m of the same disk and column
  if (in != out) {
    out[g] = in[g2];
  } else if (m > 0) {
    const cplx a = out[g];
    out[g] = out[g2];
    out[g2] = a;
  }
}
}  // namespace

extern "C" size_t mudiff_matvec_workspace_size(mudiff_t h, int R) {
  if (!h || R < 1) return 0;
  // apply scratch, then room for the flipped input of MUDIFF_OP_LT
  return apply_scratch_bytes(h, R) + align256((size_t)R * h->N_all * 16);
}

extern "C" int mudiff_matvec(mudiff_t h, int R, const void* x, void* y, int op, void* workspace,
                             size_t ws_bytes, void* stream) {
  if (!h || !x || !y) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  if (R < 1) return fail(MUDIFF_ERR_INVALID, "R < 1");
  if (x == y) return fail(MUDIFF_ERR_INVALID, "x and y must be distinct buffers");
  if (op != MUDIFF_OP_L && op != MUDIFF_OP_A && op != MUDIFF_OP_LT)
    return fail(MUDIFF_ERR_INVALID, "unknown op");
  if (op == MUDIFF_OP_LT && h->dv.op_col)
    return fail(MUDIFF_ERR_INVALID, "MUDIFF_OP_LT applies the single layer only (reset the operator first)");
  const size_t need = apply_scratch_bytes(h, R);
  const size_t need_all = mudiff_matvec_workspace_size(h, R);
  if (!workspace) return fail(MUDIFF_ERR_INVALID, "workspace is NULL");
  if (ws_bytes < (op == MUDIFF_OP_LT ? need_all : need))
    return fail(MUDIFF_ERR_NOMEM, "matvec workspace needs " + std::to_string(need_all) + " bytes");
  apply_forget_upload(h);
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)workspace;
  const cplx* xin = (const cplx*)x;
  const int64_t tot = (int64_t)R * h->N_all;
  const unsigned fb = (unsigned)((tot + 255) / 256);
  if (op == MUDIFF_OP_LT) {  // L^T x = P L (P x)
    cplx* xf = (cplx*)(w + need);
    hipLaunchKernelGGL(k_flip_modes, dim3(fb), dim3(256), 0, s, h->dv, R, xin, xf);
    HIP_TRY(hipGetLastError());
    xin = xf;
  }
  const int aop = op == MUDIFF_OP_LT ? MUDIFF_OP_L : op;
  int rc;
  if (use_mfma(h, R)) {
    rc = mfma_prepare(h, R, xin, (cplx*)y, w, s);  // autotunes on first use of R
    if (rc == MUDIFF_OK) rc = mfma_launch(h, h->mfma_sched, xin, (cplx*)y, aop, nullptr, s);
  } else {
    size_t part_bytes = need - align256((size_t)R * h->M_all * 4);
    int32_t* counters = (int32_t*)(w + part_bytes);  // zero on first use, left zero
    rc = apply_operator(h, R, xin, (cplx*)y, aop, (cplx*)w, counters, nullptr, s);
  }
  if (rc != MUDIFF_OK || op != MUDIFF_OP_LT) return rc;
  hipLaunchKernelGGL(k_flip_modes, dim3(fb), dim3(256), 0, s, h->dv, R, (const cplx*)y, (cplx*)y);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}

extern "C" int mudiff_apply_config(mudiff_t h, int R, int* kind, int* ct, int* rp, int* qs,
                                   int* threads, float* ms) {
  if (!h) return fail(MUDIFF_ERR_INVALID, "NULL handle");
  if (R < 1) return fail(MUDIFF_ERR_INVALID, "R < 1");
  int k = 2, c = 0, r = 0, q = 0, t = 0;
  float tm = 0.0f;
  if (use_mfma(h, R)) {
    k = 1;
    auto f = h->mfma_choice.find(R);
    MfmaChoice ch = f != h->mfma_choice.end() ? f->second : mfma_default(R);
    if (f == h->mfma_choice.end()) ch.circ = circ_usable(h, R);
    if (ch.circ) k = 3;
    c = ch.CT;
    r = ch.RP;
    q = ch.QS;
    t = ch.threads;
    auto g = h->mfma_time_ms.find(R);
    if (g != h->mfma_time_ms.end()) tm = g->second;
  } else {
    PlanHost H;
    make_plan(h->B, h->idisk.data(), h->N.data(), H);
    k = H.lane ? 0 : 2;
  }
  if (kind) *kind = k;
  if (ct) *ct = c;
  if (rp) *rp = r;
  if (qs) *qs = q;
  if (threads) *threads = t;
  if (ms) *ms = tm;
  return MUDIFF_OK;
}

extern "C" int mudiff_set_apply_config(mudiff_t h, int R, int ct, int rp, int qs, int threads) {
  if (!h) return fail(MUDIFF_ERR_INVALID, "NULL handle");
  if (R < 1) return fail(MUDIFF_ERR_INVALID, "R < 1");
  if (!use_mfma(h, R)) return fail(MUDIFF_ERR_INVALID, "this apply does not run on MFMA");
  MfmaChoice want{ct, rp, qs, threads, false};
  for (const MfmaChoice& c : mfma_candidates(R))
    if (c == want) {
      auto f = h->circ_modes.find(R);
      want.circ = circ_usable(h, R) && (f == h->circ_modes.end() || f->second != 0);
      h->mfma_choice[R] = want;
      h->mfma_time_ms.erase(R);
      return MUDIFF_OK;
    }
  return fail(MUDIFF_ERR_INVALID, "MFMA tile not among the candidates");
}

extern "C" int mudiff_set_circulant(mudiff_t h, int R, int mode) {
  if (!h) return fail(MUDIFF_ERR_INVALID, "NULL handle");
  if (R < 1) return fail(MUDIFF_ERR_INVALID, "R < 1");
  if (mode < -1 || mode > 1) return fail(MUDIFF_ERR_INVALID, "mode must be -1, 0 or 1");
  if (!h->circ) return fail(MUDIFF_ERR_INVALID, "the handle was built without MUDIFF_TABLES_CIRCULANT");
  h->circ_modes[R] = mode;
  auto f = h->mfma_choice.find(R);
  if (f != h->mfma_choice.end()) {
    if (h->mfma_time_ms.count(R)) {  // timed choice: time again with the new mode
      h->mfma_choice.erase(f);
      h->mfma_time_ms.erase(R);
    } else {  // fixed tile: keep it, switch the form
      f->second.circ = mode != 0 && circ_usable(h, R);
    }
  }
  if (h->mfma_sched.R == R) h->mfma_sched.R = 0;  // rebuild at the next apply
  return MUDIFF_OK;
}

extern "C" int mudiff_circulant_tile(mudiff_t h, int R, int* rows, int* cols, int* kstep,
                                     int* stages, int* threads, int* mults) {
  if (!h) return fail(MUDIFF_ERR_INVALID, "NULL handle");
  if (R < 1) return fail(MUDIFF_ERR_INVALID, "R < 1");
  int bm = 0, bn = 0, bk = 0, db = 0, nt = 0, mu = 0;
  if (use_mfma(h, R)) {
    auto f = h->mfma_choice.find(R);
    MfmaChoice ch = f != h->mfma_choice.end() ? f->second : mfma_default(R);
    if (f == h->mfma_choice.end()) ch.circ = circ_usable(h, R);
    if (ch.circ) circ_var_dims(ch.cvar >= 0 ? ch.cvar : circ_variant(R), &bm, &bn, &bk, &db, &nt, &mu);
  }
  if (rows) *rows = bm;
  if (cols) *cols = bn;
  if (kstep) *kstep = bk;
  if (stages) *stages = db;
  if (threads) *threads = nt;
  if (mults) *mults = mu;
  return MUDIFF_OK;
}

extern "C" int mudiff_set_circulant_tile(mudiff_t h, int R, int rows, int cols, int kstep,
                                         int stages, int threads, int mults) {
  if (!h) return fail(MUDIFF_ERR_INVALID, "NULL handle");
  if (R < 1) return fail(MUDIFF_ERR_INVALID, "R < 1");
  if (!use_mfma(h, R) || !circ_usable(h, R))
    return fail(MUDIFF_ERR_INVALID, "this apply does not use the circulant form");
  for (int v : circ_variants(R)) {
    int bm, bn, bk, db, nt, mu;
    circ_var_dims(v, &bm, &bn, &bk, &db, &nt, &mu);
    if (bm == rows && bn == cols && bk == kstep && db == stages && nt == threads && mu == mults) {
      auto f = h->mfma_choice.find(R);
      MfmaChoice ch = f != h->mfma_choice.end() ? f->second : mfma_default(R);
      ch.circ = true;
      ch.cvar = v;
      h->mfma_choice[R] = ch;
      h->mfma_time_ms.erase(R);
      h->circ_modes[R] = 1;
      if (h->mfma_sched.R == R) h->mfma_sched.R = 0;
      return MUDIFF_OK;
    }
  }
  return fail(MUDIFF_ERR_INVALID, "product tile not among the candidates for this R");
}

// ------------------------------------------------------------------ phase timing
void prof_open(mudiff_ctx* h, hipStream_t s) {
  h->prof_cur = -1;
  if (h->prof_n >= h->prof_max) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  h->prof_cur = h->prof_n++;
  (void)hipEventRecord(h->prof_ev[(size_t)h->prof_cur * (MUDIFF_N_PHASES + 1)], s);
}

void prof_mark(mudiff_ctx* h, hipStream_t s, int k) {
  if (h->prof_cur < 0) return;
  (void)hipEventRecord(h->prof_ev[(size_t)h->prof_cur * (MUDIFF_N_PHASES + 1) + k], s);
  if (k == MUDIFF_N_PHASES) h->prof_cur = -1;
}

static void prof_release(mudiff_ctx* h) {
  for (hipEvent_t e : h->prof_ev) (void)hipEventDestroy(e);
  h->prof_ev.clear();
  h->prof_max = h->prof_n = 0;
  h->prof_cur = -1;
}

extern "C" int mudiff_profile_begin(mudiff_t h, int max_applies) {
  if (!h) return fail(MUDIFF_ERR_INVALID, "NULL handle");
  if (max_applies < 1 || max_applies > 100000) return fail(MUDIFF_ERR_INVALID, "max_applies out of range");
  prof_release(h);
  h->prof_ev.resize((size_t)max_applies * (MUDIFF_N_PHASES + 1));
  for (size_t k = 0; k < h->prof_ev.size(); ++k) {
    if (hipEventCreate(&h->prof_ev[k]) != hipSuccess) {
      h->prof_ev.resize(k);
      prof_release(h);
      return fail(MUDIFF_ERR_DEVICE, "hipEventCreate failed");
    }
  }
  h->prof_max = max_applies;
  return MUDIFF_OK;
}

extern "C" int mudiff_profile_end(mudiff_t h, int* n_applies, double* ms) {
  if (!h || !n_applies || !ms) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  for (int k = 0; k < MUDIFF_N_PHASES; ++k) ms[k] = 0.0;
  *n_applies = h->prof_n;
  if (h->prof_n > 0) {
    const hipEvent_t last = h->prof_ev[(size_t)(h->prof_n - 1) * (MUDIFF_N_PHASES + 1) + MUDIFF_N_PHASES];
    if (hipEventSynchronize(last) != hipSuccess) {
      prof_release(h);
      return fail(MUDIFF_ERR_DEVICE, "profile: event synchronisation failed");
    }
    for (int a = 0; a < h->prof_n; ++a)
      for (int k = 0; k < MUDIFF_N_PHASES; ++k) {
        float t = 0.0f;
        const size_t b = (size_t)a * (MUDIFF_N_PHASES + 1);
        if (hipEventElapsedTime(&t, h->prof_ev[b + k], h->prof_ev[b + k + 1]) == hipSuccess) ms[k] += t;
      }
  }
  prof_release(h);
  return MUDIFF_OK;
}

// ------------------------------------------------------------------ no-allocation apply
// Apply scratch of mudiff_matvec_noalloc: a file-scope device array, one copy
// per device, held until the process ends.  Host code never hands the array's
// name to a kernel (on the host it is only a stand-in for the symbol): its
// device address comes from hipGetSymbolAddress, once per device.
#define NOALLOC_SCRATCH_BYTES ((size_t)MUDIFF_NOALLOC_SCRATCH_MB << 20)
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, char*> g_scratch_ptr;  // device -> address of its copy of scratch

static int scratch_address(char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto f = g_scratch_ptr.find(dev);
  if (f != g_scratch_ptr.end()) {
    *out = f->second;
    return MUDIFF_OK;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(MUDIFF_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[dev] = (char*)ptr;
  *out = (char*)ptr;
  return MUDIFF_OK;
}

extern "C" int mudiff_matvec_noalloc(mudiff_t h, int R, const void* x, void* y, int op,
                                     void* stream) {
  if (!h || !x || !y) return fail(MUDIFF_ERR_INVALID, "NULL argument");
  if (R < 1) return fail(MUDIFF_ERR_INVALID, "R < 1");
  if (x == y) return fail(MUDIFF_ERR_INVALID, "x and y must be distinct buffers");
  if (op != MUDIFF_OP_L && op != MUDIFF_OP_A && op != MUDIFF_OP_LT)
    return fail(MUDIFF_ERR_INVALID, "unknown op");
  if (op == MUDIFF_OP_LT && h->dv.op_col)
    return fail(MUDIFF_ERR_INVALID, "MUDIFF_OP_LT applies the single layer only (reset the operator first)");
  if (use_mfma(h, R))
    return fail(MUDIFF_ERR_INVALID, "the no-allocation apply covers the one-lane and generic kernels "
                                    "(R < 8, or N_p > 31); use mudiff_matvec");
  if (!h->plan.ready) return fail(MUDIFF_ERR_INVALID, "no operator plan for this handle");
  const size_t need = apply_scratch_bytes(h, R);
  const size_t flip = op == MUDIFF_OP_LT ? align256((size_t)R * h->N_all * 16) : 0;
  if (need + flip > NOALLOC_SCRATCH_BYTES)
    return fail(MUDIFF_ERR_NOMEM, "the no-allocation apply needs " + std::to_string(need + flip) +
                                      " bytes of scratch, more than its " +
                                      std::to_string(NOALLOC_SCRATCH_BYTES));
  char* w = nullptr;
  int rc = scratch_address(&w);
  if (rc != MUDIFF_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  const size_t part_bytes = need - align256((size_t)R * h->M_all * 4);
  int32_t* counters = (int32_t*)(w + part_bytes);
  // the generic kernel's counters start at zero (a fill kernel: no memset node
  // if the caller captures this call)
  if ((rc = launch_fill_zero(counters, (size_t)R * h->M_all * 4, s)) != MUDIFF_OK) return rc;
  const cplx* xin = (const cplx*)x;
  const int64_t tot = (int64_t)R * h->N_all;
  const unsigned fb = (unsigned)((tot + 255) / 256);
  if (op == MUDIFF_OP_LT) {  // L^T x = P L (P x)
    cplx* xf = (cplx*)(w + need);
    hipLaunchKernelGGL(k_flip_modes, dim3(fb), dim3(256), 0, s, h->dv, R, xin, xf);
    HIP_TRY(hipGetLastError());
    xin = xf;
  }
  rc = apply_operator(h, R, xin, (cplx*)y, op == MUDIFF_OP_LT ? MUDIFF_OP_L : op, (cplx*)w, counters,
                      nullptr, s);
  if (rc != MUDIFF_OK || op != MUDIFF_OP_LT) return rc;
  hipLaunchKernelGGL(k_flip_modes, dim3(fb), dim3(256), 0, s, h->dv, R, (const cplx*)y, (cplx*)y);
  HIP_TRY(hipGetLastError());
  return MUDIFF_OK;
}
