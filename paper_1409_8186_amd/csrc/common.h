// Shared definitions of the gfx950 multiple-scattering library: complex128
// helpers, the device view of the tables and the host handle.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <map>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/mudiff.h"

// ------------------------------------------------------------------ complex128
typedef double2 cplx;  // (x, y) = (re, im), 16-byte aligned

__host__ __device__ __forceinline__ cplx cmk(double re, double im) { return make_double2(re, im); }
__host__ __device__ __forceinline__ cplx cadd(cplx a, cplx b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ cplx csub(cplx a, cplx b) { return cmk(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ cplx cscale(cplx a, double s) { return cmk(a.x * s, a.y * s); }
__host__ __device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return cmk(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__host__ __device__ __forceinline__ cplx cconj(cplx a) { return cmk(a.x, -a.y); }
// acc += a * b
__host__ __device__ __forceinline__ void cmac(cplx& acc, cplx a, cplx b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
__host__ __device__ __forceinline__ void cmacc(cplx& acc, cplx a, cplx b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}
__host__ __device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return cmk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  double r = b.x / b.y, d = b.x * r + b.y;
  return cmk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__host__ __device__ __forceinline__ double cabs2(cplx a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ cplx cexpi(double t) {
  double s, c;
  sincos(t, &s, &c);
  return cmk(c, s);
}

// ------------------------------------------------------------------ device view
// Plain pointers into the tables workspace, passed to kernels by value.
struct DevView {
  int B, M_all;
  int64_t N_all;              // unknowns of one column set (sum over instances)
  const double* cx;           // [M_all] center x
  const double* cy;           // [M_all] center y
  const double* a;            // [M_all] radius
  const double* kd;           // [M_all] wavenumber of the disk's instance
  const int32_t* N;           // [M_all] truncation order N_p
  const int32_t* inst;        // [M_all] instance of the disk
  const int64_t* moff;        // [M_all] offset of the disk's modes inside its instance vector
  const int64_t* dtab;        // [M_all] offset of the disk in the J/H diagonal tables
  const int64_t* idisk;       // [B+1] first disk of each instance
  const int64_t* imode;       // [B+1] unknown offset of each instance (one column)
  const int64_t* ipair;       // [B+1] first unordered pair of each instance
  const int64_t* toff;        // [P_all] offset of each pair's symbol row in t
  cplx* t;                    // [T_all] separation symbols, rows t_s, s = -S..S
  double* Jd;                 // [sum (N_p+2)] J_m(k a_p), m = 0..N_p+1
  cplx* Hd;                   // [sum (N_p+2)] H_m(k a_p)
  double* sJ;                 // [N_all] sqrt(a_p) J_m(k a_p)
  cplx* invSH;                // [N_all] 1 / (sqrt(a_p) H_m(k a_p))
  cplx* Ldiag;                // [N_all] (i pi a_p / 2) J_m(k a_p) H_m(k a_p)
  int32_t* udisk;             // [N_all] disk of each unknown
  // Lane-interleaved pair records for uniform N (lane_N >= 0, else unused):
  // for every row disk p and chunk c of 64 column disks, rows [k][lane] of
  // H_0(k b_pq), H_1(k b_pq), e^{i alpha_pq} and (2 / (k b_pq), 0); chunk
  // (p, c) starts at ltoff[p] + c * 64 * LANE_REC.
  int lane_N;
  cplx* lt;
  const int64_t* ltoff;       // [M_all]
  // Operator set by mudiff_set_operator, or NULL for the built-in single layer
  // (EFIE).  Per unknown: the column factor of the off-diagonal blocks, row
  // factor / diagonal, row factor, diagonal, right-hand-side factor (raw and
  // divided by the diagonal) and the far-field factor.
  const cplx* op_col = nullptr;
  const cplx* op_rowA = nullptr;
  const cplx* op_row = nullptr;
  const cplx* op_diag = nullptr;
  const cplx* op_rhs = nullptr;
  const cplx* op_rhsp = nullptr;
  const cplx* op_ff = nullptr;
  // Circulant-embedded form of the well-separated blocks (MUDIFF_TABLES_CIRCULANT,
  // sec. 5 Toeplitz products through discrete Fourier transforms), per instance b:
  // embedding length L_b (0: none), offset of its transformed symbol matrices
  // [L_b][M_b][M_b] in cT, of its transformed panels ([L_b][M_b][R], times R)
  // and of its twiddles w^j = e^{2 pi i j / L_b}, j < L_b, in ctw.
  const int32_t* cL = nullptr;
  const int64_t* cTo = nullptr;
  const int64_t* cZo = nullptr;
  const int64_t* cWo = nullptr;
  const cplx* cT = nullptr;
  const cplx* ctw = nullptr;
};

#define LANE_CHUNK 64
#define LANE_REC 4   // complex values per pair record
// One-lane work item, int32 words: p, chunk, q_begin, q_end, instance b, its
// first disk, then int64 at word 6: first unknown of b, unknowns of b, record
// offset of (p, chunk) in lt, partial-sum offset of (p, chunk); word 14: 0.
// All the kernel needs before its vector loads comes from this one record.
#define LANE_ITEM_INTS 16
#define LANE_NMAX 12

// Column c = b * R + r of a packed [B][R][N_b] vector starts at
// R * imode[b] + r * N_b.
__host__ __device__ __forceinline__ int64_t col_base(const int64_t* imode, int b, int R, int r) {
  return (int64_t)R * imode[b] + (int64_t)r * (imode[b + 1] - imode[b]);
}

// Unordered pair index of disks (p, q), p != q, of instance b (global disk ids).
__host__ __device__ __forceinline__ int64_t pair_index(const int64_t* idisk, const int64_t* ipair,
                                                       int b, int p, int q) {
  int64_t d0 = idisk[b], M = idisk[b + 1] - d0;
  int64_t i = (p < q ? p : q) - d0, j = (p < q ? q : p) - d0;
  return ipair[b] + i * (2 * M - i - 1) / 2 + (j - i - 1);
}

// ------------------------------------------------------------------ host side
struct MatvecPlan {
  bool ready = false;
  int lane = 0;                  // one-lane-per-pair kernel
  int waves = 1;                 // waves per workgroup of the one-lane-per-pair kernel
  int Bt = 0;                   // outputs per thread of the generic kernel
  int spec_N = -1;              // >= 0: uniform-N specialised kernel
  int zs = 0, ts = 0;            // LDS row strides (z rows, symbol rows)
  int ppcap = 1;                 // most column disks staged per pass
  int n_items = 0;
  size_t lds_bytes = 0;
  int64_t part_total = 0;       // complex partials per right-hand side
  int32_t* d_items = nullptr;   // [n_items][4] : p, chunk, q_begin, q_end (generic);
                                // [n_items][LANE_ITEM_INTS] on the one-lane path
  int32_t* d_nchunk = nullptr;  // [M_all]
  int64_t* d_partoff = nullptr; // [M_all]
};

// MFMA apply tile choice: CT sub-tiles of 8 right-hand sides, RP row disks per
// work item (RP * CT waves), column-disk segment length QS (0: whole
// instance), workgroup size.
// circ: well-separated pairs of the instances marked in the schedule go
// through the circulant-embedded form, their close pairs through the MFMA
// items (column lists).
// cvar: variant of the per-frequency product (-1: the default for R).
struct MfmaChoice {
  int CT = 1, RP = 4, QS = 0, threads = 256;
  bool circ = false;
  int cvar = -1;
  bool operator==(const MfmaChoice& o) const {
    return CT == o.CT && RP == o.RP && QS == o.QS && threads == o.threads && circ == o.circ &&
           cvar == o.cvar;
  }
};

// Host schedule of the MFMA apply: work items (p0, rp, tile, q0, q1, partial
// block) sorted by decreasing cost, the row group of every disk, and per group
// its first disk, segment count and first partial block.
struct MfmaSched {
  int R = 0;
  MfmaChoice c{};
  int ntile = 0, n_items = 0, npad = 0;
  int64_t blk = 0, n_pb = 0;
  std::vector<int32_t> items, dgrp, grow, gnseg, drow;  // grow: RP row disks per group (-1: none)
  std::vector<int64_t> gbase;
  // circulant form: column lists of the close-pair items ((q << 8) | mask of
  // the group rows close to q), per-frequency product items (instance,
  // frequency, row tile, column tile) and the instances that use the form
  std::vector<int32_t> qlist, citems, con;
  // 8-column tiles in the circulant form: the close pairs run one wave per
  // (row disk, tile) over the row's close list (nptr [M_all + 1] offsets into
  // nq, global disk indices), not as work-queue items
  bool close_rows = false;
  std::vector<int32_t> nptr, nq;
  std::vector<int32_t> rord;  // row disks by decreasing close-pair work (launch order)
  int n_citems = 0, cvar = 0;
  void* dev_base = nullptr;  // apply scratch the device copy lives in
};

struct mudiff_ctx {
  int B = 0, M_all = 0, Nmax = 0;
  int64_t N_all = 0, P_all = 0, T_all = 0, D_all = 0;
  std::vector<int64_t> idisk, imode, ipair, moff, toff, dtab, ltoff;
  std::vector<int32_t> N, inst;
  std::vector<double> k, cx, cy, a;
  DevView dv{};
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // schedule area inside the tables workspace
  char* sched_base = nullptr;
  size_t sched_bytes = 0;
  MatvecPlan plan;
  int64_t plan_part = -1;       // partial sums per right-hand side of the plan
  bool mfma_enabled = true;     // multi-RHS applies on FP64 MFMA
  bool mfma_tune = true;        // time the MFMA tile candidates on first use of an R
  int n_cu = 256;               // compute units of the device (persistent grid size)
  std::map<int, MfmaChoice> mfma_choice;  // tile choice per R
  std::map<int, float> mfma_time_ms;      // timed apply of the choice (autotuned R only)
  std::map<int, size_t> mfma_bytes;       // apply scratch per R (largest candidate)
  MfmaSched mfma_sched;                   // current schedule (host copy + upload location)
  hipEvent_t sched_ev = nullptr;          // recorded after the last schedule upload
  // in the straggler phase the circulant form's close pairs run beside its
  // transforms and products: a second stream (default priority) forked after
  // the input scaling and joined before the output pass
  hipStream_t aux = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  bool sched_pending = false;             // its copies may still read the host vectors
  bool mfma_tail = false;                 // straggler schedule (few columns still iterating)
  std::vector<int32_t> mfma_tail_cols;    // columns of the straggler schedule
  // circulant-embedded form (MUDIFF_TABLES_CIRCULANT): host copies of the
  // embedding lengths and of the close-pair lists (CSR over the disks)
  bool circ = false;
  std::map<int, int> circ_modes;          // per R: -1 timed, 0 off, 1 on (mudiff_set_circulant)
  std::vector<int32_t> cL;                // [B]
  std::vector<int64_t> cZo;               // [B]
  int64_t cZ_all = 0;                     // sum_b L_b M_b
  std::vector<int64_t> near_off;          // [M_all + 1]
  std::vector<int32_t> near;              // close column disks of each row disk
  std::vector<uint8_t> circ_on;           // [B] instance worth the circulant form
  std::vector<uint8_t> circ_nearflag;     // [P_all] 1: close unordered pair (host copy)
  const uint8_t* circ_near_dev = nullptr; // the same on the device
  int64_t n_far = 0, n_near = 0;          // ordered pairs of each kind
  // phase timing (mudiff_profile_begin/end): MUDIFF_N_PHASES + 1 events per
  // profiled apply, the slot of the apply in flight (-1: none)
  std::vector<hipEvent_t> prof_ev;
  int prof_max = 0, prof_n = 0, prof_cur = -1;
  // penetrable disks (set by mudiff_set_penetrable, in its workspace): interior
  // wavenumbers [M_all] and J_n(k- a), n = 0..N_p+1, at dtab offsets
  const double* pen_k = nullptr;
  const double* pen_J = nullptr;
};

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
int fail(int status, const std::string& msg);
#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(MUDIFF_ERR_DEVICE, std::string(#expr ": ") + hipGetErrorString(_e));  \
  } while (0)

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ------------------------------------------------------------------ apply epilogue
// Output value of the operator apply at unknown i from the coupling sum
// w_m = sum_{q != p} sum_n t^{pq}_{n-m} sqrt(a_q) J_n(k a_q) x^q_n:
//   MUDIFF_OP_A: x + w / (sqrt(a_p) H_m)        (A = D^{-1} L = I + K)
//   OP_RAW_W:    w
//   MUDIFF_OP_L: L^{pp}_{mm} x + (i pi / 2) sqrt(a_p) J_m w
#define OP_RAW_W 7
__device__ __forceinline__ cplx finalize(const DevView& v, int op, int64_t i, cplx xv, cplx w) {
  if (v.op_rowA) {  // operator set by mudiff_set_operator
    if (op == MUDIFF_OP_A) return cadd(xv, cmul(v.op_rowA[i], w));
    if (op == OP_RAW_W) return w;
    return cadd(cmul(v.op_diag[i], xv), cmul(v.op_row[i], w));
  }
  if (op == MUDIFF_OP_A) return cadd(xv, cmul(v.invSH[i], w));
  if (op == OP_RAW_W) return w;
  const double f = 0.5 * 3.14159265358979323846 * v.sJ[i];  // (i pi / 2) s_m w
  return cadd(cmul(v.Ldiag[i], xv), cmk(-f * w.y, f * w.x));
}

// Affine epilogue of a shifted apply: alpha_c y + beta_c x, (alpha, beta) the
// pair of column c in ab.
__device__ __forceinline__ cplx affine(const cplx* __restrict__ ab, int c, cplx y, cplx x) {
  return cadd(cmul(ab[2 * c], y), cmul(ab[2 * c + 1], x));
}

// Input x_n scaled by the column factor of unknown i: sqrt(a_q) J_n(k a_q)
// for the single layer, the set operator's factor otherwise.
__device__ __forceinline__ cplx col_scale(const DevView& v, int64_t i, cplx x) {
  return v.op_col ? cmul(x, v.op_col[i]) : cscale(x, v.sJ[i]);
}

// Sum, in chunk order, of the one-lane-per-pair partial sums of unknown i
// (instance b) for one right-hand side (part points at that column's block).
__device__ __forceinline__ cplx lane_chunk_sum(const DevView& v, const cplx* __restrict__ part,
                                               const int32_t* __restrict__ nchunk,
                                               const int64_t* __restrict__ partoff, int b,
                                               int64_t i) {
  const int p = v.udisk[i];
  const int64_t m = i - v.imode[b] - v.moff[p];
  const int np = 2 * v.N[p] + 1;
  const cplx* pr = part + partoff[p] + m;
  cplx w = cmk(0.0, 0.0);
  const int nch = nchunk[p];
#pragma unroll 8
  for (int k = 0; k < nch; ++k) w = cadd(w, pr[(int64_t)k * np]);
  return w;
}

// ------------------------------------------------------------------ lane reductions
// Reduce-scatter of NV doubles over the 64 lanes of a wave: lane l ends with
// the sum over all lanes of value l >> (6 - log2 NV).  At each step the lanes
// pair up and each keeps one half of the remaining values (the upper half
// where the step's lane bit is set) plus its partner's copy of that half.
// Steps 32 and 16 use the gfx950 lane swaps (v_permlane32/16_swap), which hand
// every lane both of its addends at once; steps 8, 4, 2, 1 read the partner by
// DPP (row mirror, half-row mirror, quad permutations: partners differ in the
// step's bit, and the partner sets stay disjoint).  Steps past NV are plain
// sums over the remaining lanes.  All VALU: no LDS traffic.
template <int CTRL>
__device__ __forceinline__ double dpp_read(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

template <int O>
__device__ __forceinline__ double lane_partner(double v) {
  if constexpr (O == 8) return dpp_read<0x140>(v);       // row_mirror: l <-> 15 - l
  else if constexpr (O == 4) return dpp_read<0x141>(v);  // row_half_mirror: l <-> 7 - l
  else if constexpr (O == 2) return dpp_read<0x4E>(v);   // quad_perm [2,3,0,1]
  else return dpp_read<0xB1>(v);                          // quad_perm [1,0,3,2]
}

// a in the lower, b in the upper lane half (of 64 for O = 32, of each 32 for
// O = 16): returns own + partner's copy of the half the lane keeps.
template <int O>
__device__ __forceinline__ double swap_add(double a, double b) {
  if constexpr (O == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
  } else {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
    return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
  }
}

template <int O, int CNT>
__device__ __forceinline__ void rs_dpp_step(double* val, int lane) {
  if constexpr (CNT > 1) {
    const bool upper = (lane & O) != 0;
#pragma unroll
    for (int k = 0; k < CNT / 2; ++k) {
      const double send = upper ? val[k] : val[CNT / 2 + k];
      const double keep = upper ? val[CNT / 2 + k] : val[k];
      val[k] = keep + lane_partner<O>(send);
    }
  } else {
    val[0] += lane_partner<O>(val[0]);
  }
}

template <int NV>
__device__ __forceinline__ void lane_reduce_scatter(double* val, int lane) {
  static_assert(NV >= 8 && NV <= 64 && (NV & (NV - 1)) == 0, "NV: 8, 16, 32 or 64");
#pragma unroll
  for (int k = 0; k < NV / 2; ++k) val[k] = swap_add<32>(val[k], val[NV / 2 + k]);
#pragma unroll
  for (int k = 0; k < NV / 4; ++k) val[k] = swap_add<16>(val[k], val[NV / 4 + k]);
  rs_dpp_step<8, NV / 4>(val, lane);
  rs_dpp_step<4, (NV / 8 > 1 ? NV / 8 : 1)>(val, lane);
  rs_dpp_step<2, (NV / 16 > 1 ? NV / 16 : 1)>(val, lane);
  rs_dpp_step<1, (NV / 32 > 1 ? NV / 32 : 1)>(val, lane);
}

// ------------------------------------------------------------------ internal API
// Operator apply on R columns. `part`/`counters` come from the caller's scratch
// (mudiff_matvec_workspace_size); counters must be zero on entry and are left
// zero. `active` (optional, [B*R]) skips columns whose entry is 0.  `shift`
// (optional, [B*R][2]) makes column c of the result alpha_c (op x) + beta_c x
// with (alpha_c, beta_c) = (shift[2c], shift[2c+1]): the scaled Newton steps
// (A - theta) x / sigma of s-step GMRES.
int apply_operator(mudiff_ctx* h, int R, const cplx* x, cplx* y, int op, cplx* part,
                   int32_t* counters, const int32_t* active, hipStream_t s,
                   const cplx* shift = nullptr);
// Same, except that on the one-lane-per-pair path only the chunk partial sums
// are written (*pending = true): the caller adds them (lane_chunk_sum) and
// applies finalize itself.
int apply_operator_split(mudiff_ctx* h, int R, const cplx* x, cplx* y, int op, cplx* part,
                         int32_t* counters, const int32_t* active, hipStream_t s,
                         bool* pending);
size_t apply_scratch_bytes(mudiff_ctx* h, int R);
// Forget where the MFMA schedule was last uploaded: the next apply uploads it
// into its scratch again.  Every entry point that takes an apply scratch from
// the caller calls this first, so a buffer whose memory was used for anything
// else between calls (or a new buffer at a recycled address) never runs on a
// stale schedule.
void apply_forget_upload(mudiff_ctx* h);
// Wait until the last schedule upload has read its host vectors (before they
// are rebuilt or released).
void sched_wait(mudiff_ctx* h);
// Lane-record layout of the one-lane-per-pair apply: total size in complex
// values (0 when N is not uniform or out of range), the common N, and per disk
// the offset of its first chunk.
int64_t lane_layout(int B, const int64_t* disk_off, const int32_t* n_modes, int* lane_N,
                    std::vector<int64_t>* ltoff);
int ensure_plan(mudiff_ctx* h, hipStream_t s);
// Schedule for R applies made current (one-lane/generic plan, or the MFMA
// schedule uploaded into `scratch`, the apply scratch later passed as `part`).
// On the MFMA path the first use of R times the tile candidates on x -> y
// (y is overwritten) when x and y are given.  Synchronises; not for use under
// graph capture.
int prepare_apply(mudiff_ctx* h, int R, const cplx* x, cplx* y, cplx* scratch, hipStream_t s);
// Switch the MFMA schedule of R between the tuned form and the straggler form
// (short column segments, only the tiles holding a column c with
// cols[c] != 0, c = b * R + r); uploads into `scratch` and synchronises.
int apply_set_tail(mudiff_ctx* h, int R, bool tail, cplx* scratch, hipStream_t s,
                   const int32_t* cols);
struct PlanHost;
void make_plan(int B, const int64_t* idisk, const int32_t* N, PlanHost& P);
size_t plan_sched_bytes(const PlanHost& P, int M);

int launch_rhs(mudiff_ctx* h, int R, const double* beta, cplx* out, int precond, int point,
               hipStream_t s);
int launch_fill_zero(void* p, size_t bytes, hipStream_t s);

// Phase marks of a profiled apply: prof_open picks the apply's event slot
// (none when profiling is off, full, or the stream is being captured) and
// records mark 0; prof_mark(k) records mark k (1..MUDIFF_N_PHASES) after phase k-1.
void prof_open(mudiff_ctx* h, hipStream_t s);
void prof_mark(mudiff_ctx* h, hipStream_t s, int k);
