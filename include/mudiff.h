/*
 * mudiff.h - C ABI of the MI355X (gfx950) multiple-scattering library.
 *
 * The library computes the spectral (Fourier-mode) boundary-integral solution
 * of sound-soft multiple scattering by M disjoint disks, following Thierry,
 * Antoine, Chniti & Alzubaidi, "mu-diff: an open-source Matlab toolbox for
 * computing multiple scattering problems by disks" (arXiv:1409.8186):
 *
 *   problem    exterior Dirichlet Helmholtz problem, plane wave
 *              u_inc = exp(i k beta_hat . x), time dependence exp(-i w t) (sec. 2);
 *   unknowns   Fourier coefficients rho^p_m, m = -N_p..N_p, of the EFIE density
 *              on every disk p (sec. 4.1 basis, sec. 5 truncation);
 *   operator   truncated EFIE matrix L (sec. 4.2 block formulas):
 *                L^{pp}_{mm} = (i pi a_p/2) J_m(k a_p) H_m(k a_p)
 *                L^{pq}_{mn} = (i pi sqrt(a_p a_q)/2) J_m(k a_p) t^{pq}_{n-m} J_n(k a_q)
 *                t^{pq}_nu   = H^(1)_nu(k b_pq) exp(i nu alpha_pq),
 *              b_pq, alpha_pq the length and angle of O_p - O_q (sec. 4.1);
 *   system     L rho = -U, U the plane-wave coefficients (Prop. 4), solved by
 *              restarted GMRES with the single-scattering (block-diagonal)
 *              preconditioner (sec. 5);
 *   output     far field a(theta) = sum_p sum_m (a_L)^p_m(theta) rho^p_m (sec. 4.4).
 *
 * Conventions for every entry point
 *   complex128  interleaved (re, im) doubles, 16-byte aligned (== C99 double
 *               _Complex == torch.complex128).
 *   [host]      pointers marked so are read synchronously during the call;
 *               every other pointer is device memory (HIP / torch tensors).
 *   streams     `stream` is a hipStream_t (NULL = default stream).  Calls
 *               validate on the host, enqueue on `stream` and return; device
 *               outputs are valid after the stream is synchronised.
 *               mudiff_gmres and mudiff_grad synchronise `stream` themselves
 *               (once per restart cycle) to test convergence.  In the
 *               straggler phase of a solve on the circulant form, part of an
 *               apply runs on a second stream of the handle, forked from and
 *               joined back into `stream` by events (so still ordered with
 *               the caller's work); a handle is used by one host thread at a
 *               time.
 *   batching    B independent instances (own disks, own k) share one handle.
 *               Instance b owns disks [disk_off[b], disk_off[b+1]).  Vectors
 *               are packed [B][R][N_b] with N_b = sum_{p in b} (2 N_p + 1):
 *               inside a vector disks come in order and modes m = -N_p..N_p
 *               ascending (sec. 5 block vector).  R is the number of
 *               right-hand sides per instance (incidence angles).
 *   memory      the library never allocates device memory: every device
 *               buffer, workspaces included, is owned by the caller and must
 *               outlive the calls that use it (the handle keeps pointers into
 *               the tables workspace).  Workspace sizes come from the
 *               *_workspace_size queries (bytes, 256-byte aligned base).
 *   errors      the return value is a mudiff_status; mudiff_last_error()
 *               returns a thread-local message for the last failing call.
 *               Validation errors are detected before anything is enqueued.
 */
#ifndef MUDIFF_H
#define MUDIFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mudiff_ctx* mudiff_t;

typedef enum {
  MUDIFF_OK = 0,
  MUDIFF_ERR_INVALID = 1,        /* bad count, pointer, non-finite value, k<=0, a<=0, N_p<0 ... */
  MUDIFF_ERR_OVERLAP = 2,        /* two disks of one instance intersect or touch */
  MUDIFF_ERR_NOMEM = 3,          /* workspace smaller than the queried size */
  MUDIFF_ERR_DEVICE = 4,         /* a HIP runtime error (text in mudiff_last_error) */
  MUDIFF_ERR_NOT_CONVERGED = 5   /* mudiff_grad: a forward or adjoint solve did not converge */
} mudiff_status;

/* matvec operators */
enum {
  MUDIFF_OP_L = 0,      /* y = L x                 (sec. 4.2, truncated as in sec. 5)        */
  MUDIFF_OP_A = 1,      /* y = D^{-1} L x = x + K x, D = diag(L^{pp}) (sec. 5 preconditioner) */
  MUDIFF_OP_LT = 2      /* y = L^T x (plain transpose) = P L P x, P: m -> -m in every disk   */
};

/* mudiff_gmres flags */
enum {
  MUDIFF_X0 = 1,        /* rho holds the initial guess on entry (else x0 = 0)          */
  MUDIFF_GRAPH = 2,     /* replay each restart cycle as one captured HIP graph          */
  MUDIFF_POINT_SOURCE = 4, /* beta holds point-source positions [B][R][2] (Prop. 5)  */
  MUDIFF_NO_PRECOND = 8, /* GMRES on L rho = -U itself (no single-scattering preconditioner) */
  MUDIFF_BLOCK = 16,     /* block GMRES: blocks of consecutive columns of an instance share one
                            block Krylov space (block size: MUDIFF_BLOCK_SIZE, default 8) */
  MUDIFF_SSTEP = 32      /* s-step GMRES: after the first cycle, the Krylov basis grows s vectors
                            at a time (s: MUDIFF_SSTEP_SIZE, default 8) */
};
/* Newton vectors per block of a MUDIFF_SSTEP solve, or'ed into the flags:
 * 2 <= s <= 16, restart <= 64. */
#define MUDIFF_SSTEP_SIZE(s) (((s) & 0xff) << 16)
/* Block size s of a MUDIFF_BLOCK solve, or'ed into the flags: 1 <= s <= 16 and
 * restart * s <= 2048 (a block never exceeds the instance's R columns). */
#define MUDIFF_BLOCK_SIZE(s) (((s) & 0xff) << 8)

/* mudiff_tables flags */
enum {
  MUDIFF_TABLES_CIRCULANT = 1  /* also build the circulant-embedded form of the
                                  well-separated blocks (see mudiff_tables) */
};

/* Largest accepted truncation order N_p and GMRES restart length. */
#define MUDIFF_MAX_NP 200
#define MUDIFF_MAX_RESTART 512

/* ---------------------------------------------------------------- tables */

/* Bytes of device workspace mudiff_tables needs for this batch and flags
 * (pure host computation, no device call).  Returns 0 for invalid arguments,
 * including MUDIFF_TABLES_CIRCULANT with an order N_p > 31. */
size_t mudiff_tables_workspace_size(int B, const int64_t* disk_off /*[host] B+1*/,
                                    const int32_t* n_modes /*[host] M_tot*/, int flags);

/* Geometry, Bessel/Hankel tables and the operator schedule (sec. 4.1-4.2).
 *   B          number of instances, >= 1
 *   disk_off   [host] B+1 disk offsets, disk_off[0] = 0, strictly increasing
 *   centers    [host] [M_tot][2] disk centers (x, y)
 *   radii      [host] [M_tot] radii a_p > 0
 *   n_modes    [host] [M_tot] truncation orders 0 <= N_p <= MUDIFF_MAX_NP
 *   k          [host] [B] wavenumbers > 0
 *   workspace  device buffer of at least mudiff_tables_workspace_size bytes;
 *              it holds the tables for the lifetime of the handle
 *   flags      0 or MUDIFF_TABLES_CIRCULANT
 *   out        receives the handle (host object; free with mudiff_destroy)
 * Computes on the device: per disk J_m(k a_p), H_m(k a_p) (m = 0..N_p+1,
 * Miller's downward recurrence for J, Neumann series / Hankel's expansion and
 * upward recurrence for Y) and per unordered pair p<q the separation symbols
 * t^{pq}_s, |s| <= N_p + N_q.
 * With MUDIFF_TABLES_CIRCULANT (the Toeplitz products through FFTs of sec. 5):
 * every instance b with M_b >= 2 gets an embedding length L_b >= L_min =
 * 2 (N' + N'') + 1, N' >= N'' its two largest orders (L_b >= n_p + n_q - 1 for
 * every pair, so the circulant of length L_b holds each Toeplitz block
 * exactly): the shortest 2^i 3^j >= L_min (fast transforms) when that is at
 * most 128 and at most 1.2 L_min, else L_min itself; and for every
 * frequency f < L_b the matrix
 *   T_f[p][q] = (1/L_b) sum_{|s| <= N_p+N_q} t^{pq}_s w^{f (s + N_q - N_p)},
 *   w = e^{2 pi i / L_b},
 * over the ordered pairs that are well separated, k b_pq >= N_p + N_q (zero on
 * the diagonal and for close pairs: there the symbols grow by orders of
 * magnitude and a transform would spread their rounding over every mode).
 * Then for a well-separated pair the Toeplitz product is
 *   sum_n t^{pq}_{n-m} z_n = sum_f w^{f j} T_f[p][q] Z_f,  Z_f = sum_k w^{-f k} z_k,
 * with k = n + N_q, j = m + N_p.  This costs sum_b L_b M_b^2 complex values of
 * workspace (about 1.3 GB for 1,000 disks at N_p <= 20); multi-right-hand-side
 * applies (R >= 8, N_p <= 31) may then run those pairs as one dense complex
 * product per frequency on the matrix cores and the close pairs directly
 * (chosen per R by timing: mudiff_apply_config, mudiff_set_circulant).  The
 * flag requires N_p <= 31.
 * Errors: INVALID, OVERLAP (b_pq <= a_p + a_q), NOMEM, DEVICE. */
int mudiff_tables(int B, const int64_t* disk_off, const double* centers, const double* radii,
                  const int32_t* n_modes, const double* k, void* workspace, size_t ws_bytes,
                  int flags, void* stream, mudiff_t* out);

/* Classification of the ordered disk pairs of a handle built with
 * MUDIFF_TABLES_CIRCULANT (host outputs, any may be NULL): well-separated
 * pairs (k b_pq >= N_p + N_q, circulant form), close pairs (direct form) and
 * the largest embedding length.  Zeros for a handle built without the flag. */
int mudiff_circulant_info(mudiff_t h, int64_t* far_pairs, int64_t* near_pairs, int* L_max);

/* Form of the R-column apply on a handle built with MUDIFF_TABLES_CIRCULANT:
 * mode -1 (default) times the direct and the circulant forms on the first
 * apply with this R and keeps the faster, 0 keeps every pair in the direct
 * form, 1 uses the circulant form.  The circulant form covers the instances
 * whose well-separated pairs hold at least half of the direct form's work;
 * the others stay direct.  Takes effect at the next call with this R.
 * Errors: MUDIFF_ERR_INVALID (mode, no circulant tables). */
int mudiff_set_circulant(mudiff_t h, int R, int mode);

/* Tile of the per-frequency products of the R-column apply when it uses the
 * circulant form (host outputs, any may be NULL; zeros otherwise): rows and
 * complex columns of a workgroup's output tile, K step (column disks staged
 * per step), staging depth (1: one LDS buffer; 2: two LDS buffers; 3: two LDS
 * buffers and two register sets, loads two steps ahead), workgroup size, and
 * real matrix products per complex product: 4 (Re and Im of T against
 * [Re Z | Im Z]) or 3 (Gauss's form: Re T Re Z, Im T Im Z and
 * (Re T + Im T)(Re Z + Im Z); a quarter fewer matrix-core operations, rounding
 * error normwise of the same order).
 * The candidates for R are timed with the rest of the apply on first use. */
int mudiff_circulant_tile(mudiff_t h, int R, int* rows, int* cols, int* kstep, int* stages,
                          int* threads, int* mults);

/* Fixes that tile (one of the candidates for R, as listed by
 * Problem.circulant_tiles in the Python binding: for R >= 48 with four
 * products, 64x32 K16 or K8, 128x32 K16, K8 or K4 on 512 threads, 128x32 K8 on
 * 1024 threads, 128x64 K8 or K16, 256x32 K8, and with three, 128x32 K8 or K16,
 * 128x64 K8, 256x32 K8, 64x32 K8; other sets for smaller R) and switches the
 * circulant form on for R.
 * MUDIFF_ERR_INVALID for other tiles or when the form is not available. */
int mudiff_set_circulant_tile(mudiff_t h, int R, int rows, int cols, int kstep, int stages,
                              int threads, int mults);

/* Releases the host handle (not the caller's device memory); NULL is a no-op. */
int mudiff_destroy(mudiff_t h);

/* Unknowns per instance: n_tot[b] = N_b (host array of B entries). */
int mudiff_sizes(mudiff_t h, int64_t* n_tot /*[host] B*/);

/* Copies the per-disk diagonal values to device arrays (either may be NULL):
 * J [sum_p (N_p+2)] = J_m(k a_p), H [sum_p (N_p+2)] complex128 = H_m(k a_p),
 * m = 0..N_p+1, disks in order.  Used to check the tables. */
int mudiff_disk_tables(mudiff_t h, double* J, void* H, void* stream);

/* Copies the separation symbols of every unordered pair p<q (instance by
 * instance, p-major) to `t` (complex128, device): pair after pair,
 * t^{pq}_s for s = -(N_p+N_q)..(N_p+N_q).  `count` receives the number of
 * complex values (host). `t` may be NULL to query `count`. */
int mudiff_pair_tables(mudiff_t h, void* t, int64_t* count /*[host]*/, void* stream);

/* ---------------------------------------------------------------- operator */

size_t mudiff_matvec_workspace_size(mudiff_t h, int R);

/* y = op(x) for R right-hand sides per instance (sec. 4.2 / sec. 5).
 *   x, y       device complex128 [B][R][N_b], distinct buffers
 *   op         MUDIFF_OP_L, MUDIFF_OP_A or MUDIFF_OP_LT (the single layer only:
 *              MUDIFF_ERR_INVALID after mudiff_set_operator / mudiff_set_penetrable)
 *   workspace  device scratch of mudiff_matvec_workspace_size(h, R) bytes; it
 *              must be zero-filled before its first use and every call leaves
 *              it ready for the next one (its counters return to zero), so
 *              one buffer serves any number of calls on one stream.  Calls
 *              that overlap in time (several streams) need separate buffers.
 *              No state is kept in it between calls beyond those zeros: for
 *              R >= 8 (FP64 MFMA) each call uploads the tile schedule into it
 *              again, asynchronously, from host memory the handle keeps.  The
 *              call enqueues and returns; only the first call with a new R
 *              synchronises (it times the candidate tiles and forms).
 * Off-diagonal blocks are applied as Toeplitz products in the mode
 * difference n - m (the diagonal.Toeplitz.diagonal structure of sec. 5). */
int mudiff_matvec(mudiff_t h, int R, const void* x, void* y, int op,
                  void* workspace, size_t ws_bytes, void* stream);

/* No-allocation variant of mudiff_matvec, for callers that cannot allocate
 * or hand over device memory between calls (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the apply scratch is
 * a static device array of MUDIFF_NOALLOC_SCRATCH_MB MiB inside the library,
 * one copy per device, held until the process ends; the call itself allocates
 * nothing and does not synchronise.  Same operands and results as
 * mudiff_matvec (x, y, op, stream); it covers the one-lane and generic kernels
 * (R < 8, or a batch with N_p > 31).  Every call on a device shares that
 * device's array and leaves its contents behind (it clears what must start at
 * zero itself): calls that overlap in time on one device (several streams or
 * threads) race.  Errors: MUDIFF_ERR_INVALID (as mudiff_matvec, or R >= 8 with
 * N_p <= 31: use mudiff_matvec), MUDIFF_ERR_NOMEM (the apply needs more scratch
 * than the array holds: about 16 R sum_p (2N_p+1) ceil((M-1)/64) bytes on the
 * one-lane path), MUDIFF_ERR_DEVICE. */
#define MUDIFF_NOALLOC_SCRATCH_MB 64
int mudiff_matvec_noalloc(mudiff_t h, int R, const void* x, void* y, int op, void* stream);

/* Kernel configuration of the R-column operator apply, as chosen on this
 * handle (host outputs; any pointer may be NULL):
 *   kind       0 one lane per pair (uniform N_p <= 12, R < 8), 1 FP64-MFMA
 *              work queue (R >= 8, N_p <= 31), 2 generic LDS-staged kernel,
 *              3 circulant form on the FP64 matrix cores for the well-separated
 *              pairs and the MFMA work queue for the close ones
 *   ct, rp     MFMA tile: 8*ct right-hand sides x rp row disks per work item
 *   qs         MFMA column-disk segment length (0: whole instance)
 *   threads    MFMA workgroup size
 *   ms         timed duration of one apply when the MFMA tile was autotuned
 *              (the first mudiff_matvec / mudiff_gmres / mudiff_grad with this
 *              R times every candidate on the real data), else 0
 * Fields that do not apply to `kind` are set to 0.  Before the first call
 * with this R, the MFMA fields hold the default tile. */
int mudiff_apply_config(mudiff_t h, int R, int* kind, int* ct, int* rp, int* qs, int* threads,
                        float* ms);

/* Fixes the MFMA tile of the R-column apply on this handle instead of timing
 * the candidates (ct in {1,2,4} with ct <= max(1, ceil(R/8)), rp = waves/ct
 * with waves in {4, 8} and threads = 64 * waves, qs in {0, 32}).  Returns
 * MUDIFF_ERR_INVALID for a tile outside that set or when the R-column apply
 * does not run on MFMA.  Takes effect at the next call with this R. */
int mudiff_set_apply_config(mudiff_t h, int R, int ct, int rp, int qs, int threads);

/* Plane-wave right-hand side (Prop. 4) for R incidence angles per instance.
 *   beta       device [B][R] angles (radians), beta_hat = (cos beta, sin beta)
 *   out        device complex128 [B][R][N_b]: U (precond = 0) or the GMRES
 *              right-hand side f = -D^{-1} U (precond = 1). */
int mudiff_rhs(mudiff_t h, int R, const double* beta, void* out, int precond, void* stream);

/* Point-source right-hand side (Prop. 5): the incident wave is the Green's
 * function G(x, s) = (i/4) H_0(k |x - s|) of a source s outside every disk, with
 *   U^p_m = (i/4) sqrt(2 pi a_p) J_m(k a_p) H_m(k r_p) e^{-i m theta_p},
 * (r_p, theta_p) the polar coordinates of s - O_p (the printed
 * (i pi a/2) J H conj(Phi~(s)) with Phi~ = e^{i m theta} / sqrt(2 pi a)).
 *   src        device double [B][R][2] source positions
 *   out        as for mudiff_rhs (also after mudiff_set_operator /
 *              mudiff_set_penetrable: their right-hand side from this U, dU)
 * A source inside or on disk p (r_p <= a_p, where the expansion does not hold)
 * gives NaN coefficients for that disk; mudiff_gmres then ends the column with
 * flag 2. */
int mudiff_rhs_point(mudiff_t h, int R, const double* src, void* out, int precond, void* stream);

/* ---------------------------------------------------------------- operators */

/* Replaces the handle's operator, right-hand side and far field by a linear
 * combination of the identity and the four boundary integral operators
 * (sec. 3 formulations, sec. 4.2 block formulas, Prop. 4, sec. 4.4):
 *   op    = w_I I + w_L L + w_M M + w_N N + w_D D
 *   b     = w_U U + w_dU dU      (U = d J, dU = k d J' of the plane wave, Prop. 4)
 *   a(th) = f_L a_L + f_M a_M    (a_M: double-layer far field, the sign of the
 *                                 double-layer potential's large-r form)
 * after which mudiff_matvec applies op (MUDIFF_OP_L) or D^{-1} op with D the
 * diagonal blocks of op (MUDIFF_OP_A), mudiff_rhs returns b (or D^{-1} b),
 * mudiff_gmres solves op rho = b (from incidence angles) or op rho = -rhs (from
 * a given rhs, as for the single layer), and mudiff_farfield uses (f_L, f_M).
 * Examples: MFIE  op (1/2) I + N, b = -dU;  CFIE (alpha eta) L + (1-alpha)(I/2 + N),
 * b = -alpha eta U - (1-alpha) dU;  Brakhage-Werner (1/2) I - eta L - M,
 * b = -U, a = -(eta a_L + a_M);  sound-hard single layer -(1/2) I + N,
 * b = -dU;  sound-hard double layer D, b = -dU, a = a_M.
 *   op_w       [host] 5 complex (re, im pairs): w_I, w_L, w_M, w_N, w_D, or NULL
 *              to return to the built-in single layer (EFIE)
 *   rhs_w      [host] 2 complex: w_U, w_dU;  ff_w  [host] 2 complex: f_L, f_M
 *   workspace  device, 256-byte aligned, >= mudiff_operator_workspace_size(h);
 *              holds the per-unknown factor tables and must outlive their use
 * The operators with nonzero weight among L, M, N, D must share their row
 * factor (L and M: J; N and D: J') or their column factor (L and N: J; M and D:
 * J'), so that the off-diagonal blocks stay one diagonal-Toeplitz-diagonal
 * product; otherwise MUDIFF_ERR_INVALID.  The D diagonal is
 * -(i pi k^2 a / 2) J'_m H'_m (the normal derivative of the double-layer
 * potential of a mode; the printed + sign contradicts the off-diagonal D
 * blocks).  mudiff_grad requires the single layer (MUDIFF_ERR_INVALID otherwise).
 * Enqueues the table kernel on `stream`. */
size_t mudiff_operator_workspace_size(mudiff_t h);
int mudiff_set_operator(mudiff_t h, const double* op_w, const double* rhs_w, const double* ff_w,
                        void* workspace, size_t ws_bytes, void* stream);

/* Named formulations of sec. 3 (with the right-hand sides of Prop. 4 and the
 * far fields of sec. 4.4), set through mudiff_set_operator:
 *   MUDIFF_FORM_EFIE         L rho = -U (the built-in single layer; the
 *                            workspace is not used)
 *   MUDIFF_FORM_MFIE         (I/2 + N) rho = -dU,                  a = a_L rho
 *   MUDIFF_FORM_CFIE         (alpha eta L + (1 - alpha)(I/2 + N)) rho
 *                              = -alpha eta U - (1 - alpha) dU,     a = a_L rho
 *   MUDIFF_FORM_BWIE         Brakhage-Werner, u = -(eta L + M) psi:
 *                            (I/2 - eta L - M) psi = -U,           a = -(eta a_L + a_M) psi
 *   MUDIFF_FORM_SOUND_HARD_SINGLE  sound-hard boundary, u = L rho:
 *                            (-I/2 + N) rho = -dU,                 a = a_L rho
 *   MUDIFF_FORM_SOUND_HARD_DOUBLE  sound-hard boundary, u = M lambda:
 *                            D lambda = -dU,                       a = a_M lambda
 *   alpha      CFIE mixing weight (other kinds ignore it)
 *   eta        coupling constant eta_re + i eta_im of CFIE and Brakhage-Werner,
 *              nonzero there (i k is the usual choice)
 *   workspace  as for mudiff_set_operator
 * Errors: MUDIFF_ERR_INVALID (kind, non-finite alpha or eta, eta = 0 where it
 * is used), and those of mudiff_set_operator. */
enum {
  MUDIFF_FORM_EFIE = 0, MUDIFF_FORM_MFIE = 1, MUDIFF_FORM_CFIE = 2, MUDIFF_FORM_BWIE = 3,
  MUDIFF_FORM_SOUND_HARD_SINGLE = 4, MUDIFF_FORM_SOUND_HARD_DOUBLE = 5
};
int mudiff_set_formulation(mudiff_t h, int kind, double alpha, double eta_re, double eta_im,
                           void* workspace, size_t ws_bytes, void* stream);

/* Penetrable disks (sec. 7, Example II): replaces the handle's operator,
 * right-hand side and far field by those of the transmission problem with
 * interior wavenumber k-_p and contrast mu_p in disk p (u+ - u- = -u_inc,
 * d_n u+ - mu d_n u- = -d_n u_inc; u+ = L+ rho+ with the exterior wavenumber,
 * u- = L- rho- with k-_p).  The interior operators act within one disk, so
 * rho- is eliminated mode by mode; the equation solved is, per mode (any
 * scaling of its two weights),
 *   [J_m(k- a) (N+ - I/2) - mu k- J'_m(k- a) L+] rho+ = -J_m(k- a) dU + mu k- J'_m(k- a) U,
 * and mudiff_farfield / mudiff_nearfield return the exterior scattered field
 * (mudiff_interior_field the field inside the disks)
 * a_L rho+ / L+ rho+.  The second row's interior block is -mu (I/2 + N-): the
 * sign that the jump relations give, with which a matched medium (k- = k,
 * mu = 1) scatters nothing; the printed + sign does not.  The interior density
 * of mode m is rho-_m = (L+ rho+ + U)_m / ((i pi a / 2) J_m(k- a) H_m(k- a)).
 *   k_int      [host] double [M_all] interior wavenumbers, > 0
 *   mu         [host] double [M_all] contrasts, > 0, or NULL for all 1
 *   workspace  as for mudiff_set_operator (same size), must outlive its use
 * Undone by mudiff_set_operator(h, NULL, ...).  MUDIFF_ERR_INVALID on a
 * wavenumber or contrast that is not finite and positive.  Enqueues two table
 * kernels on `stream` and waits for them. */
int mudiff_set_penetrable(mudiff_t h, const double* k_int, const double* mu, void* workspace,
                          size_t ws_bytes, void* stream);

/* Interior field of penetrable disks (sec. 7, Example II): at points inside
 * disk p, u-(x) = sum_m c_m J_m(k-_p r) e^{i m theta}, (r, theta) the polar
 * coordinates of x - O_p, with c_m = (U + L+ rho+)_m / (sqrt(2 pi a_p) J_m(k-_p a_p))
 * from the transmission condition u- = u+ + u_inc on the circle (the same field
 * as L- rho- with rho- from the first block row).  Points outside every disk
 * are left untouched, so that after mudiff_nearfield with the total field
 * `out` holds the total field everywhere.
 *   rho        device complex128 [B][R][N_b] exterior densities (mudiff_gmres
 *              after mudiff_set_penetrable)
 *   inc, flags the incidence of rho: [B][R] angles (flags 0) or [B][R][2] point
 *              sources (MUDIFF_POINT_SOURCE)
 *   pts, out   device double [n_pts][2]; device complex128 [B][R][n_pts]
 *   workspace  device, 256-byte aligned, >= mudiff_interior_workspace_size(h, R)
 * MUDIFF_ERR_INVALID when the handle has no penetrable disks set.  Where
 * J_m(k- a) = 0 for a kept order (k- an interior Dirichlet eigenvalue) the
 * field of that disk is not finite. */
size_t mudiff_interior_workspace_size(mudiff_t h, int R);
int mudiff_interior_field(mudiff_t h, int R, const void* rho, const double* inc, int flags, int n_pts,
                          const double* pts, void* out, void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- solver */

size_t mudiff_gmres_workspace_size(mudiff_t h, int R, int restart, int flags);

/* Restarted GMRES(restart) on A x = f, A = D^{-1} L, f = -D^{-1} U (sec. 5), or with
 * MUDIFF_NO_PRECOND on L x = -U itself (after mudiff_set_operator: op x = b),
 * one independent Krylov space per (instance, right-hand side) column, all
 * columns sharing every operator application (lockstep batching).
 *   beta       device [B][R] incidence angles, or with MUDIFF_POINT_SOURCE
 *              [B][R][2] point-source positions (mudiff_rhs_point), or NULL to
 *              use `rhs`
 *   rhs        device complex128 [B][R][N_b]: the right-hand side U of
 *              L rho = -U (used when beta == NULL)
 *   rho        device complex128 [B][R][N_b] output density; with MUDIFF_X0
 *              it holds the initial guess on entry
 *   restart    1..MUDIFF_MAX_RESTART;  tol > 0;  maxit >= 1 counts inner
 *              iterations (operator applications in the Arnoldi process)
 *   flag       device int32 [B][R]: 0 converged (relres <= tol), 1 maxit
 *              reached, 2 breakdown without convergence or a non-finite value
 *   relres     device double [B][R]: true ||f - A x|| / ||f|| at exit (A = L, f = -U
 *              with MUDIFF_NO_PRECOND)
 *   iters      device int32 [B][R]: inner iterations performed
 *   resvec     device double [B][R][maxit+1] Arnoldi residual estimates
 *              |g_{j+1}| / ||f|| (entry 0 = initial), or NULL
 * Non-convergence is not an error: the call returns MUDIFF_OK with flag != 0.
 * Columns that converge stop iterating (their Krylov work is skipped).
 * With MUDIFF_BLOCK the columns r = k s .. k s + s - 1 of each instance form
 * block k (the last one may be narrower) and share one block Krylov space
 * (block Arnoldi; the paper's solver is single-vector GMRES, sec. 5): each step
 * applies the operator to the block's s basis vectors in one batched apply,
 * orthogonalises against the block basis (classical Gram-Schmidt twice), and
 * factors the new block by Cholesky QR twice, dropping directions whose pivot
 * falls below 1e-14 of the column's squared norm.  The least-squares problem
 * is triangularised by Householder reflectors as it grows, giving each column's
 * residual estimate after every step; a block stops when all its columns meet
 * tol (or at maxit), and at a restart the columns whose true residual meets
 * tol leave the block.  iters counts block steps, resvec the estimates.  The
 * restart cycle is one block step sequence of up to `restart` steps (block
 * Krylov dimension restart * s).  The straggler compaction of the lockstep
 * solver is not used.
 * With MUDIFF_SSTEP (s-step GMRES; same iterates as the one-vector process up
 * to rounding) the first cycle runs as above and gives each column s shifts,
 * the Ritz values of its Hessenberg matrix in Leja order; every later cycle
 * builds its basis s vectors at a time, v_i = (op - theta_i) v_{i-1} / sigma_i
 * (sigma_i the largest distance from theta_i to a Ritz value) by s operator
 * applies back to back, then orthogonalises the s vectors at once
 * (classical Gram-Schmidt against the basis and Cholesky QR within, both
 * twice) and derives the s Hessenberg columns from the coefficients; each
 * column's residual estimate and stopping test still follow every column.
 * A cycle that raises some column's true residual (a basis that lost
 * orthogonality) is undone for that column, and the solve continues with
 * one-vector cycles.
 * Fewer, larger reductions per step: for latency-bound sizes (one right-hand
 * side) the reductions, for bandwidth-bound ones (many right-hand sides) the
 * sweeps over the basis (two per s steps instead of two per step).  Every
 * apply path takes the shift (one-lane, generic, FP64-MFMA direct and
 * circulant forms); not with MUDIFF_BLOCK.
 * Errors: MUDIFF_ERR_INVALID for a block or s-step size out of range, or
 * unknown flags. */
int mudiff_gmres(mudiff_t h, int R, const double* beta, const void* rhs, void* rho,
                 int restart, double tol, int maxit, int flags,
                 void* workspace, size_t ws_bytes,
                 int32_t* flag, double* relres, int32_t* iters, double* resvec,
                 void* stream);

/* ---------------------------------------------------------------- far field */

/* a(theta_j) = sum_p sum_m (a_L)^p_m(theta_j) rho^p_m (sec. 4.4), for the
 * single-layer density rho [B][R][N_b] (complex128, device).
 *   theta      device [n_theta] angles (radians), direction (cos, sin)
 *   a_out      device complex128 [B][R][n_theta] */
int mudiff_farfield(mudiff_t h, int R, const void* rho, int n_theta, const double* theta,
                    void* a_out, void* stream);

/* ---------------------------------------------------------------- near field */

/* Field at points of the propagation domain (sec. 4.4, Graf's addition theorem):
 *   u(x) = sum_p sum_m (i sqrt(pi/8)) F^p_m rho^p_m H_m(k r_p) e^{i m theta_p},
 * (r_p, theta_p) the polar coordinates of x - O_p, F^p_m = sqrt(a_p) J_m(k a_p)
 * (single-layer potential) or, after mudiff_set_operator, f_L sqrt(a) J_m -
 * f_M k sqrt(a) J'_m (its far-field weights: single- plus double-layer potential).
 *   rho    device complex128 [B][R][N_b] densities
 *   pts    device double [n_pts][2], shared by all instances
 *   beta   device [B][R] incidence angles: the total field u_inc + u; or NULL:
 *          the scattered field u
 *   flags  0, or MUDIFF_POINT_SOURCE: beta holds [B][R][2] source positions and
 *          u_inc = (i/4) H_0(k |x - s|) (infinite at x = s)
 *   out    device complex128 [B][R][n_pts]; 0 at points inside a disk
 * Errors: MUDIFF_ERR_INVALID (also for other flags). */
int mudiff_nearfield(mudiff_t h, int R, const void* rho, int n_pts, const double* pts,
                     const double* beta, int flags, void* out, void* stream);

/* ---------------------------------------------------------------- gradient */

size_t mudiff_grad_workspace_size(mudiff_t h, int R, int n_rec, int restart, int flags);

/* Misfit loss_b = sum_{r, j} |a_b(theta_j; beta_{b,r}) - target_{b,r,j}|^2 of the
 * far field of every instance, and its gradient with respect to every disk
 * center, radius and the wavenumber (truncation orders held fixed), by one
 * forward and one adjoint solve per column.  The adjoint solve reuses the
 * forward operator through L^T = P L P (P flips m -> -m in every disk).
 *   beta       device [B][R] incidence angles
 *   theta_rec  device [n_rec] receiver angles
 *   target     device complex128 [B][R][n_rec]
 *   loss       device double [B]
 *   d_centers  device double [M_tot][2];  d_radii [M_tot];  d_k [B]
 * flags: MUDIFF_GRAPH and MUDIFF_SSTEP (with MUDIFF_SSTEP_SIZE) apply to both
 * solves as in mudiff_gmres; mudiff_grad_workspace_size takes the same flags.
 * Returns MUDIFF_ERR_NOT_CONVERGED (outputs undefined) if a solve fails to
 * reach tol within maxit. */
int mudiff_grad(mudiff_t h, int R, const double* beta, int n_rec, const double* theta_rec,
                const void* target, int restart, double tol, int maxit, int flags,
                void* workspace, size_t ws_bytes,
                double* loss, double* d_centers, double* d_radii, double* d_k, void* stream);

/* ---------------------------------------------------------------- time reversal */

/* The far-field mirror of sec. 7 (Example III): N_alpha cells at the angles
 * alpha_j send plane waves (incidence alpha_j) and record the far field in the
 * opposite direction, so that F[i][j] = a(alpha_i + pi; alpha_j) (obtained with
 * mudiff_gmres for R = N_alpha incidences and mudiff_farfield at the angles
 * alpha_i + pi).  In these calls F is passed as X = F^T, X[j][i] = F[i][j]:
 * complex128, row-major [n][m] (n incidences, m receivers), which is exactly
 * mudiff_farfield's output for one instance. */

/* T = conj(F)^T F, the time-reversal matrix: T[a][b] = sum_i conj(X[a][i]) X[b][i].
 *   X  device complex128 [n][m];  T  device complex128 [n][n] (Hermitian, PSD)
 * FP64 matrix-core kernel; enqueues on `stream`.  Errors: MUDIFF_ERR_INVALID. */
int mudiff_tro(int n, int m, const void* X, void* T, void* stream);

/* Eigen-decomposition of T = conj(F)^T F without forming T: one-sided Jacobi
 * rotations orthogonalise the columns of F (rows of X), F V = [f_1 .. f_n] with
 * f_j^H f_k = 0, so T V = V diag(|f_j|^2).
 *   X          device complex128 [n][m], overwritten with (F V)^T
 *   w          device double [n]: eigenvalues of T, decreasing
 *   evec       device complex128 [n][n]: row j = unit eigenvector of w[j]
 *              (component index second), unique up to a phase where w[j] is simple
 *   max_sweeps >= 1; tol > 0: a column pair counts as orthogonal when
 *              |f_p^H f_q| <= tol |f_p| |f_q|, or <= eps |F|_F^2 (the rounding
 *              level of the entries of T; eps = 2^-52)
 *   workspace  device, 256-byte aligned, >= mudiff_tro_eigh_workspace_size(n, m)
 *   sweeps     [host] out: sweeps used, or -1 if max_sweeps ran out (the outputs
 *              are then the last iterate)
 * Synchronises `stream` once per sweep.  Errors: MUDIFF_ERR_INVALID,
 * MUDIFF_ERR_NOMEM, MUDIFF_ERR_DEVICE. */
size_t mudiff_tro_eigh_workspace_size(int n, int m);
int mudiff_tro_eigh(int n, int m, void* X, double* w, void* evec, int max_sweeps, double tol,
                    void* workspace, size_t ws_bytes, int32_t* sweeps, void* stream);

/* Discrete Herglotz waves u_t(x) = sum_j h f_t[j] exp(i k (x_1 cos alpha_j + x_2 sin alpha_j))
 * (sec. 7) for n_f parameter vectors at n_pts points.
 *   alpha  device double [n_alpha];  f  device complex128 [n_f][n_alpha]
 *   pts    device double [n_pts][2];  u  device complex128 [n_f][n_pts]
 * Errors: MUDIFF_ERR_INVALID (sizes, k <= 0, NULL pointers). */
int mudiff_herglotz(int n_alpha, const double* alpha, int n_f, const void* f, double k, double h,
                    int n_pts, const double* pts, void* u, void* stream);

/* ---------------------------------------------------------------- device probes */

/* Achievable throughput of the current device, so that kernel rates can be
 * reported against measured as well as published peaks.  Not part of the
 * method (the paper has no counterpart).
 *   kind       MUDIFF_PROBE_FP64_FMA   loop of independent FP64 fused multiply-adds
 *                                      on the vector ALUs (8 workgroups per CU)
 *              MUDIFF_PROBE_FP64_MFMA  loop of v_mfma_f64_16x16x4f64 on the matrix
 *                                      cores (8 independent accumulators per wave)
 *              MUDIFF_PROBE_COPY       device-to-device copy of `bytes` bytes
 *                                      (rounded down to a multiple of 16)
 *   bytes      COPY only (>= 16); ignored otherwise
 *   workspace  device, 256-byte aligned, >= mudiff_probe_workspace_size(kind, bytes)
 *              bytes (its contents are overwritten)
 *   rate       [host] out: TFLOP/s (FMA, MFMA) or GB/s of read + write (COPY)
 * One warm-up launch, then three launches timed with HIP events on `stream`;
 * synchronises the stream.  Errors: MUDIFF_ERR_INVALID (kind, NULL pointer,
 * alignment), MUDIFF_ERR_NOMEM (workspace too small), MUDIFF_ERR_DEVICE. */
enum { MUDIFF_PROBE_FP64_FMA = 0, MUDIFF_PROBE_FP64_MFMA = 1, MUDIFF_PROBE_COPY = 2 };
size_t mudiff_probe_workspace_size(int kind, size_t bytes);
int mudiff_probe(int kind, size_t bytes, void* workspace, size_t ws_bytes, double* rate,
                 void* stream);

/* Phase timing of the operator apply (a measurement aid; the paper has no
 * counterpart).  Between mudiff_profile_begin and mudiff_profile_end, the first
 * max_applies complete operator applies on this handle that are not being
 * captured into a graph (those of mudiff_matvec, the multi-right-hand-side
 * ones inside the solvers, and the residual applies of a restart cycle) record
 * HIP events on their stream between their phases:
 *   0 input scaled by its column factors (multi-right-hand-side applies),
 *   1 forward transforms and 2 per-frequency products (circulant form),
 *   3 the MFMA work queue, or the one-lane / generic kernel,
 *   4 output pass (partial sums, inverse transforms, epilogue).
 * Recording adds no synchronisation.  mudiff_profile_end synchronises on the
 * last event and returns the number of profiled applies and the summed
 * milliseconds of each phase (phases an apply does not have count 0), then
 * releases the events.  Errors: MUDIFF_ERR_INVALID, MUDIFF_ERR_DEVICE. */
#define MUDIFF_N_PHASES 5
int mudiff_profile_begin(mudiff_t h, int max_applies);
int mudiff_profile_end(mudiff_t h, int* n_applies, double* ms /*[host] MUDIFF_N_PHASES*/);

/* Thread-local message of the last failing call on this thread. */
const char* mudiff_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MUDIFF_H */
