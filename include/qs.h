/*
 * qs.h -- C ABI of libqs, batched state-vector simulation of parameterised
 * quantum circuits on AMD MI355X (gfx950), forward and adjoint gradient.
 *
 * Definitions the calls implement (standard sources, restated):
 *   - Gates: Pauli rotations R_P(t) = exp(-i t P / 2) for P in {X, Y, Z}
 *     (Nielsen & Chuang, Quantum Computation and Quantum Information, 2010,
 *     sec. 4.2, eqs. 4.4-4.6); Paulis, Hadamard, CNOT and CZ (sec. 4.3).
 *   - Qubit q is bit q of the amplitude index (little-endian).
 *   - Amplitude encoding |x> = x / ||x||_2, zero-padded to 2^n (Schuld &
 *     Petruccione, Supervised Learning with Quantum Computers, 2018, sec. 5.2).
 *   - Readout <Z_q> = sum_i |psi_i|^2 (1 - 2 bit_q(i)).
 *   - Adjoint gradient (Jones & Gacon, arXiv:2009.02823, sec. 3): with a state
 *     cotangent lam (dL = 2 Re <lam|d psi>), dL/dtheta_g = Im <lam_g|P_g|psi_g>.
 *
 * Layouts. A batch of states is `[B][2^n]` complex numbers stored as
 * interleaved (re, im) pairs of `float` (QS_C64) or `double` (QS_C128), row b
 * contiguous, amplitude index i in logical order. Parameters and features use
 * the real type of the state dtype: float for QS_C64, double for QS_C128.
 *
 * Ownership. Every pointer argument marked (device) is caller-owned device
 * memory that must stay valid until the stream reaches the call; (host)
 * pointers are read before the call returns. Input buffers must not alias
 * output buffers, except `state`, which is in/out by design. The library owns
 * only its plan caches (device copies of planned gate programs; for uneven
 * batches also a queue counter, an adjoint workspace and up to three side
 * streams with their events), released by qs_shutdown().
 *
 * Errors. Every call returns a qs_status; nothing throws across the ABI.
 * Launch-side calls are asynchronous on the given stream (a hipStream_t
 * passed as void*, NULL = the default stream). Shape and descriptor errors
 * are detected on the host before anything is enqueued. NaN or Inf values in
 * the inputs propagate into the outputs; they are not errors.
 */
#ifndef QS_H
#define QS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
typedef enum qs_status {
  QS_OK = 0,
  QS_ERR_INVALID = -1,     /* bad descriptor, shape, pointer or flag        */
  QS_ERR_UNSUPPORTED = -2, /* valid request the library does not implement */
  QS_ERR_WORKSPACE = -3,   /* workspace missing or smaller than required    */
  QS_ERR_ZERO_NORM = -4,   /* amplitude input row with norm 0               */
  QS_ERR_LAUNCH = -5,      /* a HIP runtime call or kernel launch failed    */
  QS_ERR_NOMEM = -6,       /* the plan cache could not allocate             */
  QS_ERR_CAPTURE = -7,     /* a new plan would have to be uploaded while the
                              call's stream is being captured into a graph:
                              nothing was enqueued and the capture stays
                              valid; run the call once before capturing     */
  QS_ERR_NOT_PLANNED = -8  /* a call that may not allocate met a shape with
                              no cached plan; nothing was enqueued          */
} qs_status;

/* ------------------------------------------------------------- descriptor */
/* Gate kinds (numbering is part of the descriptor format). */
enum {
  QS_OP_RX = 0, QS_OP_RY = 1, QS_OP_RZ = 2, /* R_P(theta), P = X, Y, Z      */
  QS_OP_X = 3, QS_OP_Y = 4, QS_OP_Z = 5,    /* Paulis                        */
  QS_OP_H = 6,                              /* Hadamard                      */
  QS_OP_CNOT = 7,                           /* q0 = control, q1 = target     */
  QS_OP_CZ = 8,                             /* symmetric in q0, q1           */
  QS_OP_RESET = 9,   /* mid-circuit channels on qubit q0, see below          */
  QS_OP_MEASURE = 10
};

/* Mid-circuit channels (one quantum trajectory per sample; the projective
 * measurement postulate, Nielsen & Chuang sec. 2.2.3). Qubit q0 is measured
 * in the Z basis: with p_m the FP64 sum of |psi_i|^2 over the amplitudes
 * whose bit q0 is m, the outcome is the smallest m with
 * u (p_0 + p_1) < p_0 + ... + p_m (else the last m with p_m > 0), u being
 * the sample's uniform feats[b][feat] in [0, 1) (random numbers are inputs);
 * the state is projected on bit q0 = m and divided by sqrt(p_m), and
 * QS_OP_RESET then moves it to bit q0 = 0 (Kraus operator |0><m|) while
 * QS_OP_MEASURE keeps it. Gradients hold the drawn outcome fixed (pathwise):
 * through the renormalisation, the cotangent in front of the channel is
 * K^dagger (lam' - Re<lam'|psi'> psi') / sqrt(p_m); no gradient reaches u.
 * A channel gate needs q1 = -1 and 0 <= feat < n_features (p_w, p_b, scale
 * are ignored). Circuits with channels run on the register/LDS engine
 * (QS_PATH_AUTO or QS_PATH_FUSED; other paths, QS_FLAG_INVERSE, the planning
 * and tuning calls and uneven-batch programs return QS_ERR_UNSUPPORTED or
 * QS_ERR_INVALID), and qs_forward / qs_adjoint_backward need a checkpoint at
 * every channel's gate index (the state in front of it, which the adjoint
 * restarts from; QS_ERR_INVALID otherwise). */

/* One gate, 32 bytes. The angle of a rotation on sample b is
 *   theta_b = scale * (w * f + bias),
 *   w    = params[p_w]        (1 when p_w  < 0),
 *   f    = feats[b][feat]     (1 when feat < 0),
 *   bias = params[p_b]        (0 when p_b  < 0).
 * With QS_FLAG_PER_SAMPLE_PARAMS, params is [B][n_params] and row b is used.
 * Non-rotation gates ignore p_w, feat, p_b and scale. */
typedef struct qs_gate {
  int32_t op;
  int32_t q0;
  int32_t q1;     /* -1 for 1-qubit gates */
  int32_t p_w;
  int32_t feat;
  int32_t p_b;
  float scale;
  int32_t flags;  /* reserved, must be 0 */
} qs_gate;

/* A circuit: `gates` is a host array of n_gates records. */
typedef struct qs_circuit {
  int32_t n_qubits;   /* 1 .. 30 */
  int32_t n_gates;    /* >= 0    */
  int32_t n_params;   /* >= 0; every p_w / p_b < n_params    */
  int32_t n_features; /* >= 0; every feat < n_features       */
  const qs_gate* gates;
} qs_circuit;

/* State dtypes. */
enum { QS_C64 = 0, QS_C128 = 1 };
/* Encodings for qs_encode. */
enum { QS_ENC_AMPLITUDE = 0, QS_ENC_ZERO = 1 };

/* Flags for qs_forward / qs_adjoint_backward / qs_workspace_size (and the
 * planning calls that take flags). The low byte selects the execution path.
 * QS_FLAG_INVERSE runs the circuit's inverse U^dagger: its gates in reverse
 * order with every rotation angle negated; checkpoint gate counts then count
 * gates of that reversed list, and gradients are those of U^dagger's
 * parameters (the same parameter vector). */
enum {
  QS_PATH_AUTO = 0,   /* register/LDS-resident engine when it fits, else HBM */
  QS_PATH_FUSED = 1,  /* register/LDS-resident engine (n <= 14)              */
  QS_PATH_PLAIN = 2,  /* one kernel launch per gate, state in HBM            */
  QS_PATH_HBM = 3,    /* state in HBM, run as epochs of gathered m-qubit
                         tiles through the register/LDS engine (n > 14)     */
  QS_PATH_MFMA = 4,   /* state in HBM, gates fused into dense 5-qubit blocks,
                         each applied in one pass as a complex matrix product
                         on MFMA (complex64, angles shared by the batch,
                         n >= 10); QS_PATH_AUTO takes it for large states
                         when qs_autotune found it faster than QS_PATH_HBM */
  QS_PATH_MASK = 0xff,
  QS_FLAG_PER_SAMPLE_PARAMS = 0x100, /* params is [B][n_params]           */
  QS_FLAG_INVERSE = 0x200            /* run U^dagger instead of U          */
};

/* ------------------------------------------------------------------ calls */

/* Version of the library, major * 10000 + minor * 100 + patch. */
int qs_version(void);

/* Static text for a status code. Never NULL. */
const char* qs_status_string(int status);

/* Host only, never touches a GPU. Checks that the descriptor is well formed:
 * 1 <= n_qubits <= 30, known op codes, qubits in range, distinct qubits for
 * CNOT/CZ, q1 = -1 for 1-qubit gates, parameter and feature indices in range
 * for rotations, flags = 0. Returns QS_OK or QS_ERR_INVALID. */
int qs_validate(const qs_circuit* circuit);

/* Encode a batch into states (qs_forward's input form).
 *   enc      QS_ENC_AMPLITUDE: state[b] = pad(x[b]) / ||x[b]||_2, with the
 *            squared norm accumulated in FP64 (D <= 2^n required);
 *            QS_ENC_ZERO: state[b] = |0...0> (x, D, x_stride ignored).
 *   dtype    QS_C64 or QS_C128.
 *   x        (device) [B][x_stride] real inputs, first D used per row;
 *            float32 when x_is_f64 == 0, float64 otherwise.
 *   state    (device) [B][2^n] complex output.
 *   bad_rows (device, optional) int32 counter; the number of zero-norm rows
 *            is ADDED to it (those rows become NaN). The host cannot see this
 *            without a sync, so the call itself returns QS_OK for them;
 *            qs_encode_check reads the counter. */
int qs_encode(int enc, int dtype, int n_qubits, int64_t B, int64_t D,
              int x_is_f64, const void* x, int64_t x_stride, void* state,
              int32_t* bad_rows, void* stream);

/* Synchronous: waits for `stream`, then reads the bad_rows counter that
 * qs_encode / qs_program_encode added to (device, int32). Returns
 * QS_ERR_ZERO_NORM when it is non-zero (some amplitude input row had norm 0
 * and became NaN), QS_OK when it is zero, QS_ERR_INVALID for a NULL counter,
 * QS_ERR_CAPTURE while the stream is being captured (a capture cannot wait),
 * QS_ERR_LAUNCH when the wait or the copy fails. */
int qs_encode_check(const int32_t* bad_rows, void* stream);

/* Forward sweep: state[b] <- U_G(theta_G(b)) ... U_1(theta_1(b)) state[b].
 *   params   (device) [n_params] or [B][n_params] (QS_FLAG_PER_SAMPLE_PARAMS)
 *   feats    (device) [B][n_features] or NULL when n_features == 0
 *   state    (device) [B][2^n] complex, in: encoded input, out: final state
 *   expz     (device, optional) [B][n] double, receives <Z_q>_b summed in FP64
 *   ckpt_gates (host, optional) n_ckpt strictly increasing gate counts in
 *            (0, n_gates) (0 is allowed when gate 0 is a channel); after the
 *            first ckpt_gates[i] gates the state is copied to
 *            ckpt + i * B * 2^n (complex elements)
 *   ckpt     (device) [n_ckpt][B][2^n] complex, required when n_ckpt > 0
 *   flags    path selection (QS_PATH_*) | QS_FLAG_PER_SAMPLE_PARAMS */
int qs_forward(const qs_circuit* circuit, int dtype, int64_t B,
               const void* params, const void* feats, void* state,
               double* expz, const int32_t* ckpt_gates, int32_t n_ckpt,
               void* ckpt, int flags, void* stream);

/* Amplitude encoding and forward sweep in one call (the input of the
 * sweep's first step, then the sweep): state[b] <- U(theta(b)) pad(x[b]) /
 * ||x[b]||_2, with qs_encode's QS_ENC_AMPLITUDE definition of the encoded
 * state (squared norm summed in FP64, zero padding to 2^n). The encoded
 * state is never stored: the register/LDS engine normalises each sample as
 * it loads it when x is in the state's precision (float32 for QS_C64,
 * float64 for QS_C128); every other case runs qs_encode into `state` first.
 *   x, x_is_f64, D, x_stride  as qs_encode (device [B][x_stride] reals, the
 *            first D <= 2^n of each row used)
 *   bad_rows (device, optional) int32 counter; zero-norm rows become NaN and
 *            add one each, as in qs_encode (read it with qs_encode_check)
 *   state    (device) [B][2^n] complex output: the final state only
 *   other arguments and errors as qs_forward; QS_ERR_INVALID also for a
 *   NULL x, D outside [1, 2^n] or x_stride < D when B > 0. */
int qs_forward_amplitude(const qs_circuit* circuit, int dtype, int64_t B,
                         const void* params, const void* feats, const void* x,
                         int x_is_f64, int64_t D, int64_t x_stride, int32_t* bad_rows,
                         void* state, double* expz, const int32_t* ckpt_gates,
                         int32_t n_ckpt, void* ckpt, int flags, void* stream);

/* Mean-squared-error loss on one qubit's readout and its upstream gradient
 * (the regression loss of the training step; one kernel):
 *   loss[0]        = (1/B) sum_b (expz[b][q] - y[b])^2, FP64, summed in a
 *                    fixed order (bitwise reproducible)
 *   dexpz[b][k]    = (2/B)(expz[b][q] - y[b]) for k == q, 0 for k != q
 *   expz  (device) [B][n] double, y (device) [B] double,
 *   dexpz (device) [B][n] double output (may be NULL), loss (device) [1]
 *   double output (may be NULL). QS_ERR_INVALID for n < 1, q outside
 *   [0, n), B < 0 or a NULL expz / y when B > 0. B == 0 writes loss = 0. */
int qs_loss_mse_z(int n_qubits, int64_t B, int q, const double* expz, const double* y,
                  double* dexpz, double* loss, void* stream);

/* A training step with the MSE loss on one qubit in one engine launch:
 * the forward sweep from the amplitude encoding of x (qs_forward_amplitude's
 * definition) or, with x NULL, from |0...0>; <Z> in FP64; the loss and its
 * upstream gradient (qs_loss_mse_z's definitions, loss_q = q); the adjoint
 * (qs_adjoint_backward's gradients). The state stays in registers from the
 * encoding to the last gradient: no state is read from or written to HBM.
 * Results equal those of qs_forward_amplitude (or qs_encode + qs_forward),
 * qs_loss_mse_z and qs_adjoint_backward up to rounding order.
 *   x, x_is_f64, D, x_stride, bad_rows  as qs_forward_amplitude, or x NULL
 *   y        (device) [B] double labels
 *   expz     (device, optional) [B][n] double, receives <Z_q>_b
 *   loss     (device) [1] double, receives (1/B) sum_b (<Z_q>_b - y_b)^2,
 *            summed per workgroup in sample order, then over workgroups in
 *            a fixed order
 *   grad_params (device) [n_params] double (overwritten), grad_feats
 *            (device, optional) [B][n_features] double (overwritten)
 *   ws, ws_bytes  (device) at least qs_train_workspace_size() bytes
 * Runs only where that kernel exists: complex64, parameters shared by the
 * batch, no channels, and a register/LDS engine shape with register tile
 * 2^4 or 2^5 staging whole amplitudes (the adjoint's tuned shape). Other
 * cases return QS_ERR_UNSUPPORTED before any device work (callers then use
 * the three calls above), as does a float64 x. B == 0 does nothing. */
int qs_train_step_mse(const qs_circuit* circuit, int dtype, int64_t B, const void* params,
                      const void* feats, const void* x, int x_is_f64, int64_t D,
                      int64_t x_stride, int32_t* bad_rows, const double* y, int q,
                      double* expz, double* loss, double* grad_params, double* grad_feats,
                      void* ws, size_t ws_bytes, int flags, void* stream);

/* Workspace bytes of qs_train_step_mse for this shape (host only); 0 when
 * the one-launch training step does not run for it. */
size_t qs_train_workspace_size(const qs_circuit* circuit, int dtype, int64_t B, int flags);

/* Bytes of device workspace qs_adjoint_backward needs for this shape. */
size_t qs_workspace_size(const qs_circuit* circuit, int dtype, int64_t B,
                         int flags);

/* Adjoint backward from the final state of qs_forward.
 *   state    (device) [B][2^n] final state psi_G (read only)
 *   dexpz    (device) [B][n] double dL/d<Z_q>_b, giving lam = sum_q dexpz Z_q psi_G
 *   dstate   (device) [B][2^n] complex state cotangent lam (dL = 2Re<lam|dpsi>)
 *            exactly one of dexpz / dstate is non-NULL
 *   grad_params (device) [n_params] double, batch-summed in FP64; with
 *            QS_FLAG_PER_SAMPLE_PARAMS [B][n_params]. Overwritten.
 *   grad_feats  (device, optional) [B][n_features] double. Overwritten.
 *   ckpt_gates / n_ckpt / ckpt  the checkpoints qs_forward stored (optional);
 *            when given, psi is re-anchored to them on the way back
 *   ws, ws_bytes  (device) workspace of qs_workspace_size() bytes */
int qs_adjoint_backward(const qs_circuit* circuit, int dtype, int64_t B,
                        const void* params, const void* feats,
                        const void* state, const double* dexpz,
                        const void* dstate, double* grad_params,
                        double* grad_feats, const int32_t* ckpt_gates,
                        int32_t n_ckpt, const void* ckpt, void* ws,
                        size_t ws_bytes, int flags, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): qs_adjoint_backward
 * without a workspace argument. The per-block gradient partial sums go to a
 * library-owned device array of QS_NOALLOC_SCRATCH_BYTES per GPU (a static
 * device global, held until the process ends); the call allocates nothing.
 * Same arguments, results and errors as qs_adjoint_backward, plus:
 *   - only the register/LDS engine path runs (QS_PATH_AUTO choosing it, or
 *     QS_PATH_FUSED); another path gives QS_ERR_UNSUPPORTED;
 *   - the partial sums of this shape must fit QS_NOALLOC_SCRATCH_BYTES
 *     (qs_workspace_size() <= that), else QS_ERR_WORKSPACE;
 *   - the shape's plan must already be cached by an earlier allocating call
 *     (qs_adjoint_backward with the same circuit, dtype, flags and
 *     checkpoints), else QS_ERR_NOT_PLANNED; the autotuner never runs.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (different streams, or host threads) race on it and must not be
 * issued. Calls ordered on one stream are safe. */
#define QS_NOALLOC_SCRATCH_BYTES (32u << 20)
int qs_adjoint_backward_noalloc(const qs_circuit* circuit, int dtype, int64_t B,
                                const void* params, const void* feats,
                                const void* state, const double* dexpz,
                                const void* dstate, double* grad_params,
                                double* grad_feats, const int32_t* ckpt_gates,
                                int32_t n_ckpt, const void* ckpt, int flags,
                                void* stream);

/* Readout alone: expz[b][q] = <Z_q>_b of state [B][2^n], FP64 sums. */
int qs_expz(int dtype, int n_qubits, int64_t B, const void* state,
            double* expz, void* stream);

/* Autoencoder fidelity with the top n_trash qubits reset to |0> (Romero,
 * Olson & Aspuru-Guzik, Quantum Sci. Technol. 2, 045001, 2017): with
 * psi = U|x> and chi = V|x> (the decoder being V^dagger),
 *   c_m = <chi_0|psi_m>,  F_b = sum_m |c_m|^2   (FP64),
 * where psi_m is the slice of psi whose trash bits equal m and chi_0 the slice
 * of chi whose trash bits are 0.
 *   fid      (device) [B] double output
 *   dfid     (device, optional) [B] double dL/dF_b; when given, the state
 *            cotangents lam_psi = dfid_b sum_m c_m |m>|chi_0> and
 *            lam_chi = dfid_b |0> sum_m conj(c_m) psi_m are written
 *            (both [B][2^n] complex, device).
 * 0 <= n_trash <= 6, < n. B = 0 does nothing. Returns QS_ERR_INVALID for a
 * bad dtype or size, or a missing pointer when B > 0. */
int qs_fidelity_reset(int dtype, int n_qubits, int n_trash, int64_t B,
                      const void* psi, const void* chi, double* fid,
                      const double* dfid, void* lam_psi, void* lam_chi,
                      void* stream);

/* Post-selected autoencoder fidelity: the top n_trash qubits are measured
 * and only the all-zero outcome is kept, renormalised (the projective
 * measurement postulate, Nielsen & Chuang sec. 2.2.3). With psi_0 and chi_0
 * the trash-0 slices (the first 2^(n - n_trash) amplitudes), in FP64:
 *   c = <chi_0|psi_0>,  p = ||psi_0||^2,  F'_b = |c|^2 / p;
 * a row with p = 0 (the outcome cannot occur) gives NaN.
 *   psi, chi (device) [B][2^n] complex, read only; 0 <= n_trash < n
 *   fid      (device) [B] double output
 *   dfid     (device, optional) [B] double dL/dF'_b; when given, the state
 *            cotangents (dL = 2 Re<lam|d psi>)
 *              lam_psi = dfid_b ((c/p) chi_0 - (F'/p) psi_0),
 *              lam_chi = dfid_b (conj(c)/p) psi_0
 *            on the trash-0 slice and zero elsewhere are written (both
 *            [B][2^n] complex, device, caller-owned).
 * B = 0 does nothing. Returns QS_ERR_INVALID for a bad dtype or size, or a
 * missing pointer when B > 0. */
int qs_fidelity_postselect(int dtype, int n_qubits, int n_trash, int64_t B,
                           const void* psi, const void* chi, double* fid,
                           const double* dfid, void* lam_psi, void* lam_chi,
                           void* stream);

/* One quantum trajectory of the reset channel (its unravelling into
 * measurement outcomes: Dalibard, Castin & Molmer, PRL 68, 580, 1992): the
 * top n_trash qubits are measured, outcome m drawn from the Born
 * probabilities by the caller's uniform u_b in [0, 1), then reset to |0>.
 * With psi_m the slice of psi whose trash bits equal m, in FP64:
 *   p_m = ||psi_m||^2,  m_b = the smallest m with u_b sum_j p_j < p_0 + ... + p_m
 *   (the sums in m order; the last m with p_m > 0 if rounding leaves none),
 *   c = <chi_0|psi_m>,  F_b = |c|^2 / p_m.
 * Its average over outcomes (weights p_m / sum p) is the reset-channel
 * fidelity of qs_fidelity_reset. A row of zeros gives NaN (outcome 0).
 *   psi, chi (device) [B][2^n] complex, read only; 0 <= n_trash <= 6, < n
 *   u        (device) [B] double uniforms (the random numbers are inputs)
 *   fid      (device) [B] double output
 *   outcome  (device, optional) [B] int32 output, the drawn m_b
 *   dfid     (device, optional) [B] double dL/dF_b; when given, the state
 *            cotangents for the drawn outcome (dL = 2 Re<lam|d psi>)
 *              lam_psi = dfid_b ((c/p) chi_0 - (F/p) psi_m) on slice m,
 *              lam_chi = dfid_b (conj(c)/p) psi_m on slice 0,
 *            zero elsewhere, are written (both [B][2^n] complex, device).
 * B = 0 does nothing. Returns QS_ERR_INVALID for a bad dtype or size, or a
 * missing pointer when B > 0. */
int qs_fidelity_trajectory(int dtype, int n_qubits, int n_trash, int64_t B,
                           const void* psi, const void* chi, const double* u,
                           double* fid, int32_t* outcome, const double* dfid,
                           void* lam_psi, void* lam_chi, void* stream);

/* ------------------------------------------------------- uneven batches */
/* Many circuits of uneven qubit count and depth in one persistent launch.
 * Circuits are grouped into classes of identical structure (same gate list);
 * class k has counts[k] circuits, each with its own parameter set and state.
 * Device buffers are packed class after class, circuit-major inside a class:
 *   states        [sum_k counts[k] * 2^n_k]   complex (c64 / c128)
 *   x (encode)    [sum_k counts[k] * 2^n_k]   real, same offsets as states
 *   params        [sum_k counts[k] * P_k]     real (P_k = n_params of class k)
 *   expz, dexpz   [sum_k counts[k] * n_k]     double
 *   grad_params   [sum_k counts[k] * P_k]     double (overwritten)
 * Workgroups pull work items (a run of circuits of one class) from an atomic
 * queue ordered longest first, so the uneven costs balance across the chip.
 * A class whose 2^n_k amplitudes need more than one workgroup (QS_C128 at 14
 * qubits) runs through qs_forward / qs_adjoint_backward on its slices of the
 * same buffers, on up to three library-owned side streams that are forked
 * from `stream` before the persistent launch and joined back into it (with
 * events) before the call returns: all work of the call is ordered on
 * `stream` as usual.
 * Restrictions: no features; 5 <= n_k <= 14 for QS_C64, 4 <= n_k <= 14 for
 * QS_C128. Calls on the same program must not overlap in time (they share
 * the library-owned queue counter and adjoint workspace). */
typedef struct qs_program {
  int32_t n_classes;
  const qs_circuit* circuits; /* [n_classes] (host) */
  const int64_t* counts;      /* [n_classes] circuits per class (host) */
} qs_program;

/* Host only: offsets (in elements) of each class inside the packed buffers,
 * and totals[3] = {state elements, parameter elements, expz elements}. Any
 * output pointer may be NULL. */
int qs_program_layout(const qs_program* prog, int64_t* state_off,
                      int64_t* param_off, int64_t* expz_off, int64_t* totals);

/* Amplitude-encode every circuit's input (x packed like states, real). */
int qs_program_encode(const qs_program* prog, int dtype, const void* x,
                      int x_is_f64, void* states, int32_t* bad_rows,
                      void* stream);

/* Forward sweep of every circuit in one persistent launch; expz optional. */
int qs_program_forward(const qs_program* prog, int dtype, const void* params,
                       void* states, double* expz, void* stream);

/* Adjoint of every circuit in one persistent launch, from the final states
 * and dL/d<Z> rows; per-circuit parameter gradients. */
int qs_program_adjoint(const qs_program* prog, int dtype, const void* params,
                       const void* states, const double* dexpz,
                       double* grad_params, void* stream);

/* What the planner decided for a circuit on the fused engine (host only).
 * The forward and the adjoint may use different register tiles (both read
 * and write states in logical order, so they need not agree). */
typedef struct qs_plan_info {
  int32_t path;              /* QS_PATH_FUSED or QS_PATH_PLAIN / QS_PATH_HBM */
  int32_t log2_regs;         /* amplitudes per thread = 2^log2_regs          */
  int32_t log2_threads;      /* threads per sample = 2^log2_threads          */
  int32_t samples_per_block; /* samples per workgroup                        */
  int32_t block_threads;     /* threads per workgroup                        */
  int32_t n_segments;        /* register-resident segments                   */
  int32_t n_remaps;          /* LDS remaps between segments (forward)        */
  int32_t n_ops;             /* gates as scheduled (qs_plan_export rows)     */
  int64_t lds_bytes;         /* dynamic LDS per workgroup                    */
  int32_t adj_log2_regs;     /* the adjoint's amplitudes-per-thread exponent */
  int32_t adj_samples_per_block;
  int32_t adj_block_threads;
  int32_t n_engine_ops;      /* engine operations after grouping gates into
                                layer ops (fused single-qubit blocks on all
                                register bits; CZ sets as one sign pattern) */
} qs_plan_info;

/* Fill `out` with the plan the engine would use (host only, no GPU). */
int qs_plan_info_get(const qs_circuit* circuit, int dtype, int64_t B,
                     int flags, qs_plan_info* out);

/* Host only: what a large-state path (QS_PATH_HBM or QS_PATH_MFMA) runs for
 * this circuit with these checkpoints (the same gate counts qs_forward and
 * qs_adjoint_backward take; ckpt_gates may be NULL when n_ckpt == 0).
 * Returns QS_ERR_UNSUPPORTED when the circuit takes neither path. */
typedef struct qs_hbm_info {
  int32_t path;              /* QS_PATH_HBM or QS_PATH_MFMA                  */
  int32_t n_passes;          /* epochs (QS_PATH_HBM) or dense blocks
                                (QS_PATH_MFMA): kernel launches over the
                                whole state per direction                    */
  int32_t tile_qubits;       /* qubits of a tile-sample (m), or of a block  */
  int32_t reserved;
  int64_t max_partial_bytes; /* largest gradient partial-sum area any adjoint
                                pass of this plan writes                     */
  int64_t ws_bytes;          /* qs_workspace_size() for these flags: covers
                                every checkpoint placement                   */
} qs_hbm_info;
int qs_hbm_info_get(const qs_circuit* circuit, int dtype, int64_t B, int flags,
                    const int32_t* ckpt_gates, int32_t n_ckpt, qs_hbm_info* out);

/* Host only: the dense-block plan of QS_PATH_MFMA, for inspection and for
 * checking the planner on the CPU. Call with NULL arrays to get *n_blocks;
 * then, with arrays of these sizes, fills
 *   blk_qubits [n_blocks][5] the block's qubits, ascending (local bit i of
 *              the block's 32 x 32 matrix = qubit blk_qubits[b][i]),
 *   blk_begin  [n_blocks + 1] ranges of blk_gates,
 *   blk_gates  [n_gates] descriptor gate indices in the order each block
 *              multiplies them (every gate exactly once),
 *   blk_ckpt   [n_blocks] checkpoint slot stored after the block, or -1.
 * Returns QS_ERR_UNSUPPORTED when the circuit cannot take QS_PATH_MFMA. */
int qs_block_plan_export(const qs_circuit* circuit, int dtype, int flags,
                         const int32_t* ckpt_gates, int32_t n_ckpt, int32_t* n_blocks,
                         int32_t* blk_qubits, int32_t* blk_begin, int32_t* blk_gates,
                         int32_t* blk_ckpt);

/* Host only: export the fused engine's plan for inspection (tests, tools).
 * Fills `info` like qs_plan_info_get; then, when the arrays are non-NULL,
 * copies  ops [info->n_ops][4] int32 = (gate kind, physical position a,
 * physical position b, descriptor gate index) in execution order,
 * seg_begin [info->n_segments + 1] int32 op ranges, and
 * seg_map [info->n_segments][16] uint8 = logical qubit at each physical bit
 * position (positions below log2_regs are register bits). Returns
 * QS_ERR_UNSUPPORTED when the circuit does not take the fused path. */
int qs_plan_export(const qs_circuit* circuit, int dtype, int64_t B, int flags,
                   qs_plan_info* info, int32_t* ops, int32_t* seg_begin,
                   uint8_t* seg_map);

/* Host only: the engine program itself, for inspection and for checking the
 * planner on the CPU (a test can execute it and compare with a reference).
 * `adjoint` selects the register split of the adjoint's plan instead of the
 * forward's. Call once with NULL arrays to get the sizes in `info`, then with
 * arrays of those sizes:
 *   ops        [n_ops][5] int32  kind, a, b, aux, gate: kind 16 (a layer
 *                                op), a = mask of register bits with a
 *                                block, aux bit 0 = per-sample angles,
 *                                gate = its l1q record
 *   seg_begin  [n_segments + 1] int32 op ranges
 *   seg_lay    [n_segments][32] uint16 logical index mask of each physical
 *              bit: 16 for reading the segment in, 16 for writing it out
 *   l1q        [n_l1q][16] int32 words 0..4: block id per register bit (-1:
 *              none); word 5: sign pattern applied before the blocks, word
 *              7: after them (diag record, -1: none); words 8..12: the
 *              block's fused-matrix slot (-1: none or built per sample)
 *   diag       [n_diag][24] uint32 sign-pattern records (CZ sets)
 *   blk_begin  [n_blocks + 1] int32, blk_gates [n_block_gates] int32: the
 *              gates of each block in application order
 * Returns QS_ERR_UNSUPPORTED when the circuit does not take the fused path. */
typedef struct qs_engine_dump {
  int32_t n_qubits, log2_regs, n_ops, n_segments;
  int32_t n_l1q, n_diag, n_blocks, n_block_gates;
} qs_engine_dump;
int qs_plan_dump(const qs_circuit* circuit, int dtype, int64_t B, int flags, int adjoint,
                 qs_engine_dump* info, int32_t* ops, int32_t* seg_begin, uint16_t* seg_lay,
                 int32_t* l1q, uint32_t* diag, int32_t* blk_begin, int32_t* blk_gates);

/* ------------------------------------------------------------- autotuner */
typedef struct qs_tune_info {
  int32_t path;           /* QS_PATH_FUSED or QS_PATH_HBM                    */
  int32_t fwd_log2_regs;  /* chosen forward register tile (fused path)       */
  int32_t adj_log2_regs;  /* chosen adjoint register tile (fused path)       */
  int32_t tile_qubits;    /* chosen tile size (large-state path)             */
  float fwd_ms;           /* best forward time measured                      */
  float adj_ms;           /* best adjoint time measured                      */
  int32_t n_candidates;   /* configurations timed                            */
  int32_t fwd_samples_cap; /* chosen cap on samples per workgroup, forward
                              (0: as many as the LDS holds)                  */
  int32_t adj_samples_cap; /* the same for the adjoint                       */
  int32_t fwd_half_staging; /* 1: the forward stages one state component at a
                               time in LDS (half the LDS per sample)        */
  int32_t adj_half_staging; /* the same for the adjoint                      */
  int32_t reserved;
} qs_tune_info;

/* Time every feasible launch configuration of this circuit at batch size B
 * (register tile and samples per workgroup per direction on the fused path,
 * tile size and register tiles on the large-state path) on library-allocated scratch buffers, synchronously on
 * `stream`, and use the fastest for later calls with the same circuit, dtype,
 * flags and a batch of the same power-of-two size class. When the environment
 * variable QS_AUTOTUNE_CACHE names a file, the choice is appended to it and
 * such files are read back at the first tuning lookup of a process. With
 * QS_AUTOTUNE=1 a forward or adjoint call tunes itself on its first use.
 * Allocates device memory: not to be called during a stream capture. */
int qs_autotune(const qs_circuit* circuit, int dtype, int64_t B, int flags,
                void* stream, qs_tune_info* out);

/* Release the plan caches (device memory, and the side streams and events of
 * uneven-batch programs). No call may be in flight on any stream. Safe to
 * call more than once; later calls plan again. */
void qs_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* QS_H */
