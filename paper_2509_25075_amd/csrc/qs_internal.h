// Internal declarations shared by the host API, the planner and the kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "qs.h"

namespace qs {

// One operation of the register-resident engine: a layer op (L1Q). Positions
// are PHYSICAL bit positions inside a sample's state: 0 .. r-1 are register
// bits (amplitude index within a thread), r .. n-1 are thread bits (thread
// index within the sample's thread group). The scheduler's intermediate
// single-gate ops use the same record.
//   kind  kOpL1Q (single-gate ops: the gate kind QS_OP_*)
//   a     L1Q: mask of register bits with a block (single gate: position of
//         q0)
//   b     single gate: position of q1, unused otherwise
//   aux   bit 0: some angle of the op differs per sample
//   gate  L1Q: record index (single gate: descriptor gate)
struct SvOp {
  uint8_t kind, a, b, aux;
  int32_t gate;
};
static_assert(sizeof(SvOp) == 8, "SvOp layout");

// An L1Q op applies, in order, an optional sign pattern (DIAG record), on
// every register bit j at once the product of a run of consecutive
// single-qubit gates ("block") acting on the qubit held there, and an
// optional second sign pattern. Its record is kL1QWords int32: the block id
// per register bit (-1: none; identity), then at kL1QPreDiag and
// kL1QPostDiag the DIAG records (-1: none), and from kL1QFused the block's
// fused-matrix slot per register bit (-1: built per sample; n_fu: the
// identity, for a bit without a block). The record of op o is record o. A DIAG record (a set of CZs as
// one sign pattern over the amplitude index) is kDiagWords uint32:
//   [0]      sign parity of register index k (bit k) from register-register CZs
//   [1]      thread-bit mask of single thread-bit sign terms
//   [2 + j]  thread bits paired with register bit j (register-thread CZs)
//   [7 + i]  higher thread bits paired with thread bit i (thread-thread CZs)
constexpr uint8_t kOpL1Q = 16;
constexpr int kL1QWords = 16;  // one 64-byte scalar load
constexpr int kL1QPreDiag = 5;
constexpr int kL1QPostDiag = 7;
constexpr int kL1QFused = 8;
constexpr int kDiagWords = 24;

constexpr int kMaxQubitsFused = 14;  // 2^14 complex64 = 128 KiB LDS staging
constexpr int kMapStride = 16;       // bytes per segment mapping record
constexpr int kLayWords = 32;        // uint16 per segment layout record

// A planned gate program: a sequence of segments, each with a fixed
// placement of the logical qubits onto physical bit positions, such that
// every single-qubit gate of the segment acts on a register-resident qubit.
// Within a segment the gates are grouped into L1Q layer ops. CNOTs are
// folded into the remap that closes their segment. `exec` lists
// every gate once in execution order with its physical positions (-1, -1 for
// a folded CNOT, listed after its segment's ops), for inspection.
struct SvPlan {
  int n = 0, r = 0, t = 0;            // qubits, log2 regs, log2 threads/sample
  int n_gates = 0;
  std::vector<uint8_t> seg_map;       // [nseg][16]: physical pos -> logical q
  // [nseg][32]: logical index mask of each physical bit when the segment's
  // state is read from LDS (first 16: 1 << seg_map) and when it is written
  // at its end (last 16: mapped through the CNOTs folded there).
  std::vector<uint16_t> seg_lay;
  std::vector<std::vector<int>> seg_folded;  // CNOT gates folded at each end
  std::vector<int32_t> seg_begin;     // [nseg + 1] op ranges
  std::vector<int32_t> seg_ckpt;      // [nseg] checkpoint slot after segment
  std::vector<SvOp> ops;
  std::vector<int32_t> gate_slot;     // [G] per-sample angle slot, or -1
  std::vector<int32_t> slot_gate;     // [n_slots] gate of a per-sample slot
  std::vector<int32_t> l1q;           // [n_l1q][kL1QWords]
  std::vector<uint32_t> diag;         // [n_diag][kDiagWords]
  std::vector<int32_t> blk_begin;     // [n_blocks + 1] ranges of blk_gates
  std::vector<int32_t> blk_gates;     // gates of each block, forward order
  std::vector<int32_t> blk_fu;        // [n_blocks] slot of the block's fused matrix
                                      // (angles shared), -1: built per sample
  std::vector<int32_t> blk_gen;       // [n_blocks] first generator-frame slot of a
                                      // block with shared angles (one slot per
                                      // gate), -1: built per sample
  std::vector<int32_t> exec;          // [G][3] gate, physical a, physical b
  std::vector<int32_t> exec_seg;      // [nseg + 1] ranges of exec rows
  std::vector<int32_t> grad_cols;     // shared parameter of each gradient column
  std::vector<int32_t> gate_cols;     // [G][2] columns of p_w and p_b, or -1
  int n_remaps = 0;
  bool layered = true;                // every op is an L1Q op
  int nseg() const { return (int)seg_begin.size() - 1; }
  int n_fu = 0;                       // blocks with a fused-matrix slot
  int n_gen = 0;                      // generator-frame slots
  int n_blocks() const { return (int)blk_fu.size(); }
};

// Plans `c` for 2^r amplitudes per thread. `per_sample_angles_all` marks every
// rotation's angle per-sample (per-sample parameter sets); otherwise only
// rotations with a feature are. Checkpoint boundaries force segment ends.
SvPlan plan_sv(const qs_circuit& c, int r, bool per_sample_angles_all,
               const int32_t* ckpt_gates, int n_ckpt);

// The shared parameters that the circuit's rotations read, ascending. The
// adjoint keeps per-block gradient sums only for these (its "gradient
// columns"); a sub-circuit of a large state touches few of the parameters.
// Empty for per-sample parameter sets, whose gradients go straight to HBM.
std::vector<int32_t> grad_columns(const qs_circuit& c, bool per_sample_params);

// A block's gate as the engine reads it: one 32-byte record per position of
// blk_gates, so a gate costs one scalar load in the kernels' inner loops.
struct BGate {
  int32_t g;          // descriptor gate
  int32_t kind_slot;  // gate kind (bits 0..3) | (per-sample angle slot + 1) << 4
  int32_t feat, p_w, p_b;
  int32_t col_w, col_b;  // gradient columns of p_w, p_b (-1: none)
  float scale;
};
static_assert(sizeof(BGate) == 32, "BGate layout");

// Large states: the gate list is cut into epochs; each epoch acts only on a
// tile set L of m qubits (sorted; always containing the `low_keep` lowest
// qubits so that a tile reads contiguous runs of 2^low_keep amplitudes), and
// runs as the register engine on 2^(n-m) gathered m-qubit "samples" per
// batch row.
struct TiledEpoch {
  std::vector<int> L;              // global qubit of each local bit
  std::vector<qs_gate> gates;      // the epoch's gates, qubits renumbered local
  std::vector<int> gate_index;     // descriptor index of each epoch gate
  int ckpt_after = -1;             // checkpoint stored after this epoch
};
std::vector<TiledEpoch> plan_tiled(const qs_circuit& c, int m, int low_keep,
                                   const int32_t* ckpt_gates, int n_ckpt);

// Large states on the dense-block path: the gate list cut into blocks of K
// qubits; each block's gates (descriptor indices, in an order that keeps
// every qubit's gate order) multiply into one 2^K x 2^K unitary applied in
// one pass over the state.
struct DenseBlock {
  std::vector<int> qubits;    // the K qubits, ascending (local bit i = qubits[i])
  std::vector<int> gates;     // descriptor gates, application order
  int ckpt_after = -1;        // checkpoint stored after this block
};
std::vector<DenseBlock> plan_blocks(const qs_circuit& c, int K, const int32_t* ckpt_gates,
                                    int n_ckpt);

// Device records of a dense-block plan. A block gate: kind, local qubits,
// angle rule (as in qs_gate, no features).
struct DbGate {
  int32_t op, q0, q1, p_w, p_b;
  float scale;
  int32_t g;        // descriptor gate (gradient slot)
  int32_t pad;
};
static_assert(sizeof(DbGate) == 32, "DbGate layout");
// Per-block tile geometry, kDbGeoWords int32 per block: [0, 5) the block
// qubits (ascending), [5, 15) the 10 address bits of a tile of 32 columns
// (the block qubits and the 5 lowest other positions, ascending; the first 5
// are always 0..4), [15, 20) the rank among those 10 of each block qubit,
// [20, 25) the rank of each column bit (column bit j sits at the j-th lowest
// position outside the block).
constexpr int kDbGeoWords = 32;
struct DbLaunch {
  int K;                      // block qubits (5)
  int n;                      // qubits of a state
  int64_t B;
  const int32_t* blk_begin;   // device [n_blocks + 1] ranges of gates
  const DbGate* gates;        // device
  const int32_t* blk_q;       // device [n_blocks][kDbGeoWords] tile geometry
  const int32_t* h_blk_q;     // host copy of blk_q
  const void* params;         // device float (complex64 states)
  int grid;                   // persistent workgroups of the pass kernels
  void* stream;
};
// Forward pass of block i over the state (in place): every workgroup builds
// the block's unitary M in FP64 from the parameters and applies it to its
// share of the state's columns on MFMA.
int launch_db_forward(const DbLaunch& L, int i, void* state);
// Adjoint pass of block i: psi <- M^dagger psi, lam <- M^dagger lam (in
// place), and per-workgroup partial sums of rho = sum psi lam^dagger over the
// state's columns (taken before the update) into `partials`
// [grid][2][2^K][2^K] float (real part, then imaginary part).
int launch_db_adjoint(const DbLaunch& L, int i, void* psi, void* lam, float* partials);
// rho (FP64, [2][2^K][2^K]) = sum over workgroups of the partials.
int launch_db_reduce(const DbLaunch& L, const float* partials, double* rho);
// Per-gate adjoint gradients dL/dtheta_g (FP64, gtheta[g] for every rotation
// g of the n_blocks blocks) from each block's rho, walking its gates
// backwards.
int launch_db_grads(const DbLaunch& L, int n_blocks, const double* rho, double* gtheta);
// grad[p] = sum of scale * gtheta over the rotations reading p (p_w or p_b).
int launch_db_chain(int n_params, const int32_t* p_begin, const int32_t* p_gate,
                    const float* p_scale, const double* gtheta, double* grad, void* stream);

// Device copy of a plan plus its launch shape.
struct SvDevPlan {
  int n, r, t, nseg, n_gates, n_slots, n_params, n_features;
  int n_remaps, n_ops;
  uint8_t* seg_map;
  uint16_t* seg_lay;
  int32_t* seg_begin;
  int32_t* seg_ckpt;
  SvOp* ops;
  qs_gate* gates;
  int32_t* gate_slot;
  int32_t* slot_gate;
  int32_t* l1q;
  uint32_t* diag;
  int32_t* blk_begin;
  BGate* blk_rec;      // [n_block_gates] the gate records of the blocks
  int32_t* blk_fu;
  int32_t* blk_gen;
  int32_t* grad_cols;  // [n_acc] parameter of each gradient column
  int n_blocks, n_fu, n_acc, n_gen;
  int ryrz = 0;        // every block is RY then RZ (hardware-efficient layers)
  // Salt vectors of one-component staging (packed six bits each), 0: none.
  uint64_t salt_half = 0;
};

// Launch geometry of the engine for a plan.
struct SvShape {
  int r, t;                 // log2 regs, log2 threads per sample
  int block_threads;        // threads per workgroup
  int samples_per_block;
  int64_t lds_bytes;
  int half = 0;             // LDS staging one state component at a time
};

// Kernel launchers (defined in the .hip files).
struct SvLaunch {
  const SvDevPlan* p;
  SvShape shape;
  int64_t B;
  int per_sample_params;
  const void* params;
  const void* feats;
  void* state;
  double* expz;
  void* ckpt;
  const double* dexpz;
  const void* dstate;
  void* ws_partials;        // [grid][n_params] shared-parameter partial sums
                            // (float for complex64, double for complex128)
  double* grad_params;
  double* grad_feats;
  // Tiled (gathered) operation on a larger state; ob = 0 for plain batches.
  int n_tot = 0, ob = 0;
  const uint8_t* tile_q = nullptr;   // device [n] global qubit per local bit
  const uint8_t* outer_q = nullptr;  // device [ob] global qubit per outer bit
  void* out_psi = nullptr;           // adjoint: final psi (may alias state)
  void* out_lam = nullptr;           // adjoint: final lam (may alias dstate)
  int accum_feats = 0;               // adjoint: add to grad_feats (segments of a
                                     // circuit with mid-circuit channels)
  // Forward: amplitude encoding fused into the state load (batched layout,
  // x in the state's real type); x_in null reads `state`.
  const void* x_in = nullptr;
  int64_t x_stride = 0, x_D = 0;
  int32_t* bad_rows = nullptr;
  // Training step (launch_sv_train): labels, loss qubit, per-workgroup
  // squared-residual sums [grid] double.
  const double* y = nullptr;
  int loss_q = 0;
  double* loss_part = nullptr;
  void* stream;
};
int launch_sv_forward(int dtype, const SvLaunch& L);
int launch_sv_adjoint(int dtype, const SvLaunch& L);
// The training step in one engine launch (complex64, whole-amplitude
// staging, register tiles 2^4 and 2^5); QS_ERR_UNSUPPORTED otherwise.
int launch_sv_train(int dtype, const SvLaunch& L);
bool sv_train_supported(int dtype, const SvShape& shape);

int launch_encode(int enc, int dtype, int n, int64_t B, int64_t D,
                  int x_is_f64, const void* x, int64_t x_stride, void* state,
                  int32_t* bad_rows, void* stream);
int launch_expz(int dtype, int n, int64_t B, const void* state, double* expz,
                void* stream);
int launch_loss_mse_z(int n, int64_t B, int q, const double* expz, const double* y,
                      double* dexpz, double* loss, void* stream);
int launch_fidelity(int dtype, int n, int n_trash, int64_t B, const void* psi,
                    const void* chi, double* fid, const double* dfid,
                    void* lam_psi, void* lam_chi, void* stream);
int launch_fidelity_postselect(int dtype, int n, int n_trash, int64_t B, const void* psi,
                               const void* chi, double* fid, const double* dfid,
                               void* lam_psi, void* lam_chi, void* stream);
int launch_fidelity_trajectory(int dtype, int n, int n_trash, int64_t B, const void* psi,
                               const void* chi, const double* u, double* fid,
                               int32_t* outcome, const double* dfid, void* lam_psi,
                               void* lam_chi, void* stream);
// out[col_param[j]] (+)= sum over rows of partials[row][j], j < cols.
// Sums [rows][cols] partials per column into out[col_param[c]] (FP64, fixed
// order); with `loss`, also loss[0] = loss_scale x the sum of loss_part[rows].
int launch_reduce_partials(int dtype, const void* partials, int64_t rows,
                           int cols, const int32_t* col_param, double* out,
                           int accumulate, void* stream, const double* loss_part = nullptr,
                           double* loss = nullptr, double loss_scale = 0.0);
int launch_obs_cot(int dtype, int n, int64_t B, const double* dexpz,
                   const void* psi, void* lam, void* stream);
int launch_fill_f64(double* p, int64_t n, void* stream);
// Mid-circuit channel on qubit q (reset or measurement), one trajectory per
// sample, its uniform at feats[b][feat]; and its backward pass.
int launch_channel(int dtype, int n, int q, int reset, int64_t B, const void* feats,
                   int n_feats, int feat, void* state, void* stream);
int launch_channel_adjoint(int dtype, int n, int q, int reset, int64_t B, const void* feats,
                           int n_feats, int feat, const void* psi_pre, void* lam,
                           void* psi_out, void* stream);
int launch_copy_state(int dtype, const void* src, void* dst, int64_t n_amp,
                      void* stream);

// Uneven batches: classes of identically-structured circuits, one parameter
// set and one state per circuit, packed class after class.
struct ProgClass {
  const uint8_t* seg_map;
  const uint16_t* seg_lay;
  const int32_t* seg_begin;
  const int32_t* seg_ckpt;
  const SvOp* ops;
  const qs_gate* gates;
  const int32_t* gate_slot;
  const int32_t* slot_gate;
  const int32_t* l1q;
  const uint32_t* diag;
  const int32_t* blk_begin;
  const BGate* blk_rec;
  const int32_t* blk_fu;
  const int32_t* blk_gen;
  int32_t n, t, nseg, n_gates, n_slots, n_params, S, n_blocks, n_fu, n_gen;
  int32_t ryrz;        // every block is RY then RZ (the adjoint's gate-at-a-time pass)
  int32_t table;       // 1: the item's angles go to an LDS table (sines and
                       // cosines once per gate and circuit); 0: each thread
                       // computes the angles of its circuit where it uses them
  int64_t count;       // circuits in the class
  int64_t state_off;   // complex-element offset of the class's first state
  int64_t param_off;   // element offset of the class's parameters [count][P]
  int64_t expz_off;    // element offset of the class's <Z> rows [count][n]
};
struct ProgItem {
  int32_t cls;
  int32_t first;       // first circuit of the class in this work item
};
struct ProgLaunch {
  const ProgClass* classes;  // device
  const ProgItem* items;     // device, longest first
  int n_items;
  int* counter;              // device work-queue counter
  int grid, block, r;
  int half;                  // LDS staging one state component at a time
  int64_t lds_bytes;
  const void* params;
  void* states;
  double* expz;
  const double* dexpz;
  double* grad_params;
  void* stream;
};
int launch_program(int dtype, const ProgLaunch& L, bool adjoint);
int launch_zero_i32(int* p, void* stream);
int launch_program_encode(int dtype, int n_classes, const int64_t* d_counts_cum,
                          const int32_t* d_nq, const int64_t* d_state_off,
                          int64_t n_circuits, const void* x, int x_is_f64,
                          void* states, int32_t* bad_rows, void* stream);

// Plain one-gate-per-launch path.
struct PlainLaunch {
  const qs_circuit* c;       // host descriptor
  const qs_gate* d_gates;    // device copy
  int dtype;
  int64_t B;
  int per_sample_params;
  const void* params;
  const void* feats;
  void* state;
  double* expz;
  const int32_t* ckpt_gates;
  int n_ckpt;
  void* ckpt;
  const double* dexpz;
  const void* dstate;
  double* grad_params;
  double* grad_feats;
  void* ws;                  // lam [B][2^n] + psi copy + gtheta [B][G]
  void* stream;
};
size_t plain_workspace_bytes(const qs_circuit& c, int dtype, int64_t B);

// The stream of the launch-side call running on this thread, set for the
// call's duration by its entry point (nested calls restore the outer one).
// Plan caches upload with synchronous allocations and copies, which a stream
// capture does not allow: on a cache miss they first ask whether that stream
// is capturing and, if so, return QS_ERR_CAPTURE instead of breaking it.
struct CallStream {
  explicit CallStream(void* stream);
  ~CallStream();
  void* prev;
  bool prev_in_call;
};
bool call_stream_capturing();

// Set for the duration of a call that must not allocate device memory: plan
// caches then refuse a miss with QS_ERR_NOT_PLANNED, and the autotuner does
// not run.
struct NoAllocCall {
  NoAllocCall();
  ~NoAllocCall();
  bool prev;
};
// QS_OK when a plan cache may upload a new plan now; otherwise the status to
// return (QS_ERR_NOT_PLANNED in a no-allocation call, QS_ERR_CAPTURE while
// the call's stream is being captured).
int plan_upload_status();

// The body of qs_adjoint_backward. With no_alloc, only the register/LDS
// engine path runs (its workspace is the caller's `ws`), plans must already
// be cached, and nothing allocates.
int adjoint_backward_impl(const qs_circuit* c, int dtype, int64_t B, const void* params,
                          const void* feats, const void* state, const double* dexpz,
                          const void* dstate, double* grad_params, double* grad_feats,
                          const int32_t* ckpt_gates, int32_t n_ckpt, const void* ckpt,
                          void* ws, size_t ws_bytes, int flags, void* stream,
                          bool no_alloc);
int run_plain_forward(const PlainLaunch& L);
int run_plain_adjoint(const PlainLaunch& L);

}  // namespace qs
