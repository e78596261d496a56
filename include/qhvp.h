/*
 * qhvp.h - C ABI of the MI355X (gfx950) library that evaluates the
 * Hilbert-Schmidt cost, its gradient and its Hessian-vector product for a
 * brickwall circuit of two-qubit gates against a reference unitary, by
 * sample-batched recursive state propagation on full statevectors.
 *
 * The method is that of arXiv 2604.20384 ("Hessian-vector products for
 * tensor networks via recursive tangent-state propagation"): forward states
 * and their tangents (Sec. II.C-E, Eq. fis / Eq. dfis), backward states and
 * their tangents (Eq. bis / Eq. dbis), per-gate environments (Eq.
 * environment) and their directional derivatives (Eq. overlap-hvp), the
 * Hilbert-Schmidt post-processing of Alg. 2 and the empirical risk over
 * Haar product states (Eq. costHS), with the Riemannian projections of
 * App. F.
 *
 * Conventions
 *   - Complex numbers are interleaved (re, im) doubles; 4x4 matrices are
 *     row-major, G[i][j] with i the output index, i = 2*b_q + b_{q+1} for a
 *     gate on qubits (q, q+1).
 *   - Brickwall: layer l (0-based, first applied) has a gate on every pair
 *     (q, q+1) with q = l (mod 2), q + 1 < n.  Gates are numbered layer by
 *     layer, by increasing q inside a layer; qhvp_num_gates(n, L) of them.
 *   - Statevector index x = sum_q b_q 2^(n-1-q) (qubit 0 most significant).
 *   - A sample is n single-qubit states (amp|0>, amp|1>): psi_s = u_s0 (x) ... (x) u_s,n-1.
 *   - Cost C = 1 - F with F = (1/N_s) sum_s |phi_s^dag G psi_s|^2 and
 *     phi_s = U_ref psi_s (Eq. costHS).  grad and hvp are the complex
 *     gradients of C (App. A convention: grad f = df/dx + i df/dy entry-wise),
 *     i.e. dC[V] = Re sum_k Tr(grad_k^dag V_k) and hvp = D(grad C)[V].
 *
 * Ownership: the caller owns every pointer it passes.  Host arrays are read
 * during the call only.  The device workspace passed to
 * qhvp_problem_create is used until qhvp_problem_destroy; the library never
 * frees it.  With a NULL workspace the library allocates (and later frees)
 * its own.
 *
 * Errors: every entry point returns a qhvp_status, never aborts, and leaves
 * its outputs untouched on error; qhvp_last_error() gives a message (per
 * thread).  Arguments are validated before any device work is launched.  The
 * device-pointer calls (*_dev) validate pointers and sizes on the host and the
 * values of G and V on the device: an invalid value leaves every output of the
 * call untouched and sets the problem's device status (qhvp_device_status).
 *
 * Host and device calls run the same device code: the host calls copy G and V
 * to the device, enqueue the device-pointer path and copy its outputs back, so
 * their results are bitwise those of the corresponding *_dev call.
 *
 * Threading: one problem is used by one host thread at a time; calls on one
 * problem are serialised on its stream.  Different problems (each on its
 * own stream) may be used from different threads concurrently.
 */
#ifndef QHVP_H
#define QHVP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qhvp_ctx qhvp_ctx;
typedef struct qhvp_problem qhvp_problem;

typedef enum {
  QHVP_OK = 0,
  QHVP_ERR_INVALID = 1,     /* bad sizes, null pointers, non-finite input, non-unitary gate in Riemannian mode */
  QHVP_ERR_NOMEM = 2,       /* workspace smaller than qhvp_workspace_bytes, or allocation failed */
  QHVP_ERR_DEVICE = 3,      /* a HIP runtime call failed */
  QHVP_ERR_UNSUPPORTED = 4  /* e.g. an HVP on a problem created without tangent storage */
} qhvp_status;

typedef enum {
  QHVP_C128 = 0,      /* complex128 states, FP64 reductions */
  QHVP_C64_ACC64 = 1  /* complex64 states and gates; products reduced in FP32 over one tile, FP64 beyond */
} qhvp_precision;

typedef enum {
  QHVP_EUCLIDEAN = 0,  /* plain complex gradient / HVP (Alg. 2) */
  QHVP_RIEMANNIAN = 1  /* projected onto the tangent space of U(4)^K (App. F); V is projected first */
} qhvp_geometry;

/* Library version (major*10000 + minor*100 + patch). */
int qhvp_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char* qhvp_last_error(void);

/* Number of gates K of an n-qubit, L-layer open brickwall (Sec. III), or -1 if n < 2 or L < 1. */
int qhvp_num_gates(int n, int L);

/* The pass plan the library uses for an n-qubit, L-layer brickwall (host only, no device needed).
 * A pass applies up to 6 gates to tiles of at most 2^10 amplitudes spanned by the low 4 index bits
 * and a window of consecutive bits; gates of several layers share a pass, in an order that keeps
 * every gate after the gates of the previous layer on overlapping qubits.  Returns the number of
 * passes (or a negative status); if gates_per_pass is non-NULL it receives that many counts
 * (capacity max_passes), and if gate_order is non-NULL it receives the K gate indices in the order
 * of application (capacity K = qhvp_num_gates(n, L)).  Errors return -QHVP_ERR_INVALID (message in
 * qhvp_last_error). */
int qhvp_plan(int n, int L, int max_passes, int* gates_per_pass, int* gate_order);

/* Create / destroy a context bound to HIP device `device`. */
qhvp_status qhvp_ctx_create(int device, qhvp_ctx** out);
void qhvp_ctx_destroy(qhvp_ctx* ctx);

/*
 * Device workspace (bytes) a problem needs.
 *   ckpt_every > 0 : keep the states at every ckpt_every-th layer boundary and
 *                    recompute the rest of a segment in the backward sweep
 *                    (layer checkpointing; Alg. 1 keeps every state instead).
 *   ckpt_every = 0 : keep the state at every pass boundary (no recomputation).
 *   ckpt_every < 0 : segments of -ckpt_every passes.
 *   ckpt_every = QHVP_CKPT_REBUILD : keep only the final forward states; the backward sweep
 *                    rebuilds every pass boundary from the one after it by undoing the pass's
 *                    gates (Eq. fis / Eq. dfis solved for the input states), so no boundary is
 *                    stored and none is recomputed: close to the speed of ckpt_every = 0 in the
 *                    memory of five state sets.  The undo errors add up over all K gates, so it
 *                    needs well-conditioned gates: |G|_F |G^-1|_F <= 4 (1 + 1e-6) for every gate
 *                    (4 exactly for a unitary up to a scale; the bound admits singular values that
 *                    differ by about 1e-3).  Gradient and HVP calls with other gates fail on the
 *                    device (QHVP_DEV_NOT_INVERTIBLE) and leave their outputs untouched.
 *   with_tangent   : 1 to allow qhvp_hvp (stores the tangent states too).
 * Returns 0 on invalid arguments.
 */
#define QHVP_CKPT_REBUILD (-(1 << 30))
size_t qhvp_workspace_bytes(int n, int L, int L_ref, int n_samples, qhvp_precision prec,
                            int ckpt_every, int with_tangent);

/*
 * Create a problem: n qubits, an L-layer ansatz, a reference brickwall U_ref of
 * L_ref layers with gates `uref_gates` (K_ref*16 complex, host), and n_samples
 * product states `samples` (n_samples*n*2 complex, host).  Computes the labels
 * phi_s = U_ref psi_s on the device (Alg. 2 takes phi^[0] as input) and keeps
 * them for every later call.  `d_workspace` (device, caller-owned, >=
 * qhvp_workspace_bytes(...) bytes, 256-byte aligned) may be NULL.
 * `hip_stream` is a hipStream_t (NULL = default stream).
 */
qhvp_status qhvp_problem_create(qhvp_ctx* ctx, int n, int L, int L_ref,
                                const double* uref_gates, const double* samples, int n_samples,
                                qhvp_precision prec, int ckpt_every, int with_tangent,
                                void* d_workspace, size_t ws_bytes, void* hip_stream,
                                qhvp_problem** out);
void qhvp_problem_destroy(qhvp_problem* p);

/* Cost C and fidelity F for gates G (K*16 complex, host).  One forward sweep (Sec. III, single-pass overlap). */
qhvp_status qhvp_cost(qhvp_problem* p, const double* G, double* cost, double* fidelity);

/* Backward sweep algorithm (gradient and HVP calls), chosen on the device for each call.  When every
 * gate satisfies |G_k|_F |G_k^-1|_F <= 8 (unitary gates: 4), each backward pass starts from the
 * forward states at the pass OUTPUT and undoes the gates on them (psi <- G^-1 psi, dpsi <- G^-1 dpsi -
 * G^-1 V G^-1 psi) while it undoes them on the backward states; the environments taken against
 * output states are mapped back in FP64 (E = Et G^-T, D = (Dt - E V^T) G^-T).  Otherwise, or when the
 * environment variable QHVP_BACKWARD is "recompute", each pass recomputes the forward states
 * inside the tile from the pass input.  Both give the same sums up to rounding. */

/* Cost, fidelity F = 1 - C and gradient (K*16 complex, host) of C at G: forward sweep, then the
 * backward sweep accumulating the environments (Eq. environment, Alg. 2 "postprocess gradient").
 * cost and fidelity may be NULL.  F is returned as computed (not as 1 - C, which cancels when F is
 * small). */
qhvp_status qhvp_grad(qhvp_problem* p, const double* G, qhvp_geometry geom,
                      double* cost, double* fidelity, double* grad);

/* Cost, fidelity, gradient and HVP H(C)[V] (each K*16 complex, host) at G along V (K*16
 * complex, host): Alg. 1 + Alg. 2 with tangent states. cost, fidelity and grad may be NULL. */
qhvp_status qhvp_hvp(qhvp_problem* p, const double* G, const double* V, qhvp_geometry geom,
                     double* cost, double* fidelity, double* grad, double* hvp);

/* ---- device-pointer calls (the same evaluations with G, V and the outputs in device memory) ----
 * d_G, d_V: K*16 complex FP64 (interleaved re, im; 2*K*16 doubles), device memory of the problem's
 * device, read during the call's device work only; outputs: device doubles (cost, fidelity: one
 * each; grad, hvp: K*16 complex), written by the call's last kernel.  The calls enqueue their work on
 * the problem's stream and return without waiting; the caller orders later use of the outputs after
 * that stream (a torch stream passed at problem creation does this for torch work on the same
 * stream).  Host-side errors (NULL or non-device pointers, sizes, a problem without tangent storage)
 * return before anything is enqueued.  Non-finite entries of G or V, or (Riemannian) gates off the
 * unitary manifold, are detected on the device: the call then writes none of its outputs and
 * qhvp_device_status reports the reason.  Cost, gradient and HVP follow Alg. 1 + Alg. 2 over the
 * samples (Eq. costHS); Riemannian outputs follow App. F with V projected first. */
qhvp_status qhvp_cost_dev(qhvp_problem* p, const double* d_G, double* d_cost, double* d_fidelity);
qhvp_status qhvp_grad_dev(qhvp_problem* p, const double* d_G, qhvp_geometry geom, double* d_cost,
                          double* d_fidelity, double* d_grad);
qhvp_status qhvp_hvp_dev(qhvp_problem* p, const double* d_G, const double* d_V, qhvp_geometry geom,
                         double* d_cost, double* d_fidelity, double* d_grad, double* d_hvp);
/* Two-phase form on device pointers (as qhvp_forward / qhvp_backward below); d_cost, d_fidelity,
 * d_grad may be NULL. */
qhvp_status qhvp_forward_dev(qhvp_problem* p, const double* d_G, const double* d_V, qhvp_geometry geom,
                             double* d_cost, double* d_fidelity);
qhvp_status qhvp_backward_dev(qhvp_problem* p, double* d_grad, double* d_hvp);

/* ---- one HVP that allocates nothing ----
 * For callers that cannot allocate memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  One HVP as qhvp_hvp_dev computes it, for a problem given in
 * full on the device (U_ref gates, K_ref*16 complex FP64, and samples, n_samples*n*2 complex FP64, as
 * for qhvp_problem_create; G, V and the outputs as for qhvp_hvp_dev), evaluated entirely inside a
 * scratch area of QHVP_NOALLOC_SCRATCH_BYTES (64 MiB) of device memory that the library holds on
 * each device from qhvp_ctx_create until the process ends.  The call allocates nothing (no device,
 * pinned or torch memory, no events); it picks the fastest layer-checkpoint policy whose workspace
 * fits the scratch, and returns QHVP_ERR_NOMEM before enqueueing anything if none does.  The labels
 * are computed by every call.  Work is enqueued on hip_stream and the call returns without waiting.
 * Every call on one device shares that device's scratch, which keeps the last call's contents (each
 * call clears what it needs cleared): calls that overlap on one device - on different streams or
 * from different threads - race, so serialise them (one stream).  d_cost, d_fidelity, d_grad may be
 * NULL; values the device rejects leave the outputs untouched, as for qhvp_hvp_dev. */
#define QHVP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
qhvp_status qhvp_hvp_noalloc(qhvp_ctx* ctx, int n, int L, int L_ref, const double* d_uref_gates,
                             const double* d_samples, int n_samples, qhvp_precision prec,
                             const double* d_G, const double* d_V, qhvp_geometry geom,
                             double* d_cost, double* d_fidelity, double* d_grad, double* d_hvp,
                             void* hip_stream);

/* Device-side input check of the last call (waits for the problem's stream): 0 if its inputs were
 * valid, else an OR of the QHVP_DEV_* reasons. */
#define QHVP_DEV_NONFINITE 1    /* a non-finite entry in G or V */
#define QHVP_DEV_NOT_UNITARY 2  /* Riemannian geometry with |G_k^dag G_k - I|_F > 1e-10 for some k */
#define QHVP_DEV_NOT_INVERTIBLE 4 /* QHVP_CKPT_REBUILD with a gate beyond its bound on |G|_F |G^-1|_F */
qhvp_status qhvp_device_status(qhvp_problem* p, int* status);

/* Fixed-G reuse and several directions (Sec. IV: the truncated-CG inner loop takes many HVPs at
 * one point; App. G: one HVP per tangent basis vector).  The forward states psi that a gradient or
 * HVP sweep leaves at the pass boundaries kept in the workspace (every boundary with ckpt_every =
 * 0, the segment checkpoints otherwise) are tagged with the gates G that produced them.  A later
 * gradient or HVP call whose G is bitwise the same reads them there and stores only the tangent
 * states over them; its results are identical to those of a call that rewrites them.  Any gradient
 * or HVP call at another G retags them; qhvp_cost never touches them.  With QHVP_CKPT_REBUILD
 * nothing is kept (the backward sweep overwrites the forward states), so every call recomputes them.
 * qhvp_hvp_batch evaluates n_dirs HVPs at one G: V and hvp hold n_dirs*K*16 complex (direction m at
 * offset m*K*16), processed one tangent sweep pair after another; hvp[m] equals qhvp_hvp(G, V[m])
 * bit for bit.  cost and grad (the gradient at G) may be NULL.  All directions are validated before
 * any device work; n_dirs < 1 is QHVP_ERR_INVALID.  The problem needs tangent storage. */
qhvp_status qhvp_hvp_batch(qhvp_problem* p, const double* G, int n_dirs, const double* V, qhvp_geometry geom,
                           double* cost, double* grad, double* hvp);
/* 1 if the kept pass-boundary states belong to G (bitwise), 0 if not, -1 for NULL arguments. */
int qhvp_states_kept_for(const qhvp_problem* p, const double* G);

/* Two-phase form of qhvp_grad / qhvp_hvp (Alg. 1: forward pass, then backward pass).
 * qhvp_forward runs the forward sweep at G (with the tangent sweep along V if V != NULL; V is
 * projected onto the tangent space first when geom is Riemannian), returns the cost and
 * fidelity, and keeps the layer checkpoints in the workspace.  qhvp_backward then runs the
 * backward sweep of that forward sweep once and returns the gradient (and, if the forward had a
 * direction, the HVP; either pointer may be NULL).  A second qhvp_backward without a new
 * qhvp_forward fails with QHVP_ERR_INVALID. */
qhvp_status qhvp_forward(qhvp_problem* p, const double* G, const double* V, qhvp_geometry geom,
                         double* cost, double* fidelity);
qhvp_status qhvp_backward(qhvp_problem* p, double* grad, double* hvp);

/* Translationally invariant brickwalls (App. E, Alg. 3): every gate of layer l is the same
 * G_(l).  G_layers, V_layers, grad_layers, hvp_layers hold L*16 complex (one 4x4 per layer,
 * row-major, interleaved re/im doubles; host memory, owned by the caller).  The gradient and HVP
 * with respect to G_(l) are the sums over the layer's gates of the per-gate ones, with the
 * direction V_(l) on every gate of layer l (a layer without gates, e.g. the odd layers at n = 2,
 * gives zero); Riemannian outputs are projected at G_(l) (App. F on U(4)^L, V projected first).
 * The layer gates are expanded and the per-layer sums taken on the device (FP64, gates added in
 * increasing order), so the cost of a call is that of qhvp_grad / qhvp_hvp on the expanded
 * circuit.  cost, fidelity and grad_layers may be NULL in qhvp_hvp_ti (grad_layers is required in
 * qhvp_grad_ti).  Errors as for qhvp_grad / qhvp_hvp: every output is left untouched. */
qhvp_status qhvp_grad_ti(qhvp_problem* p, const double* G_layers, qhvp_geometry geom, double* cost,
                         double* fidelity, double* grad_layers);
qhvp_status qhvp_hvp_ti(qhvp_problem* p, const double* G_layers, const double* V_layers, qhvp_geometry geom,
                        double* cost, double* fidelity, double* grad_layers, double* hvp_layers);
/* Device-pointer forms of the two calls above (App. E): every array and scalar is device memory of
 * the problem's device, L*16 complex per array; the work is enqueued on the problem's stream and
 * the call returns without waiting.  Inputs found invalid on the device (non-finite entries, or
 * non-unitary layer gates in Riemannian geometry) leave every output untouched and are reported by
 * qhvp_device_status. */
qhvp_status qhvp_grad_ti_dev(qhvp_problem* p, const double* d_G_layers, qhvp_geometry geom, double* d_cost,
                             double* d_fidelity, double* d_grad_layers);
qhvp_status qhvp_hvp_ti_dev(qhvp_problem* p, const double* d_G_layers, const double* d_V_layers, qhvp_geometry geom,
                            double* d_cost, double* d_fidelity, double* d_grad_layers, double* d_hvp_layers);

/* Per-sample overlaps T_s and Omega_s = D(T_s)[V] (n_samples complex each, host) of
 * the last cost/grad/hvp call (Omega is zero unless that call was an HVP). */
qhvp_status qhvp_overlaps(const qhvp_problem* p, double* T, double* Omega);

/* Problem facts: n_passes is the number of gate passes per sweep of the ansatz. */
qhvp_status qhvp_problem_info(const qhvp_problem* p, int* K, int* n_passes, size_t* ws_bytes,
                              int* segments);

/* 1 if the last gradient / HVP forward phase chose the backward sweep from pass outputs (see
 * above), 0 if it chose recomputation; -1 for a NULL problem. */
int qhvp_backward_from_outputs(const qhvp_problem* p);

/* Milliseconds spent on the device by the last cost / forward(+backward) evaluation (HIP events). */
double qhvp_last_device_ms(const qhvp_problem* p);

/* ---- per-kernel timing (HIP events around every launch on the problem's stream) ---- */

typedef enum {
  QHVP_KERNEL_FORWARD = 0,    /* forward passes of the ansatz sweep (Eq. fis / Eq. dfis) */
  QHVP_KERNEL_RECOMPUTE = 1,  /* forward passes recomputing a segment from its layer checkpoint */
  QHVP_KERNEL_BACKWARD = 2,   /* backward passes with environment sums (Eq. bis / dbis / environment) */
  QHVP_KERNEL_REDUCE = 3,     /* fixed-order reductions of the per-workgroup environment partials */
  QHVP_KERNEL_KINDS = 4
} qhvp_kernel_kind;

/* Switch per-launch timing on (1) or off (0) for later calls; either way resets the statistics. */
qhvp_status qhvp_set_profiling(qhvp_problem* p, int on);

/* Accumulated statistics of one kernel kind since the last qhvp_set_profiling: total device
 * milliseconds, number of launches, and the algorithmic HBM bytes and flops of those launches
 * (states read and written once per pass; gate arithmetic without the in-tile recomputation). */
qhvp_status qhvp_kernel_stats(const qhvp_problem* p, int kind, double* total_ms, long long* launches,
                              double* alg_bytes, double* alg_flops);

/* ---- FP64 host utilities on gate vectors (App. F); all arrays K*16 complex ---- */

/* out = P_G(X) = X/2 - G X^dag G / 2, gate by gate (Eq. projec). */
qhvp_status qhvp_project(int K, const double* G, const double* X, double* out);

/* out = P_G(hvp - V grad^dag G / 2 - G grad^dag V / 2), gate by gate (App. F), for tangent V. */
qhvp_status qhvp_riemannian_hvp(int K, const double* G, const double* grad, const double* hvp,
                                const double* V, double* out);

/* Polar retraction out = U W^dag where G + xi = U S W^dag (the paper names no retraction). */
qhvp_status qhvp_retract(int K, const double* G, const double* xi, double* out);

/* Max over gates of ||G_k^dag G_k - I||_F. */
double qhvp_unitarity_error(int K, const double* G);

#ifdef __cplusplus
}
#endif

#endif /* QHVP_H */
