// Internal declarations shared by the host runtime (qhvp_host.cpp) and the
// gfx950 kernels (qhvp_kernels.hip).
#pragma once

#include <cstddef>
#include <cstdint>

namespace qhvp {

// A pass applies up to kMaxGates gates (in dependency order) to a tile of
// 2^mb amplitudes (mb <= kMaxTileBits) of one sample.  The tile's "active"
// bits abit[0..mb) are statevector index bits (ascending); the low kCoalesce
// bits are always active so that global loads and stores touch contiguous
// runs.  The remaining (inactive) bits ibit[0..n-mb) enumerate the tiles.
constexpr int kMaxGates = 6;
constexpr int kSmallMaxGates = 4;   // passes of at most this many gates use a lighter kernel instance
constexpr int kMaxTileBits = 10;
constexpr int kMaxQubits = 30;
constexpr int kThreads = 256;     // 4 wave64s; one 4-amplitude group per thread per gate at mb = 10
constexpr int kEnvVals = 64;      // 16 complex E + 16 complex D per gate, as 64 doubles

// complex64 LDS tile layout (8-byte elements): tile element t sits at t + sum of kLdsPadC64[b] over
// the set bits b of t, i.e. tile bit b at element offset 2^b + kLdsPadC64[b] = 1, 2, 4, 8, 16, 34,
// 68, 136, 270, 552 (one-to-one on the 1024 elements, extent 1092; index 32 stays free for the
// kernels' dummy slot), and the second state array kTspC64 elements after the first.  The pads and
// kTspC64 minimise, under the measured LDS bank model (32-bit accesses: 32 lanes over 32 banks;
// 64-bit reads: 32 lanes over 64 banks; 64-bit writes: 16 lanes over 32 banks), the conflict cycles
// of a backward gate step with the host's per-gate choice of lane bits at n = 20, plus those of the
// tile puts and reads.
constexpr int kLdsPadC64[kMaxTileBits] = {0, 0, 0, 0, 0, 2, 4, 8, 14, 40};
constexpr int kTspC64 = 1093;

// complex128 LDS tile layout (16-byte elements): tile bit b at element offset 2^b + kLdsPadC128[b] =
// 1, 2, 4, 8, 17, 40, 74, 148, 306, 604 (one-to-one on the 1024 elements, extent 1205; index
// kDummyC128 stays free), the second state array kTspC128 elements after the first.  Only the
// offsets modulo 16 elements (256 bytes) decide bank conflicts.  Measured on gfx950: 128-bit writes
// are served 8 lanes at a time over 32 banks; the environment operand reads (ds_read2st64_b64) as
// two 64-bit accesses, each 16 lanes at a time over 32 banks; 128-bit reads roughly 16 lanes at a
// time over 64 banks.  The environment reads of a gate on tile bits lo, hi then depend only on the
// residues of lo, hi and kTspC128; the group reads and writes on the tile bits the host puts under
// the lanes.  The residues (1, 8, 10, 4, 2, 12 for bits 4..9, 5 for kTspC128) are those with the
// fewest modelled conflict cycles of the forward and backward gate steps of the pass plans at
// n = 12 .. 22 among layouts whose two tile buffers (four state arrays) leave two workgroups of the
// backward kernel room on a CU; the multiples of 16 added keep the layout one-to-one.  Bits 0..3
// stay unpadded: the tile transfers move 16 consecutive elements per 16 lanes.
constexpr int kLdsPadC128[kMaxTileBits] = {0, 0, 0, 0, 1, 8, 10, 20, 50, 92};
constexpr int kTspC128 = 1205;
constexpr int kDummyC128 = 16;

struct PassDesc {
  int n;      // qubits
  int mb;     // tile bits
  int ng;     // gates in this pass
  int gidx[kMaxGates];          // global gate index of each gate, in application order
  int tlo[kMaxGates];           // tile bit of qubit q+1 (less significant bit of the pair)
  int thi[kMaxGates];           // tile bit of qubit q   (more significant bit of the pair)
  int abit[kMaxTileBits];       // statevector bit of each tile bit
  int ibit[kMaxQubits];         // statevector bits that index tiles, ascending
  unsigned long long imask;     // OR of 1 << ibit[i]: tile w of a sample starts at pdep(w, imask)
  // Padded LDS offsets (element units of the problem's precision) for gate slot j, filled by the
  // host for the kernels' tile layout: a group index (the 8 tile bits other than tlo, thi) maps to
  // the sum of goff[j][i] over its set bits i; tile bits tlo / thi add aoff[j][0] / aoff[j][1].
  int goff[kMaxGates][8];
  int aoff[kMaxGates][2];
  int wave_local;               // 1: each wave owns the groups with its index in bits 6, 7 for all gates
};

enum Prec { P_C128 = 0, P_C64 = 1 };

// Forward pass: states (psi, dpsi) -> W psi (Eq. fis / Eq. dfis).  src_psi == nullptr means
// "generate the product state psi^[0] from `samples`, with dpsi = 0".  dst_psi and dst_dpsi are
// stored independently (null: not stored).  If ov_part != nullptr the
// result is not stored; instead per-tile partial overlaps with phi0 are written:
// ov_part[s*tiles + w] = (sum conj(phi0) psi, sum conj(phi0) dpsi) as 4 doubles.
struct FwdArgs {
  PassDesc pd;
  int n_samples;
  int tangent;
  const void* gates;   // K*16 complex (precision of the pass)
  const void* dirs;    // K*16 complex or null
  const void* src_psi; const void* src_dpsi;
  const void* samples; // N_s * n * 2 complex
  void* dst_psi; void* dst_dpsi;
  const void* phi0;
  double* ov_part;
  int* sched;          // tile-schedule counter of this launch (zero before the launch)
  int chunk;           // set by launch_fwd: > 0 dynamic chunks of that many tiles; < 0 static ranges of -chunk tiles
  // decisions taken on the device for this call (null: none): psi is not stored if *psi_skip != 0
  // (the boundary already holds psi for these gates); nothing is stored if *store_if == 0
  const int* psi_skip;
  const int* store_if;
};

// Backward pass over the same tile structure: (a, b) at the pass output -> at the pass input
// (Eq. bis / Eq. dbis with the folded boundary a = T phi, b = Omega phi), accumulating the
// per-gate environment sums.  env_part[wg][j][0..64) (doubles) receives, for gate slot j,
// sum conj(a) psi^T (16 complex) and sum conj(b) psi^T + conj(a) dpsi^T (16 complex).
struct BwdArgs {
  PassDesc pd;
  int n_samples;
  int tangent;
  const void* gates; const void* dirs;
  const void* src_psi; const void* src_dpsi;  // pass-input forward states (null -> generated)
  const void* samples;
  void* ab_a; void* ab_b;                     // in/out backward states (in place)
  const void* phi0; const double* tov;        // fold: a = T_s phi0, b = Omega_s phi0 when fold != 0
  int fold;
  int store_ab;
  double* env_part;
  // launch_bwd_out only: forward states are the pass OUTPUT (src_*), igates = G^-1 | -G^-1 V G^-1
  // per gate (32 complex), fold passes read src_* too (no generated states)
  const void* igates;
  int turns;           // set by the launchers: 1 when two workgroups share each CU (priority turns)
  // the launch does nothing unless *run_flag == run_when (null: always runs); the host launches both
  // backward kernels of a pass and the device-side choice (kFlagInverse) picks one
  const int* run_flag;
  int run_when;
  // launch_bwd_out only: if not null, the forward states at the pass INPUT, which the kernel rebuilds
  // by undoing every gate of the pass, are stored here (may equal src_*: a tile writes only the
  // amplitudes it read)
  void* dst_psi; void* dst_dpsi;
};

// Upper bound of the workgroup count of any pass kernel over `items` tiles (sizes per-workgroup
// buffers); fwd_grid / bwd_grid give the count actually launched on the current device (at most
// the workgroups that are resident at once; 0 for a gate count outside 1..kMaxGates).
int grid_size(long long items);
int fwd_grid(Prec prec, int tangent, int ng, long long items);
int bwd_grid(Prec prec, int tangent, int ng, long long items, int from_output);


// Launchers (return a hipError_t as int).
int launch_fwd(Prec prec, const FwdArgs& a, void* stream);
int launch_bwd(Prec prec, const BwdArgs& a, void* stream);
// Backward pass from the pass-output forward states (see k_bwd_out); same grid as launch_bwd.
int launch_bwd_out(Prec prec, const BwdArgs& a, void* stream);
// p[0..n) = 0 (a kernel, not a memset).
int launch_zero_ints(int* p, int n, void* stream);
// tov[s] = (T_s, Omega_s) = sum over tiles of ov_part.
int launch_reduce_overlaps(const double* ov_part, int n_samples, int tiles, double* tov, void* stream);
// env[gidx[j]][0..64) = sum over wg of env_part[wg][j][0..64), for j < ng, over n_wg_set workgroups if
// flag is null or *flag != 0, else over n_wg_clear (the two backward kernels have different grids).
int launch_reduce_env(const double* env_part, int n_wg_set, int n_wg_clear, const int* flag, const PassDesc& pd,
                      double* env, void* stream);

// ---- per-call FP64 work on the device (qhvp_post.hip) ----
// Per-call flags (ints in the workspace), written by k_prep and read by the sweeps and k_post.
constexpr int kFlagInverse = 0;    // 1: the backward sweep runs from pass outputs (k_bwd_out)
constexpr int kFlagStatus = 1;     // input check on the device: OR of kStat* (0: valid)
constexpr int kFlagKeptValid = 2;  // the kept pass-boundary states belong to the gates in kept_g
constexpr int kFlagKeep = 3;       // this sweep's gates equal kept_g bitwise: store tangents only there
constexpr int kFlagCount = 8;
constexpr int kStatNonFinite = 1;  // a non-finite entry in G or V
constexpr int kStatNotUnitary = 2; // Riemannian geometry with |G^dag G - I|_F > 1e-10 for some gate
constexpr int kStatNotInvertible = 4;   // the rebuilding backward sweep with a gate beyond kRebuildCond
// The backward sweep undoes gates on pass outputs only if every gate has |G|_F |G^-1|_F <= this (4 for a
// unitary gate), so that undoing the at most kMaxGates gates of a pass loses at most a few bits.
constexpr double kInverseCond = 8.0;
// The backward sweep that rebuilds every pass boundary undoes all K gates in a row, so their
// rounding errors add up over the circuit instead of over one pass, and each step may amplify them
// by the gate's condition number.  |G|_F |G^-1|_F >= 4, with equality exactly for a unitary up to a
// scale, and near it the excess is second order: singular values 1 +- d give about 4 (1 + d^2).  So
// this bound admits condition numbers up to about 1.002 (amplification below 1.5 over 190 gates).
constexpr double kRebuildCond = 4.0 * (1.0 + 1e-6);

// Prepare a call's gates: G_in, V_in (K*16 complex FP64, device) -> device precision gates / dirs
// (V projected onto the tangent space at G when riem), FP64 copies g64 / v64, and, when with_inverse,
// G^-1 (gi64, FP64) and igates (G^-1 | -G^-1 V G^-1, device precision) with flags[kFlagInverse] = 1
// if every gate qualifies.  keep_mode (gradient / HVP sweeps): flags[kFlagKeep] = kept states valid
// and G_in == kept_g bitwise (and !invalidate_kept); then kept_g = G_in.
struct PrepArgs {
  int K, prec, tangent, riem, with_inverse, keep_mode, invalidate_kept;
  int rebuild;   // the backward sweep rebuilds the pass boundaries: kRebuildCond or kStatNotInvertible
  const double* G_in;
  const double* V_in;
  void* gates;
  void* dirs;
  void* igates;
  double* g64;
  double* v64;
  double* gi64;
  double* kept_g;
  int* flags;
};
constexpr int kPostCost = 1, kPostDeriv = 2;
// Post-processing: (mode & kPostCost) fidelity and cost from the overlaps tov; (mode & kPostDeriv)
// gradient (and HVP if tangent) from the environment sums env, Riemannian if riem.  Null outputs are
// skipped; nothing is written if flags[kFlagStatus] != 0.
struct PostArgs {
  int K, Ns, tangent, riem, mode;
  const double* tov;
  const double* env;
  const int* flags;
  const double* g64;
  const double* v64;
  const double* gi64;
  double* cost;
  double* fidelity;
  double* grad;
  double* hvp;
};
int launch_prep(const PrepArgs& a, void* stream);
int launch_post(const PostArgs& a, void* stream);
// dst = src (n_complex complex FP64 values, device) in the given precision.
int launch_convert(const double* src, void* dst, long long n_complex, int prec, void* stream);
// Translationally invariant brickwalls (App. E).  The K gates of a brickwall are numbered layer by
// layer, and within a layer by their first qubit: even layers hold the n/2 gates on (0,1), (2,3), ...,
// odd layers the (n-1)/2 gates on (1,2), (3,4), ...; so a pair of layers holds n-1 gates.
constexpr int ti_first_gate(int l, int n) { return (l / 2) * (n - 1) + ((l & 1) ? n / 2 : 0); }
constexpr int ti_gate_count(int l, int n) { return (l & 1) ? (n - 1) / 2 : n / 2; }
constexpr int ti_layer_of(int k, int n) { return 2 * (k / (n - 1)) + ((k % (n - 1)) >= n / 2 ? 1 : 0); }
// gates[k] = layers[ti_layer_of(k, n)] for the K gates of
// an n-qubit brickwall (16 complex FP64 per gate, device).
int launch_ti_expand(const double* layers, int n, int K, double* gates, void* stream);
// out[l] = sum over the gates k of layer l, in increasing k, of per_gate[k] (16 complex FP64 each;
// L layers); a layer without gates gives zero.  Nothing is written if flags[kFlagStatus] != 0.
int launch_ti_reduce(const double* per_gate, int n, int L, const int* flags, double* out, void* stream);

// Scratch of the entry point that allocates nothing (a file-scope device array in qhvp_post.hip).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
// Looks up the array's address on `device` (which must be current) once; returns a hipError_t.
int noalloc_scratch_init(int device);
// The array's address on `device` (null before noalloc_scratch_init succeeded there).
void* noalloc_scratch(int device);

}  // namespace qhvp
