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
// env[gidx[j]][0..64) = sum over wg of env_part[wg][j][0..64), for j < ng.
int launch_reduce_env(const double* env_part, int n_wg, const PassDesc& pd, double* env, void* stream);

}  // namespace qhvp
