// gfx950 kernels for sample-batched recursive state propagation on brickwall
// circuits (arXiv 2604.20384, Sec. II.C-F and Sec. III; Alg. 1 restructured
// into tiled passes).
//
// Data layout: a state set is N_s contiguous statevectors of 2^n complex
// amplitudes (sample-major).  A pass loads, for one sample at a time, a tile
// of 2^mb amplitudes spanned by the pass's active index bits into LDS,
// applies its gates (possibly from several layers, in dependency order) one
// after another, and writes the tile back (or reduces it against phi0).  When
// two tile bits are untouched by every gate of the pass, they index the waves
// and each wave works on its own quarter of the tile with no barrier between
// gates; otherwise a workgroup barrier separates gates.  The low index bits are
// always active, so each global access covers contiguous runs of amplitudes.
//
// Backward pass: the tile holds the backward states (a, b) at the pass output
// and the forward states (psi, dpsi) at the pass input.  The forward states
// in front of each gate are recomputed inside the tile (instead of caching
// one state per gate, as Alg. 1 does), then the gates are undone in reverse
// order: for gate k the environment sum conj(a) psi^T and its directional
// derivative sum conj(b) psi^T + conj(a) dpsi^T (Eq. environment, Eq.
// overlap-hvp) are accumulated first, then (a, b) <- (G^dag a, G^dag b + V^dag a)
// (Eq. bis, Eq. dbis).  The accumulation is a contraction over (sample,
// rest-of-qubits) of 16-row x 16-column real operands, done with
// v_mfma_*_16x16x4 so that the cross-lane reduction costs nothing; complex64
// runs accumulate one tile in FP32 and add that into FP64 registers.
//
// Folding: the first backward pass starts from a = T_s phi0 and
// b = Omega_s phi0, which carries Alg. 2's per-sample weights through the
// (linear) backward recursion, so the environment sums over samples directly
// give -(N_s/2) conj(grad C) and -(N_s/2) conj(H(C)[V]).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdlib>
#include <cstring>

#include <type_traits>
#include <utility>

#include "qhvp_internal.h"

namespace qhvp {

template <typename R> struct CT;
template <> struct CT<float> { using T = float2; };
template <> struct CT<double> { using T = double2; };

template <typename R> struct Mfma;
// Output row held in accumulator item r by a lane of 16-lane block `blk` (= lane / 16); the
// column is lane % 16 for both.  A operand: lane holds A[lane % 16][lane / 16]; B: B[lane / 16][lane % 16].
template <> struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int out_row(int blk, int r) { return 4 * blk + r; }
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int out_row(int blk, int r) { return 4 * r + blk; }
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <typename T> __device__ __forceinline__ T cz() { T r; r.x = 0; r.y = 0; return r; }

// acc + a*b
template <typename T> __device__ __forceinline__ T cfma(T a, T b, T acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc + conj(a)*b
template <typename T> __device__ __forceinline__ T cfmac(T a, T b, T acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
template <typename T> __device__ __forceinline__ T cmul(T a, T b) {
  T r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

// Uniform pointer to gate entries, made opaque to the optimiser so that the (scalar) loads of the
// entries stay next to their use instead of being hoisted out of the tile loop into vector registers.
template <typename R>
using cptr = const __attribute__((address_space(4))) R*;   // constant address space: scalar loads

// Gate entries as interleaved (re, im) scalars behind an opaque constant-address-space pointer.
template <typename T>
__device__ __forceinline__ cptr<decltype(T::x)> opaque(const T* p) {
  asm volatile("" : "+s"(p));
  return (cptr<decltype(T::x)>)p;
}
template <typename T>
__device__ __forceinline__ T centry(cptr<decltype(T::x)> m, int k) {
  T r;
  r.x = m[2 * k];
  r.y = m[2 * k + 1];
  return r;
}

// (p, d) <- (G p, G d + V p) on one 4-amplitude group (Eq. fis / Eq. dfis); the V terms come after a
// compiler barrier so that only one matrix's scalar entries are live at a time.
template <typename T, bool TANG>
__device__ __forceinline__ void apply_w(cptr<decltype(T::x)> G, cptr<decltype(T::x)> V, T (&p)[4], T (&d)[4]) {
  T np[4], nd[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    np[i] = cz<T>();
    nd[i] = cz<T>();
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const T g = centry<T>(G, 4 * i + m);
      np[i] = cfma(g, p[m], np[i]);
      if (TANG) nd[i] = cfma(g, d[m], nd[i]);
    }
  }
  if (TANG) {
    // V's scalar loads may not start before the G phase is done (bounds live scalar registers);
    // a register-only dependency, so no wait on outstanding memory operations is implied
    asm volatile("" : "+s"(V) : "v"(np[3].y));
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int m = 0; m < 4; ++m) nd[i] = cfma(centry<T>(V, 4 * i + m), p[m], nd[i]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) { p[i] = np[i]; if (TANG) d[i] = nd[i]; }
}

// (a, b) <- (G^dag a, G^dag b + V^dag a) (Eq. bis / Eq. dbis), same phase split.
template <typename T, bool TANG>
__device__ __forceinline__ void apply_wdag(cptr<decltype(T::x)> G, cptr<decltype(T::x)> V, T (&a)[4], T (&b)[4]) {
  T na[4], nb[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    na[i] = cz<T>();
    nb[i] = cz<T>();
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const T g = centry<T>(G, 4 * m + i);   // (G^dag)_{im} = conj(G_{mi})
      na[i] = cfmac(g, a[m], na[i]);
      if (TANG) nb[i] = cfmac(g, b[m], nb[i]);
    }
  }
  if (TANG) {
    asm volatile("" : "+s"(V) : "v"(na[3].y));
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int m = 0; m < 4; ++m) nb[i] = cfmac(centry<T>(V, 4 * m + i), a[m], nb[i]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) { a[i] = na[i]; if (TANG) b[i] = nb[i]; }
}


// LDS index of tile element t.  Both layouts are additive over index values with disjoint bits
// (used to split MFMA operand addresses into a per-lane and a wave-uniform part), and leave index
// DUMMY unused (a sink for writes of elements beyond a tile of fewer than 2^kMaxTileBits).
template <typename T> struct Lds;
// complex64: per-bit offsets chosen under the measured bank model (kLdsPadC64); TSP elements per
// state array.
template <> struct Lds<float2> {
  static constexpr int TSMAX = 1 << kMaxTileBits;
  static constexpr int TSP = kTspC64;
  static constexpr int DUMMY = 32;
  static __device__ __forceinline__ int at(int t) {
    int r = t;
#pragma unroll
    for (int b = 5; b < kMaxTileBits; ++b) r += ((t >> b) & 1) * kLdsPadC64[b];
    return r;
  }
};
// complex128: per-bit offsets chosen under the same bank model (kLdsPadC128).
template <> struct Lds<double2> {
  static constexpr int TSMAX = 1 << kMaxTileBits;
  static constexpr int TSP = kTspC128;
  static constexpr int DUMMY = kDummyC128;
  static __device__ __forceinline__ int at(int t) {
    int r = t;
#pragma unroll
    for (int b = 4; b < kMaxTileBits; ++b) r += ((t >> b) & 1) * kLdsPadC128[b];
    return r;
  }
};

// Global <-> LDS transfer of one state of a tile in 16-byte vectors: thread tid moves tile
// elements EPV*(tid + kThreads*v) .. +EPV-1 for v < NV.  Tile bit 0 is always statevector bit 0,
// so those elements are adjacent in memory.  Loads are unconditional: indices beyond a tile of
// fewer than 2^kMaxTileBits elements alias to in-tile elements (deposit ignores bits >= mb), so
// every address is in bounds and all loads can be in flight together; only the LDS writes and
// global stores of such indices are skipped.
typedef float qv4f __attribute__((ext_vector_type(4)));
typedef double qv2d __attribute__((ext_vector_type(2)));

// Global state traffic: every state array a pass touches is read or written once per pass and is
// many times larger than the caches, so these accesses are marked non-temporal (streaming).
template <typename V> __device__ __forceinline__ V gld(const V* p) { return __builtin_nontemporal_load(p); }
template <typename V> __device__ __forceinline__ void gst(V* p, V v) { __builtin_nontemporal_store(v, p); }

template <typename T> struct TileIO {
  using V = typename std::conditional<sizeof(T) == 8, qv4f, qv2d>::type;   // 16 bytes
  static constexpr int EPV = 16 / (int)sizeof(T);
  static constexpr int NV = (1 << kMaxTileBits) / EPV / kThreads;
  static __device__ __forceinline__ int elem(int tid, int v) { return EPV * (tid + kThreads * v); }
  // LDS slot of tile element t, or for t >= TS the (never read) dummy slot; the write is then
  // unconditional, which keeps the loads from being sunk into guarded blocks.
  static __device__ __forceinline__ int slot(int t, int TS) { return t < TS ? Lds<T>::at(t) : Lds<T>::DUMMY; }
  static __device__ __forceinline__ T part(const V& r, int e) {
    T o;
    if constexpr (sizeof(T) == 8) { o.x = e ? r[2] : r[0]; o.y = e ? r[3] : r[1]; }
    else { o.x = r[0]; o.y = r[1]; }
    return o;
  }
  // element-wise LDS access of one 16-byte vector (complex64 elements need not be 16-byte aligned).
  // complex64: 64-bit LDS writes are served 16 lanes at a time over 32 banks of 4 bytes, and the 16
  // lanes of a group hold 32 consecutive elements, so if every lane wrote its element t first,
  // elements r and r + 16 would meet on the same banks.  Lanes 8..15 of each group write t + 1
  // first, which makes both write instructions conflict-free.
  static __device__ __forceinline__ void put(T* lds, int t, int TS, const V& r) {
    if constexpr (sizeof(T) == 8) {
      const int sw = (threadIdx.x >> 3) & 1;
      lds[slot(t + sw, TS)] = part(r, sw);
      lds[slot(t + 1 - sw, TS)] = part(r, 1 - sw);
    } else {
#pragma unroll
      for (int e = 0; e < EPV; ++e) lds[slot(t + e, TS)] = part(r, e);
    }
  }
  static __device__ __forceinline__ V get(const T* lds, int t) {
    V r;
    if constexpr (sizeof(T) == 8) {
      const T a = lds[Lds<T>::at(t)], b = lds[Lds<T>::at(t + 1)];
      r[0] = a.x; r[1] = a.y; r[2] = b.x; r[3] = b.y;
    } else {
      const T a = lds[Lds<T>::at(t)];
      r[0] = a.x; r[1] = a.y;
    }
    return r;
  }
  static __device__ __forceinline__ void load(T* lds, const T* g, long long base, const int* xv, int TS, int tid) {
    V r[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) r[v] = gld((const V*)(g + base + xv[v]));
#pragma unroll
    for (int v = 0; v < NV; ++v) put(lds, elem(tid, v), TS, r[v]);
  }
  static __device__ __forceinline__ void store(T* g, const T* lds, long long base, const int* xv, int TS, int tid) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const V r = get(lds, elem(tid, v));
      if (elem(tid, v) < TS) gst((V*)(g + base + xv[v]), r);
    }
  }
  // Stores split in two halves (LDS -> registers, registers -> memory), so that a tile's global
  // stores can be issued after the next tile's loads have been waited for.
  static __device__ __forceinline__ void read(V (&r)[NV], const T* lds, int tid) {
#pragma unroll
    for (int v = 0; v < NV; ++v) r[v] = get(lds, elem(tid, v));
  }
  static __device__ __forceinline__ void write(T* g, const V (&r)[NV], long long base, const int* xv, int TS, int tid) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (elem(tid, v) < TS) gst((V*)(g + base + xv[v]), r[v]);
  }
};

// A register-only use of 16 values: the loads producing them are issued back to back and
// waited for once, instead of one load-and-wait per use under register pressure.
template <typename R>
__device__ __forceinline__ void pin16(R (&v)[16]) {
  asm volatile("" ::"v"(v[0]), "v"(v[1]), "v"(v[2]), "v"(v[3]), "v"(v[4]), "v"(v[5]), "v"(v[6]), "v"(v[7]),
               "v"(v[8]), "v"(v[9]), "v"(v[10]), "v"(v[11]), "v"(v[12]), "v"(v[13]), "v"(v[14]), "v"(v[15]));
}


// --------------------------------------------------------------------------------------------
// complex64 gate application on the matrix cores
// --------------------------------------------------------------------------------------------
// Per group (the 4 amplitudes of a qubit pair), W = [[X, 0], [Y, X]] acts on the 16 reals of the
// state pair (p, d) as one real 16x16 matrix: the block-triangular operator of App. D, with X = G,
// Y = V in the forward recursion (Eq. fis / Eq. dfis) and X = G^dag, Y = V^dag in the backward one
// (Eq. bis / Eq. dbis).  Each lane owns one group (lane l of wave w: group 64 w + l) and keeps its
// 16 input reals in registers.  v_mfma_f32_4x4x1_16b_f32 multiplies, in each of its 16 blocks of 4
// lanes, a 4-row column A by the 4 lanes' own input reals; with one block's A broadcast to all
// blocks (CBSZ = 4, ABID = that block) an instruction adds one input real's contribution to 4
// output reals of all 64 groups of the wave, and every lane receives its own group's outputs, so no
// data crosses lanes.  Inputs are taken as (amplitude m, re | im) = kappa = 2 m + part; outputs in
// quads f = 0, 1 (main state, amplitudes 2f, 2f+1, re and im each) and f = 2, 3 (tangent state).
// The zero block (main outputs from tangent inputs) is never issued: 16 instructions for X on p,
// 16 for Y on p and 16 for X on d, 48 against the 64 a dense 16x16 product needs.
//
// Operand registers: block b = 2 kappa + f (the ABID) of register x holds rows 4f..4f+3 of column
// kappa of the real form of X ([[Re, -Im], [Im, Re]] per complex entry), register y the same of Y;
// the X columns serve both diagonal blocks.  Lane 4 b + i holds row i of block b.
__device__ __forceinline__ float w4_op(const float2* Z, int l, bool ct) {
  const int blk = l >> 2, i = l & 3;
  const int f = blk & 1, kap = blk >> 1;
  const int o = 2 * f + (i >> 1), co = i & 1, m = kap >> 1, ci = kap & 1;
  float2 z = ct ? Z[4 * m + o] : Z[4 * o + m];
  if (ct) z.y = -z.y;
  return co == ci ? z.x : (co == 0 ? -z.y : z.y);
}

template <int ABID>
__device__ __forceinline__ Mfma<float>::acc_t mfma4(float a, float b, Mfma<float>::acc_t c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 4, ABID, 0);
}

// Byte offsets ad[m] of this lane's amplitude m, shared by every state array of the tile: the lane
// part (its group's index bits) plus the wave-uniform parts am[m] (the wave's group bits and the
// pair bits).  The lane part is made opaque so that the compiler keeps each array's LDS base as an
// instruction offset (one add per amplitude for all arrays) instead of folding it into a base
// register per array.
__device__ __forceinline__ void tile_addr(int tl, const int (&am)[4], int (&ad)[4]) {
  int tb = 8 * tl;
  asm volatile("" : "+v"(tb));
#pragma unroll
  for (int c = 0; c < 4; ++c) ad[c] = tb + 8 * am[c];
}

// (p, d) <- W (p, d) on the 64 groups of one wave.  All LDS reads first (pinned, so that they are in
// flight together rather than read-and-wait one at a time), then the MFMAs, then the writes.  Groups
// beyond the tile (tiles of fewer than 2^kMaxTileBits amplitudes) hold tile indices >= 2^mb only:
// they are transformed and written back like the others, which leaves a zeroed tail zero (W 0 = 0)
// and never touches an index below 2^mb.
template <bool TANG>
struct WTile {
  float2 p[4], d[4];            // amplitudes 0..3 of the lane's group, main and tangent state
  Mfma<float>::acc_t r[4];      // output quads: main (0, 1), (2, 3); tangent (0, 1), (2, 3)
  __device__ __forceinline__ void load(const float2* sP, const float2* sD, const int (&ad)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      p[c] = *(const float2*)((const char*)sP + ad[c]);
      if (TANG) d[c] = *(const float2*)((const char*)sD + ad[c]);
    }
  }
  __device__ __forceinline__ void pin() {
    if (TANG)
      asm volatile("" ::"v"(p[0].x), "v"(p[0].y), "v"(p[1].x), "v"(p[1].y), "v"(p[2].x), "v"(p[2].y), "v"(p[3].x),
                   "v"(p[3].y), "v"(d[0].x), "v"(d[0].y), "v"(d[1].x), "v"(d[1].y), "v"(d[2].x), "v"(d[2].y),
                   "v"(d[3].x), "v"(d[3].y));
    else
      asm volatile("" ::"v"(p[0].x), "v"(p[0].y), "v"(p[1].x), "v"(p[1].y), "v"(p[2].x), "v"(p[2].y), "v"(p[3].x),
                   "v"(p[3].y));
  }
  // Main-input column kappa (all four output quads: X and Y on p), then the tangent-input columns
  // (X on d, tangent quads only): the main outputs are complete after the first 32 instructions, so
  // their stores overlap the last 16, and the tangent inputs are needed last.
  template <int KAP>
  __device__ __forceinline__ void column_p(float x, float y) {
    const float ip = (KAP & 1) ? p[KAP >> 1].y : p[KAP >> 1].x;
    r[0] = mfma4<2 * KAP>(x, ip, r[0]);
    r[1] = mfma4<2 * KAP + 1>(x, ip, r[1]);
    if constexpr (TANG) {
      r[2] = mfma4<2 * KAP>(y, ip, r[2]);
      r[3] = mfma4<2 * KAP + 1>(y, ip, r[3]);
    }
  }
  template <int KAP>
  __device__ __forceinline__ void column_d(float x) {
    const float id = (KAP & 1) ? d[KAP >> 1].y : d[KAP >> 1].x;
    r[2] = mfma4<2 * KAP>(x, id, r[2]);
    r[3] = mfma4<2 * KAP + 1>(x, id, r[3]);
  }
  template <int... K>
  __device__ __forceinline__ void columns(float x, float y, std::integer_sequence<int, K...>) {
    (column_p<K>(x, y), ...);
    if constexpr (TANG) (column_d<K>(x), ...);
  }
  __device__ __forceinline__ void mfma(float x, float y) {
#pragma unroll
    for (int c = 0; c < 4; ++c) { r[c][0] = 0; r[c][1] = 0; r[c][2] = 0; r[c][3] = 0; }
    columns(x, y, std::make_integer_sequence<int, 8>{});
  }
  __device__ __forceinline__ void store(float2* sP, float2* sD, const int (&ad)[4]) const {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const Mfma<float>::acc_t& q = r[c >> 1];
      *(float2*)((char*)sP + ad[c]) = (c & 1) ? make_float2(q[2], q[3]) : make_float2(q[0], q[1]);
      if (TANG) {
        const Mfma<float>::acc_t& u = r[2 + (c >> 1)];
        *(float2*)((char*)sD + ad[c]) = (c & 1) ? make_float2(u[2], u[3]) : make_float2(u[0], u[1]);
      }
    }
  }
};

template <bool TANG>
__device__ __forceinline__ void apply_w_mfma(float x, float y, float2* sP, float2* sD, int tl, const int (&am)[4]) {
  int ad[4];
  tile_addr(tl, am, ad);
  WTile<TANG> w;
  w.load(sP, sD, ad);
  w.pin();
  w.mfma(x, y);
  w.store(sP, sD, ad);
}

__device__ __forceinline__ int bitsel(int v, int b, int off) { return ((v >> b) & 1) ? off : 0; }

// Gate boundary inside a wave-local pass (every wave reads and writes only its own quarter of the
// tile): the LDS accesses of one wave are performed in issue order, so only the compiler has to be
// kept from moving LDS accesses across the boundary.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-gate LDS offsets of a pass, staged in LDS once per workgroup (kOffs ints per gate slot:
// goff[0..8), aoff[0..2)).  Read back after a barrier, they cannot be hoisted out of the tile loop
// (where they would occupy, then spill, scalar registers); readfirstlane keeps them scalar.
constexpr int kOffs = 10;
__device__ __forceinline__ void stage_offsets(const PassDesc& pd, int* sOff, int tid) {
  for (int j = 0; j < pd.ng; ++j) {
    if (tid < 8) sOff[kOffs * j + tid] = pd.goff[j][tid];
    else if (tid < 10) sOff[kOffs * j + tid] = pd.aoff[j][tid - 8];
  }
}
struct GateOff {
  int go[8], ao[2];
};
// complex64 operand tables of the gate applications (w4_op): per gate slot and lane, the x and y
// operands of each W the kernel applies, built once per launch, so that a gate step loads them with
// one LDS read (k_fwd: W = [[G, 0], [V, G]]; k_bwd_out: W^dag = [[G^dag, 0], [V^dag, G^dag]] and the
// inverse [[G^-1, 0], [Y, G^-1]]).
//
// What one gate step reads from the per-pass LDS tables, loaded ahead so that the step does not start
// with a chain of LDS round trips: the gate's offsets (made scalar with readfirstlane when used) and,
// for complex64, this lane's operands (k_fwd: x, y of W in op[0], op[1]; k_bwd_out: x, y of W^dag,
// then x, y of the inverse) and packed lane offsets.
struct StepRaw {
  int off[kOffs];
  qv4f op;
  int lanep;      // complex64: this lane's packed offsets of the gate (lane_offsets)
};
__device__ __forceinline__ void load_fwd_step(const int* sOff, const float2* sW, const int* sLane, int j, int lane,
                                              StepRaw& r) {
#pragma unroll
  for (int i = 0; i < kOffs; ++i) r.off[i] = sOff[kOffs * j + i];
  const float2 w = sW[64 * j + lane];
  r.op[0] = w.x; r.op[1] = w.y; r.op[2] = 0.f; r.op[3] = 0.f;
  r.lanep = sLane[64 * j + lane];
}
__device__ __forceinline__ void load_step(const int* sOff, const qv4f* sW, int j, int lane, bool with_gates,
                                          StepRaw& r) {
#pragma unroll
  for (int i = 0; i < kOffs; ++i) r.off[i] = sOff[kOffs * j + i];
  if (with_gates) r.op = sW[64 * j + lane];
}

// Padded LDS indices of the 4 amplitudes of group g (2*b_hi + b_lo order).
__device__ __forceinline__ void group_index(const GateOff& o, int g, int (&ix)[4]) {
  int t = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) t += bitsel(g, i, o.go[i]);
  ix[0] = t; ix[1] = t + o.ao[0]; ix[2] = t + o.ao[1]; ix[3] = t + o.ao[0] + o.ao[1];
}
__device__ __forceinline__ GateOff gate_offsets_raw(const int (&raw)[kOffs]) {
  GateOff o;
#pragma unroll
  for (int i = 0; i < 8; ++i) o.go[i] = __builtin_amdgcn_readfirstlane(raw[i]);
  o.ao[0] = __builtin_amdgcn_readfirstlane(raw[8]);
  o.ao[1] = __builtin_amdgcn_readfirstlane(raw[9]);
  return o;
}
__device__ __forceinline__ GateOff gate_offsets(const int* sOff, int j) {
  GateOff o;
#pragma unroll
  for (int i = 0; i < 8; ++i) o.go[i] = __builtin_amdgcn_readfirstlane(sOff[kOffs * j + i]);
  o.ao[0] = __builtin_amdgcn_readfirstlane(sOff[kOffs * j + 8]);
  o.ao[1] = __builtin_amdgcn_readfirstlane(sOff[kOffs * j + 9]);
  return o;
}

// Wave-uniform offsets of the 4 amplitudes of the W tile: the wave's group bits 6, 7 and the pair
// bits of the gate.
__device__ __forceinline__ void w_amps(const GateOff& o, int wave, int (&am)[4]) {
  const int wv = bitsel(wave, 0, o.go[6]) + bitsel(wave, 1, o.go[7]);
  am[0] = wv;
  am[1] = wv + o.ao[0];
  am[2] = wv + o.ao[1];
  am[3] = wv + o.ao[0] + o.ao[1];
}
// LDS offsets of gate slot j for the MFMA gate application of this lane / wave (group 64 wave + lane:
// its bits 0..5 are the lane's), from the pass constants goff / aoff.
__device__ __forceinline__ void w_offsets(const GateOff& o, int wave, int lane, int& tl, int (&am)[4]) {
  tl = 0;
#pragma unroll
  for (int i = 0; i < 6; ++i) tl += bitsel(lane, i, o.go[i]);
  w_amps(o, wave, am);
}

// complex64 per-lane offsets of a pass, computed once per launch (they depend on the gate slot and
// the lane only): sLane[64 j + l] packs, for lane l and gate slot j, the byte index of the lane's
// environment operand (low 16 bits; elements of R, second state array included) and 8x the
// element index of its group in the W tile (high 16 bits), both without the wave-uniform parts.
// The environment operand of lane l is real part cri of amplitude cidx of state cst of group sub
// (comp = l % 16 = 8 cst + 4 cri + cidx, sub = l / 16: group bits 0, 1), the layout of k_bwd_out's
// MFMA operands (A: rows = lane % 16, B: columns = lane % 16).
__device__ __forceinline__ int lane_offsets(const PassDesc& pd, int j, int l, int tsp, bool tang) {
  const int* go = pd.goff[j];
  const int* ao = pd.aoff[j];
  const int comp = l & 15, sub = l >> 4;
  const int cst = comp >> 3, cri = (comp >> 2) & 1, cidx = comp & 3;
  const int tl = bitsel(sub, 0, go[0]) + bitsel(sub, 1, go[1]) + bitsel(cidx, 0, ao[0]) + bitsel(cidx, 1, ao[1]);
  const int eb = 4 * (2 * (tang ? cst : 0) * tsp + cri + 2 * tl);
  int tw = 0;
#pragma unroll
  for (int i = 0; i < 6; ++i) tw += bitsel(l, i, go[i]);
  return eb | ((8 * tw) << 16);
}
// Tile byte offsets ad[c] from the lane's packed offsets (high half: 8x its element index).
__device__ __forceinline__ void tile_addr_packed(int lanep, const int (&am)[4], int (&ad)[4]) {
  int tb = (int)((unsigned)lanep >> 16);
  asm volatile("" : "+v"(tb));
#pragma unroll
  for (int c = 0; c < 4; ++c) ad[c] = tb + 8 * am[c];
}

// Stage the G (and V) entries of the pass's gates in LDS: sGV[32 j + e] = G_(gidx j)[e],
// sGV[32 j + 16 + e] = V_(gidx j)[e] (0 without tangent).  Visible after the next barrier.
template <bool TANG>
__device__ __forceinline__ void stage_gates(const PassDesc& pd, const float2* G, const float2* V, float2* sGV, int tid) {
  for (int j = 0; j < pd.ng; ++j) {
    const int k = pd.gidx[j];
    if (tid < 16) sGV[32 * j + tid] = G[16 * k + tid];
    else if (tid < 32) sGV[32 * j + tid] = TANG ? V[16 * k + tid - 16] : make_float2(0.f, 0.f);
  }
}

// The forward kernel's operand table (complex64): per gate slot j and lane l, the operands x, y of
// W = [[G, 0], [V, G]] (y = 0 without tangent).  Visible after the next barrier.
template <bool TANG>
__device__ __forceinline__ void stage_fwd_op_tables(const PassDesc& pd, const float2* G, const float2* V, float2* sW,
                                                    int tid) {
  for (int i = tid; i < pd.ng * 64; i += kThreads) {
    const int j = i >> 6, l = i & 63, k = pd.gidx[j];
    sW[i] = make_float2(w4_op(G + 16 * k, l, false), TANG ? w4_op(V + 16 * k, l, false) : 0.f);
  }
}

// Scatter the low `cnt` bits of v to the statevector bit positions pos[0..cnt).
__device__ __forceinline__ long long deposit(long long v, const int* pos, int cnt) {
  long long x = 0;
  for (int i = 0; i < cnt; ++i) x |= ((v >> i) & 1LL) << pos[i];
  return x;
}

// Next tile offset in enumeration order: pdep(w + 1, mask) from x = pdep(w, mask); 0 after the last.
__device__ __forceinline__ unsigned next_tile(unsigned x, unsigned mask) { return ((x | ~mask) + 1u) & mask; }

// Product state amplitude at statevector index x: prod_q u_q[bit of qubit q] (Sec. IV, Haar product states).
template <typename T>
__device__ __forceinline__ T product_amp(const T* u, int n, long long x) {
  T v = cz<T>();
  v.x = 1;
  for (int q = 0; q < n; ++q) {
    int bit = (int)((x >> (n - 1 - q)) & 1);
    v = cmul(v, u[2 * q + bit]);
  }
  return v;
}

// --------------------------------------------------------------------------------------------
// Forward pass
// --------------------------------------------------------------------------------------------
// NG > 0: an instance for passes of exactly NG gates (complex64), whose gate steps are unrolled
// into straight-line code; NG = 0: any gate count (complex128).
template <typename R, bool TANG, int NG>
// complex64: at least 4 waves per SIMD (registers <= 128), which the latency-bound forward needs
__global__ void __launch_bounds__(kThreads)
    __attribute__((amdgpu_waves_per_eu(std::is_same<R, float>::value ? 4 : 1, 8))) k_fwd(FwdArgs a) {
  using T = typename CT<R>::T;
  using LD = Lds<T>;
  using IO = TileIO<T>;
  constexpr bool kF32 = std::is_same<R, float>::value;
  __shared__ __attribute__((aligned(16))) T sP[LD::TSP];
  __shared__ __attribute__((aligned(16))) T sD[TANG ? LD::TSP : 1];
  __shared__ T sU[2 * kMaxQubits];
  __shared__ double sRed[kThreads / 64][4];
  __shared__ float2 sW[kF32 ? kMaxGates * 64 : 1];   // per gate slot and lane: operands x, y of W
  __shared__ int sLane[kF32 ? kMaxGates * 64 : 1];
  __shared__ int sOff[kMaxGates * kOffs];
  __shared__ int sSch[2];

  const PassDesc& pd = a.pd;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = pd.n, mb = pd.mb, ng = pd.ng;
  const int TS = 1 << mb, ngroups = TS >> 2;
  const long long dim = 1LL << n;
  const int tiles = 1 << (n - mb);
  const long long items = (long long)a.n_samples * tiles;
  const T* __restrict__ G = (const T*)a.gates;
  const T* __restrict__ V = (const T*)a.dirs;
  const T* srcP = (const T*)a.src_psi;
  const T* srcD = (const T*)a.src_dpsi;
  T* dstP = (T*)a.dst_psi;
  T* dstD = (T*)a.dst_dpsi;
  const T* __restrict__ phi0 = (const T*)a.phi0;
  const T* __restrict__ samp = (const T*)a.samples;
  const bool gen = (srcP == nullptr);
  const bool ovl = (a.ov_part != nullptr);
  // psi and dpsi are stored independently: a tangent sweep may leave psi in a boundary buffer that
  // already holds it (same gates) and store dpsi only; both decisions can come from the device
  const bool st_ok = a.store_if == nullptr || *a.store_if != 0;
  const bool stP = st_ok && dstP != nullptr && !(a.psi_skip != nullptr && *a.psi_skip != 0);
  const bool stD = st_ok && TANG && dstD != nullptr;
  const unsigned imask = (unsigned)pd.imask;
  const bool wl = pd.wave_local != 0;
  static_assert(NG >= 0 && NG <= kMaxGates && (NG > 0) == kF32, "complex64 instances have a fixed gate count");
  if (NG > 0 && ng != NG) return;   // the launcher picks the instance by the pass's gate count

  if constexpr (kF32) {
    stage_fwd_op_tables<TANG>(pd, (const float2*)G, (const float2*)V, sW, tid);
    for (int i = tid; i < ng * 64; i += kThreads) sLane[i] = lane_offsets(pd, i >> 6, i & 63, LD::TSP, TANG);
  }
  stage_offsets(pd, sOff, tid);

  int xv[IO::NV];
#pragma unroll
  for (int v = 0; v < IO::NV; ++v) xv[v] = (int)deposit(IO::elem(tid, v), pd.abit, mb);

  // Dynamic schedule: tiles are handed out in chunks of CH consecutive tiles from the launch's
  // counter (zeroed by the host), so a workgroup that runs ahead takes more and all finish together
  // (several workgroups share a CU and the hardware serves the oldest first: with a static split the
  // younger ones finished last, on a half-empty CU).  Thread 0 requests the next chunk at the start
  // of a chunk's first tile and publishes it in LDS at that tile's end, hiding the request's
  // latency; from then on the chunk's last tile can prefetch the next chunk's first tile.
  // (tile indices fit in 32 bits: the host checks items < 2^31).  Launches with few tiles per
  // workgroup use a static split instead (chunk < 0: workgroup b takes range b of -chunk tiles),
  // where the counter's round trips would not pay for themselves.
  const bool dyn = a.chunk > 0;
  const int nit = (int)items, CH = dyn ? a.chunk : -a.chunk;
  const int nch = (nit + CH - 1) / CH;
  if (dyn) {
    if (tid == 0) sSch[0] = atomicAdd(a.sched, 1);
    __syncthreads();
  }
  int c = dyn ? sSch[0] : (int)blockIdx.x, cn = -1;   // current chunk; the next one once known
  int it = c * CH;                            // current tile (item)
  int cend = c < nch ? min(it + CH, nit) : it;
  int pend = 0;                               // thread 0: the next chunk, requested at a chunk's start
  // current tile: sample s, offset x = pdep(tile index within the sample, imask)
  int s = 0;
  unsigned x = 0;
  if (c < nch) {
    s = it / tiles;
    x = (unsigned)deposit(it - s * tiles, pd.ibit, n - mb);
  }

  // complex64: the next tile's loads are in flight while the current tile is computed, and a tile's
  // stores wait until the next tile's loads are in; complex128 loads and stores at the tile's ends
  // (the registers those take would halve its occupancy; the other workgroups on the CU cover it)
  typename IO::V pf0[kF32 ? IO::NV : 1], pf1[kF32 ? IO::NV : 1];
#define QHVP_FWD_PREFETCH(S, X)                                                                     \
  {                                                                                                 \
    const long long bn_ = (long long)(S) * dim + (X);                                               \
    _Pragma("unroll") for (int v = 0; v < IO::NV; ++v) {                                            \
      pf0[v] = gld((const typename IO::V*)(srcP + bn_ + xv[v]));                                    \
      if (TANG) pf1[v] = gld((const typename IO::V*)(srcD + bn_ + xv[v]));                          \
    }                                                                                               \
  }
  if constexpr (kF32) {
    if (!gen && c < nch) QHVP_FWD_PREFETCH(s, x);
  }
  // The stores of tile t are issued after tile t+1's loads have been waited for: vmcnt counts
  // stores too, so stores issued right before that wait would be waited for as well.
  typename IO::V st0[kF32 ? IO::NV : 1], st1[kF32 ? IO::NV : 1];
  long long st_base = -1;
  StepRaw nxt;
  if constexpr (kF32) {
    __syncthreads();   // the staged tables
    load_fwd_step(sOff, sW, sLane, 0, lane, nxt);
  }

  while (c < nch) {
    const bool firstt = (it == c * CH);
    if (firstt && tid == 0) pend = dyn ? atomicAdd(a.sched, 1) : nch;
    const long long sbase = (long long)s * dim;
    const long long base = sbase + x;
    // the next tile: the next one of this chunk, else the first of the next chunk (known from the
    // end of this chunk's first tile; unknown during a chunk of one tile)
    bool hn = false;
    int sn = 0;
    unsigned xn = 0;
    if (it + 1 < cend) {
      hn = true;
      xn = next_tile(x, imask);
      sn = s + (xn == 0u ? 1 : 0);
    } else if (!firstt && cn < nch) {
      hn = true;
      const int itn = cn * CH;
      sn = itn / tiles;
      xn = (unsigned)deposit(itn - sn * tiles, pd.ibit, n - mb);
    }
    if (gen) {
      if (tid < 2 * n) sU[tid] = samp[(long long)s * 2 * n + tid];
      __syncthreads();
#pragma unroll
      for (int v = 0; v < IO::NV; ++v)
#pragma unroll
        for (int e = 0; e < IO::EPV; ++e) {
          const int t = IO::elem(tid, v) + e;
          if (t < TS) {
            sP[LD::at(t)] = product_amp(sU, n, (long long)x + xv[v] + e);
            if (TANG) sD[LD::at(t)] = cz<T>();
          }
        }
    } else if constexpr (kF32) {
#pragma unroll
      for (int v = 0; v < IO::NV; ++v) {
        IO::put(sP, IO::elem(tid, v), TS, pf0[v]);
        if (TANG) IO::put(sD, IO::elem(tid, v), TS, pf1[v]);
      }
    } else {
      typename IO::V l0[IO::NV], l1[IO::NV];
#pragma unroll
      for (int v = 0; v < IO::NV; ++v) {
        l0[v] = gld((const typename IO::V*)(srcP + base + xv[v]));
        if (TANG) l1[v] = gld((const typename IO::V*)(srcD + base + xv[v]));
      }
#pragma unroll
      for (int v = 0; v < IO::NV; ++v) {
        IO::put(sP, IO::elem(tid, v), TS, l0[v]);
        if (TANG) IO::put(sD, IO::elem(tid, v), TS, l1[v]);
      }
    }
    if constexpr (kF32) {
      if (st_base >= 0) {
        if (stP) IO::write(dstP, st0, st_base, xv, TS, tid);
        if (stD) IO::write(dstD, st1, st_base, xv, TS, tid);
      }
    }
    __syncthreads();
    if constexpr (kF32) {
      if (!gen && hn) QHVP_FWD_PREFETCH(sn, xn);
    }

    auto gate_step = [&](int j) {
      if constexpr (kF32) {
        // this step's tables were loaded one step ahead; load the next step's (the next tile's
        // first after the last gate: the tables do not change between tiles)
        const StepRaw cur = nxt;
        load_fwd_step(sOff, sW, sLane, j + 1 < NG ? j + 1 : 0, lane, nxt);
        const GateOff O = gate_offsets_raw(cur.off);
        int am[4], ad[4];
        w_amps(O, wave, am);
        tile_addr_packed(cur.lanep, am, ad);
        WTile<TANG> w;
        w.load(sP, sD, ad);
        w.mfma(cur.op[0], cur.op[1]);
        w.store(sP, sD, ad);
      } else {
        const GateOff O = gate_offsets(sOff, j);
        const auto Gk = opaque(G + 16 * pd.gidx[j]);
        const auto Vk = opaque(TANG ? V + 16 * pd.gidx[j] : G);
        if (tid < ngroups) {
          int ix[4];
          group_index(O, tid, ix);
          T p[4], d[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) { p[i] = sP[ix[i]]; if (TANG) d[i] = sD[ix[i]]; }
          apply_w<T, TANG>(Gk, Vk, p, d);
#pragma unroll
          for (int i = 0; i < 4; ++i) { sP[ix[i]] = p[i]; if (TANG) sD[ix[i]] = d[i]; }
        }
      }
      if (wl && j + 1 < ng) wave_sync();
      else __syncthreads();
    };
    if constexpr (NG > 0) {
#pragma unroll
      for (int j = 0; j < NG; ++j) gate_step(j);
    } else {
      for (int j = 0; j < ng; ++j) gate_step(j);
    }

    if (ovl) {
      double tr = 0, ti = 0, orr = 0, oi = 0;
      typename IO::V ph[IO::NV];
#pragma unroll
      for (int v = 0; v < IO::NV; ++v) ph[v] = gld((const typename IO::V*)(phi0 + base + xv[v]));
#pragma unroll
      for (int v = 0; v < IO::NV; ++v)
#pragma unroll
        for (int e = 0; e < IO::EPV; ++e) {
          const int t = IO::elem(tid, v) + e;
          if (t < TS) {
            const T f = IO::part(ph[v], e);
            const T ps = sP[LD::at(t)];
            tr += (double)f.x * ps.x + (double)f.y * ps.y;
            ti += (double)f.x * ps.y - (double)f.y * ps.x;
            if (TANG) {
              const T dp = sD[LD::at(t)];
              orr += (double)f.x * dp.x + (double)f.y * dp.y;
              oi += (double)f.x * dp.y - (double)f.y * dp.x;
            }
          }
        }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        tr += __shfl_xor(tr, off);
        ti += __shfl_xor(ti, off);
        orr += __shfl_xor(orr, off);
        oi += __shfl_xor(oi, off);
      }
      if ((tid & 63) == 0) {
        sRed[tid >> 6][0] = tr; sRed[tid >> 6][1] = ti; sRed[tid >> 6][2] = orr; sRed[tid >> 6][3] = oi;
      }
      __syncthreads();
      if (tid < 4) {
        double v = 0;
        for (int wv = 0; wv < kThreads / 64; ++wv) v += sRed[wv][tid];
        a.ov_part[(long long)it * 4 + tid] = v;
      }
    }
    if (stP || stD) {
      if constexpr (kF32) {
        if (stP) IO::read(st0, sP, tid);
        if (stD) IO::read(st1, sD, tid);
        st_base = base;
      } else {
        if (stP) IO::store(dstP, sP, base, xv, TS, tid);
        if (stD) IO::store(dstD, sD, base, xv, TS, tid);
      }
    }
    if (firstt && tid == 0) sSch[1] = pend;
    __syncthreads();
    if (firstt) cn = sSch[1];
    if (it + 1 < cend) {
      ++it;
      s = sn;
      x = xn;
    } else {
      c = cn;
      cn = -1;
      it = c * CH;
      cend = c < nch ? min(it + CH, nit) : it;
      if (c < nch) {
        if (hn) {
          s = sn;
          x = xn;
        } else {
          s = it / tiles;
          x = (unsigned)deposit(it - s * tiles, pd.ibit, n - mb);
          if constexpr (kF32) {
            if (!gen) QHVP_FWD_PREFETCH(s, x);
          }
        }
      }
    }
  }
  if constexpr (kF32) {
    if (st_base >= 0) {
      if (stP) IO::write(dstP, st0, st_base, xv, TS, tid);
      if (stD) IO::write(dstD, st1, st_base, xv, TS, tid);
    }
  }
}

// complex64 environment accumulation.  A wave's FP32 MFMA accumulator holds one tile's partial sums
// of one gate slot (64 products per element); right after its step the wave stages it in LDS
// (stg[(w * MAXG + j) * 256 + 4 * lane + r]), so no accumulator outlives its step.  k_bwd reduces
// after every tile, k_bwd_out after every pair of tiles (the second adds its partial to the first's
// in FP32: 128 products per element).  Between the end of that tile (pair) and the next tile's
// first barrier every thread adds the four waves' values of its own element e = 4 * lane + r, in
// wave order and in FP64, into one FP64 running sum per gate slot (sAcc[j * 256 + e]): the
// workgroup keeps 256 doubles per gate.
template <int MAXG>
__device__ __forceinline__ void env_put(const Mfma<float>::acc_t& e, float* stg, int j, int tid) {
  const int wave = tid >> 6, lane = tid & 63;
  *(qv4f*)(stg + (wave * MAXG + j) * 256 + 4 * lane) = e;
}
// All MAXG slots are reduced, used or not (an unused slot's sum is never read): without a branch
// per slot the loads of every slot are in flight together.
// The same, added to what the wave staged for the previous tile: k_bwd_out stages the sum of a pair
// of tiles (128 products per element in FP32) before the FP64 reduction.
template <int MAXG>
__device__ __forceinline__ void env_put_add(const Mfma<float>::acc_t& e, float* stg, int j, int tid) {
  const int wave = tid >> 6, lane = tid & 63;
  qv4f* p = (qv4f*)(stg + (wave * MAXG + j) * 256 + 4 * lane);
  const qv4f prev = *p;
  qv4f sum;
#pragma unroll
  for (int r = 0; r < 4; ++r) sum[r] = prev[r] + e[r];
  *p = sum;
}
template <int MAXG>
__device__ __forceinline__ void env_reduce(const float* stg, double* sAcc, int tid) {
  double v[MAXG], acc[MAXG];
#pragma unroll
  for (int j = 0; j < MAXG; ++j) {
    v[j] = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) v[j] += (double)stg[(w * MAXG + j) * 256 + tid];
    acc[j] = sAcc[j * 256 + tid];
  }
#pragma unroll
  for (int j = 0; j < MAXG; ++j) sAcc[j * 256 + tid] = acc[j] + v[j];
}

// Per-workgroup environment partials after the tile loop: sum the 4 waves' 16x16 MFMA blocks of
// each gate slot (FP64, fixed order), then combine the real blocks into the 16 complex entries of
// E = sum conj(a) psi^T and of D = sum conj(b) psi^T + conj(a) dpsi^T:
// env_part[wg][j][0..32) = E (re, im interleaved, entry 4x + y), [32..64) = D.
// sRed: kThreads * 4 doubles of LDS that the tile loop no longer uses.
template <typename R, int MAXG>
__device__ __forceinline__ void env_partials(const typename Mfma<R>::acc_t* acc, const double* sAcc, double* sRed,
                                             double* sM, int ng, int tid, double* env_part) {
  using M = Mfma<R>;
  constexpr bool kF32 = std::is_same<R, float>::value;
  const int wave = tid >> 6, lane = tid & 63, comp = lane & 15, sub = lane >> 4;
#pragma unroll
  for (int j = 0; j < MAXG; ++j) {
    if (j < ng) {
      if constexpr (kF32) {
        // the workgroup's sum of element e = 4 * lane_e + r is already in sAcc (see env_reduce)
        const int le = tid >> 2, r = tid & 3;
        sM[M::out_row(le >> 4, r) * 16 + (le & 15)] = sAcc[j * 256 + tid];
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) sRed[(wave * 64 + lane) * 4 + r] = (double)acc[j][r];
        __syncthreads();
        if (wave == 0) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double v = 0;
            for (int wv = 0; wv < kThreads / 64; ++wv) v += sRed[(wv * 64 + lane) * 4 + r];
            sM[M::out_row(sub, r) * 16 + comp] = v;
          }
        }
      }
      __syncthreads();
      if (tid < kEnvVals) {
        const int which = tid >> 5, e = (tid >> 1) & 15, part = tid & 1;
        const int ex = e >> 2, ey = e & 3;
        // row of A component (st: 0 a, 1 b; ri: 0 re, 1 im; amplitude k), column of B (0 psi, 1 dpsi)
#define RI(st, ri, k) (8 * (st) + 4 * (ri) + (k))
#define P(r, c) sM[(r) * 16 + (c)]
        double v;
        if (which == 0) {
          v = part == 0 ? P(RI(0, 0, ex), RI(0, 0, ey)) + P(RI(0, 1, ex), RI(0, 1, ey))
                        : P(RI(0, 0, ex), RI(0, 1, ey)) - P(RI(0, 1, ex), RI(0, 0, ey));
        } else {
          v = part == 0 ? P(RI(1, 0, ex), RI(0, 0, ey)) + P(RI(1, 1, ex), RI(0, 1, ey)) +
                              P(RI(0, 0, ex), RI(1, 0, ey)) + P(RI(0, 1, ex), RI(1, 1, ey))
                        : P(RI(1, 0, ex), RI(0, 1, ey)) - P(RI(1, 1, ex), RI(0, 0, ey)) +
                              P(RI(0, 0, ex), RI(1, 1, ey)) - P(RI(0, 1, ex), RI(1, 0, ey));
        }
#undef P
#undef RI
        env_part[((long long)blockIdx.x * kMaxGates + j) * kEnvVals + tid] = v;
      }
      __syncthreads();
    }
  }
}

// Two workgroups share each CU in the backward kernels (registers and LDS allow no more), and the
// hardware serves the older one first: with an even static split of the tiles the younger one fell
// behind and finished its share alone, on a half-empty CU.  The grid's two halves (workgroups b and
// b + grid/2, dispatched one round apart, so one older and one younger per CU) therefore take turns
// at the higher wave priority, in windows of 2^13 ticks (82 us) of the device's 100 MHz clock, so
// that both progress at the same average rate.  Which tiles a workgroup computes does not change,
// so results are unaffected.
__device__ __forceinline__ void share_cu_turns(unsigned half) {
  const unsigned rt = (unsigned)__builtin_amdgcn_s_memrealtime();
  if (((rt >> 13) ^ half) & 1u) __builtin_amdgcn_s_setprio(1);
  else __builtin_amdgcn_s_setprio(0);
}

// --------------------------------------------------------------------------------------------
// Backward pass with environment accumulation
// --------------------------------------------------------------------------------------------
// MAXG: most gates a pass may hold (the per-gate MFMA operands and accumulators are registers).
template <typename R, bool TANG, int MAXG>
__global__ void __launch_bounds__(kThreads) k_bwd(BwdArgs a) {
  using T = typename CT<R>::T;
  using M = Mfma<R>;
  using acc_t = typename M::acc_t;
  using LD = Lds<T>;
  using IO = TileIO<T>;
  constexpr int TSMAX = LD::TSMAX, TSP = LD::TSP;
  constexpr int NST = TANG ? 2 : 1;
  constexpr bool kF32 = std::is_same<R, float>::value;
  // sX: forward states (psi | dpsi), sY: backward states (a | b); element t of state st at
  // [st*TSP + LD::at(t)]
  __shared__ __attribute__((aligned(16))) T sX[NST * TSP];
  __shared__ __attribute__((aligned(16))) T sY[NST * TSP];
  __shared__ T sU[2 * kMaxQubits];
  __shared__ double sM[16 * 16];
  // complex64: FP64 running sums of the per-tile FP32 MFMA accumulators, one column per thread
  __shared__ double sAcc[kF32 ? MAXG * 256 : 1];
  __shared__ __attribute__((aligned(16))) float sStg[kF32 ? 4 * MAXG * 256 : 1];
  __shared__ float2 sGV[kF32 ? kMaxGates * 32 : 1];
  __shared__ int sOff[kMaxGates * kOffs];

  if (a.run_flag != nullptr && *a.run_flag != a.run_when) return;   // the other backward kernel runs
  const PassDesc& pd = a.pd;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int uwave = __builtin_amdgcn_readfirstlane(wave);
  const int n = pd.n, mb = pd.mb, ng = pd.ng;
  const int TS = 1 << mb, ngroups = TS >> 2;
  const long long dim = 1LL << n;
  const int tiles = 1 << (n - mb);
  const long long items = (long long)a.n_samples * tiles;
  const T* __restrict__ G = (const T*)a.gates;
  const T* __restrict__ V = (const T*)a.dirs;
  const T* srcP = (const T*)a.src_psi;
  const T* srcD = (const T*)a.src_dpsi;
  T* abA = (T*)a.ab_a;
  T* abB = (T*)a.ab_b;
  const T* __restrict__ phi0 = (const T*)a.phi0;
  const T* __restrict__ samp = (const T*)a.samples;
  const bool gen = (srcP == nullptr);
  const unsigned imask = (unsigned)pd.imask;
  const bool wl = pd.wave_local != 0;

  if constexpr (kF32) stage_gates<TANG>(pd, (const float2*)G, (const float2*)V, sGV, tid);
  stage_offsets(pd, sOff, tid);

  int xv[IO::NV];
#pragma unroll
  for (int v = 0; v < IO::NV; ++v) xv[v] = (int)deposit(IO::elem(tid, v), pd.abit, mb);

  // MFMA operand of this lane for the environment sums: real part cri of amplitude cidx (pair
  // index 2*b_hi + b_lo) of state cst, for group 64*wave + 4*c + sub in chunk c (A: rows =
  // lane%16, B: columns = lane%16).
  const int comp = lane & 15, sub = lane >> 4;
  const int cst = comp >> 3, cri = (comp >> 2) & 1, cidx = comp & 3;
  // Without tangent states the b rows / dpsi columns only feed the unused D sums; those lanes read
  // the a / psi arrays (in bounds) and their products are discarded.
  const int lane_scalar_off = 2 * (TANG ? cst : 0) * TSP + cri;  // in units of R

  acc_t acc[kF32 ? 1 : MAXG];   // complex128: FP64 sums over all tiles; complex64 stages per step
#pragma unroll
  for (int j = 0; j < MAXG; ++j) {
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[j][r] = 0;
  }
  if constexpr (kF32) {
    for (int i = tid; i < MAXG * 256; i += kThreads) sAcc[i] = 0;
  }
  // Groups g >= ngroups (only when mb < kMaxTileBits) map to tile indices >= 2^mb: zero them once so
  // that their MFMA operands are zero (the gate applications keep them zero).
  for (int t = TS + tid; t < TSMAX; t += kThreads) {
    sX[LD::at(t)] = cz<T>(); sY[LD::at(t)] = cz<T>();
    if (TANG) { sX[TSP + LD::at(t)] = cz<T>(); sY[TSP + LD::at(t)] = cz<T>(); }
  }
  __syncthreads();

  const long long it0 = items * blockIdx.x / gridDim.x;
  const long long it1 = items * (blockIdx.x + 1) / gridDim.x;
  int s = 0;
  unsigned x = 0;
  if (it0 < it1) {
    s = (int)(it0 / tiles);
    x = (unsigned)deposit(it0 - (long long)s * tiles, pd.ibit, n - mb);
  }

  // Common case (all four states come from memory): the next tile's loads are issued right
  // after the current tile is in LDS, so they are in flight during the current tile's compute.
  const bool common = !a.fold && !gen;
  typename IO::V pfa[IO::NV], pfb[IO::NV], pfp[IO::NV], pfd[IO::NV];
#define QHVP_BWD_PREFETCH(S, X)                                                                     \
  {                                                                                                 \
    const long long bn_ = (long long)(S) * dim + (X);                                               \
    _Pragma("unroll") for (int v = 0; v < IO::NV; ++v) {                                            \
      pfa[v] = gld((const typename IO::V*)(abA + bn_ + xv[v]));                                     \
      if (TANG) pfb[v] = gld((const typename IO::V*)(abB + bn_ + xv[v]));                           \
      pfp[v] = gld((const typename IO::V*)(srcP + bn_ + xv[v]));                                    \
      if (TANG) pfd[v] = gld((const typename IO::V*)(srcD + bn_ + xv[v]));                          \
    }                                                                                               \
  }
  if (common && it0 < it1) QHVP_BWD_PREFETCH(s, x);
  // deferred stores of the previous tile's (a, b), as in k_fwd (not with 5-gate passes, where the
  // registers they hold would halve the occupancy)
  constexpr bool kDefer = MAXG <= kSmallMaxGates;
  typename IO::V st0[IO::NV], st1[IO::NV];
  long long st_base = -1;

  const unsigned half = blockIdx.x >= gridDim.x / 2 ? 1u : 0u;
  for (long long it = it0; it < it1; ++it) {
    if (a.turns) share_cu_turns(half);
    const long long sbase = (long long)s * dim;
    const long long base = sbase + x;
    const unsigned xn = next_tile(x, imask);
    const int sn = s + (xn == 0u ? 1 : 0);

    if (common) {
#pragma unroll
      for (int v = 0; v < IO::NV; ++v) {
        IO::put(sY, IO::elem(tid, v), TS, pfa[v]);
        if (TANG) IO::put(sY + TSP, IO::elem(tid, v), TS, pfb[v]);
        IO::put(sX, IO::elem(tid, v), TS, pfp[v]);
        if (TANG) IO::put(sX + TSP, IO::elem(tid, v), TS, pfd[v]);
      }
    } else {
    // ---- backward states (a, b) at the pass output
    if (a.fold) {
      T Ts, Os;
      Ts.x = (R)a.tov[4 * s + 0]; Ts.y = (R)a.tov[4 * s + 1];
      Os.x = (R)a.tov[4 * s + 2]; Os.y = (R)a.tov[4 * s + 3];
      typename IO::V ph[IO::NV];
#pragma unroll
      for (int v = 0; v < IO::NV; ++v) ph[v] = gld((const typename IO::V*)(phi0 + base + xv[v]));
#pragma unroll
      for (int v = 0; v < IO::NV; ++v)
#pragma unroll
        for (int e = 0; e < IO::EPV; ++e) {
          const int t = IO::elem(tid, v) + e;
          const int at = t < TS ? LD::at(t) : LD::DUMMY;    // dummy slot when outside the tile
          const T f = IO::part(ph[v], e);
          sY[at] = cmul(Ts, f);
          if (TANG) sY[TSP + at] = cmul(Os, f);
        }
    } else {
      IO::load(sY, abA, base, xv, TS, tid);
      if (TANG) IO::load(sY + TSP, abB, base, xv, TS, tid);
    }
    // ---- forward states (psi, dpsi) at the pass input
    if (gen) {
      if (tid < 2 * n) sU[tid] = samp[(long long)s * 2 * n + tid];
      __syncthreads();
#pragma unroll
      for (int v = 0; v < IO::NV; ++v)
#pragma unroll
        for (int e = 0; e < IO::EPV; ++e) {
          const int t = IO::elem(tid, v) + e;
          if (t < TS) {
            sX[LD::at(t)] = product_amp(sU, n, (long long)x + xv[v] + e);
            if (TANG) sX[TSP + LD::at(t)] = cz<T>();
          }
        }
    } else {
      IO::load(sX, srcP, base, xv, TS, tid);
      if (TANG) IO::load(sX + TSP, srcD, base, xv, TS, tid);
    }
    }
    if (st_base >= 0) {
      IO::write(abA, st0, st_base, xv, TS, tid);
      if (TANG) IO::write(abB, st1, st_base, xv, TS, tid);
    }
    if constexpr (kF32) {
      // the previous tile's staged partials (staged before its final barrier; this tile stages after
      // the next one)
      if (it > it0) env_reduce<MAXG>(sStg, sAcc, tid);
    }
    __syncthreads();
    if (common && it + 1 < it1) QHVP_BWD_PREFETCH(sn, xn);

    // ---- forward recompute inside the tile; keep this lane's MFMA B operands of every gate
    R bop[MAXG][16];
#pragma unroll
    for (int j = 0; j < MAXG; ++j) {
      if (j < ng) {
        const GateOff O = gate_offsets(sOff, j);
        const int* go = O.go;
        const int* ao = O.ao;
        // LDS offset of this lane's operand in chunk 0 (group bits 0, 1 = sub; 6, 7 = wave) and the
        // wave-uniform offsets of the chunks (group bits 2..5)
        const int tl = bitsel(sub, 0, go[0]) + bitsel(sub, 1, go[1]) + bitsel(cidx, 0, ao[0]) +
                       bitsel(cidx, 1, ao[1]) + bitsel(uwave, 0, go[6]) + bitsel(uwave, 1, go[7]);
        const R* xs = (const R*)sX + lane_scalar_off + 2 * tl;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const int uo = ((c & 1) ? go[2] : 0) + ((c & 2) ? go[3] : 0) + ((c & 4) ? go[4] : 0) + ((c & 8) ? go[5] : 0);
          bop[j][c] = xs[2 * uo];
        }
        pin16(bop[j]);
        if (j + 1 < ng) {
          if constexpr (kF32) {
            int tw, am[4];
            w_offsets(O, uwave, lane, tw, am);
            const float wx = w4_op(sGV + 32 * j, lane, false);
            const float wy = TANG ? w4_op(sGV + 32 * j + 16, lane, false) : 0.f;
            apply_w_mfma<TANG>(wx, wy, sX, sX + TSP, tw, am);
          } else {
            const auto Gk = opaque(G + 16 * pd.gidx[j]);
            const auto Vk = opaque(TANG ? V + 16 * pd.gidx[j] : G);
            if (tid < ngroups) {
              int ix[4];
              group_index(O, tid, ix);
              T p[4], d[4];
#pragma unroll
              for (int i = 0; i < 4; ++i) { p[i] = sX[ix[i]]; if (TANG) d[i] = sX[TSP + ix[i]]; }
              apply_w<T, TANG>(Gk, Vk, p, d);
#pragma unroll
              for (int i = 0; i < 4; ++i) { sX[ix[i]] = p[i]; if (TANG) sX[TSP + ix[i]] = d[i]; }
            }
          }
          if (wl) wave_sync();
          else __syncthreads();
        }
      }
    }

    // ---- backward through the pass: accumulate environments, then undo the gate
#pragma unroll
    for (int j = MAXG - 1; j >= 0; --j) {
      if (j < ng) {
        const GateOff O = gate_offsets(sOff, j);
        const int* go = O.go;
        const int* ao = O.ao;
        const int tl = bitsel(sub, 0, go[0]) + bitsel(sub, 1, go[1]) + bitsel(cidx, 0, ao[0]) +
                       bitsel(cidx, 1, ao[1]) + bitsel(uwave, 0, go[6]) + bitsel(uwave, 1, go[7]);
        const R* ys = (const R*)sY + lane_scalar_off + 2 * tl;
        // all 16 A operands in flight together (one wait), then the 16 accumulating MFMAs
        R av[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const int uo = ((c & 1) ? go[2] : 0) + ((c & 2) ? go[3] : 0) + ((c & 4) ? go[4] : 0) + ((c & 8) ? go[5] : 0);
          av[c] = ys[2 * uo];
        }
        pin16(av);
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          if constexpr (kF32) acc[0] = M::step(av[c], bop[j][c], acc[0]);
          else acc[j] = M::step(av[c], bop[j][c], acc[j]);
        }
        if constexpr (kF32) {
          env_put<MAXG>(acc[0], sStg, j, tid);
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[0][r] = 0;
        }
        if constexpr (kF32) {
          int tw, am[4];
          w_offsets(O, uwave, lane, tw, am);
          const float wx = w4_op(sGV + 32 * j, lane, true);
          const float wy = TANG ? w4_op(sGV + 32 * j + 16, lane, true) : 0.f;
          apply_w_mfma<TANG>(wx, wy, sY, sY + TSP, tw, am);
        } else {
          const auto Gk = opaque(G + 16 * pd.gidx[j]);
          const auto Vk = opaque(TANG ? V + 16 * pd.gidx[j] : G);
          if (tid < ngroups) {
            int ix[4];
            group_index(O, tid, ix);
            T pa[4], pb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) { pa[i] = sY[ix[i]]; if (TANG) pb[i] = sY[TSP + ix[i]]; }
            apply_wdag<T, TANG>(Gk, Vk, pa, pb);
#pragma unroll
            for (int i = 0; i < 4; ++i) { sY[ix[i]] = pa[i]; if (TANG) sY[TSP + ix[i]] = pb[i]; }
          }
        }
        if (wl && j > 0) wave_sync();
        else __syncthreads();
      }
    }


    if (a.store_ab) {
      if constexpr (kDefer) {
        IO::read(st0, sY, tid);
        if (TANG) IO::read(st1, sY + TSP, tid);
        st_base = base;
      } else {
        IO::store(abA, sY, base, xv, TS, tid);
        if (TANG) IO::store(abB, sY + TSP, base, xv, TS, tid);
      }
    }
    __syncthreads();
    s = sn;
    x = xn;
  }
  if (st_base >= 0) {
    IO::write(abA, st0, st_base, xv, TS, tid);
    if (TANG) IO::write(abB, st1, st_base, xv, TS, tid);
  }

  if constexpr (kF32) {
    if (it1 > it0) env_reduce<MAXG>(sStg, sAcc, tid);   // staged by the last tile, after its barrier
  }
  env_partials<R, MAXG>(acc, sAcc, (double*)sY, sM, ng, tid, a.env_part);
}

// --------------------------------------------------------------------------------------------
// Backward pass from the pass-output forward states (gates with a well-conditioned inverse)
// --------------------------------------------------------------------------------------------
// Instead of recomputing the forward states inside the tile from the pass input (and holding each
// gate's operands until its environment is taken), this variant loads the forward states at the
// pass OUTPUT and undoes every gate on them in the same step that undoes it on the backward states:
// (psi, dpsi) <- (G^-1 psi, G^-1 dpsi + Y psi) with Y = -G^-1 V G^-1 (Eq. fis / Eq. dfis inverted).
// The environment sums of gate k are then taken against its output states,
//   Et = sum conj(a) psi_out^T,   Dt = sum conj(b) psi_out^T + conj(a) dpsi_out^T,
// which the host maps to the input-side sums (psi_in = G^-1 psi_out, dpsi_in = G^-1 (dpsi_out -
// V psi_in)): E = Et G^-T and D = (Dt - E V^T) G^-T.  Each step runs three independent products
// (environment, W^dag on (a, b), W^-1 on (psi, dpsi)).  igates holds G^-1 | Y per gate (32 complex).
// complex128: two workgroups per CU (two waves per SIMD) need at most 256 registers per lane; left to
// itself the compiler took 268 for the 6-gate instance, and then one workgroup fits.
template <typename R, bool TANG, int MAXG>
__global__ void __launch_bounds__(kThreads, sizeof(R) == 8 ? 2 : 1) k_bwd_out(BwdArgs a) {
  using T = typename CT<R>::T;
  using M = Mfma<R>;
  using acc_t = typename M::acc_t;
  using LD = Lds<T>;
  using IO = TileIO<T>;
  constexpr int TSMAX = LD::TSMAX, TSP = LD::TSP;
  constexpr int NST = TANG ? 2 : 1;
  constexpr bool kF32 = std::is_same<R, float>::value;
  // sX: forward states (psi | dpsi) at the current gate's output, sY: backward states (a | b).
  // Both start on a 512-byte boundary: the environment operands of sY and sX sit at the same index
  // of each array, so each pair is one ds_read2st64 (offsets in units of 256 / 512 bytes).
  __shared__ __attribute__((aligned(512))) T sX[NST * TSP];
  __shared__ __attribute__((aligned(512))) T sY[NST * TSP];
  __shared__ double sAcc[kF32 ? MAXG * 256 : 1];
  __shared__ int sLane[kF32 ? MAXG * 64 : 1];
  __shared__ __attribute__((aligned(16))) float sStg[kF32 ? 4 * MAXG * 256 : 1];
  __shared__ qv4f sW[kF32 ? kMaxGates * 64 : 1];   // per gate slot and lane: x, y of W^dag, x, y of the inverse
  __shared__ int sOff[kMaxGates * kOffs];

  if (a.run_flag != nullptr && *a.run_flag != a.run_when) return;   // the other backward kernel runs
  const PassDesc& pd = a.pd;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int uwave = __builtin_amdgcn_readfirstlane(wave);
  const int n = pd.n, mb = pd.mb, ng = pd.ng;
  const int TS = 1 << mb, ngroups = TS >> 2;
  const long long dim = 1LL << n;
  const int tiles = 1 << (n - mb);
  const long long items = (long long)a.n_samples * tiles;
  const T* __restrict__ G = (const T*)a.gates;
  const T* __restrict__ V = (const T*)a.dirs;
  const T* __restrict__ GI = (const T*)a.igates;
  const T* srcP = (const T*)a.src_psi;
  const T* srcD = (const T*)a.src_dpsi;
  T* abA = (T*)a.ab_a;
  T* abB = (T*)a.ab_b;
  T* dstP = (T*)a.dst_psi;
  T* dstD = (T*)a.dst_dpsi;
  const bool store_x = dstP != nullptr;   // the first gate is undone too, and the pass input stored
  const T* __restrict__ phi0 = (const T*)a.phi0;
  const unsigned imask = (unsigned)pd.imask;
  const bool wl = pd.wave_local != 0;
  // complex64 instances are compiled for exactly MAXG gates (the launcher picks the instance by the
  // pass's gate count), so that the gate steps are straight-line code
  if (kF32 && ng != MAXG) return;

  if constexpr (kF32) {
    // operand tables: W^dag = [[G^dag, 0], [V^dag, G^dag]] and the inverse [[G^-1, 0], [Y, G^-1]]
    for (int i = tid; i < ng * 64; i += kThreads) {
      const int j = i >> 6, l = i & 63, k = pd.gidx[j];
      const float2* Gk = (const float2*)G + 16 * k;
      const float2* GIk = (const float2*)GI + 32 * k;
      qv4f w;
      w[0] = w4_op(Gk, l, true);
      w[1] = TANG ? w4_op((const float2*)V + 16 * k, l, true) : 0.f;
      w[2] = w4_op(GIk, l, false);
      w[3] = TANG ? w4_op(GIk + 16, l, false) : 0.f;
      sW[i] = w;
    }
    for (int i = tid; i < ng * 64; i += kThreads) sLane[i] = lane_offsets(pd, i >> 6, i & 63, TSP, TANG);
  }
  stage_offsets(pd, sOff, tid);

  int xv[IO::NV];
#pragma unroll
  for (int v = 0; v < IO::NV; ++v) xv[v] = (int)deposit(IO::elem(tid, v), pd.abit, mb);

  const int comp = lane & 15, sub = lane >> 4;
  const int cst = comp >> 3, cri = (comp >> 2) & 1, cidx = comp & 3;
  const int lane_scalar_off = 2 * (TANG ? cst : 0) * TSP + cri;  // in units of R

  acc_t acc[kF32 ? 1 : MAXG];   // complex128: FP64 sums over all tiles; complex64 stages per step
#pragma unroll
  for (int j = 0; j < MAXG; ++j) {
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[j][r] = 0;
  }
  if constexpr (kF32) {
    for (int i = tid; i < MAXG * 256; i += kThreads) sAcc[i] = 0;
  }
  for (int t = TS + tid; t < TSMAX; t += kThreads) {
    sX[LD::at(t)] = cz<T>(); sY[LD::at(t)] = cz<T>();
    if (TANG) { sX[TSP + LD::at(t)] = cz<T>(); sY[TSP + LD::at(t)] = cz<T>(); }
  }
  __syncthreads();

  const long long it0 = items * blockIdx.x / gridDim.x;
  const long long it1 = items * (blockIdx.x + 1) / gridDim.x;
  int s = 0;
  unsigned x = 0;
  if (it0 < it1) {
    s = (int)(it0 / tiles);
    x = (unsigned)deposit(it0 - (long long)s * tiles, pd.ibit, n - mb);
  }

  const bool common = !a.fold;
  typename IO::V pfa[IO::NV], pfb[IO::NV], pfp[IO::NV], pfd[IO::NV];
  if (common && it0 < it1) QHVP_BWD_PREFETCH(s, x);
  // complex64 defers a tile's (a, b) stores until the next tile's loads are in; complex128 stores them
  // straight from LDS (the registers of the deferred copy would not let two workgroups share a CU)
  typename IO::V st0[kF32 ? IO::NV : 1], st1[kF32 ? IO::NV : 1];
  long long st_base = -1;

  const unsigned half = blockIdx.x >= gridDim.x / 2 ? 1u : 0u;
  for (long long it = it0; it < it1; ++it) {
    if (a.turns) share_cu_turns(half);
    const long long base = (long long)s * dim + x;
    const unsigned xn = next_tile(x, imask);
    const int sn = s + (xn == 0u ? 1 : 0);

    if (common) {
#pragma unroll
      for (int v = 0; v < IO::NV; ++v) {
        IO::put(sY, IO::elem(tid, v), TS, pfa[v]);
        if (TANG) IO::put(sY + TSP, IO::elem(tid, v), TS, pfb[v]);
        IO::put(sX, IO::elem(tid, v), TS, pfp[v]);
        if (TANG) IO::put(sX + TSP, IO::elem(tid, v), TS, pfd[v]);
      }
    } else {
      // last pass: a = T_s phi0, b = Omega_s phi0 (the folded boundary); forward states from memory
      T Ts, Os;
      Ts.x = (R)a.tov[4 * s + 0]; Ts.y = (R)a.tov[4 * s + 1];
      Os.x = (R)a.tov[4 * s + 2]; Os.y = (R)a.tov[4 * s + 3];
      typename IO::V ph[IO::NV];
#pragma unroll
      for (int v = 0; v < IO::NV; ++v) ph[v] = gld((const typename IO::V*)(phi0 + base + xv[v]));
#pragma unroll
      for (int v = 0; v < IO::NV; ++v)
#pragma unroll
        for (int e = 0; e < IO::EPV; ++e) {
          const int t = IO::elem(tid, v) + e;
          const int at = t < TS ? LD::at(t) : LD::DUMMY;
          const T f = IO::part(ph[v], e);
          sY[at] = cmul(Ts, f);
          if (TANG) sY[TSP + at] = cmul(Os, f);
        }
      IO::load(sX, srcP, base, xv, TS, tid);
      if (TANG) IO::load(sX + TSP, srcD, base, xv, TS, tid);
    }
    if constexpr (kF32) {
      if (st_base >= 0) {
        IO::write(abA, st0, st_base, xv, TS, tid);
        if (TANG) IO::write(abB, st1, st_base, xv, TS, tid);
      }
    }
    if constexpr (kF32) {
      // the staged partials of the previous pair of tiles (staged before the pair's final barrier;
      // odd-numbered tiles of the workgroup add to what their predecessor staged)
      if (it > it0 && ((it - it0) & 1) == 0) env_reduce<MAXG>(sStg, sAcc, tid);
    }
    __syncthreads();
    if (common && it + 1 < it1) QHVP_BWD_PREFETCH(sn, xn);

    if constexpr (kF32) {
      // The gate steps, software-pipelined inside each wave.  Region A of gate j applies the W
      // products to (a, b) and (psi, dpsi), whose operands were read earlier, and stores them in
      // place; after the step barrier, region B issues the reads of gate j-1's W operands (the states
      // just stored), runs gate j's environment chain on operands read before region A (its 16 MFMAs
      // cover those reads), stages the chain's sum, and issues the reads of gate j-1's environment
      // operands (covered by the 32 MFMAs of gate j-1's region A).  Every step still reads the
      // states its predecessor stored, and the arithmetic and its order are those of the plain
      // sequence: only the issue order changes.  Offsets and gate entries are loaded two steps ahead.
      StepRaw rw[2];
      load_step(sOff, sW, MAXG - 1, lane, true, rw[(MAXG - 1) & 1]);
      rw[(MAXG - 1) & 1].lanep = sLane[64 * (MAXG - 1) + lane];
      if (MAXG > 1) {
        load_step(sOff, sW, MAXG > 1 ? MAXG - 2 : 0, lane, true, rw[(MAXG - 2) & 1]);
        rw[(MAXG - 2) & 1].lanep = sLane[64 * (MAXG > 1 ? MAXG - 2 : 0) + lane];
      }
      R av[16], bx[16];
      WTile<TANG> wy, wx;
      int ad[4];
      // environment operands of a gate: one byte index for both state arrays, opaque so that their
      // LDS bases stay instruction offsets (one add per operand address); per-lane selects on the
      // loaded offsets, wave-uniform parts scalar
      auto env_reads = [&](const StepRaw& st, const GateOff& O) {
        const int wv = bitsel(uwave, 0, O.go[6]) + bitsel(uwave, 1, O.go[7]);
        int eb = (st.lanep & 0xffff) + 2 * (int)sizeof(R) * wv;
        asm volatile("" : "+v"(eb));
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const int uo = ((c & 1) ? O.go[2] : 0) + ((c & 2) ? O.go[3] : 0) + ((c & 4) ? O.go[4] : 0) +
                         ((c & 8) ? O.go[5] : 0);
          const int ib = eb + 2 * (int)sizeof(R) * uo;
          av[c] = *(const R*)((const char*)sY + ib);
          bx[c] = *(const R*)((const char*)sX + ib);
        }
      };
      // W operands of a gate (the tile addresses ad are kept for the stores)
      auto w_reads = [&](const StepRaw& st, const GateOff& O, bool ab, bool xs) {
        int am[4];
        w_amps(O, uwave, am);
        tile_addr_packed(st.lanep, am, ad);
        if (ab) wy.load(sY, sY + TSP, ad);
        if (xs) wx.load(sX, sX + TSP, ad);
      };
      {
        const GateOff O = gate_offsets_raw(rw[(MAXG - 1) & 1].off);
        env_reads(rw[(MAXG - 1) & 1], O);
        w_reads(rw[(MAXG - 1) & 1], O, MAXG > 1 || a.store_ab, MAXG > 1 || store_x);
      }
#pragma unroll
      for (int j = MAXG - 1; j >= 0; --j) {
        const StepRaw& cur = rw[j & 1];
        const bool undo_ab = j > 0 || a.store_ab;   // (a, b) at the pass input are needed
        // region A
        if (undo_ab) {
          wy.mfma(cur.op[0], cur.op[1]);
          wy.store(sY, sY + TSP, ad);
        }
        if (j > 0 || store_x) {
          wx.mfma(cur.op[2], cur.op[3]);
          wx.store(sX, sX + TSP, ad);
        }
        if (wl && j > 0) wave_sync();
        else __syncthreads();
        // region B
        GateOff On{};   // gate j-1's offsets
        if (j > 0) {
          On = gate_offsets_raw(rw[(j + 1) & 1].off);
          w_reads(rw[(j + 1) & 1], On, j > 1 || a.store_ab, j > 1 || store_x);
        }
        pin16(av);
        pin16(bx);
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[0] = M::step(av[c], bx[c], acc[0]);
        if ((it - it0) & 1) env_put_add<MAXG>(acc[0], sStg, j, tid);
        else env_put<MAXG>(acc[0], sStg, j, tid);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[0][r] = 0;
        if (j > 0) {
          env_reads(rw[(j + 1) & 1], On);
          if (j > 1) {   // gate j's are done
            load_step(sOff, sW, j > 1 ? j - 2 : 0, lane, true, rw[j & 1]);
            rw[j & 1].lanep = sLane[64 * (j > 1 ? j - 2 : 0) + lane];
          }
        }
      }
    } else {
#pragma unroll
    for (int j = MAXG - 1; j >= 0; --j) {
      if (j < ng) {
        StepRaw cur;
        load_step(sOff, sW, j, lane, false, cur);
        const GateOff O = gate_offsets_raw(cur.off);
        const int* go = O.go;
        const int tl = bitsel(sub, 0, cur.off[0]) + bitsel(sub, 1, cur.off[1]) + bitsel(cidx, 0, cur.off[8]) +
                       bitsel(cidx, 1, cur.off[9]) + bitsel(uwave, 0, go[6]) + bitsel(uwave, 1, go[7]);
        int eb = (int)sizeof(R) * (lane_scalar_off + 2 * tl);
        asm volatile("" : "+v"(eb));
        const bool undo_ab = j > 0 || a.store_ab;   // (a, b) at the pass input are needed
        R av[16], bx[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const int uo = ((c & 1) ? go[2] : 0) + ((c & 2) ? go[3] : 0) + ((c & 4) ? go[4] : 0) + ((c & 8) ? go[5] : 0);
          const int ib = eb + 2 * (int)sizeof(R) * uo;
          av[c] = *(const R*)((const char*)sY + ib);
          bx[c] = *(const R*)((const char*)sX + ib);
        }
        pin16(av);
        pin16(bx);
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[j] = M::step(av[c], bx[c], acc[j]);
        const auto Gk = opaque(G + 16 * pd.gidx[j]);
        const auto Vk = opaque(TANG ? V + 16 * pd.gidx[j] : G);
        const auto GIk = opaque(GI + 32 * pd.gidx[j]);
        const auto YIk = opaque(GI + 32 * pd.gidx[j] + 16);
        if (tid < ngroups) {
          int ix[4];
          group_index(O, tid, ix);
          if (undo_ab) {
            T pa[4], pb[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) { pa[i] = sY[ix[i]]; if (TANG) pb[i] = sY[TSP + ix[i]]; }
            apply_wdag<T, TANG>(Gk, Vk, pa, pb);
#pragma unroll
            for (int i = 0; i < 4; ++i) { sY[ix[i]] = pa[i]; if (TANG) sY[TSP + ix[i]] = pb[i]; }
          }
          if (j > 0 || store_x) {
            T p[4], d[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) { p[i] = sX[ix[i]]; if (TANG) d[i] = sX[TSP + ix[i]]; }
            apply_w<T, TANG>(GIk, YIk, p, d);
#pragma unroll
            for (int i = 0; i < 4; ++i) { sX[ix[i]] = p[i]; if (TANG) sX[TSP + ix[i]] = d[i]; }
          }
        }
        if (wl && j > 0) wave_sync();
        else __syncthreads();
      }
    }
    }

    if (a.store_ab) {
      if constexpr (kF32) {
        IO::read(st0, sY, tid);
        if (TANG) IO::read(st1, sY + TSP, tid);
        st_base = base;
      } else {
        IO::store(abA, sY, base, xv, TS, tid);
        if (TANG) IO::store(abB, sY + TSP, base, xv, TS, tid);
      }
    }
    if (store_x) {   // the rebuilt pass-input forward states, over the pass-output states this tile read
      IO::store(dstP, sX, base, xv, TS, tid);
      if (TANG) IO::store(dstD, sX + TSP, base, xv, TS, tid);
    }
    __syncthreads();
    s = sn;
    x = xn;
  }
  if constexpr (kF32) {
    if (st_base >= 0) {
      IO::write(abA, st0, st_base, xv, TS, tid);
      if (TANG) IO::write(abB, st1, st_base, xv, TS, tid);
    }
  }
  if constexpr (kF32) {
    if (it1 > it0) env_reduce<MAXG>(sStg, sAcc, tid);   // staged by the last one or two tiles, after their barrier
  }
  env_partials<R, MAXG>(acc, sAcc, (double*)sY, (double*)sX, ng, tid, a.env_part);   // sX, sY free now
}

#undef QHVP_FWD_PREFETCH
#undef QHVP_BWD_PREFETCH

// --------------------------------------------------------------------------------------------
// Deterministic fixed-order reductions
// --------------------------------------------------------------------------------------------
// One block per sample: thread t sums tiles w = t/4, t/4 + 64, ... of component t%4, then the 64
// partial sums are added in a fixed order.
__global__ void __launch_bounds__(256) k_reduce_overlaps(const double* __restrict__ ov_part, int n_samples,
                                                         int tiles, double* __restrict__ tov) {
  __shared__ double red[64][4];
  const int s = blockIdx.x;
  const int c = threadIdx.x & 3, chunk = threadIdx.x >> 2;
  double v = 0;
  for (int w = chunk; w < tiles; w += 64) v += ov_part[((long long)s * tiles + w) * 4 + c];
  red[chunk][c] = v;
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = 0;
    for (int k = 0; k < 64; ++k) t += red[k][c];
    tov[4 * s + c] = t;
  }
}

// One block per gate slot j: thread t sums workgroups wg = t/64, t/64 + 16, ... for output t%64,
// then the 16 partial sums are added in a fixed order.
__global__ void __launch_bounds__(1024) k_reduce_env(const double* __restrict__ env_part, int n_wg_set,
                                                     int n_wg_clear, const int* flag, PassDesc pd,
                                                     double* __restrict__ env) {
  __shared__ double red[16][kEnvVals];
  const int j = blockIdx.x;
  const int n_wg = (flag == nullptr || *flag != 0) ? n_wg_set : n_wg_clear;
  const int o = threadIdx.x & 63, chunk = threadIdx.x >> 6;
  double v = 0;
  for (int wg = chunk; wg < n_wg; wg += 16) v += env_part[((long long)wg * kMaxGates + j) * kEnvVals + o];
  red[chunk][o] = v;
  __syncthreads();
  if (threadIdx.x < kEnvVals) {
    double t = 0;
    for (int c = 0; c < 16; ++c) t += red[c][o];
    env[(long long)pd.gidx[j] * kEnvVals + o] = t;
  }
}

// --------------------------------------------------------------------------------------------
int grid_size(long long items) { return (int)(items < 2048 ? items : 2048); }

namespace {
// Occupancy cache slots: k_fwd complex64 0..11 (2 (ng - 1) + tangent), complex128 12..13; k_bwd
// 14..21; k_bwd_out complex128 22..25, complex64 26..37 (26 + 2 (ng - 1) + tangent).
constexpr int kKernelSlots = 48;
// Workgroups of `kern` that fit on the current device at once (all CUs), cached per device.  The
// persistent kernels split their tiles evenly over the grid, so a grid of exactly this many
// workgroups runs in one round instead of leaving a partial second round.
// Host threads may launch concurrently: the caches are relaxed atomics (every thread computes the
// same value, so a lost race only repeats the query).
int resident_wgs(const void* kern, int slot) {
  static std::atomic<int> cache[16][kKernelSlots] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return 2048;
  std::atomic<int>& c = cache[dev][slot];
  int v = c.load(std::memory_order_relaxed);
  if (v == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1 || cus < 1)
      return 2048;
    v = per_cu * cus;
    c.store(v, std::memory_order_relaxed);
  }
  return v;
}

// Compute units of the current device (cached per device).
int device_cus() {
  static std::atomic<int> cache[16] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) return 0;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v == 0) {
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    cache[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}
int pick_grid(long long items, int resident) {
  const long long g = items < resident ? items : resident;
  return (int)(g < 2048 ? g : 2048);
}

template <int NG>
const void* fwd_kernel_c64(int tangent) {
  return tangent ? (const void*)k_fwd<float, true, NG> : (const void*)k_fwd<float, false, NG>;
}
// The instance for a pass of ng gates (complex64: one per gate count), or null for an invalid count.
const void* fwd_kernel(Prec prec, int tangent, int ng, int* slot) {
  if (ng < 1 || ng > kMaxGates) return nullptr;
  if (prec == P_C64) {
    *slot = 2 * (ng - 1) + (tangent ? 1 : 0);
    switch (ng) {
      case 1: return fwd_kernel_c64<1>(tangent);
      case 2: return fwd_kernel_c64<2>(tangent);
      case 3: return fwd_kernel_c64<3>(tangent);
      case 4: return fwd_kernel_c64<4>(tangent);
      case 5: return fwd_kernel_c64<5>(tangent);
      default: return fwd_kernel_c64<6>(tangent);
    }
  }
  *slot = 12 + (tangent ? 1 : 0);
  return tangent ? (const void*)k_fwd<double, true, 0> : (const void*)k_fwd<double, false, 0>;
}

template <int MAXG>
const void* bwd_kernel_g(Prec prec, int tangent) {
  if (prec == P_C64) return tangent ? (const void*)k_bwd<float, true, MAXG> : (const void*)k_bwd<float, false, MAXG>;
  return tangent ? (const void*)k_bwd<double, true, MAXG> : (const void*)k_bwd<double, false, MAXG>;
}

const void* bwd_kernel(Prec prec, int tangent, int ng, int* slot) {
  if (ng < 1 || ng > kMaxGates) return nullptr;
  const bool small = ng <= kSmallMaxGates;
  *slot = 14 + (prec == P_C64 ? 0 : 2) + (tangent ? 1 : 0) + (small ? 4 : 0);
  return small ? bwd_kernel_g<kSmallMaxGates>(prec, tangent) : bwd_kernel_g<kMaxGates>(prec, tangent);
}
}  // namespace

int fwd_grid(Prec prec, int tangent, int ng, long long items) {
  int slot = 0;
  const void* k = fwd_kernel(prec, tangent, ng, &slot);
  return k ? pick_grid(items, resident_wgs(k, slot)) : 0;
}

template <int MAXG>
const void* bwd_out_kernel_c128(int tangent) {
  return tangent ? (const void*)k_bwd_out<double, true, MAXG> : (const void*)k_bwd_out<double, false, MAXG>;
}

template <int NG>
const void* bwd_out_kernel_c64(int tangent) {
  return tangent ? (const void*)k_bwd_out<float, true, NG> : (const void*)k_bwd_out<float, false, NG>;
}
// complex64: one instance per gate count (straight-line gate steps); complex128: passes of at most
// kSmallMaxGates gates use the lighter instance.  Null for an invalid count.
const void* bwd_out_kernel(Prec prec, int tangent, int ng, int* slot) {
  if (ng < 1 || ng > kMaxGates) return nullptr;
  if (prec == P_C64) {
    *slot = 26 + 2 * (ng - 1) + (tangent ? 1 : 0);
    switch (ng) {
      case 1: return bwd_out_kernel_c64<1>(tangent);
      case 2: return bwd_out_kernel_c64<2>(tangent);
      case 3: return bwd_out_kernel_c64<3>(tangent);
      case 4: return bwd_out_kernel_c64<4>(tangent);
      case 5: return bwd_out_kernel_c64<5>(tangent);
      default: return bwd_out_kernel_c64<6>(tangent);
    }
  }
  const bool small = ng <= kSmallMaxGates;
  *slot = 22 + (tangent ? 1 : 0) + (small ? 2 : 0);
  return small ? bwd_out_kernel_c128<kSmallMaxGates>(tangent) : bwd_out_kernel_c128<kMaxGates>(tangent);
}

int bwd_grid(Prec prec, int tangent, int ng, long long items, int from_output) {
  int slot = 0;
  const void* k = from_output ? bwd_out_kernel(prec, tangent, ng, &slot) : bwd_kernel(prec, tangent, ng, &slot);
  return k ? pick_grid(items, resident_wgs(k, slot)) : 0;
}

// Tiles per chunk of the dynamic schedule: about 32 chunks per workgroup (a late workgroup's tail is
// at most one chunk), between 4 and 64 tiles (from the second tile of a chunk on, the next chunk is
// known and its first tile can be prefetched; a chunk of one tile would load its successor
// without overlap).
int sched_chunk(long long items, int grid) {
  long long c = items / ((long long)grid * 32);
  return (int)(c < 4 ? 4 : (c > 64 ? 64 : c));
}
int launch_fwd(Prec prec, const FwdArgs& a0, void* stream) {
  const long long items = (long long)a0.n_samples << (a0.pd.n - a0.pd.mb);
  int slot = 0;
  const void* k = fwd_kernel(prec, a0.tangent, a0.pd.ng, &slot);
  if (k == nullptr || a0.sched == nullptr || items >= (1LL << 31)) return (int)hipErrorInvalidValue;
  dim3 grid(pick_grid(items, resident_wgs(k, slot))), block(kThreads);
  FwdArgs a = a0;
  // dynamic chunks when every workgroup has at least 16 tiles on average, else a static split
  // (QHVP_SCHEDULE=static, read at every launch, forces the static split; the results are the
  // same either way)
  const char* sched_env = std::getenv("QHVP_SCHEDULE");
  const bool force_static = sched_env != nullptr && std::strcmp(sched_env, "static") == 0;
  const bool dyn = !force_static && items >= 16LL * grid.x;
  a.chunk = dyn ? sched_chunk(items, (int)grid.x) : -(int)((items + grid.x - 1) / grid.x);
  void* args[] = {(void*)&a};
  return (int)hipLaunchKernel(k, grid, block, args, 0, (hipStream_t)stream);
}

int launch_bwd(Prec prec, const BwdArgs& a, void* stream) {
  const long long items = (long long)a.n_samples << (a.pd.n - a.pd.mb);
  int slot = 0;
  const void* k = bwd_kernel(prec, a.tangent, a.pd.ng, &slot);
  if (k == nullptr) return (int)hipErrorInvalidValue;
  dim3 grid(pick_grid(items, resident_wgs(k, slot))), block(kThreads);
  BwdArgs b = a;
  b.turns = (int)grid.x > device_cus() ? 1 : 0;   // two workgroups per CU
  void* args[] = {(void*)&b};
  return (int)hipLaunchKernel(k, grid, block, args, 0, (hipStream_t)stream);
}

int launch_bwd_out(Prec prec, const BwdArgs& a, void* stream) {
  const long long items = (long long)a.n_samples << (a.pd.n - a.pd.mb);
  int slot = 0;
  const void* k = bwd_out_kernel(prec, a.tangent, a.pd.ng, &slot);
  if (k == nullptr) return (int)hipErrorInvalidValue;
  dim3 grid(pick_grid(items, resident_wgs(k, slot))), block(kThreads);
  BwdArgs b = a;
  b.turns = (int)grid.x > device_cus() ? 1 : 0;   // two workgroups per CU
  void* args[] = {(void*)&b};
  return (int)hipLaunchKernel(k, grid, block, args, 0, (hipStream_t)stream);
}

// Zero n ints (the tile-schedule counters) with a kernel rather than a memset node, which stays
// correct when the caller captures the stream into a graph.
__global__ void __launch_bounds__(256) k_zero_ints(int* __restrict__ p, int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) p[i] = 0;
}
int launch_zero_ints(int* p, int n, void* stream) {
  const int blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_zero_ints, dim3(blocks < 64 ? blocks : 64), dim3(256), 0, (hipStream_t)stream, p, n);
  return (int)hipGetLastError();
}

int launch_reduce_overlaps(const double* ov_part, int n_samples, int tiles, double* tov, void* stream) {
  hipLaunchKernelGGL(k_reduce_overlaps, dim3(n_samples), dim3(256), 0, (hipStream_t)stream, ov_part, n_samples,
                     tiles, tov);
  return (int)hipGetLastError();
}

int launch_reduce_env(const double* env_part, int n_wg_set, int n_wg_clear, const int* flag, const PassDesc& pd,
                      double* env, void* stream) {
  hipLaunchKernelGGL(k_reduce_env, dim3(pd.ng), dim3(1024), 0, (hipStream_t)stream, env_part, n_wg_set, n_wg_clear,
                     flag, pd, env);
  return (int)hipGetLastError();
}

}  // namespace qhvp
