// Host runtime of the qhvp C ABI (include/qhvp.h): pass planning, workspace
// layout with layer checkpoints, the launch sequence of one cost / gradient /
// HVP evaluation, and the FP64 post-processing of Alg. 2 and App. F.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qhvp.h"
#include "qhvp_internal.h"

using cd = std::complex<double>;

namespace {

thread_local std::string g_err;

qhvp_status fail(qhvp_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(QHVP_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LAUNCH_TRY(expr)                                                                \
  do {                                                                                  \
    int e_ = (expr);                                                                    \
    if (e_ != 0) return fail(QHVP_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString((hipError_t)e_)); \
  } while (0)

constexpr int kCoalesceBits = 4;   // always-active low index bits: runs of >= 16 amplitudes
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int num_gates(int n, int L) {
  if (n < 2 || L < 1) return -1;
  return ((L + 1) / 2) * (n / 2) + (L / 2) * ((n - 1) / 2);
}

// Circuit -> passes.  Gate k of the brickwall (layers in order, qubits q = l%2, l%2+2, ... within
// layer l) acts on statevector bits lo = n-2-q and lo+1 and must follow the gates of layer l-1 on
// bits lo-1..lo+1.  A pass applies up to kMaxGates gates, in an order that respects these
// dependencies, to tiles spanned by 2^mb index bits: the low kCoalesceBits bits (runs of >= 16
// amplitudes per global access) plus a window of mb - kCoalesceBits consecutive bits.  The planner
// is greedy: each pass takes the window that admits the most gates (scanning gates in index order,
// so a gate may join once the gates it follows are done or already in the pass), and - at full
// tile size - at most mb - 2 touched tile bits, so that two untouched bits index the waves and the
// pass runs without workgroup barriers (wave-local).  In the plan's tail (at most kTailGates gates
// left) each window is instead scored by the passes a greedy plan of the rest would then need
// (ties: more gates now), which lets the last passes merge.  Gates of several layers share a pass,
// which cuts the number of HBM round trips (n=20, L=20: 32 passes for 190 gates, the fewest at 6
// gates per pass; one layer per pass would need 60).  gates_before[q] = gates in the passes before
// q (np + 1 entries).
constexpr int kTailGates = 48;
std::vector<qhvp::PassDesc> plan_circuit(int n, int L, std::vector<int>* gates_before) {
  const int K = num_gates(n, L);
  std::vector<int> glo(K), glayer(K);
  std::vector<std::vector<int>> at(L, std::vector<int>(n, -1));   // at[l][lo] = gate index
  for (int l = 0, k = 0; l < L; ++l)
    for (int q = l % 2; q + 1 < n; q += 2, ++k) {
      glo[k] = n - 2 - q;
      glayer[k] = l;
      at[l][glo[k]] = k;
    }
  std::vector<std::vector<int>> deps(K);
  for (int k = 0; k < K; ++k)
    if (glayer[k] > 0)
      for (int b = glo[k] - 1; b <= glo[k] + 1; ++b)
        if (b >= 0 && b < n && at[glayer[k] - 1][b] >= 0) deps[k].push_back(at[glayer[k] - 1][b]);

  const int mb = std::min(n, qhvp::kMaxTileBits);
  const int cb = std::min(kCoalesceBits, mb);
  std::vector<std::vector<int>> cands;   // tile bits of each candidate, ascending
  if (n <= mb) {
    std::vector<int> all(n);
    for (int b = 0; b < n; ++b) all[b] = b;
    cands.push_back(all);
  } else {
    for (int w = cb; w + (mb - cb) <= n; ++w) {
      std::vector<int> t;
      for (int b = 0; b < cb; ++b) t.push_back(b);
      for (int b = w; b < w + mb - cb; ++b) t.push_back(b);
      cands.push_back(t);
    }
  }
  const int max_touched = mb == qhvp::kMaxTileBits ? mb - 2 : mb;

  std::vector<qhvp::PassDesc> passes;
  std::vector<char> done(K, 0);
  // the gates a pass over tile bits `bits` takes, greedily in gate index order
  auto take_for = [&](const std::vector<int>& bits, const std::vector<char>& dn, std::vector<int>& take) {
    std::vector<char> in_tile(n, 0), touched(n, 0), in_pass(K, 0);
    for (int b : bits) in_tile[b] = 1;
    take.clear();
    int nt = 0;
    for (int k = 0; k < K && (int)take.size() < qhvp::kMaxGates; ++k) {
      if (dn[k] || !in_tile[glo[k]] || !in_tile[glo[k] + 1]) continue;
      bool ready = true;
      for (int d : deps[k]) ready = ready && (dn[d] || in_pass[d]);
      if (!ready) continue;
      const int add = (touched[glo[k]] ? 0 : 1) + (touched[glo[k] + 1] ? 0 : 1);
      if (nt + add > max_touched) continue;
      touched[glo[k]] = touched[glo[k] + 1] = 1;
      nt += add;
      in_pass[k] = 1;
      take.push_back(k);
    }
  };
  // the window a greedy pass takes (most gates, the first such window)
  auto greedy_pick = [&](const std::vector<char>& dn, std::vector<int>& best, std::vector<int>& best_bits) {
    std::vector<int> take;
    best.clear();
    for (const auto& bits : cands) {
      take_for(bits, dn, take);
      if (take.size() > best.size()) { best = take; best_bits = bits; }
    }
  };
  // passes a greedy plan needs for the gates not in dn
  auto greedy_count = [&](std::vector<char> dn, int left) {
    int np = 0;
    std::vector<int> best, best_bits;
    while (left > 0) {
      greedy_pick(dn, best, best_bits);
      if (best.empty()) return 1 << 20;   // (cannot happen: the first pending gate always fits)
      for (int k : best) dn[k] = 1;
      left -= (int)best.size();
      ++np;
    }
    return np;
  };
  if (gates_before) gates_before->assign(1, 0);
  int remaining = K, total = 0;
  while (remaining > 0) {
    std::vector<int> best, best_bits;
    if (remaining > kTailGates) {
      greedy_pick(done, best, best_bits);
    } else {
      int best_cost = -1;
      std::vector<int> take;
      for (const auto& bits : cands) {
        take_for(bits, done, take);
        if (take.empty()) continue;
        std::vector<char> dn = done;
        for (int k : take) dn[k] = 1;
        const int cost = 1 + greedy_count(dn, remaining - (int)take.size());
        if (best_cost < 0 || cost < best_cost || (cost == best_cost && take.size() > best.size())) {
          best_cost = cost;
          best = take;
          best_bits = bits;
        }
      }
      if (best.empty()) greedy_pick(done, best, best_bits);
    }
    if (best.empty()) break;   // (cannot happen: the first pending gate always fits a window)
    qhvp::PassDesc pd;
    std::memset(&pd, 0, sizeof(pd));
    pd.n = n;
    pd.mb = (int)best_bits.size();
    std::vector<int> tpos(n, -1);
    std::vector<char> act(n, 0);
    for (int b : best_bits) act[b] = 1;
    for (int b = 0, ti = 0, ii = 0; b < n; ++b) {
      if (act[b]) { pd.abit[ti] = b; tpos[b] = ti++; }
      else pd.ibit[ii++] = b;
    }
    pd.ng = (int)best.size();
    for (int g = 0; g < pd.ng; ++g) {
      const int k = best[g];
      pd.gidx[g] = k;
      pd.tlo[g] = tpos[glo[k]];
      pd.thi[g] = tpos[glo[k] + 1];
      done[k] = 1;
    }
    remaining -= pd.ng;
    total += pd.ng;
    passes.push_back(pd);
    if (gates_before) gates_before->push_back(total);
  }
  return passes;
}

// LDS index of tile element t in the kernels' layout: complex64 per-bit offsets (kLdsPadC64),
// complex128 16 spare bytes after every 256 bytes.
int lds_at(int t, int elem_bytes) {
  if (elem_bytes == 8) {
    int r = t;
    for (int b = 5; b < qhvp::kMaxTileBits; ++b) r += ((t >> b) & 1) * qhvp::kLdsPadC64[b];
    return r;
  }
  return t + (t >> 4);
}

// gfx950 LDS bank model, fitted to the hardware's bank-conflict counter on probe access patterns:
// a wave's access of `width` bytes per lane is served a group of lanes at a time (32-bit: 32 lanes
// over 32 banks of 4 bytes; 64-bit reads: 32 lanes over 64 banks; 64-bit writes: 16 lanes over 32
// banks; 128-bit reads: 16 lanes over 64 banks; 128-bit writes: 8 lanes over 32 banks), and a group
// takes as many cycles as its most used bank holds distinct dwords.  Returns the wave's cycles.
int lds_cycles(const int (&addr)[64], int width, bool write) {
  int group = 32, banks = 32;
  if (width == 8) { group = write ? 16 : 32; banks = write ? 32 : 64; }
  if (width == 16) { group = write ? 8 : 16; banks = write ? 32 : 64; }
  int total = 0;
  for (int s = 0; s < 64; s += group) {
    int dw[64 * 4], n = 0;
    for (int l = s; l < s + group; ++l)
      for (int k = 0; k < width / 4; ++k) dw[n++] = addr[l] / 4 + k;
    std::sort(dw, dw + n);
    n = (int)(std::unique(dw, dw + n) - dw);
    int cnt[64] = {0}, worst = 0;
    for (int i = 0; i < n; ++i) worst = std::max(worst, ++cnt[dw[i] % banks]);
    total += worst;
  }
  return total;
}

// Modelled bank-conflict cycles of one complex64 backward gate step (k_bwd_out) for a gate on tile
// bits lo, hi whose group bits 0..3 sit on tile bits p0..p3: the environment operand reads (32-bit,
// 32 wave accesses per step; lanes over the amplitude bits lo, hi, the state arrays, real / imaginary
// part and group bits 0, 1) and the W-tile reads and writes (64-bit, 16 each; lanes over group bits
// 0..3 and lo, hi).  Wave-uniform parts of the addresses shift every lane alike and drop out.
int c64_step_conflicts(int lo, int hi, int p0, int p1, int p2, int p3) {
  auto O = [](int b) { return lds_at(1 << b, 8); };
  auto sel = [](int v, int bit, int off) { return ((v >> bit) & 1) ? off : 0; };
  int env[64], w[64];
  for (int l = 0; l < 64; ++l) {
    const int comp = l & 15, sub = l >> 4;
    const int cst = comp >> 3, cri = (comp >> 2) & 1, cidx = comp & 3;
    const int tl = sel(sub, 0, O(p0)) + sel(sub, 1, O(p1)) + sel(cidx, 0, O(lo)) + sel(cidx, 1, O(hi));
    env[l] = 4 * (2 * cst * qhvp::kTspC64 + cri + 2 * tl);
    const int col = l & 15, g = l >> 4;
    const int tw = sel(col, 0, O(p0)) + sel(col, 1, O(p1)) + sel(col, 2, O(p2)) + sel(col, 3, O(p3)) +
                   sel(g, 0, O(lo)) + sel(g, 1, O(hi));
    w[l] = 8 * tw;
  }
  return 32 * (lds_cycles(env, 4, false) - 2) + 16 * (lds_cycles(w, 8, false) - 2) +
         16 * (lds_cycles(w, 8, true) - 4);
}

// Per-pass constants of the kernels' tile addressing: the tile-enumeration mask and, per gate, the
// padded LDS offsets of the group-index bits (zero bits inserted at tlo < thi) and of tlo / thi.
//
// Group index bits 6, 7 select the wave.  Wave-local layout (full tile, two tile bits f0 < f1 that
// no gate of the pass touches): bits 6, 7 sit on f0, f1 for every gate and bits 0..5 on the other
// free bits in ascending order, so each wave only ever touches its own quarter of the tile.
// Otherwise group bit i sits on the i-th tile bit other than tlo, thi (bits beyond the tile for
// tiles of fewer than 2^kMaxTileBits amplitudes).
void fill_tile_offsets(std::vector<qhvp::PassDesc>& passes, int elem_bytes) {
  for (auto& pd : passes) {
    pd.imask = 0;
    for (int i = 0; i < pd.n - pd.mb; ++i) pd.imask |= 1ULL << pd.ibit[i];
    bool used[qhvp::kMaxTileBits] = {};
    for (int j = 0; j < pd.ng; ++j) used[pd.tlo[j]] = used[pd.thi[j]] = true;
    int f1 = -1, f0 = -1;
    if (pd.mb == qhvp::kMaxTileBits) {
      for (int b = qhvp::kMaxTileBits - 1; b >= 0 && f0 < 0; --b)
        if (!used[b]) { if (f1 < 0) f1 = b; else f0 = b; }
    }
    pd.wave_local = f0 >= 0 ? 1 : 0;
    for (int j = 0; j < pd.ng; ++j) {
      const int lo = pd.tlo[j], hi = pd.thi[j];
      int pos[8];
      if (pd.wave_local) {
        int avail[6], k = 0;
        for (int b = 0; b < qhvp::kMaxTileBits; ++b)
          if (b != lo && b != hi && b != f0 && b != f1) avail[k++] = b;
        for (int i = 0; i < 6; ++i) pos[i] = avail[i];
        if (elem_bytes == 8) {
          // complex64: choose the tile bits the lanes run over (group bits 0, 1: the sub-rows of
          // the environment operands; 0..3: the 16 columns of the gate application; the order of
          // 2 and 3 does not matter) with the fewest modelled bank-conflict cycles per gate step
          int best = -1;
          for (int a0 = 0; a0 < 6; ++a0)
            for (int a1 = 0; a1 < 6; ++a1)
              for (int a2 = 0; a2 < 6; ++a2)
                for (int a3 = a2 + 1; a3 < 6; ++a3) {
                  if (a0 == a1 || a0 == a2 || a0 == a3 || a1 == a2 || a1 == a3) continue;
                  const int c = c64_step_conflicts(lo, hi, avail[a0], avail[a1], avail[a2], avail[a3]);
                  if (best < 0 || c < best) {
                    best = c;
                    pos[0] = avail[a0]; pos[1] = avail[a1]; pos[2] = avail[a2]; pos[3] = avail[a3];
                    int r = 4;
                    for (int i = 0; i < 6; ++i)
                      if (i != a0 && i != a1 && i != a2 && i != a3) pos[r++] = avail[i];
                  }
                }
        }
        pos[6] = f0;
        pos[7] = f1;
      } else {
        for (int i = 0; i < 8; ++i) {
          pos[i] = i + (i >= lo ? 1 : 0);
          pos[i] += (pos[i] >= hi ? 1 : 0);
        }
      }
      for (int i = 0; i < 8; ++i) pd.goff[j][i] = lds_at(1 << pos[i], elem_bytes);
      pd.aoff[j][0] = lds_at(1 << lo, elem_bytes);
      pd.aoff[j][1] = lds_at(1 << hi, elem_bytes);
    }
  }
}

// Segments of the backward sweep (pass index ranges); each segment starts at a stored
// checkpoint (pass 0's input is regenerated from the samples).
std::vector<std::pair<int, int>> plan_segments(int n, int L, int ckpt_every) {
  std::vector<int> gb;
  auto passes = plan_circuit(n, L, &gb);
  const int np = (int)passes.size();
  std::vector<std::pair<int, int>> seg;
  if (ckpt_every > 0) {
    // a checkpoint about every ckpt_every layers' worth of gates: a segment ends before the first
    // pass that starts at or beyond the next multiple of ckpt_every * K / L gates
    const double step = (double)ckpt_every * num_gates(n, L) / L;
    double next = step;
    int start = 0;
    for (int q = 1; q < np; ++q)
      if (gb[q] >= next - 1e-9) {
        seg.push_back({start, q});
        start = q;
        while (next <= gb[q] + 1e-9) next += step;
      }
    seg.push_back({start, np});
  } else {
    int c = ckpt_every == 0 ? 1 : -ckpt_every;
    for (int p = 0; p < np; p += c) seg.push_back({p, std::min(np, p + c)});
  }
  return seg;
}

struct Layout {
  size_t state_bytes = 0;   // one state set: N_s * 2^n amplitudes
  int n_ckpt = 0;           // stored segment-start checkpoints (segments 1..J-1)
  int n_seg = 0;            // in-segment boundary buffers (max segment length - 1)
  int slot_states = 1;      // state sets per slot (2 with tangent)
  int n_wg_max = 0;
  int tiles_max = 0;
  size_t off_phi0 = 0, off_slots = 0, off_small = 0, total = 0;
  size_t slot_bytes = 0;
  // small buffers (offsets from off_small)
  size_t o_samples, o_gates, o_dirs, o_igates, o_uref, o_tov, o_ovpart, o_envpart, o_env, o_sched;
};

// Tile-schedule counters (one int per launch, zeroed at the start of every sweep)
constexpr int kSchedSlots = 4096;

bool make_layout(int n, int L, int L_ref, int Ns, qhvp_precision prec, int ckpt_every, int tangent,
                 Layout& lay) {
  if (n < 2 || n > qhvp::kMaxQubits || L < 1 || L_ref < 1 || Ns < 1) return false;
  const size_t amp = prec == QHVP_C64_ACC64 ? 8 : 16;
  const int K = num_gates(n, L), Kr = num_gates(n, L_ref);
  auto seg = plan_segments(n, L, ckpt_every);
  int maxlen = 0;
  for (auto& s : seg) maxlen = std::max(maxlen, s.second - s.first);
  lay.state_bytes = align_up((size_t)Ns * ((size_t)1 << n) * amp);
  lay.slot_states = tangent ? 2 : 1;
  lay.slot_bytes = lay.state_bytes * lay.slot_states;
  lay.n_ckpt = (int)seg.size() - 1;
  lay.n_seg = maxlen - 1;
  const int mb = std::min(n, qhvp::kMaxTileBits);
  lay.tiles_max = 1 << (n - mb);
  lay.n_wg_max = qhvp::grid_size((long long)Ns * lay.tiles_max);
  lay.off_phi0 = 0;
  lay.off_slots = lay.state_bytes;
  const int nslots = lay.n_ckpt + lay.n_seg + 1;   // + working / backward (a, b) slot
  lay.off_small = lay.off_slots + (size_t)nslots * lay.slot_bytes;
  size_t o = 0;
  lay.o_samples = o; o = align_up(o + (size_t)Ns * n * 2 * amp);
  lay.o_gates = o;   o = align_up(o + (size_t)K * 16 * amp);
  lay.o_dirs = o;    o = align_up(o + (size_t)K * 16 * amp);
  lay.o_igates = o;  o = align_up(o + (size_t)K * 32 * amp);
  lay.o_uref = o;    o = align_up(o + (size_t)Kr * 16 * amp);
  lay.o_tov = o;     o = align_up(o + (size_t)Ns * 4 * sizeof(double));
  // overlap partials: the ansatz and U_ref plans share the tile count of their passes
  lay.o_ovpart = o;  o = align_up(o + (size_t)Ns * lay.tiles_max * 4 * sizeof(double) * 2);
  lay.o_envpart = o; o = align_up(o + (size_t)lay.n_wg_max * qhvp::kMaxGates * qhvp::kEnvVals * sizeof(double));
  lay.o_env = o;     o = align_up(o + (size_t)K * qhvp::kEnvVals * sizeof(double));
  lay.o_sched = o;   o = align_up(o + (size_t)kSchedSlots * sizeof(int));
  lay.total = lay.off_small + o;
  return true;
}

bool finite_all(const double* x, size_t cnt) {
  for (size_t i = 0; i < cnt; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

// ---- 4x4 complex helpers (FP64, host)
typedef cd M4[16];
void load4(const double* p, cd* m) { for (int i = 0; i < 16; ++i) m[i] = cd(p[2 * i], p[2 * i + 1]); }
void store4(const cd* m, double* p) { for (int i = 0; i < 16; ++i) { p[2 * i] = m[i].real(); p[2 * i + 1] = m[i].imag(); } }
void mul4(const cd* a, const cd* b, cd* c) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cd s = 0;
      for (int k = 0; k < 4; ++k) s += a[4 * i + k] * b[4 * k + j];
      c[4 * i + j] = s;
    }
}
void dag4(const cd* a, cd* b) { for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) b[4 * i + j] = std::conj(a[4 * j + i]); }
// P_G(X) = X/2 - G X^dag G / 2 (Eq. projec)
void project4(const cd* G, const cd* X, cd* out) {
  M4 Xd, t, u;
  dag4(X, Xd);
  mul4(G, Xd, t);
  mul4(t, G, u);
  for (int i = 0; i < 16; ++i) out[i] = 0.5 * X[i] - 0.5 * u[i];
}
// P_G(H - V grad^dag G / 2 - G grad^dag V / 2) (App. F)
void riem_hvp4(const cd* G, const cd* gr, const cd* H, const cd* V, cd* out) {
  M4 grd, t1, t2, t3, t4, inner;
  dag4(gr, grd);
  mul4(V, grd, t1); mul4(t1, G, t2);
  mul4(G, grd, t3); mul4(t3, V, t4);
  for (int i = 0; i < 16; ++i) inner[i] = H[i] - 0.5 * t2[i] - 0.5 * t4[i];
  project4(G, inner, out);
}
double unitarity_err4(const cd* G) {
  M4 Gd, P;
  dag4(G, Gd);
  mul4(Gd, G, P);
  double e = 0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) e += std::norm(P[4 * i + j] - (i == j ? 1.0 : 0.0));
  return std::sqrt(e);
}
// Polar factor of A via Newton iteration X <- (X + X^-dag)/2 with scaling (Higham); FP64.
bool inv4(const cd* a, cd* out) {
  cd m[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 8; ++j) m[i][j] = j < 4 ? a[4 * i + j] : (j - 4 == i ? 1.0 : 0.0);
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r) if (std::abs(m[r][c]) > std::abs(m[piv][c])) piv = r;
    if (std::abs(m[piv][c]) < 1e-300) return false;
    if (piv != c) for (int j = 0; j < 8; ++j) std::swap(m[c][j], m[piv][j]);
    cd d = m[c][c];
    for (int j = 0; j < 8; ++j) m[c][j] /= d;
    for (int r = 0; r < 4; ++r)
      if (r != c) {
        cd f = m[r][c];
        for (int j = 0; j < 8; ++j) m[r][j] -= f * m[c][j];
      }
  }
  for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) out[4 * i + j] = m[i][j + 4];
  return true;
}
double fro4(const cd* a) { double s = 0; for (int i = 0; i < 16; ++i) s += std::norm(a[i]); return std::sqrt(s); }
bool polar4(const cd* A, cd* U) {
  M4 X, Xi, Xid;
  for (int i = 0; i < 16; ++i) X[i] = A[i];
  for (int it = 0; it < 100; ++it) {
    if (!inv4(X, Xi)) return false;
    dag4(Xi, Xid);
    double g = std::sqrt(fro4(Xi) / fro4(X));   // Frobenius scaling
    M4 Y;
    double diff = 0;
    for (int i = 0; i < 16; ++i) {
      Y[i] = 0.5 * (g * X[i] + Xid[i] / g);
      diff += std::norm(Y[i] - X[i]);
    }
    for (int i = 0; i < 16; ++i) X[i] = Y[i];
    if (it > 2 && std::sqrt(diff) < 1e-15) break;
  }
  // two unscaled steps to settle at full accuracy
  for (int it = 0; it < 2; ++it) {
    if (!inv4(X, Xi)) return false;
    dag4(Xi, Xid);
    for (int i = 0; i < 16; ++i) X[i] = 0.5 * (X[i] + Xid[i]);
  }
  for (int i = 0; i < 16; ++i) U[i] = X[i];
  return true;
}

}  // namespace

// --------------------------------------------------------------------------------------------
struct qhvp_ctx {
  int device;
};

struct qhvp_problem {
  qhvp_ctx* ctx;
  int n, L, L_ref, Ns, K, Kr;
  qhvp_precision prec;
  int ckpt_every, tangent;
  hipStream_t stream;
  std::vector<qhvp::PassDesc> passes, ref_passes;
  std::vector<std::pair<int, int>> seg;
  Layout lay;
  char* ws;
  bool owns_ws;
  // host staging (pinned)
  void* h_gates;   // K*16 amplitudes (device precision)
  void* h_dirs;
  void* h_igates;  // K*32 amplitudes: G^-1 | -G^-1 V G^-1 per gate (device precision)
  double* h_tov;   // Ns*4
  double* h_env;   // K*64
  std::vector<double> last_T, last_Om;
  // two-phase evaluation: a forward sweep leaves its checkpoints for one backward sweep
  int fwd_ready = 0, fwd_tangent = 0;
  // backward from pass-output states (all gates well conditioned): FP64 G^-1 and V of that sweep
  int bwd_inverse = 0;
  std::vector<cd> bwd_Gi, bwd_V;
  qhvp_geometry fwd_geom = QHVP_EUCLIDEAN;
  std::vector<double> fwd_G, fwd_V;
  // The forward states psi at the pass boundaries that stay in the workspace between calls (every
  // boundary when there is one segment, else the segment checkpoints) belong to the gates kept_G
  // while kept_valid: a later gradient / HVP sweep at bitwise the same G stores only tangents there.
  int kept_valid = 0;
  std::vector<double> kept_G;
  hipEvent_t ev0, ev1;
  double last_ms;
  // optional per-launch timing: events bracket every launch of the call; stats accumulate per kind
  int profiling = 0;
  int sched_used = 0;   // tile-schedule counters handed out since the last reset
  std::vector<hipEvent_t> evpool;
  size_t ev_used = 0;
  struct Pending { int kind; size_t e0; double bytes, flops; };
  std::vector<Pending> pending;
  double k_ms[QHVP_KERNEL_KINDS] = {0}, k_bytes[QHVP_KERNEL_KINDS] = {0}, k_flops[QHVP_KERNEL_KINDS] = {0};
  long long k_count[QHVP_KERNEL_KINDS] = {0};

  char* phi0() { return ws + lay.off_phi0; }
  char* slot(int i) { return ws + lay.off_slots + (size_t)i * lay.slot_bytes; }
  char* small(size_t o) { return ws + lay.off_small + o; }
  // slot indices: [0, n_ckpt) checkpoints of segments 1..J-1; [n_ckpt, n_ckpt+n_seg) in-segment
  // boundaries 1..maxlen-1; last: working / backward (a, b)
  char* ckpt(int segment) { return slot(segment - 1); }
  char* segbuf(int i) { return slot(lay.n_ckpt + i - 1); }
  char* work() { return slot(lay.n_ckpt + lay.n_seg); }
  char* second(char* slotp) { return slotp + lay.state_bytes; }
  qhvp::Prec dprec() const { return prec == QHVP_C64_ACC64 ? qhvp::P_C64 : qhvp::P_C128; }
  size_t amp() const { return prec == QHVP_C64_ACC64 ? 8 : 16; }
};

namespace {

// Per-launch timing (only when profiling is on): an event before and after the launch.
hipError_t prof_begin(qhvp_problem* p) {
  if (!p->profiling) return hipSuccess;
  while (p->evpool.size() < p->ev_used + 2) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    p->evpool.push_back(e);
  }
  return hipEventRecord(p->evpool[p->ev_used], p->stream);
}
hipError_t prof_end(qhvp_problem* p, int kind, double bytes, double flops) {
  if (!p->profiling) return hipSuccess;
  hipError_t r = hipEventRecord(p->evpool[p->ev_used + 1], p->stream);
  p->pending.push_back({kind, p->ev_used, bytes, flops});
  p->ev_used += 2;
  return r;
}
hipError_t prof_collect(qhvp_problem* p) {
  for (auto& q : p->pending) {
    float ms = 0;
    hipError_t r = hipEventElapsedTime(&ms, p->evpool[q.e0], p->evpool[q.e0 + 1]);
    if (r != hipSuccess) return r;
    p->k_ms[q.kind] += ms;
    p->k_bytes[q.kind] += q.bytes;
    p->k_flops[q.kind] += q.flops;
    p->k_count[q.kind] += 1;
  }
  p->pending.clear();
  p->ev_used = 0;
  return hipSuccess;
}

// Algorithmic traffic and arithmetic of one pass (what the method must move / compute for
// it, not counting the in-tile recomputation): S bytes per state set read or written; per gate
// and amplitude 32 flop for psi <- G psi, 96 with the tangent; the backward adds the environment
// products (32 flop, 96 with the tangent).
// Tile-schedule counters: zeroed at the start of each sweep; every kernel launch takes a fresh one
// (all in stream order, so a re-zeroing when the slots run out follows the launches that used them).
hipError_t sched_reset(qhvp_problem* p) {
  p->sched_used = 0;
  return (hipError_t)qhvp::launch_zero_ints((int*)p->small(p->lay.o_sched), kSchedSlots, p->stream);
}
int* sched_slot(qhvp_problem* p) {
  if (p->sched_used == kSchedSlots && sched_reset(p) != hipSuccess) return nullptr;
  return (int*)p->small(p->lay.o_sched) + p->sched_used++;
}

double state_bytes_alg(const qhvp_problem* p) { return (double)p->Ns * std::ldexp(1.0, p->n) * (double)p->amp(); }
double pass_flops(const qhvp_problem* p, const qhvp::PassDesc& pd, int tangent, bool backward) {
  const double per = tangent ? 96.0 : 32.0;
  return (backward ? 2.0 : 1.0) * per * pd.ng * (double)p->Ns * std::ldexp(1.0, p->n);
}

void to_device_precision(const qhvp_problem* p, const double* src, size_t n_complex, void* dst) {
  if (p->prec == QHVP_C64_ACC64) {
    float* d = (float*)dst;
    for (size_t i = 0; i < 2 * n_complex; ++i) d[i] = (float)src[i];
  } else {
    std::memcpy(dst, src, 2 * n_complex * sizeof(double));
  }
}

// Forward sweep of `passes` (gates at device pointer `gates`).  mode: 0 = labels (write result to
// phi0), 1 = ansatz sweep storing checkpoints for a later backward sweep, 2 = ansatz cost only.
// keep_psi (mode 1): the kept boundaries already hold psi for these gates; store dpsi only there.
qhvp_status forward_sweep(qhvp_problem* p, const std::vector<qhvp::PassDesc>& passes, const void* gates,
                          const void* dirs, int tangent, int mode, bool keep_psi = false) {
  const int np = (int)passes.size();
  const char* samples = p->small(p->lay.o_samples);
  double* ovpart = (double*)p->small(p->lay.o_ovpart);
  const size_t sb = p->lay.state_bytes;
  (void)sb;
  // segment lookup for mode 1
  std::vector<int> seg_of(np, 0);
  for (size_t j = 0; j < p->seg.size(); ++j)
    for (int q = p->seg[j].first; q < p->seg[j].second; ++q) seg_of[q] = (int)j;
  const int J = (int)p->seg.size();
  HIP_TRY(sched_reset(p));
  for (int q = 0; q < np; ++q) {
    qhvp::FwdArgs a;
    std::memset(&a, 0, sizeof(a));
    a.pd = passes[q];
    a.sched = sched_slot(p);
    a.n_samples = p->Ns;
    a.tangent = tangent;
    a.gates = gates;
    a.dirs = dirs;
    a.samples = samples;
    char* src = nullptr;
    char* dst = nullptr;
    bool dst_kept = false;   // dst is a boundary that later calls find unchanged
    if (mode == 0) {
      src = q == 0 ? nullptr : p->phi0();
      dst = p->phi0();
    } else if (mode == 2) {
      src = q == 0 ? nullptr : p->work();
      dst = q == np - 1 ? nullptr : p->work();
    } else {
      const int j = seg_of[q];
      const int s0 = p->seg[j].first, s1 = p->seg[j].second;
      const bool last_seg = (j == J - 1);
      if (q == s0) src = (j == 0) ? nullptr : p->ckpt(j);
      else src = last_seg ? p->segbuf(q - s0) : p->work();
      if (q == np - 1) dst = nullptr;
      else if (q + 1 == s1) dst = p->ckpt(j + 1);
      else dst = last_seg ? p->segbuf(q + 1 - s0) : p->work();
      // checkpoints are only written here; with several segments the backward sweep recomputes
      // into the in-segment buffers, so those are kept only when there is a single segment
      dst_kept = dst != nullptr && (q + 1 == s1 || J == 1);
    }
    a.src_psi = src;
    a.src_dpsi = src ? p->second(src) : nullptr;
    if (mode != 0 && q == np - 1) {
      // the backward sweep from pass outputs starts from the final states (kept in the working slot)
      a.dst_psi = (mode == 1 && p->bwd_inverse) ? p->work() : nullptr;
      a.dst_dpsi = a.dst_psi ? p->second(p->work()) : nullptr;
      a.phi0 = p->phi0();
      a.ov_part = ovpart;
    } else {
      a.dst_psi = (keep_psi && dst_kept) ? nullptr : dst;
      a.dst_dpsi = p->second(dst);
    }
    {
      const double S = state_bytes_alg(p), nst = tangent ? 2 : 1;
      const double bytes = (a.src_psi ? nst * S : 0) + (a.ov_part ? S : 0) + (a.dst_psi ? S : 0) +
                           (tangent && a.dst_dpsi ? S : 0);
      HIP_TRY(prof_begin(p));
      LAUNCH_TRY(qhvp::launch_fwd(p->dprec(), a, p->stream));
      HIP_TRY(prof_end(p, QHVP_KERNEL_FORWARD, bytes, pass_flops(p, a.pd, tangent, false)));
    }
  }
  if (mode != 0) {
    const int tiles = 1 << (p->n - passes[np - 1].mb);
    LAUNCH_TRY(qhvp::launch_reduce_overlaps(ovpart, p->Ns, tiles, (double*)p->small(p->lay.o_tov), p->stream));
  }
  return QHVP_OK;
}

qhvp_status backward_sweep(qhvp_problem* p, int tangent) {
  const int np = (int)p->passes.size();
  const int J = (int)p->seg.size();
  const void* gates = p->small(p->lay.o_gates);
  const void* dirs = p->small(p->lay.o_dirs);
  const char* samples = p->small(p->lay.o_samples);
  double* envpart = (double*)p->small(p->lay.o_envpart);
  double* env = (double*)p->small(p->lay.o_env);
  char* ab = p->work();
  HIP_TRY(sched_reset(p));
  for (int j = J - 1; j >= 0; --j) {
    const int s0 = p->seg[j].first, s1 = p->seg[j].second;
    char* start = j == 0 ? nullptr : p->ckpt(j);
    if (j < J - 1) {
      // recompute the segment's inner boundaries from its checkpoint
      for (int q = s0; q + 1 < s1; ++q) {
        qhvp::FwdArgs a;
        std::memset(&a, 0, sizeof(a));
        a.pd = p->passes[q];
        a.sched = sched_slot(p);
        a.n_samples = p->Ns;
        a.tangent = tangent;
        a.gates = gates;
        a.dirs = dirs;
        a.samples = samples;
        char* src = q == s0 ? start : p->segbuf(q - s0);
        char* dst = p->segbuf(q + 1 - s0);
        a.src_psi = src;
        a.src_dpsi = src ? p->second(src) : nullptr;
        a.dst_psi = dst;
        a.dst_dpsi = p->second(dst);
        const double S = state_bytes_alg(p), nst = tangent ? 2 : 1;
        HIP_TRY(prof_begin(p));
        LAUNCH_TRY(qhvp::launch_fwd(p->dprec(), a, p->stream));
        HIP_TRY(prof_end(p, QHVP_KERNEL_RECOMPUTE, (src ? nst * S : 0) + nst * S, pass_flops(p, a.pd, tangent, false)));
      }
    }
    for (int q = s1 - 1; q >= s0; --q) {
      qhvp::BwdArgs b;
      std::memset(&b, 0, sizeof(b));
      b.pd = p->passes[q];
      b.n_samples = p->Ns;
      b.tangent = tangent;
      b.gates = gates;
      b.dirs = dirs;
      b.igates = p->small(p->lay.o_igates);
      // forward states: the pass input (recomputing kernel) or the pass output (inverse kernel)
      char* src = q == s0 ? start : p->segbuf(q - s0);
      if (p->bwd_inverse) src = q + 1 < s1 ? p->segbuf(q + 1 - s0) : (j == J - 1 ? ab : p->ckpt(j + 1));
      b.src_psi = src;
      b.src_dpsi = src ? p->second(src) : nullptr;
      b.samples = samples;
      b.ab_a = ab;
      b.ab_b = p->second(ab);
      b.phi0 = p->phi0();
      b.tov = (const double*)p->small(p->lay.o_tov);
      b.fold = (q == np - 1);
      b.store_ab = (q > 0);
      b.env_part = envpart;
      const double S = state_bytes_alg(p), nst = tangent ? 2 : 1;
      const double bytes = (b.fold ? S : nst * S) + (src ? nst * S : 0) + (b.store_ab ? nst * S : 0);
      HIP_TRY(prof_begin(p));
      if (p->bwd_inverse) LAUNCH_TRY(qhvp::launch_bwd_out(p->dprec(), b, p->stream));
      else LAUNCH_TRY(qhvp::launch_bwd(p->dprec(), b, p->stream));
      HIP_TRY(prof_end(p, QHVP_KERNEL_BACKWARD, bytes, pass_flops(p, b.pd, tangent, true)));
      const int nwg = qhvp::bwd_grid(p->dprec(), tangent, b.pd.ng, (long long)p->Ns << (p->n - b.pd.mb), p->bwd_inverse);
      HIP_TRY(prof_begin(p));
      LAUNCH_TRY(qhvp::launch_reduce_env(envpart, nwg, b.pd, env, p->stream));
      HIP_TRY(prof_end(p, QHVP_KERNEL_REDUCE, (double)nwg * b.pd.ng * qhvp::kEnvVals * 8, 0));
    }
  }
  return QHVP_OK;
}

qhvp_status check_gates(const qhvp_problem* p, const double* G, const char* what) {
  if (!G) return fail(QHVP_ERR_INVALID, std::string(what) + " is NULL");
  if (!finite_all(G, (size_t)p->K * 32)) return fail(QHVP_ERR_INVALID, std::string(what) + " has non-finite entries");
  return QHVP_OK;
}

qhvp_status finish_call(qhvp_problem* p, int copy_env, int tangent) {
  if (copy_env)
    HIP_TRY(hipMemcpyAsync(p->h_env, p->small(p->lay.o_env), (size_t)p->K * qhvp::kEnvVals * sizeof(double),
                           hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipEventRecord(p->ev1, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, p->ev0, p->ev1));
  p->last_ms += ms;
  HIP_TRY(prof_collect(p));
  (void)tangent;
  return QHVP_OK;
}

// The backward sweep may start each pass from its OUTPUT forward states and undo the gates on them
// (k_bwd_out) when every gate is well conditioned: then the inverse gates G^-1 and Y = -G^-1 V G^-1
// (FP64 here, device precision on the device) are staged.  Condition: |G|_F |G^-1|_F <= 8 (4 for a
// unitary gate), so that undoing the at most kMaxGates gates of a pass loses at most a few bits.
void prepare_inverse(qhvp_problem* p, const double* G, const double* V) {
  p->bwd_inverse = 0;
  const char* choice = std::getenv("QHVP_BACKWARD");
  if (choice && std::strcmp(choice, "recompute") == 0) return;
  p->bwd_Gi.assign((size_t)p->K * 16, cd(0));
  p->bwd_V.assign((size_t)p->K * 16, cd(0));
  std::vector<double> stage((size_t)p->K * 64);
  for (int k = 0; k < p->K; ++k) {
    M4 g, gi, v, t, y;
    load4(G + (size_t)k * 32, g);
    if (!inv4(g, gi) || fro4(g) * fro4(gi) > 8.0) return;
    if (V) load4(V + (size_t)k * 32, v);
    else for (int i = 0; i < 16; ++i) v[i] = 0;
    mul4(gi, v, t);
    mul4(t, gi, y);
    for (int i = 0; i < 16; ++i) {
      p->bwd_Gi[(size_t)k * 16 + i] = gi[i];
      p->bwd_V[(size_t)k * 16 + i] = v[i];
      stage[(size_t)k * 64 + 2 * i] = gi[i].real();
      stage[(size_t)k * 64 + 2 * i + 1] = gi[i].imag();
      stage[(size_t)k * 64 + 32 + 2 * i] = -y[i].real();
      stage[(size_t)k * 64 + 32 + 2 * i + 1] = -y[i].imag();
    }
  }
  to_device_precision(p, stage.data(), (size_t)p->K * 32, p->h_igates);
  p->bwd_inverse = 1;
}

// Output-side environment sums of the inverse backward sweep -> input-side ones, per gate (FP64):
// E = Et G^-T, D = (Dt - E V^T) G^-T, in place in h_env (E at [0, 32), D at [32, 64), entry 4x+y).
void map_output_envs(qhvp_problem* p, int tangent) {
  for (int k = 0; k < p->K; ++k) {
    double* e = p->h_env + (size_t)k * 64;
    const cd* gi = &p->bwd_Gi[(size_t)k * 16];
    const cd* v = &p->bwd_V[(size_t)k * 16];
    cd Et[16], Dt[16], E[16], W[16];
    for (int i = 0; i < 16; ++i) { Et[i] = cd(e[2 * i], e[2 * i + 1]); Dt[i] = cd(e[32 + 2 * i], e[32 + 2 * i + 1]); }
    for (int x = 0; x < 4; ++x)
      for (int y = 0; y < 4; ++y) {
        cd sE = 0;
        for (int z = 0; z < 4; ++z) sE += Et[4 * x + z] * gi[4 * y + z];
        E[4 * x + y] = sE;
      }
    for (int x = 0; x < 4; ++x)   // W = Dt - E V^T
      for (int z = 0; z < 4; ++z) {
        cd w = Dt[4 * x + z];
        if (tangent)
          for (int u = 0; u < 4; ++u) w -= E[4 * x + u] * v[4 * z + u];
        W[4 * x + z] = w;
      }
    for (int x = 0; x < 4; ++x)
      for (int y = 0; y < 4; ++y) {
        cd sD = 0;
        for (int z = 0; z < 4; ++z) sD += W[4 * x + z] * gi[4 * y + z];
        e[2 * (4 * x + y)] = E[4 * x + y].real();
        e[2 * (4 * x + y) + 1] = E[4 * x + y].imag();
        e[32 + 2 * (4 * x + y)] = sD.real();
        e[32 + 2 * (4 * x + y) + 1] = sD.imag();
      }
  }
}

// Forward phase.  mode 0: cost only (no checkpoints kept); 1: gradient sweep; 2: HVP sweep.  Uploads
// G (and V), sweeps, and brings the per-sample overlaps T_s (and Omega_s) back to the host.
qhvp_status phase_forward(qhvp_problem* p, const double* G, const double* V, int mode) {
  HIP_TRY(hipSetDevice(p->ctx->device));
  p->fwd_ready = 0;
  p->last_ms = 0;
  const size_t gn = (size_t)p->K * 32;
  const bool keep = mode != 0 && p->kept_valid && p->kept_G.size() == gn &&
                    std::memcmp(p->kept_G.data(), G, gn * sizeof(double)) == 0;
  if (mode != 0 && !keep) p->kept_valid = 0;   // this sweep overwrites the kept boundaries
  to_device_precision(p, G, (size_t)p->K * 16, p->h_gates);
  HIP_TRY(hipEventRecord(p->ev0, p->stream));
  HIP_TRY(hipMemcpyAsync(p->small(p->lay.o_gates), p->h_gates, (size_t)p->K * 16 * p->amp(), hipMemcpyHostToDevice, p->stream));
  if (mode == 2) {
    to_device_precision(p, V, (size_t)p->K * 16, p->h_dirs);
    HIP_TRY(hipMemcpyAsync(p->small(p->lay.o_dirs), p->h_dirs, (size_t)p->K * 16 * p->amp(), hipMemcpyHostToDevice, p->stream));
  }
  const int tangent = mode == 2 ? 1 : 0;
  if (mode != 0) {
    prepare_inverse(p, G, tangent ? V : nullptr);
    if (p->bwd_inverse)
      HIP_TRY(hipMemcpyAsync(p->small(p->lay.o_igates), p->h_igates, (size_t)p->K * 32 * p->amp(), hipMemcpyHostToDevice,
                             p->stream));
  }
  qhvp_status st = mode == 0 ? forward_sweep(p, p->passes, p->small(p->lay.o_gates), nullptr, 0, 2)
                             : forward_sweep(p, p->passes, p->small(p->lay.o_gates), p->small(p->lay.o_dirs), tangent, 1,
                                             keep);
  if (st) return st;
  HIP_TRY(hipMemcpyAsync(p->h_tov, p->small(p->lay.o_tov), (size_t)p->Ns * 4 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  st = finish_call(p, 0, tangent);
  if (st) return st;
  p->last_T.assign(2 * p->Ns, 0.0);
  p->last_Om.assign(2 * p->Ns, 0.0);
  for (int s = 0; s < p->Ns; ++s) {
    p->last_T[2 * s] = p->h_tov[4 * s];
    p->last_T[2 * s + 1] = p->h_tov[4 * s + 1];
    if (tangent) {
      p->last_Om[2 * s] = p->h_tov[4 * s + 2];
      p->last_Om[2 * s + 1] = p->h_tov[4 * s + 3];
    }
  }
  if (mode != 0) {
    p->fwd_ready = 1;
    p->fwd_tangent = tangent;
    if (!keep) p->kept_G.assign(G, G + gn);
    p->kept_valid = 1;
  }
  return QHVP_OK;
}

// Backward phase of the last gradient / HVP forward phase (its checkpoints are consumed).
qhvp_status phase_backward(qhvp_problem* p) {
  HIP_TRY(hipSetDevice(p->ctx->device));
  if (!p->fwd_ready) return fail(QHVP_ERR_INVALID, "no forward sweep to differentiate (call qhvp_forward first)");
  p->fwd_ready = 0;
  HIP_TRY(hipEventRecord(p->ev0, p->stream));
  qhvp_status st = backward_sweep(p, p->fwd_tangent);
  if (st) return st;
  st = finish_call(p, 1, p->fwd_tangent);
  if (st) return st;
  if (p->bwd_inverse) map_output_envs(p, p->fwd_tangent);
  return QHVP_OK;
}

// Alg. 2 post-processing over samples: F = mean |T_s|^2; with the folded environments
// Ehat_k = sum_s conj(T_s) dT_s/dG_k and Dhat_k = sum_s conj(Omega_s) dT_s/dG_k + conj(T_s) D(dT_s/dG_k)[V],
// grad C = -(2/N_s) conj(Ehat) and H(C)[V] = -(2/N_s) conj(Dhat) (cost 1 - F differentiated).
double fidelity_of(const qhvp_problem* p) {
  double F = 0;
  for (int s = 0; s < p->Ns; ++s) F += p->h_tov[4 * s] * p->h_tov[4 * s] + p->h_tov[4 * s + 1] * p->h_tov[4 * s + 1];
  return F / p->Ns;
}

void env_to_output(const qhvp_problem* p, int which, double* out) {
  const double f = -2.0 / p->Ns;
  for (int k = 0; k < p->K; ++k)
    for (int e = 0; e < 16; ++e) {
      const double re = p->h_env[(size_t)k * 64 + which * 32 + 2 * e];
      const double im = p->h_env[(size_t)k * 64 + which * 32 + 2 * e + 1];
      out[(size_t)k * 32 + 2 * e] = f * re;
      out[(size_t)k * 32 + 2 * e + 1] = -f * im;
    }
}

}  // namespace

// --------------------------------------------------------------------------------------------
extern "C" {

int qhvp_version(void) { return 100; }

const char* qhvp_last_error(void) { return g_err.c_str(); }

int qhvp_num_gates(int n, int L) { return num_gates(n, L); }

int qhvp_plan(int n, int L, int max_passes, int* gates_per_pass, int* gate_order) {
  if (n < 2 || n > qhvp::kMaxQubits || L < 1) {
    fail(QHVP_ERR_INVALID, "n must be in [2, 30] and L >= 1");
    return -QHVP_ERR_INVALID;
  }
  const auto passes = plan_circuit(n, L, nullptr);
  const int np = (int)passes.size();
  if (gates_per_pass && max_passes < np) {
    fail(QHVP_ERR_INVALID, "gates_per_pass holds " + std::to_string(max_passes) + " entries, the plan has " +
                               std::to_string(np) + " passes");
    return -QHVP_ERR_INVALID;
  }
  int k = 0;
  for (int q = 0; q < np; ++q) {
    if (gates_per_pass) gates_per_pass[q] = passes[q].ng;
    for (int j = 0; j < passes[q].ng; ++j, ++k)
      if (gate_order) gate_order[k] = passes[q].gidx[j];
  }
  return np;
}

qhvp_status qhvp_ctx_create(int device, qhvp_ctx** out) {
  if (!out) return fail(QHVP_ERR_INVALID, "out is NULL");
  int cnt = 0;
  HIP_TRY(hipGetDeviceCount(&cnt));
  if (device < 0 || device >= cnt) return fail(QHVP_ERR_INVALID, "no such HIP device");
  HIP_TRY(hipSetDevice(device));
  *out = new qhvp_ctx{device};
  return QHVP_OK;
}

void qhvp_ctx_destroy(qhvp_ctx* ctx) { delete ctx; }

size_t qhvp_workspace_bytes(int n, int L, int L_ref, int n_samples, qhvp_precision prec, int ckpt_every,
                            int with_tangent) {
  if (prec != QHVP_C128 && prec != QHVP_C64_ACC64) return 0;
  Layout lay;
  if (!make_layout(n, L, L_ref, n_samples, prec, ckpt_every, with_tangent ? 1 : 0, lay)) return 0;
  return lay.total;
}

qhvp_status qhvp_problem_create(qhvp_ctx* ctx, int n, int L, int L_ref, const double* uref_gates,
                                const double* samples, int n_samples, qhvp_precision prec, int ckpt_every,
                                int with_tangent, void* d_workspace, size_t ws_bytes, void* hip_stream,
                                qhvp_problem** out) {
  if (!ctx || !out) return fail(QHVP_ERR_INVALID, "ctx or out is NULL");
  if (n < 2 || n > qhvp::kMaxQubits) return fail(QHVP_ERR_INVALID, "n must be in [2, 30]");
  if (L < 1 || L_ref < 1) return fail(QHVP_ERR_INVALID, "L and L_ref must be >= 1");
  if (n_samples < 1) return fail(QHVP_ERR_INVALID, "n_samples must be >= 1");
  if (prec != QHVP_C128 && prec != QHVP_C64_ACC64) return fail(QHVP_ERR_INVALID, "unknown precision");
  if (!uref_gates || !samples) return fail(QHVP_ERR_INVALID, "uref_gates or samples is NULL");
  const int Kr = num_gates(n, L_ref);
  if (!finite_all(uref_gates, (size_t)Kr * 32)) return fail(QHVP_ERR_INVALID, "uref_gates has non-finite entries");
  if (!finite_all(samples, (size_t)n_samples * n * 4)) return fail(QHVP_ERR_INVALID, "samples has non-finite entries");
  Layout lay;
  if (!make_layout(n, L, L_ref, n_samples, prec, ckpt_every, with_tangent ? 1 : 0, lay))
    return fail(QHVP_ERR_INVALID, "invalid problem shape");
  if (d_workspace && ws_bytes < lay.total)
    return fail(QHVP_ERR_NOMEM, "workspace has " + std::to_string(ws_bytes) + " bytes, needs " + std::to_string(lay.total));
  if (d_workspace && ((uintptr_t)d_workspace % kAlign) != 0) return fail(QHVP_ERR_INVALID, "workspace must be 256-byte aligned");
  HIP_TRY(hipSetDevice(ctx->device));

  qhvp_problem* p = new qhvp_problem();
  p->ctx = ctx;
  p->n = n; p->L = L; p->L_ref = L_ref; p->Ns = n_samples;
  p->K = num_gates(n, L); p->Kr = Kr;
  p->prec = prec; p->ckpt_every = ckpt_every; p->tangent = with_tangent ? 1 : 0;
  p->stream = (hipStream_t)hip_stream;
  p->passes = plan_circuit(n, L, nullptr);
  p->ref_passes = plan_circuit(n, L_ref, nullptr);
  fill_tile_offsets(p->passes, (int)p->amp());
  fill_tile_offsets(p->ref_passes, (int)p->amp());
  p->seg = plan_segments(n, L, ckpt_every);
  p->lay = lay;
  p->last_ms = 0;
  p->h_gates = p->h_dirs = p->h_igates = nullptr;
  p->h_tov = p->h_env = nullptr;
  p->ev0 = p->ev1 = nullptr;
  auto cleanup_fail = [&](qhvp_status st, const std::string& msg) {
    qhvp_problem_destroy(p);
    return fail(st, msg);
  };
  if (d_workspace) {
    p->ws = (char*)d_workspace;
    p->owns_ws = false;
  } else {
    p->ws = nullptr;
    p->owns_ws = true;
    hipError_t e = hipMalloc((void**)&p->ws, lay.total);
    if (e != hipSuccess) { p->ws = nullptr; return cleanup_fail(QHVP_ERR_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)); }
  }
  const size_t amp = p->amp();
  const size_t stage = std::max((size_t)std::max(p->K, Kr) * 16, (size_t)n_samples * n * 2) * amp;
  if (hipHostMalloc(&p->h_gates, stage) != hipSuccess || hipHostMalloc(&p->h_dirs, stage) != hipSuccess ||
      hipHostMalloc(&p->h_igates, (size_t)p->K * 32 * amp) != hipSuccess ||
      hipHostMalloc((void**)&p->h_tov, (size_t)n_samples * 4 * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&p->h_env, (size_t)p->K * qhvp::kEnvVals * sizeof(double)) != hipSuccess)
    return cleanup_fail(QHVP_ERR_NOMEM, "pinned host allocation failed");
  if (hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess)
    return cleanup_fail(QHVP_ERR_DEVICE, "hipEventCreate failed");

  // samples and U_ref gates to the device, then labels phi0 = U_ref psi (a forward sweep of U_ref)
  to_device_precision(p, samples, (size_t)n_samples * n * 2, p->h_gates);
  if (hipMemcpyAsync(p->small(lay.o_samples), p->h_gates, (size_t)n_samples * n * 2 * amp, hipMemcpyHostToDevice, p->stream) != hipSuccess ||
      hipStreamSynchronize(p->stream) != hipSuccess)
    return cleanup_fail(QHVP_ERR_DEVICE, "copy of samples failed");
  to_device_precision(p, uref_gates, (size_t)Kr * 16, p->h_gates);
  if (hipMemcpyAsync(p->small(lay.o_uref), p->h_gates, (size_t)Kr * 16 * amp, hipMemcpyHostToDevice, p->stream) != hipSuccess)
    return cleanup_fail(QHVP_ERR_DEVICE, "copy of U_ref failed");
  qhvp_status st = forward_sweep(p, p->ref_passes, p->small(lay.o_uref), nullptr, 0, 0);
  if (st != QHVP_OK) { std::string m = g_err; qhvp_problem_destroy(p); return fail(st, m); }
  if (hipStreamSynchronize(p->stream) != hipSuccess) return cleanup_fail(QHVP_ERR_DEVICE, "label sweep failed");
  *out = p;
  return QHVP_OK;
}

void qhvp_problem_destroy(qhvp_problem* p) {
  if (!p) return;
  if (p->stream) hipStreamSynchronize(p->stream);
  else hipDeviceSynchronize();
  if (p->owns_ws && p->ws) hipFree(p->ws);
  if (p->h_gates) hipHostFree(p->h_gates);
  if (p->h_dirs) hipHostFree(p->h_dirs);
  if (p->h_igates) hipHostFree(p->h_igates);
  if (p->h_tov) hipHostFree(p->h_tov);
  if (p->h_env) hipHostFree(p->h_env);
  if (p->ev0) hipEventDestroy(p->ev0);
  if (p->ev1) hipEventDestroy(p->ev1);
  for (auto e : p->evpool) hipEventDestroy(e);
  delete p;
}

qhvp_status qhvp_cost(qhvp_problem* p, const double* G, double* cost, double* fidelity) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  qhvp_status st = check_gates(p, G, "G");
  if (st) return st;
  st = phase_forward(p, G, nullptr, 0);
  if (st) return st;
  const double F = fidelity_of(p);
  if (cost) *cost = 1.0 - F;
  if (fidelity) *fidelity = F;
  return QHVP_OK;
}

qhvp_status qhvp_forward(qhvp_problem* p, const double* G, const double* V, qhvp_geometry geom, double* cost,
                         double* fidelity) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (geom != QHVP_EUCLIDEAN && geom != QHVP_RIEMANNIAN) return fail(QHVP_ERR_INVALID, "unknown geometry");
  qhvp_status st = check_gates(p, G, "G");
  if (st) return st;
  if (V) {
    if (!p->tangent) return fail(QHVP_ERR_UNSUPPORTED, "problem was created without tangent storage");
    st = check_gates(p, V, "V");
    if (st) return st;
  }
  if (geom == QHVP_RIEMANNIAN && qhvp_unitarity_error(p->K, G) > 1e-10)
    return fail(QHVP_ERR_INVALID, "Riemannian geometry needs unitary gates");
  p->fwd_G.assign(G, G + (size_t)p->K * 32);
  p->fwd_V.clear();
  if (V) {
    p->fwd_V.assign(V, V + (size_t)p->K * 32);
    // the Riemannian HVP formula assumes a tangent direction: project V first
    if (geom == QHVP_RIEMANNIAN) qhvp_project(p->K, G, V, p->fwd_V.data());
  }
  p->fwd_geom = geom;
  st = phase_forward(p, G, V ? p->fwd_V.data() : nullptr, V ? 2 : 1);
  if (st) return st;
  const double F = fidelity_of(p);
  if (cost) *cost = 1.0 - F;
  if (fidelity) *fidelity = F;
  return QHVP_OK;
}

qhvp_status qhvp_backward(qhvp_problem* p, double* grad, double* hvp) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (!p->fwd_ready) return fail(QHVP_ERR_INVALID, "no forward sweep to differentiate (call qhvp_forward first)");
  if (hvp && !p->fwd_tangent) return fail(QHVP_ERR_INVALID, "the last forward sweep had no direction V");
  const int tangent = p->fwd_tangent;
  qhvp_status st = phase_backward(p);
  if (st) return st;
  std::vector<double> g((size_t)p->K * 32), h;
  env_to_output(p, 0, g.data());
  if (tangent) {
    h.resize((size_t)p->K * 32);
    env_to_output(p, 1, h.data());
  }
  if (p->fwd_geom == QHVP_RIEMANNIAN) {
    if (grad) qhvp_project(p->K, p->fwd_G.data(), g.data(), grad);
    if (hvp) return qhvp_riemannian_hvp(p->K, p->fwd_G.data(), g.data(), h.data(), p->fwd_V.data(), hvp);
    return QHVP_OK;
  }
  if (grad) std::memcpy(grad, g.data(), g.size() * sizeof(double));
  if (hvp) std::memcpy(hvp, h.data(), h.size() * sizeof(double));
  return QHVP_OK;
}

qhvp_status qhvp_hvp_batch(qhvp_problem* p, const double* G, int n_dirs, const double* V, qhvp_geometry geom,
                           double* cost, double* grad, double* hvp) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (n_dirs < 1) return fail(QHVP_ERR_INVALID, "n_dirs must be positive");
  if (!V || !hvp) return fail(QHVP_ERR_INVALID, "V and hvp must not be NULL");
  if (!p->tangent) return fail(QHVP_ERR_UNSUPPORTED, "problem was created without tangent storage");
  if (geom != QHVP_EUCLIDEAN && geom != QHVP_RIEMANNIAN) return fail(QHVP_ERR_INVALID, "unknown geometry");
  qhvp_status st = check_gates(p, G, "G");
  if (st) return st;
  const size_t gn = (size_t)p->K * 32;
  if (!finite_all(V, gn * (size_t)n_dirs)) return fail(QHVP_ERR_INVALID, "V has non-finite entries");
  if (geom == QHVP_RIEMANNIAN && qhvp_unitarity_error(p->K, G) > 1e-10)
    return fail(QHVP_ERR_INVALID, "Riemannian geometry needs unitary gates");
  // the first direction stores psi at the kept boundaries (unless they already belong to G); the
  // others read it there
  std::vector<double> out(gn * (size_t)n_dirs), g(gn);
  double c = 0;
  for (int m = 0; m < n_dirs; ++m) {
    st = qhvp_forward(p, G, V + gn * m, geom, &c, nullptr);
    if (st) return st;
    st = qhvp_backward(p, m == 0 ? g.data() : nullptr, out.data() + gn * m);
    if (st) return st;
  }
  std::memcpy(hvp, out.data(), out.size() * sizeof(double));
  if (grad) std::memcpy(grad, g.data(), gn * sizeof(double));
  if (cost) *cost = c;
  return QHVP_OK;
}

int qhvp_states_kept_for(const qhvp_problem* p, const double* G) {
  if (!p || !G) return -1;
  const size_t gn = (size_t)p->K * 32;
  return p->kept_valid && p->kept_G.size() == gn && std::memcmp(p->kept_G.data(), G, gn * sizeof(double)) == 0;
}

qhvp_status qhvp_grad(qhvp_problem* p, const double* G, qhvp_geometry geom, double* cost, double* grad) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (!grad) return fail(QHVP_ERR_INVALID, "grad is NULL");
  qhvp_status st = qhvp_forward(p, G, nullptr, geom, cost, nullptr);
  if (st) return st;
  return qhvp_backward(p, grad, nullptr);
}

qhvp_status qhvp_hvp(qhvp_problem* p, const double* G, const double* V, qhvp_geometry geom, double* cost,
                     double* grad, double* hvp) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (!hvp) return fail(QHVP_ERR_INVALID, "hvp is NULL");
  if (!V) return fail(QHVP_ERR_INVALID, "V is NULL");
  qhvp_status st = qhvp_forward(p, G, V, geom, cost, nullptr);
  if (st) return st;
  return qhvp_backward(p, grad, hvp);
}

// ---- translationally invariant circuits (App. E): one gate G_(l) per layer ----------------------

namespace {
// gate k of the brickwall belongs to layer layer_of[k]
std::vector<int> gate_layers(int n, int L) {
  std::vector<int> out;
  for (int l = 0; l < L; ++l)
    for (int q = l % 2; q + 1 < n; q += 2) out.push_back(l);
  return out;
}
void ti_expand(const qhvp_problem* p, const double* layers, std::vector<double>& gates) {
  const auto lay = gate_layers(p->n, p->L);
  gates.resize((size_t)p->K * 32);
  for (int k = 0; k < p->K; ++k) std::memcpy(&gates[(size_t)k * 32], layers + (size_t)lay[k] * 32, 32 * sizeof(double));
}
void ti_reduce(const qhvp_problem* p, const double* per_gate, double* layers) {
  const auto lay = gate_layers(p->n, p->L);
  std::memset(layers, 0, (size_t)p->L * 32 * sizeof(double));
  for (int k = 0; k < p->K; ++k)
    for (int e = 0; e < 32; ++e) layers[(size_t)lay[k] * 32 + e] += per_gate[(size_t)k * 32 + e];
}
}  // namespace

qhvp_status qhvp_grad_ti(qhvp_problem* p, const double* G_layers, qhvp_geometry geom, double* cost,
                         double* grad_layers) {
  if (!p || !G_layers || !grad_layers) return fail(QHVP_ERR_INVALID, "bad arguments");
  if (geom != QHVP_EUCLIDEAN && geom != QHVP_RIEMANNIAN) return fail(QHVP_ERR_INVALID, "unknown geometry");
  if (!finite_all(G_layers, (size_t)p->L * 32)) return fail(QHVP_ERR_INVALID, "G_layers has non-finite entries");
  if (geom == QHVP_RIEMANNIAN && qhvp_unitarity_error(p->L, G_layers) > 1e-10)
    return fail(QHVP_ERR_INVALID, "Riemannian geometry needs unitary gates");
  std::vector<double> G, g((size_t)p->K * 32), gl((size_t)p->L * 32);
  ti_expand(p, G_layers, G);
  qhvp_status st = qhvp_grad(p, G.data(), QHVP_EUCLIDEAN, cost, g.data());
  if (st) return st;
  ti_reduce(p, g.data(), gl.data());
  if (geom == QHVP_RIEMANNIAN) return qhvp_project(p->L, G_layers, gl.data(), grad_layers);
  std::memcpy(grad_layers, gl.data(), gl.size() * sizeof(double));
  return QHVP_OK;
}

qhvp_status qhvp_hvp_ti(qhvp_problem* p, const double* G_layers, const double* V_layers, qhvp_geometry geom,
                        double* cost, double* grad_layers, double* hvp_layers) {
  if (!p || !G_layers || !V_layers || !hvp_layers) return fail(QHVP_ERR_INVALID, "bad arguments");
  if (geom != QHVP_EUCLIDEAN && geom != QHVP_RIEMANNIAN) return fail(QHVP_ERR_INVALID, "unknown geometry");
  if (!finite_all(G_layers, (size_t)p->L * 32) || !finite_all(V_layers, (size_t)p->L * 32))
    return fail(QHVP_ERR_INVALID, "non-finite layer gates or directions");
  std::vector<double> Vl(V_layers, V_layers + (size_t)p->L * 32);
  if (geom == QHVP_RIEMANNIAN) {
    if (qhvp_unitarity_error(p->L, G_layers) > 1e-10) return fail(QHVP_ERR_INVALID, "Riemannian geometry needs unitary gates");
    qhvp_project(p->L, G_layers, V_layers, Vl.data());   // tangent direction first (App. F)
  }
  std::vector<double> G, V, g((size_t)p->K * 32), h((size_t)p->K * 32), gl((size_t)p->L * 32), hl((size_t)p->L * 32);
  ti_expand(p, G_layers, G);
  ti_expand(p, Vl.data(), V);
  qhvp_status st = qhvp_hvp(p, G.data(), V.data(), QHVP_EUCLIDEAN, cost, g.data(), h.data());
  if (st) return st;
  ti_reduce(p, g.data(), gl.data());
  ti_reduce(p, h.data(), hl.data());
  if (geom == QHVP_RIEMANNIAN) {
    if (grad_layers) qhvp_project(p->L, G_layers, gl.data(), grad_layers);
    return qhvp_riemannian_hvp(p->L, G_layers, gl.data(), hl.data(), Vl.data(), hvp_layers);
  }
  if (grad_layers) std::memcpy(grad_layers, gl.data(), gl.size() * sizeof(double));
  std::memcpy(hvp_layers, hl.data(), hl.size() * sizeof(double));
  return QHVP_OK;
}

qhvp_status qhvp_overlaps(const qhvp_problem* p, double* T, double* Omega) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (p->last_T.empty()) return fail(QHVP_ERR_INVALID, "no evaluation yet");
  if (T) std::memcpy(T, p->last_T.data(), p->last_T.size() * sizeof(double));
  if (Omega) std::memcpy(Omega, p->last_Om.data(), p->last_Om.size() * sizeof(double));
  return QHVP_OK;
}

qhvp_status qhvp_problem_info(const qhvp_problem* p, int* K, int* n_passes, size_t* ws_bytes, int* segments) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (K) *K = p->K;
  if (n_passes) *n_passes = (int)p->passes.size();
  if (ws_bytes) *ws_bytes = p->lay.total;
  if (segments) *segments = (int)p->seg.size();
  return QHVP_OK;
}

int qhvp_backward_from_outputs(const qhvp_problem* p) { return p ? p->bwd_inverse : -1; }

double qhvp_last_device_ms(const qhvp_problem* p) { return p ? p->last_ms : 0.0; }

qhvp_status qhvp_set_profiling(qhvp_problem* p, int on) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  p->profiling = on ? 1 : 0;
  for (int k = 0; k < QHVP_KERNEL_KINDS; ++k) { p->k_ms[k] = p->k_bytes[k] = p->k_flops[k] = 0; p->k_count[k] = 0; }
  return QHVP_OK;
}

qhvp_status qhvp_kernel_stats(const qhvp_problem* p, int kind, double* total_ms, long long* launches,
                              double* alg_bytes, double* alg_flops) {
  if (!p || kind < 0 || kind >= QHVP_KERNEL_KINDS) return fail(QHVP_ERR_INVALID, "bad arguments");
  if (total_ms) *total_ms = p->k_ms[kind];
  if (launches) *launches = p->k_count[kind];
  if (alg_bytes) *alg_bytes = p->k_bytes[kind];
  if (alg_flops) *alg_flops = p->k_flops[kind];
  return QHVP_OK;
}

qhvp_status qhvp_project(int K, const double* G, const double* X, double* out) {
  if (K < 1 || !G || !X || !out) return fail(QHVP_ERR_INVALID, "bad arguments");
  for (int k = 0; k < K; ++k) {
    M4 g, x, o;
    load4(G + 32 * (size_t)k, g);
    load4(X + 32 * (size_t)k, x);
    project4(g, x, o);
    store4(o, out + 32 * (size_t)k);
  }
  return QHVP_OK;
}

qhvp_status qhvp_riemannian_hvp(int K, const double* G, const double* grad, const double* hvp, const double* V,
                                double* out) {
  if (K < 1 || !G || !grad || !hvp || !V || !out) return fail(QHVP_ERR_INVALID, "bad arguments");
  for (int k = 0; k < K; ++k) {
    M4 g, gr, h, v, o;
    load4(G + 32 * (size_t)k, g);
    load4(grad + 32 * (size_t)k, gr);
    load4(hvp + 32 * (size_t)k, h);
    load4(V + 32 * (size_t)k, v);
    riem_hvp4(g, gr, h, v, o);
    store4(o, out + 32 * (size_t)k);
  }
  return QHVP_OK;
}

qhvp_status qhvp_retract(int K, const double* G, const double* xi, double* out) {
  if (K < 1 || !G || !xi || !out) return fail(QHVP_ERR_INVALID, "bad arguments");
  for (int k = 0; k < K; ++k) {
    M4 g, x, a, u;
    load4(G + 32 * (size_t)k, g);
    load4(xi + 32 * (size_t)k, x);
    for (int i = 0; i < 16; ++i) a[i] = g[i] + x[i];
    if (!polar4(a, u)) return fail(QHVP_ERR_INVALID, "G + xi is singular");
    store4(u, out + 32 * (size_t)k);
  }
  return QHVP_OK;
}

double qhvp_unitarity_error(int K, const double* G) {
  if (K < 1 || !G) return INFINITY;
  double e = 0;
  for (int k = 0; k < K; ++k) {
    M4 g;
    load4(G + 32 * (size_t)k, g);
    e = std::max(e, unitarity_err4(g));
  }
  return e;
}

}  // extern "C"
