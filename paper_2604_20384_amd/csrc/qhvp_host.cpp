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
#include <mutex>
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

// LDS index of tile element t in the kernels' layout: per-bit offsets kLdsPadC64 (complex64) or
// kLdsPadC128 (complex128).
int lds_at(int t, int elem_bytes) {
  const int* pad = elem_bytes == 8 ? qhvp::kLdsPadC64 : qhvp::kLdsPadC128;
  int r = t;
  for (int b = 0; b < qhvp::kMaxTileBits; ++b) r += ((t >> b) & 1) * pad[b];
  return r;
}

// gfx950 LDS bank model, fitted to the hardware's bank-conflict counter on probe access patterns:
// a wave's access of `width` bytes per lane is served a group of lanes at a time (32-bit: 32 lanes
// over 32 banks of 4 bytes; 64-bit reads: 32 lanes over 64 banks; 64-bit writes: 16 lanes over 32
// banks; 128-bit reads: 16 lanes over 64 banks; 128-bit writes: 8 lanes over 32 banks), and a group
// takes as many cycles as its most used bank holds distinct dwords.  Returns the wave's cycles.
// 128-bit reads follow it only roughly (on the complex128 kernels' group patterns it is exact for
// half of them and low by two cycles on average); a ds_read2st64_b64 is two 64-bit accesses, each
// served 16 lanes at a time over 32 banks.
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
// bits lo, hi whose group bits 0..5 sit on tile bits p[0..6).  The environment operand reads (32-bit,
// 32 wave accesses per step) run the lanes over the amplitude bits lo, hi, the state arrays, the
// real / imaginary part and group bits 0, 1; the W-tile reads and writes (64-bit, 16 each) run lane l
// over group bits 0..5 (lane l owns group l of the wave; the amplitude and the state array are
// wave-uniform).  Wave-uniform parts of the addresses shift every lane alike and drop out.
int c64_env_conflicts(int lo, int hi, int p0, int p1) {
  auto O = [](int b) { return lds_at(1 << b, 8); };
  auto sel = [](int v, int bit, int off) { return ((v >> bit) & 1) ? off : 0; };
  int env[64];
  for (int l = 0; l < 64; ++l) {
    const int comp = l & 15, sub = l >> 4;
    const int cst = comp >> 3, cri = (comp >> 2) & 1, cidx = comp & 3;
    const int tl = sel(sub, 0, O(p0)) + sel(sub, 1, O(p1)) + sel(cidx, 0, O(lo)) + sel(cidx, 1, O(hi));
    env[l] = 4 * (2 * cst * qhvp::kTspC64 + cri + 2 * tl);
  }
  return 32 * (lds_cycles(env, 4, false) - 2);
}
// W-tile reads are served 32 lanes (group bits 0..4) at a time and writes 16 lanes (bits 0..3), and
// the other lanes' addresses are the first group's shifted by a common offset, so their conflicts
// depend only on which tile bits sit on group bits 0..4 (resp. 0..3); `bits` lists those.
int c64_w_conflicts(const int* bits, int nbits, bool write) {
  int w[64];
  for (int l = 0; l < 64; ++l) {
    int t = 0;
    for (int i = 0; i < nbits; ++i)
      if ((l >> i) & 1) t += lds_at(1 << bits[i], 8);
    w[l] = 8 * t;
  }
  return 16 * (lds_cycles(w, 8, write) - (write ? 4 : 2));
}

// Modelled bank-conflict cycles of a complex128 group read (`write` false: 128-bit, 16 lanes at a
// time) or write (128-bit, 8 lanes at a time) whose lanes run over group bits 0..nbits-1 on tile bits
// `bits`.  Lane l owns group l of the wave; the other lanes' addresses are a common shift of these.
// (The environment operand reads of a backward step do not depend on this choice: their lanes run
// over the amplitude bits of the gate, the state array and the real / imaginary part.)
int c128_group_conflicts(const int* bits, int nbits, bool write) {
  int g[64];
  for (int l = 0; l < 64; ++l) {
    int t = 0;
    for (int i = 0; i < nbits; ++i)
      if ((l >> i) & 1) t += lds_at(1 << bits[i], 16);
    g[l] = 16 * t;
  }
  return lds_cycles(g, 16, write) - (write ? 8 : 4);
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
          // complex64: choose the order of the six lane bits with the fewest modelled bank-conflict
          // cycles per gate step: bits 0, 1 are the sub-rows of the environment operands; the W-tile
          // reads are served 32 lanes (bits 0..4) and its writes 16 lanes (bits 0..3) at a time, so
          // only the sets {0..4} and {0..3} matter there
          int wr[6], ww[6][6];
          for (int e = 0; e < 6; ++e) {   // read cost with avail[e] on group bit 5
            int bits[5], r = 0;
            for (int i = 0; i < 6; ++i)
              if (i != e) bits[r++] = avail[i];
            wr[e] = c64_w_conflicts(bits, 5, false);
          }
          for (int e = 0; e < 6; ++e)   // write cost with avail[e], avail[f] on group bits 4, 5
            for (int f = e + 1; f < 6; ++f) {
              int bits[4], r = 0;
              for (int i = 0; i < 6; ++i)
                if (i != e && i != f) bits[r++] = avail[i];
              ww[e][f] = ww[f][e] = c64_w_conflicts(bits, 4, true);
            }
          int best = -1;
          for (int a0 = 0; a0 < 6; ++a0)
            for (int a1 = 0; a1 < 6; ++a1) {
              if (a1 == a0) continue;
              const int ce = c64_env_conflicts(lo, hi, avail[a0], avail[a1]);
              for (int e4 = 0; e4 < 6; ++e4)
                for (int e5 = 0; e5 < 6; ++e5) {
                  if (e4 == e5 || e4 == a0 || e4 == a1 || e5 == a0 || e5 == a1) continue;
                  const int c = ce + wr[e5] + ww[e4][e5];
                  if (best < 0 || c < best) {
                    best = c;
                    pos[0] = avail[a0];
                    pos[1] = avail[a1];
                    int r = 2;
                    for (int i = 0; i < 6; ++i)
                      if (i != a0 && i != a1 && i != e4 && i != e5) pos[r++] = avail[i];
                    pos[4] = avail[e4];
                    pos[5] = avail[e5];
                  }
                }
            }
        }
        if (elem_bytes == 16) {
          // complex128: group bits 0..2 serve the writes (8 lanes) and 0..3 the reads (16 lanes);
          // a backward step issues 16 of each and a forward step 8, so both weigh the same
          int wr[64], rd[64];
          for (int m = 0; m < 64; ++m) {
            const int cnt = __builtin_popcount(m);
            if (cnt != 3 && cnt != 4) continue;
            int bits[4], r = 0;
            for (int i = 0; i < 6; ++i)
              if ((m >> i) & 1) bits[r++] = avail[i];
            if (cnt == 3) wr[m] = c128_group_conflicts(bits, 3, true);
            else rd[m] = c128_group_conflicts(bits, 4, false);
          }
          int best = -1;
          for (int m3 = 0; m3 < 64; ++m3) {
            if (__builtin_popcount(m3) != 3) continue;
            for (int a3 = 0; a3 < 6; ++a3) {
              if ((m3 >> a3) & 1) continue;
              const int m4 = m3 | (1 << a3);
              const int c = wr[m3] + rd[m4];
              if (best < 0 || c < best) {
                best = c;
                int r = 0;
                for (int i = 0; i < 6; ++i)
                  if ((m3 >> i) & 1) pos[r++] = avail[i];
                pos[r++] = avail[a3];
                for (int i = 0; i < 6; ++i)
                  if (!((m4 >> i) & 1)) pos[r++] = avail[i];
              }
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
  int rebuild = 0;          // QHVP_CKPT_REBUILD: one slot for the forward states, rebuilt backwards
  int n_ckpt = 0;           // stored segment-start checkpoints (segments 1..J-1)
  int n_seg = 0;            // in-segment boundary buffers (max segment length - 1)
  int slot_states = 1;      // state sets per slot (2 with tangent)
  int n_wg_max = 0;
  int tiles_max = 0;
  size_t off_phi0 = 0, off_slots = 0, off_small = 0, total = 0;
  size_t slot_bytes = 0;
  // small buffers (offsets from off_small)
  size_t o_samples, o_gates, o_dirs, o_igates, o_uref, o_tov, o_ovpart, o_envpart, o_env, o_sched;
  // per-call FP64 buffers: the call's G and V as given (host calls stage them here), the FP64 copies
  // the post-processing reads (G, the possibly projected V, G^-1), the gates the kept pass-boundary
  // states belong to, the per-call flags and the outputs of host calls (cost, fidelity, grad, hvp);
  // for translationally invariant calls the layer gates and directions as given and the per-layer
  // gradient and HVP
  size_t o_gin, o_vin, o_g64, o_v64, o_gi64, o_keptg, o_flags, o_out, o_tiin, o_tiout;
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
  lay.rebuild = ckpt_every == QHVP_CKPT_REBUILD ? 1 : 0;
  lay.n_ckpt = lay.rebuild ? 0 : (int)seg.size() - 1;
  lay.n_seg = lay.rebuild ? 1 : maxlen - 1;   // rebuilding: the one forward-state slot
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
  const size_t g64 = (size_t)K * 32 * sizeof(double);
  lay.o_gin = o;     o = align_up(o + g64);
  lay.o_vin = o;     o = align_up(o + g64);
  lay.o_g64 = o;     o = align_up(o + g64);
  lay.o_v64 = o;     o = align_up(o + g64);
  lay.o_gi64 = o;    o = align_up(o + g64);
  lay.o_keptg = o;   o = align_up(o + g64);
  lay.o_flags = o;   o = align_up(o + qhvp::kFlagCount * sizeof(int));
  lay.o_out = o;     o = align_up(o + 2 * sizeof(double) + 2 * g64);
  const size_t l64 = (size_t)L * 32 * sizeof(double);
  lay.o_tiin = o;    o = align_up(o + 2 * l64);
  lay.o_tiout = o;   o = align_up(o + 2 * l64);
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
  explicit qhvp_ctx(int d) : device(d) {}
  int device;
  // Pinned host buffers and events of destroyed problems, handed to later problems of this context
  // (a serving slot creates one problem per request), so that creating a problem does not pin host
  // memory or create events each time.  At most kPoolKeep of each are kept.
  static constexpr size_t kPoolKeep = 16;
  std::mutex mu;
  std::vector<std::pair<size_t, void*>> pinned;   // (bytes, pointer)
  std::vector<hipEvent_t> events;
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
  // pinned host staging: the samples and U_ref gates at creation, then G | V (FP64) of host calls;
  // the outputs of host calls (cost, fidelity, grad, hvp); the overlaps
  void* h_in;
  double* h_out;
  double* h_tov;
  size_t h_in_bytes = 0, h_out_bytes = 0, h_tov_bytes = 0;
  // two-phase evaluation: a forward sweep leaves its checkpoints for one backward sweep
  int fwd_ready = 0, fwd_tangent = 0, fwd_riem = 0;
  int last_tangent = 0, have_eval = 0;
  // set while a gradient / HVP sweep is being enqueued: if enqueueing fails part-way, the kept
  // pass-boundary states may be incomplete and the next sweep must not reuse them
  int invalidate_kept = 0;
  // device time of the last evaluation: events around its forward (0, 1) and backward (2, 3) phases
  hipEvent_t ev[4];
  int ev_fwd = 0, ev_bwd = 0;
  // optional per-launch timing: events bracket every launch of the call; stats accumulate per kind.
  // Where a device-side decision (a flag of the call) changes a launch's traffic, both figures are kept
  // and the flag picks one when the events are collected.
  int profiling = 0;
  int sched_used = 0;   // tile-schedule counters handed out since the last reset
  std::vector<hipEvent_t> evpool;
  size_t ev_used = 0;
  struct Pending { int kind; size_t e0; double bytes_set, bytes_clear, flops; int flag; };
  std::vector<Pending> pending;
  double k_ms[QHVP_KERNEL_KINDS] = {0}, k_bytes[QHVP_KERNEL_KINDS] = {0}, k_flops[QHVP_KERNEL_KINDS] = {0};
  long long k_count[QHVP_KERNEL_KINDS] = {0};

  char* phi0() { return ws + lay.off_phi0; }
  char* slot(int i) { return ws + lay.off_slots + (size_t)i * lay.slot_bytes; }
  char* small(size_t o) const { return ws + lay.off_small + o; }
  // slot indices: [0, n_ckpt) checkpoints of segments 1..J-1; [n_ckpt, n_ckpt+n_seg) in-segment
  // boundaries 1..maxlen-1; last: working / backward (a, b)
  char* ckpt(int segment) { return slot(segment - 1); }
  char* segbuf(int i) { return slot(lay.n_ckpt + i - 1); }
  // QHVP_CKPT_REBUILD: the forward states, overwritten pass by pass (forward sweep: each pass's
  // output; backward sweep: each pass's input, rebuilt)
  char* rebuilt() { return segbuf(1); }
  char* work() { return slot(lay.n_ckpt + lay.n_seg); }
  char* second(char* slotp) { return slotp + lay.state_bytes; }
  int* flags() const { return (int*)small(lay.o_flags); }
  double* dbuf(size_t o) const { return (double*)small(o); }
  qhvp::Prec dprec() const { return prec == QHVP_C64_ACC64 ? qhvp::P_C64 : qhvp::P_C128; }
  size_t amp() const { return prec == QHVP_C64_ACC64 ? 8 : 16; }
};

namespace {

// Per-launch timing (only when profiling is on): an event before and after the launch(es).
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
// flag < 0: the traffic is bytes_set; else bytes_set if that per-call flag is set, bytes_clear if not
hipError_t prof_end(qhvp_problem* p, int kind, double bytes_set, double flops, int flag = -1, double bytes_clear = 0) {
  if (!p->profiling) return hipSuccess;
  hipError_t r = hipEventRecord(p->evpool[p->ev_used + 1], p->stream);
  p->pending.push_back({kind, p->ev_used, bytes_set, bytes_clear, flops, flag});
  p->ev_used += 2;
  return r;
}
// Waits for the pending launches (the last call's) and adds them to the statistics.
hipError_t prof_collect(qhvp_problem* p) {
  if (p->pending.empty()) return hipSuccess;
  int fl[qhvp::kFlagCount];
  hipError_t r = hipMemcpyAsync(fl, p->flags(), sizeof(fl), hipMemcpyDeviceToHost, p->stream);
  if (r == hipSuccess) r = hipStreamSynchronize(p->stream);
  if (r != hipSuccess) return r;
  for (auto& q : p->pending) {
    float ms = 0;
    r = hipEventElapsedTime(&ms, p->evpool[q.e0], p->evpool[q.e0 + 1]);
    if (r != hipSuccess) return r;
    p->k_ms[q.kind] += ms;
    p->k_bytes[q.kind] += (q.flag < 0 || fl[q.flag] != 0) ? q.bytes_set : q.bytes_clear;
    p->k_flops[q.kind] += q.flops;
    p->k_count[q.kind] += 1;
  }
  p->pending.clear();
  p->ev_used = 0;
  return hipSuccess;
}

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

// Algorithmic traffic and arithmetic of one pass (what the method must move / compute for
// it, not counting the in-tile recomputation): S bytes per state set read or written; per gate
// and amplitude 32 flop for psi <- G psi, 96 with the tangent; the backward adds the environment
// products (32 flop, 96 with the tangent).
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
// Mode 1 leaves two decisions to the flags its k_prep set: psi is not stored at the boundaries that
// stay in the workspace when they already hold it for these gates (kFlagKeep), and the final states
// are stored (for the backward sweep from pass outputs) only if that sweep runs (kFlagInverse).
qhvp_status forward_sweep(qhvp_problem* p, const std::vector<qhvp::PassDesc>& passes, const void* gates,
                          const void* dirs, int tangent, int mode) {
  const int np = (int)passes.size();
  const char* samples = p->small(p->lay.o_samples);
  double* ovpart = (double*)p->small(p->lay.o_ovpart);
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
    } else if (p->lay.rebuild) {
      // in place in one slot; the last pass's output stays there for the backward sweep
      src = q == 0 ? nullptr : p->rebuilt();
      dst = p->rebuilt();
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
    const double S = state_bytes_alg(p), nst = tangent ? 2 : 1;
    double b_set = 0, b_clear = 0;
    int flag = -1;
    if (mode != 0 && q == np - 1) {
      // the backward sweep from pass outputs starts from the final states (kept in the working slot,
      // or in the rebuilt slot, where they are always stored)
      if (mode == 1 && p->lay.rebuild) {
        a.dst_psi = dst;
        a.dst_dpsi = p->second(dst);
      } else if (mode == 1) {
        a.dst_psi = p->work();
        a.dst_dpsi = p->second(p->work());
        a.store_if = p->flags() + qhvp::kFlagInverse;
        flag = qhvp::kFlagInverse;
      }
      a.phi0 = p->phi0();
      a.ov_part = ovpart;
      b_clear = (src ? nst * S : 0) + S + (p->lay.rebuild && mode == 1 ? nst * S : 0);
      b_set = (src ? nst * S : 0) + S + (mode == 1 ? nst * S : 0);
    } else {
      a.dst_psi = dst;
      a.dst_dpsi = p->second(dst);
      if (mode == 1 && dst_kept && !p->lay.rebuild) {
        a.psi_skip = p->flags() + qhvp::kFlagKeep;
        flag = qhvp::kFlagKeep;
      }
      b_clear = (src ? nst * S : 0) + (dst ? S : 0) + (tangent && dst ? S : 0);
      b_set = flag < 0 ? b_clear : b_clear - S;   // psi not stored
    }
    HIP_TRY(prof_begin(p));
    LAUNCH_TRY(qhvp::launch_fwd(p->dprec(), a, p->stream));
    HIP_TRY(prof_end(p, QHVP_KERNEL_FORWARD, b_set, pass_flops(p, a.pd, tangent, false), flag, b_clear));
  }
  if (mode != 0) {
    const int tiles = 1 << (p->n - passes[np - 1].mb);
    LAUNCH_TRY(qhvp::launch_reduce_overlaps(ovpart, p->Ns, tiles, (double*)p->small(p->lay.o_tov), p->stream));
  }
  return QHVP_OK;
}

// Backward sweep of the last mode-1 forward sweep.  Each pass launches both backward kernels; the
// call's kFlagInverse (set by k_prep) lets exactly one of them run: k_bwd_out from the pass-output
// states, or k_bwd recomputing from the pass-input states.
qhvp_status backward_sweep(qhvp_problem* p, int tangent) {
  const int np = (int)p->passes.size();
  const int J = (int)p->seg.size();
  const void* gates = p->small(p->lay.o_gates);
  const void* dirs = p->small(p->lay.o_dirs);
  const char* samples = p->small(p->lay.o_samples);
  double* envpart = (double*)p->small(p->lay.o_envpart);
  double* env = (double*)p->small(p->lay.o_env);
  const int* finv = p->flags() + qhvp::kFlagInverse;
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
      b.samples = samples;
      b.ab_a = ab;
      b.ab_b = p->second(ab);
      b.phi0 = p->phi0();
      b.tov = (const double*)p->small(p->lay.o_tov);
      b.fold = (q == np - 1);
      b.store_ab = (q > 0);
      b.env_part = envpart;
      b.run_flag = finv;
      const double S = state_bytes_alg(p), nst = tangent ? 2 : 1;
      const double common = (b.fold ? S : nst * S) + (b.store_ab ? nst * S : 0);
      if (p->lay.rebuild) {
        // from the pass output, rebuilding the pass input in place for the next backward pass (the
        // first pass's input is not needed); k_prep has checked that every gate can be undone
        qhvp::BwdArgs bo = b;
        bo.src_psi = p->rebuilt();
        bo.src_dpsi = p->second(p->rebuilt());
        if (q > 0) {
          bo.dst_psi = p->rebuilt();
          bo.dst_dpsi = p->second(p->rebuilt());
        }
        bo.run_when = 1;
        HIP_TRY(prof_begin(p));
        LAUNCH_TRY(qhvp::launch_bwd_out(p->dprec(), bo, p->stream));
        HIP_TRY(prof_end(p, QHVP_KERNEL_BACKWARD, common + nst * S + (q > 0 ? nst * S : 0),
                         pass_flops(p, b.pd, tangent, true)));
      } else {
        // forward states: the pass input (recomputing kernel) or the pass output (inverse kernel)
        char* src_in = q == s0 ? start : p->segbuf(q - s0);
        char* src_out = q + 1 < s1 ? p->segbuf(q + 1 - s0) : (j == J - 1 ? ab : p->ckpt(j + 1));
        qhvp::BwdArgs bo = b, br = b;
        bo.src_psi = src_out;
        bo.src_dpsi = p->second(src_out);
        bo.run_when = 1;
        br.src_psi = src_in;
        br.src_dpsi = src_in ? p->second(src_in) : nullptr;
        br.run_when = 0;
        HIP_TRY(prof_begin(p));
        LAUNCH_TRY(qhvp::launch_bwd_out(p->dprec(), bo, p->stream));
        LAUNCH_TRY(qhvp::launch_bwd(p->dprec(), br, p->stream));
        HIP_TRY(prof_end(p, QHVP_KERNEL_BACKWARD, common + nst * S, pass_flops(p, b.pd, tangent, true),
                         qhvp::kFlagInverse, common + (src_in ? nst * S : 0)));
      }
      const long long items = (long long)p->Ns << (p->n - b.pd.mb);
      const int nwg_out = qhvp::bwd_grid(p->dprec(), tangent, b.pd.ng, items, 1);
      const int nwg_rec = qhvp::bwd_grid(p->dprec(), tangent, b.pd.ng, items, 0);
      HIP_TRY(prof_begin(p));
      LAUNCH_TRY(qhvp::launch_reduce_env(envpart, nwg_out, nwg_rec, finv, b.pd, env, p->stream));
      HIP_TRY(prof_end(p, QHVP_KERNEL_REDUCE, (double)nwg_out * b.pd.ng * qhvp::kEnvVals * 8, 0, qhvp::kFlagInverse,
                       (double)nwg_rec * b.pd.ng * qhvp::kEnvVals * 8));
    }
  }
  return QHVP_OK;
}

// Whether ptr lies in device memory of HIP device `device` (or in managed memory).
bool device_pointer(const void* ptr, int device) {
  if (!ptr) return false;
  hipPointerAttribute_t at;
  std::memset(&at, 0, sizeof(at));
  if (hipPointerGetAttributes(&at, ptr) != hipSuccess) {
    (void)hipGetLastError();   // plain host memory: the query fails; leave no error behind
    return false;
  }
  if (at.type == hipMemoryTypeDevice) return at.device == device;
  return at.type == hipMemoryTypeManaged;
}

bool env_recompute() {
  const char* choice = std::getenv("QHVP_BACKWARD");
  return choice && std::strcmp(choice, "recompute") == 0;
}

// Forward phase of one evaluation on device inputs d_G, d_V (K*16 complex FP64 each; d_V only for
// mode 2).  mode 0: cost sweep (nothing kept); 1: gradient sweep; 2: HVP sweep (tangent states).
// Enqueues k_prep and the sweep on the problem's stream; returns without waiting.
qhvp_status core_forward(qhvp_problem* p, const double* d_G, const double* d_V, int riem, int mode) {
  HIP_TRY(hipSetDevice(p->ctx->device));
  HIP_TRY(prof_collect(p));
  p->fwd_ready = 0;
  p->ev_fwd = p->ev_bwd = 0;
  const int tangent = mode == 2 ? 1 : 0;
  if (p->ev[0]) HIP_TRY(hipEventRecord(p->ev[0], p->stream));
  qhvp::PrepArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.K = p->K;
  pa.prec = p->dprec();
  pa.tangent = tangent;
  pa.riem = mode != 0 ? riem : 0;
  pa.rebuild = (mode != 0 && p->lay.rebuild) ? 1 : 0;
  pa.with_inverse = (mode != 0 && (pa.rebuild || !env_recompute())) ? 1 : 0;
  pa.keep_mode = (mode != 0 && !p->lay.rebuild) ? 1 : 0;   // rebuilding overwrites the forward states
  pa.invalidate_kept = p->invalidate_kept;
  pa.G_in = d_G;
  pa.V_in = tangent ? d_V : nullptr;
  pa.gates = p->small(p->lay.o_gates);
  pa.dirs = p->small(p->lay.o_dirs);
  pa.igates = p->small(p->lay.o_igates);
  pa.g64 = p->dbuf(p->lay.o_g64);
  pa.v64 = p->dbuf(p->lay.o_v64);
  pa.gi64 = p->dbuf(p->lay.o_gi64);
  pa.kept_g = p->dbuf(p->lay.o_keptg);
  pa.flags = p->flags();
  if (mode != 0) p->invalidate_kept = 1;   // cleared once the whole sweep is enqueued
  LAUNCH_TRY(qhvp::launch_prep(pa, p->stream));
  qhvp_status st = forward_sweep(p, p->passes, p->small(p->lay.o_gates), p->small(p->lay.o_dirs), tangent,
                                 mode == 0 ? 2 : 1);
  if (st) return st;
  if (mode != 0) p->invalidate_kept = 0;
  if (p->ev[1]) HIP_TRY(hipEventRecord(p->ev[1], p->stream));
  p->ev_fwd = p->ev[1] ? 1 : 0;
  p->have_eval = 1;
  p->last_tangent = tangent;
  if (mode != 0) {
    p->fwd_ready = 1;
    p->fwd_tangent = tangent;
    p->fwd_riem = riem;
  }
  return QHVP_OK;
}

// Post-processing on the device (k_post): outputs are device pointers (null: not written).
qhvp_status core_post(qhvp_problem* p, int mode, int tangent, int riem, double* cost, double* fidelity, double* grad,
                      double* hvp) {
  qhvp::PostArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.K = p->K;
  pa.Ns = p->Ns;
  pa.tangent = tangent;
  pa.riem = riem;
  pa.mode = mode;
  pa.tov = (const double*)p->small(p->lay.o_tov);
  pa.env = (const double*)p->small(p->lay.o_env);
  pa.flags = p->flags();
  pa.g64 = p->dbuf(p->lay.o_g64);
  pa.v64 = p->dbuf(p->lay.o_v64);
  pa.gi64 = p->dbuf(p->lay.o_gi64);
  pa.cost = cost;
  pa.fidelity = fidelity;
  pa.grad = grad;
  pa.hvp = hvp;
  LAUNCH_TRY(qhvp::launch_post(pa, p->stream));
  return QHVP_OK;
}

// Backward phase of the last gradient / HVP forward phase (its checkpoints are consumed), then the
// post-processing into the device outputs (cost and fidelity too when given).
qhvp_status core_backward(qhvp_problem* p, double* cost, double* fidelity, double* grad, double* hvp) {
  HIP_TRY(hipSetDevice(p->ctx->device));
  if (!p->fwd_ready) return fail(QHVP_ERR_INVALID, "no forward sweep to differentiate (call qhvp_forward first)");
  p->fwd_ready = 0;
  if (p->ev[2]) HIP_TRY(hipEventRecord(p->ev[2], p->stream));
  qhvp_status st = backward_sweep(p, p->fwd_tangent);
  if (st) return st;
  const int mode = qhvp::kPostDeriv | ((cost || fidelity) ? qhvp::kPostCost : 0);
  st = core_post(p, mode, p->fwd_tangent, p->fwd_riem, cost, fidelity, grad, hvp);
  if (st) return st;
  if (p->ev[3]) HIP_TRY(hipEventRecord(p->ev[3], p->stream));
  p->ev_bwd = p->ev[3] ? 1 : 0;
  return QHVP_OK;
}

// The context's pools (thread-safe): the smallest pooled buffer of at least `bytes`, else a new one;
// *got receives its size.
void* pool_pinned(qhvp_ctx* c, size_t bytes, size_t* got) {
  *got = bytes;
  {
    std::lock_guard<std::mutex> lock(c->mu);
    size_t best = c->pinned.size();
    for (size_t i = 0; i < c->pinned.size(); ++i)
      if (c->pinned[i].first >= bytes && (best == c->pinned.size() || c->pinned[i].first < c->pinned[best].first)) best = i;
    if (best < c->pinned.size()) {
      void* ptr = c->pinned[best].second;
      *got = c->pinned[best].first;
      c->pinned.erase(c->pinned.begin() + best);
      return ptr;
    }
  }
  void* ptr = nullptr;
  if (hipHostMalloc(&ptr, bytes) != hipSuccess) return nullptr;
  return ptr;
}
// Returns a buffer (its true size: a pooled buffer may be larger than its problem asked for).
void pool_release_pinned(qhvp_ctx* c, void* ptr, size_t bytes) {
  if (!ptr) return;
  {
    std::lock_guard<std::mutex> lock(c->mu);
    if (c->pinned.size() < qhvp_ctx::kPoolKeep) {
      c->pinned.emplace_back(bytes, ptr);
      return;
    }
  }
  hipHostFree(ptr);
}
hipEvent_t pool_event(qhvp_ctx* c) {
  {
    std::lock_guard<std::mutex> lock(c->mu);
    if (!c->events.empty()) {
      hipEvent_t e = c->events.back();
      c->events.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
void pool_release_event(qhvp_ctx* c, hipEvent_t e) {
  if (!e) return;
  {
    std::lock_guard<std::mutex> lock(c->mu);
    if (c->events.size() < 4 * qhvp_ctx::kPoolKeep) {
      c->events.push_back(e);
      return;
    }
  }
  hipEventDestroy(e);
}

// A problem's host-side description (pass plans, checkpoint segments, workspace layout), with no
// workspace, staging or events attached yet.
qhvp_problem* new_problem(qhvp_ctx* ctx, int n, int L, int L_ref, int n_samples, qhvp_precision prec, int ckpt_every,
                          int with_tangent, const Layout& lay, void* hip_stream) {
  qhvp_problem* p = new qhvp_problem();
  p->ctx = ctx;
  p->n = n; p->L = L; p->L_ref = L_ref; p->Ns = n_samples;
  p->K = num_gates(n, L); p->Kr = num_gates(n, L_ref);
  p->prec = prec; p->ckpt_every = ckpt_every; p->tangent = with_tangent ? 1 : 0;
  p->stream = (hipStream_t)hip_stream;
  p->passes = plan_circuit(n, L, nullptr);
  p->ref_passes = plan_circuit(n, L_ref, nullptr);
  fill_tile_offsets(p->passes, (int)p->amp());
  fill_tile_offsets(p->ref_passes, (int)p->amp());
  p->seg = plan_segments(n, L, ckpt_every);
  p->lay = lay;
  p->ws = nullptr;
  p->owns_ws = false;
  p->h_in = nullptr;
  p->h_out = p->h_tov = nullptr;
  for (auto& e : p->ev) e = nullptr;
  return p;
}

// ---- host calls: validated on the host, staged to the device, evaluated by the device path, and
// the outputs copied back once everything succeeded (outputs are untouched on every error path)

qhvp_status check_gates(const qhvp_problem* p, const double* G, const char* what) {
  if (!G) return fail(QHVP_ERR_INVALID, std::string(what) + " is NULL");
  if (!finite_all(G, (size_t)p->K * 32)) return fail(QHVP_ERR_INVALID, std::string(what) + " has non-finite entries");
  return QHVP_OK;
}

qhvp_status check_host_call(const qhvp_problem* p, const double* G, const double* V, qhvp_geometry geom) {
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
  return QHVP_OK;
}

// Copies host G (and V) into the workspace's input buffers through pinned staging.
qhvp_status stage_inputs(qhvp_problem* p, const double* G, const double* V) {
  HIP_TRY(hipSetDevice(p->ctx->device));
  const size_t gb = (size_t)p->K * 32 * sizeof(double);
  std::memcpy(p->h_in, G, gb);
  HIP_TRY(hipMemcpyAsync(p->small(p->lay.o_gin), p->h_in, gb, hipMemcpyHostToDevice, p->stream));
  if (V) {
    std::memcpy((char*)p->h_in + gb, V, gb);
    HIP_TRY(hipMemcpyAsync(p->small(p->lay.o_vin), (char*)p->h_in + gb, gb, hipMemcpyHostToDevice, p->stream));
  }
  return QHVP_OK;
}

// Device output staging of host calls: cost, fidelity, grad (K*32), hvp (K*32) doubles.
double* out_cost(qhvp_problem* p) { return p->dbuf(p->lay.o_out); }
double* out_grad(qhvp_problem* p) { return p->dbuf(p->lay.o_out) + 2; }
double* out_hvp(qhvp_problem* p) { return p->dbuf(p->lay.o_out) + 2 + (size_t)p->K * 32; }

// Brings the staged outputs back (cost and fidelity; the gradient, then the HVP, `gn` doubles each,
// contiguous from `src`), waits, and (only then) writes the caller's outputs.
qhvp_status finish_host_call(qhvp_problem* p, const double* src, size_t gn, double* cost, double* fidelity, double* grad,
                             double* hvp) {
  const size_t cnt = (grad || hvp) ? (hvp ? 2 * gn : gn) : 0;
  HIP_TRY(hipMemcpyAsync(p->h_out, out_cost(p), 2 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  if (cnt) HIP_TRY(hipMemcpyAsync(p->h_out + 2, src, cnt * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  int status = 0;
  HIP_TRY(hipMemcpyAsync(p->h_tov, p->flags() + qhvp::kFlagStatus, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  std::memcpy(&status, p->h_tov, sizeof(int));
  if (status != 0) return fail(QHVP_ERR_INVALID, "the device rejected the inputs (status " + std::to_string(status) + ")");
  if (cost) *cost = p->h_out[0];
  if (fidelity) *fidelity = p->h_out[1];
  if (grad) std::memcpy(grad, p->h_out + 2, gn * sizeof(double));
  if (hvp) std::memcpy(hvp, p->h_out + 2 + gn, gn * sizeof(double));
  return QHVP_OK;
}

qhvp_status host_forward(qhvp_problem* p, const double* G, const double* V, qhvp_geometry geom, double* cost,
                         double* fidelity) {
  qhvp_status st = check_host_call(p, G, V, geom);
  if (st) return st;
  st = stage_inputs(p, G, V);
  if (st) return st;
  const double* dv = V ? p->dbuf(p->lay.o_vin) : nullptr;
  st = core_forward(p, p->dbuf(p->lay.o_gin), dv, geom == QHVP_RIEMANNIAN, V ? 2 : 1);
  if (st) return st;
  st = core_post(p, qhvp::kPostCost, 0, 0, out_cost(p), out_cost(p) + 1, nullptr, nullptr);
  if (st) return st;
  return finish_host_call(p, nullptr, 0, cost, fidelity, nullptr, nullptr);
}

}  // namespace

// --------------------------------------------------------------------------------------------
extern "C" {

int qhvp_version(void) { return 200; }

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
  // the scratch of qhvp_hvp_noalloc: its address on this device, looked up once
  LAUNCH_TRY(qhvp::noalloc_scratch_init(device));
  *out = new qhvp_ctx(device);
  return QHVP_OK;
}

void qhvp_ctx_destroy(qhvp_ctx* ctx) {
  if (!ctx) return;
  for (auto& b : ctx->pinned) hipHostFree(b.second);
  for (auto e : ctx->events) hipEventDestroy(e);
  delete ctx;
}

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

  qhvp_problem* p = new_problem(ctx, n, L, L_ref, n_samples, prec, ckpt_every, with_tangent, lay, hip_stream);
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
  const size_t gl = (size_t)std::max(p->K, L);   // gates, or layers of a translationally invariant call
  const size_t in_bytes = std::max({gl * 64 * sizeof(double), (size_t)Kr * 16 * amp, (size_t)n_samples * n * 2 * amp});
  const size_t out_bytes = (2 + gl * 64) * sizeof(double);
  const size_t tov_bytes = std::max((size_t)n_samples * 4, (size_t)qhvp::kFlagCount) * sizeof(double);
  if (!(p->h_in = pool_pinned(ctx, in_bytes, &p->h_in_bytes)) ||
      !(p->h_out = (double*)pool_pinned(ctx, out_bytes, &p->h_out_bytes)) ||
      !(p->h_tov = (double*)pool_pinned(ctx, tov_bytes, &p->h_tov_bytes)))
    return cleanup_fail(QHVP_ERR_NOMEM, "pinned host allocation failed");
  for (auto& e : p->ev)
    if (!(e = pool_event(ctx))) return cleanup_fail(QHVP_ERR_DEVICE, "hipEventCreate failed");

  // per-call flags start cleared (no kept states); samples and U_ref gates to the device, then the
  // labels phi0 = U_ref psi (a forward sweep of U_ref)
  if (qhvp::launch_zero_ints(p->flags(), qhvp::kFlagCount, p->stream) != 0)
    return cleanup_fail(QHVP_ERR_DEVICE, "clearing the call flags failed");
  to_device_precision(p, samples, (size_t)n_samples * n * 2, p->h_in);
  if (hipMemcpyAsync(p->small(lay.o_samples), p->h_in, (size_t)n_samples * n * 2 * amp, hipMemcpyHostToDevice, p->stream) != hipSuccess ||
      hipStreamSynchronize(p->stream) != hipSuccess)
    return cleanup_fail(QHVP_ERR_DEVICE, "copy of samples failed");
  to_device_precision(p, uref_gates, (size_t)Kr * 16, p->h_in);
  if (hipMemcpyAsync(p->small(lay.o_uref), p->h_in, (size_t)Kr * 16 * amp, hipMemcpyHostToDevice, p->stream) != hipSuccess)
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
  pool_release_pinned(p->ctx, p->h_in, p->h_in_bytes);
  pool_release_pinned(p->ctx, p->h_out, p->h_out_bytes);
  pool_release_pinned(p->ctx, p->h_tov, p->h_tov_bytes);
  for (auto e : p->ev) pool_release_event(p->ctx, e);
  for (auto e : p->evpool) hipEventDestroy(e);
  delete p;
}

qhvp_status qhvp_cost(qhvp_problem* p, const double* G, double* cost, double* fidelity) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  qhvp_status st = check_gates(p, G, "G");
  if (st) return st;
  st = stage_inputs(p, G, nullptr);
  if (st) return st;
  st = core_forward(p, p->dbuf(p->lay.o_gin), nullptr, 0, 0);
  if (st) return st;
  st = core_post(p, qhvp::kPostCost, 0, 0, out_cost(p), out_cost(p) + 1, nullptr, nullptr);
  if (st) return st;
  return finish_host_call(p, nullptr, 0, cost, fidelity, nullptr, nullptr);
}

qhvp_status qhvp_forward(qhvp_problem* p, const double* G, const double* V, qhvp_geometry geom, double* cost,
                         double* fidelity) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  return host_forward(p, G, V, geom, cost, fidelity);
}

qhvp_status qhvp_backward(qhvp_problem* p, double* grad, double* hvp) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (!p->fwd_ready) return fail(QHVP_ERR_INVALID, "no forward sweep to differentiate (call qhvp_forward first)");
  if (hvp && !p->fwd_tangent) return fail(QHVP_ERR_INVALID, "the last forward sweep had no direction V");
  qhvp_status st = core_backward(p, nullptr, nullptr, grad ? out_grad(p) : nullptr, hvp ? out_hvp(p) : nullptr);
  if (st) return st;
  return finish_host_call(p, out_grad(p), (size_t)p->K * 32, nullptr, nullptr, grad, hvp);
}

qhvp_status qhvp_hvp_batch(qhvp_problem* p, const double* G, int n_dirs, const double* V, qhvp_geometry geom,
                           double* cost, double* grad, double* hvp) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (n_dirs < 1) return fail(QHVP_ERR_INVALID, "n_dirs must be positive");
  if (!V || !hvp) return fail(QHVP_ERR_INVALID, "V and hvp must not be NULL");
  if (!p->tangent) return fail(QHVP_ERR_UNSUPPORTED, "problem was created without tangent storage");
  qhvp_status st = check_host_call(p, G, nullptr, geom);
  if (st) return st;
  const size_t gn = (size_t)p->K * 32;
  if (!finite_all(V, gn * (size_t)n_dirs)) return fail(QHVP_ERR_INVALID, "V has non-finite entries");
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
  int fl[qhvp::kFlagCount];
  std::vector<double> kg(gn);
  if (hipSetDevice(p->ctx->device) != hipSuccess ||
      hipMemcpyAsync(fl, p->flags(), sizeof(fl), hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
      hipMemcpyAsync(kg.data(), p->small(p->lay.o_keptg), gn * sizeof(double), hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
      hipStreamSynchronize(p->stream) != hipSuccess)
    return -1;
  return (!p->invalidate_kept && fl[qhvp::kFlagKeptValid] && std::memcmp(kg.data(), G, gn * sizeof(double)) == 0) ? 1 : 0;
}

qhvp_status qhvp_grad(qhvp_problem* p, const double* G, qhvp_geometry geom, double* cost, double* fidelity,
                      double* grad) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (!grad) return fail(QHVP_ERR_INVALID, "grad is NULL");
  qhvp_status st = check_host_call(p, G, nullptr, geom);
  if (st) return st;
  st = stage_inputs(p, G, nullptr);
  if (st) return st;
  st = core_forward(p, p->dbuf(p->lay.o_gin), nullptr, geom == QHVP_RIEMANNIAN, 1);
  if (st) return st;
  st = core_backward(p, out_cost(p), out_cost(p) + 1, out_grad(p), nullptr);
  if (st) return st;
  return finish_host_call(p, out_grad(p), (size_t)p->K * 32, cost, fidelity, grad, nullptr);
}

qhvp_status qhvp_hvp(qhvp_problem* p, const double* G, const double* V, qhvp_geometry geom, double* cost,
                     double* fidelity, double* grad, double* hvp) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (!hvp) return fail(QHVP_ERR_INVALID, "hvp is NULL");
  if (!V) return fail(QHVP_ERR_INVALID, "V is NULL");
  qhvp_status st = check_host_call(p, G, V, geom);
  if (st) return st;
  st = stage_inputs(p, G, V);
  if (st) return st;
  st = core_forward(p, p->dbuf(p->lay.o_gin), p->dbuf(p->lay.o_vin), geom == QHVP_RIEMANNIAN, 2);
  if (st) return st;
  st = core_backward(p, out_cost(p), out_cost(p) + 1, out_grad(p), out_hvp(p));
  if (st) return st;
  return finish_host_call(p, out_grad(p), (size_t)p->K * 32, cost, fidelity, grad, hvp);
}

// ---- device-pointer calls: inputs and outputs in device memory, enqueued on the problem's stream

namespace {
qhvp_status check_dev_call(const qhvp_problem* p, const double* d_G, const double* d_V, qhvp_geometry geom,
                           std::initializer_list<const double*> outs) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (geom != QHVP_EUCLIDEAN && geom != QHVP_RIEMANNIAN) return fail(QHVP_ERR_INVALID, "unknown geometry");
  const int dev = p->ctx->device;
  if (!device_pointer(d_G, dev)) return fail(QHVP_ERR_INVALID, "G is not device memory of the problem's device");
  if (d_V) {
    if (!p->tangent) return fail(QHVP_ERR_UNSUPPORTED, "problem was created without tangent storage");
    if (!device_pointer(d_V, dev)) return fail(QHVP_ERR_INVALID, "V is not device memory of the problem's device");
  }
  for (const double* o : outs)
    if (o && !device_pointer(o, dev)) return fail(QHVP_ERR_INVALID, "an output is not device memory of the problem's device");
  return QHVP_OK;
}
}  // namespace

qhvp_status qhvp_cost_dev(qhvp_problem* p, const double* d_G, double* d_cost, double* d_fidelity) {
  qhvp_status st = check_dev_call(p, d_G, nullptr, QHVP_EUCLIDEAN, {d_cost, d_fidelity});
  if (st) return st;
  st = core_forward(p, d_G, nullptr, 0, 0);
  if (st) return st;
  return core_post(p, qhvp::kPostCost, 0, 0, d_cost, d_fidelity, nullptr, nullptr);
}

qhvp_status qhvp_forward_dev(qhvp_problem* p, const double* d_G, const double* d_V, qhvp_geometry geom, double* d_cost,
                             double* d_fidelity) {
  qhvp_status st = check_dev_call(p, d_G, d_V, geom, {d_cost, d_fidelity});
  if (st) return st;
  st = core_forward(p, d_G, d_V, geom == QHVP_RIEMANNIAN, d_V ? 2 : 1);
  if (st) return st;
  if (!d_cost && !d_fidelity) return QHVP_OK;
  return core_post(p, qhvp::kPostCost, 0, 0, d_cost, d_fidelity, nullptr, nullptr);
}

qhvp_status qhvp_backward_dev(qhvp_problem* p, double* d_grad, double* d_hvp) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (!p->fwd_ready) return fail(QHVP_ERR_INVALID, "no forward sweep to differentiate (call qhvp_forward_dev first)");
  if (d_hvp && !p->fwd_tangent) return fail(QHVP_ERR_INVALID, "the last forward sweep had no direction V");
  const int dev = p->ctx->device;
  if ((d_grad && !device_pointer(d_grad, dev)) || (d_hvp && !device_pointer(d_hvp, dev)))
    return fail(QHVP_ERR_INVALID, "an output is not device memory of the problem's device");
  return core_backward(p, nullptr, nullptr, d_grad, d_hvp);
}

qhvp_status qhvp_grad_dev(qhvp_problem* p, const double* d_G, qhvp_geometry geom, double* d_cost, double* d_fidelity,
                          double* d_grad) {
  if (!d_grad) return fail(QHVP_ERR_INVALID, "grad is NULL");
  qhvp_status st = check_dev_call(p, d_G, nullptr, geom, {d_cost, d_fidelity, d_grad});
  if (st) return st;
  st = core_forward(p, d_G, nullptr, geom == QHVP_RIEMANNIAN, 1);
  if (st) return st;
  return core_backward(p, d_cost, d_fidelity, d_grad, nullptr);
}

qhvp_status qhvp_hvp_dev(qhvp_problem* p, const double* d_G, const double* d_V, qhvp_geometry geom, double* d_cost,
                         double* d_fidelity, double* d_grad, double* d_hvp) {
  if (!d_hvp || !d_V) return fail(QHVP_ERR_INVALID, "V and hvp must not be NULL");
  qhvp_status st = check_dev_call(p, d_G, d_V, geom, {d_cost, d_fidelity, d_grad, d_hvp});
  if (st) return st;
  st = core_forward(p, d_G, d_V, geom == QHVP_RIEMANNIAN, 2);
  if (st) return st;
  return core_backward(p, d_cost, d_fidelity, d_grad, d_hvp);
}

qhvp_status qhvp_hvp_noalloc(qhvp_ctx* ctx, int n, int L, int L_ref, const double* d_uref_gates,
                             const double* d_samples, int n_samples, qhvp_precision prec, const double* d_G,
                             const double* d_V, qhvp_geometry geom, double* d_cost, double* d_fidelity,
                             double* d_grad, double* d_hvp, void* hip_stream) {
  if (!ctx) return fail(QHVP_ERR_INVALID, "ctx is NULL");
  if (n < 2 || n > qhvp::kMaxQubits) return fail(QHVP_ERR_INVALID, "n must be in [2, 30]");
  if (L < 1 || L_ref < 1) return fail(QHVP_ERR_INVALID, "L and L_ref must be >= 1");
  if (n_samples < 1) return fail(QHVP_ERR_INVALID, "n_samples must be >= 1");
  if (prec != QHVP_C128 && prec != QHVP_C64_ACC64) return fail(QHVP_ERR_INVALID, "unknown precision");
  if (geom != QHVP_EUCLIDEAN && geom != QHVP_RIEMANNIAN) return fail(QHVP_ERR_INVALID, "unknown geometry");
  if (!d_V || !d_hvp) return fail(QHVP_ERR_INVALID, "V and hvp must not be NULL");
  const int dev = ctx->device;
  for (const double* ptr : {d_uref_gates, d_samples, d_G, d_V})
    if (!device_pointer(ptr, dev)) return fail(QHVP_ERR_INVALID, "an input is not device memory of the context's device");
  for (const double* ptr : {d_cost, d_fidelity, d_grad, d_hvp})
    if (ptr && !device_pointer(ptr, dev)) return fail(QHVP_ERR_INVALID, "an output is not device memory of the context's device");
  void* scratch = qhvp::noalloc_scratch(dev);
  if (!scratch) return fail(QHVP_ERR_DEVICE, "no scratch on this device (qhvp_ctx_create did not finish)");
  // the fastest checkpoint policy whose workspace fits the scratch
  Layout lay;
  int ckpt = 0;
  bool fits = false;
  for (int ck : {0, -2, 1, 2, 4, 8}) {
    Layout l;
    if (make_layout(n, L, L_ref, n_samples, prec, ck, 1, l) && l.total <= qhvp::kNoAllocScratchBytes) {
      lay = l;
      ckpt = ck;
      fits = true;
      break;
    }
  }
  if (!fits)
    return fail(QHVP_ERR_NOMEM, "the problem needs more than the " + std::to_string(qhvp::kNoAllocScratchBytes >> 20) +
                                    " MiB of scratch of qhvp_hvp_noalloc (use qhvp_problem_create)");
  HIP_TRY(hipSetDevice(dev));
  qhvp_problem* p = new_problem(ctx, n, L, L_ref, n_samples, prec, ckpt, 1, lay, hip_stream);
  p->ws = (char*)scratch;
  // labels phi0 = U_ref psi (Alg. 2 takes them as input), then the HVP: all inside the scratch
  qhvp_status st = QHVP_OK;
  if (qhvp::launch_zero_ints(p->flags(), qhvp::kFlagCount, p->stream) != 0 ||
      qhvp::launch_convert(d_samples, p->small(lay.o_samples), (long long)n_samples * n * 2, p->dprec(), p->stream) != 0 ||
      qhvp::launch_convert(d_uref_gates, p->small(lay.o_uref), (long long)p->Kr * 16, p->dprec(), p->stream) != 0)
    st = fail(QHVP_ERR_DEVICE, "launch failed while setting up the scratch");
  if (st == QHVP_OK) st = forward_sweep(p, p->ref_passes, p->small(lay.o_uref), nullptr, 0, 0);
  if (st == QHVP_OK) st = core_forward(p, d_G, d_V, geom == QHVP_RIEMANNIAN, 2);
  if (st == QHVP_OK) st = core_backward(p, d_cost, d_fidelity, d_grad, d_hvp);
  delete p;   // host-side description only: the scratch stays with the device
  return st;
}

qhvp_status qhvp_device_status(qhvp_problem* p, int* status) {
  if (!p || !status) return fail(QHVP_ERR_INVALID, "bad arguments");
  HIP_TRY(hipSetDevice(p->ctx->device));
  int v = 0;
  HIP_TRY(hipMemcpyAsync(p->h_tov, p->flags() + qhvp::kFlagStatus, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  std::memcpy(&v, p->h_tov, sizeof(int));
  *status = v;
  return QHVP_OK;
}

}  // extern "C"

extern "C" {

// ---- translationally invariant circuits (App. E): one gate G_(l) per layer ----------------------
// The layer gates (and directions) are expanded to the K gates on the device, the evaluation runs as
// for any circuit, and the per-gate derivatives (post-processed, so Riemannian ones already
// projected at G_(l) with the projected V_(l): both maps are linear in the derivatives) are summed
// per layer on the device in FP64 in a fixed order.

namespace {
qhvp_status check_ti_layers(const qhvp_problem* p, const double* G_layers, const double* V_layers, qhvp_geometry geom) {
  if (geom != QHVP_EUCLIDEAN && geom != QHVP_RIEMANNIAN) return fail(QHVP_ERR_INVALID, "unknown geometry");
  if (!G_layers) return fail(QHVP_ERR_INVALID, "G_layers is NULL");
  if (!finite_all(G_layers, (size_t)p->L * 32)) return fail(QHVP_ERR_INVALID, "G_layers has non-finite entries");
  if (V_layers) {
    if (!p->tangent) return fail(QHVP_ERR_UNSUPPORTED, "problem was created without tangent storage");
    if (!finite_all(V_layers, (size_t)p->L * 32)) return fail(QHVP_ERR_INVALID, "V_layers has non-finite entries");
  }
  if (geom == QHVP_RIEMANNIAN && qhvp_unitarity_error(p->L, G_layers) > 1e-10)
    return fail(QHVP_ERR_INVALID, "Riemannian geometry needs unitary gates");
  return QHVP_OK;
}

// The whole translationally invariant evaluation on device inputs (L*16 complex each) into device
// outputs (grad_layers may be null; hvp_layers only with d_Vl).
qhvp_status core_ti(qhvp_problem* p, const double* d_Gl, const double* d_Vl, int riem, double* d_cost, double* d_fid,
                    double* d_gl, double* d_hl) {
  HIP_TRY(hipSetDevice(p->ctx->device));
  LAUNCH_TRY(qhvp::launch_ti_expand(d_Gl, p->n, p->K, p->dbuf(p->lay.o_gin), p->stream));
  if (d_Vl) LAUNCH_TRY(qhvp::launch_ti_expand(d_Vl, p->n, p->K, p->dbuf(p->lay.o_vin), p->stream));
  qhvp_status st = core_forward(p, p->dbuf(p->lay.o_gin), d_Vl ? p->dbuf(p->lay.o_vin) : nullptr, riem, d_Vl ? 2 : 1);
  if (st) return st;
  st = core_backward(p, d_cost, d_fid, d_gl ? out_grad(p) : nullptr, d_hl ? out_hvp(p) : nullptr);
  if (st) return st;
  if (d_gl) LAUNCH_TRY(qhvp::launch_ti_reduce(out_grad(p), p->n, p->L, p->flags(), d_gl, p->stream));
  if (d_hl) LAUNCH_TRY(qhvp::launch_ti_reduce(out_hvp(p), p->n, p->L, p->flags(), d_hl, p->stream));
  return QHVP_OK;
}

qhvp_status host_ti(qhvp_problem* p, const double* G_layers, const double* V_layers, qhvp_geometry geom, double* cost,
                    double* fidelity, double* grad_layers, double* hvp_layers) {
  qhvp_status st = check_ti_layers(p, G_layers, V_layers, geom);
  if (st) return st;
  HIP_TRY(hipSetDevice(p->ctx->device));
  const size_t lb = (size_t)p->L * 32 * sizeof(double);
  double* d_in = p->dbuf(p->lay.o_tiin);
  double* d_out = p->dbuf(p->lay.o_tiout);
  std::memcpy(p->h_in, G_layers, lb);
  if (V_layers) std::memcpy((char*)p->h_in + lb, V_layers, lb);
  HIP_TRY(hipMemcpyAsync(d_in, p->h_in, V_layers ? 2 * lb : lb, hipMemcpyHostToDevice, p->stream));
  st = core_ti(p, d_in, V_layers ? d_in + (size_t)p->L * 32 : nullptr, geom == QHVP_RIEMANNIAN, out_cost(p),
               out_cost(p) + 1, (grad_layers || hvp_layers) ? d_out : nullptr, hvp_layers ? d_out + (size_t)p->L * 32 : nullptr);
  if (st) return st;
  return finish_host_call(p, d_out, (size_t)p->L * 32, cost, fidelity, grad_layers, hvp_layers);
}
}  // namespace

qhvp_status qhvp_grad_ti(qhvp_problem* p, const double* G_layers, qhvp_geometry geom, double* cost, double* fidelity,
                         double* grad_layers) {
  if (!p || !grad_layers) return fail(QHVP_ERR_INVALID, "bad arguments");
  return host_ti(p, G_layers, nullptr, geom, cost, fidelity, grad_layers, nullptr);
}

qhvp_status qhvp_hvp_ti(qhvp_problem* p, const double* G_layers, const double* V_layers, qhvp_geometry geom,
                        double* cost, double* fidelity, double* grad_layers, double* hvp_layers) {
  if (!p || !V_layers || !hvp_layers) return fail(QHVP_ERR_INVALID, "bad arguments");
  return host_ti(p, G_layers, V_layers, geom, cost, fidelity, grad_layers, hvp_layers);
}

qhvp_status qhvp_grad_ti_dev(qhvp_problem* p, const double* d_G_layers, qhvp_geometry geom, double* d_cost,
                             double* d_fidelity, double* d_grad_layers) {
  if (!d_grad_layers) return fail(QHVP_ERR_INVALID, "grad_layers is NULL");
  qhvp_status st = check_dev_call(p, d_G_layers, nullptr, geom, {d_cost, d_fidelity, d_grad_layers});
  if (st) return st;
  return core_ti(p, d_G_layers, nullptr, geom == QHVP_RIEMANNIAN, d_cost, d_fidelity, d_grad_layers, nullptr);
}

qhvp_status qhvp_hvp_ti_dev(qhvp_problem* p, const double* d_G_layers, const double* d_V_layers, qhvp_geometry geom,
                            double* d_cost, double* d_fidelity, double* d_grad_layers, double* d_hvp_layers) {
  if (!d_hvp_layers || !d_V_layers) return fail(QHVP_ERR_INVALID, "V_layers and hvp_layers must not be NULL");
  qhvp_status st = check_dev_call(p, d_G_layers, d_V_layers, geom, {d_cost, d_fidelity, d_grad_layers, d_hvp_layers});
  if (st) return st;
  return core_ti(p, d_G_layers, d_V_layers, geom == QHVP_RIEMANNIAN, d_cost, d_fidelity, d_grad_layers, d_hvp_layers);
}

qhvp_status qhvp_overlaps(const qhvp_problem* p, double* T, double* Omega) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  if (!p->have_eval) return fail(QHVP_ERR_INVALID, "no evaluation yet");
  HIP_TRY(hipSetDevice(p->ctx->device));
  std::vector<double> tov((size_t)p->Ns * 4);
  HIP_TRY(hipMemcpyAsync(tov.data(), p->small(p->lay.o_tov), tov.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  for (int s = 0; s < p->Ns; ++s) {
    if (T) { T[2 * s] = tov[4 * s]; T[2 * s + 1] = tov[4 * s + 1]; }
    if (Omega) {
      Omega[2 * s] = p->last_tangent ? tov[4 * s + 2] : 0.0;
      Omega[2 * s + 1] = p->last_tangent ? tov[4 * s + 3] : 0.0;
    }
  }
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

int qhvp_backward_from_outputs(const qhvp_problem* p) {
  if (!p) return -1;
  int fl[qhvp::kFlagCount];
  if (hipSetDevice(p->ctx->device) != hipSuccess ||
      hipMemcpyAsync(fl, p->flags(), sizeof(fl), hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
      hipStreamSynchronize(p->stream) != hipSuccess)
    return -1;
  return fl[qhvp::kFlagInverse];
}

double qhvp_last_device_ms(const qhvp_problem* p) {
  if (!p || !p->ev_fwd) return 0.0;
  float a = 0, b = 0;
  if (hipEventSynchronize(p->ev[p->ev_bwd ? 3 : 1]) != hipSuccess || hipEventElapsedTime(&a, p->ev[0], p->ev[1]) != hipSuccess)
    return 0.0;
  if (p->ev_bwd && hipEventElapsedTime(&b, p->ev[2], p->ev[3]) != hipSuccess) return 0.0;
  return (double)a + (double)b;
}

qhvp_status qhvp_set_profiling(qhvp_problem* p, int on) {
  if (!p) return fail(QHVP_ERR_INVALID, "problem is NULL");
  HIP_TRY(hipSetDevice(p->ctx->device));
  HIP_TRY(prof_collect(p));   // launches timed before the reset are dropped with the statistics
  p->profiling = on ? 1 : 0;
  for (int k = 0; k < QHVP_KERNEL_KINDS; ++k) { p->k_ms[k] = p->k_bytes[k] = p->k_flops[k] = 0; p->k_count[k] = 0; }
  return QHVP_OK;
}

qhvp_status qhvp_kernel_stats(const qhvp_problem* p, int kind, double* total_ms, long long* launches,
                              double* alg_bytes, double* alg_flops) {
  if (!p || kind < 0 || kind >= QHVP_KERNEL_KINDS) return fail(QHVP_ERR_INVALID, "bad arguments");
  HIP_TRY(hipSetDevice(p->ctx->device));
  HIP_TRY(prof_collect(const_cast<qhvp_problem*>(p)));   // waits for the timed launches
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
