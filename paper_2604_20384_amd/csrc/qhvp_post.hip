// Per-call FP64 work on the device around the sweeps of one cost / gradient / HVP evaluation
// (arXiv 2604.20384): preparing the gates of a call (device precision, inverses, the tangent
// projection of App. F, the fixed-G check) and the post-processing of Alg. 2 (fidelity and cost over
// the samples, Eq. costHS; gradient and HVP from the environment sums, Eq. grad-costHS and Eq.
// hvp-costHS; the Riemannian projections of App. F).  Everything here is 4x4 arithmetic per gate or
// one sum over samples: one workgroup, fixed summation orders, so results are bitwise repeatable.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "qhvp_internal.h"

namespace qhvp {
namespace {

// Both kernels run one workgroup of kPostThreads threads; each thread keeps its 4x4 matrices in its
// own slab of LDS (kSlab complex numbers), so that no kernel here uses private (scratch) memory.
constexpr int kPostThreads = 32;
constexpr int kSlab = 240;

typedef double2 zd;
__device__ __forceinline__ zd zmk(double x, double y) { return make_double2(x, y); }
__device__ __forceinline__ zd zadd(zd a, zd b) { return zmk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ zd zsub(zd a, zd b) { return zmk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ zd zmul(zd a, zd b) { return zmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ zd zconj(zd a) { return zmk(a.x, -a.y); }
__device__ __forceinline__ zd zscale(double s, zd a) { return zmk(s * a.x, s * a.y); }
__device__ __forceinline__ double znorm(zd a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ zd zdiv(zd a, zd b) {
  const double d = znorm(b);
  return zmk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// 4x4 complex matrices, row-major: M[4 i + j]; c must not alias a or b
__device__ void mm4(const zd* a, const zd* b, zd* c) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      zd s = zmk(0, 0);
      for (int k = 0; k < 4; ++k) s = zadd(s, zmul(a[4 * i + k], b[4 * k + j]));
      c[4 * i + j] = s;
    }
}
__device__ void dag4(const zd* a, zd* b) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) b[4 * i + j] = zconj(a[4 * j + i]);
}
// P_G(X) = X/2 - G X^dag G / 2, the projection onto the tangent space of U(4) at G (App. F).
// tmp: 48 entries.
__device__ void project4(const zd* G, const zd* X, zd* out, zd* tmp) {
  zd *Xd = tmp, *t = tmp + 16, *u = tmp + 32;
  dag4(X, Xd);
  mm4(G, Xd, t);
  mm4(t, G, u);
  for (int i = 0; i < 16; ++i) out[i] = zsub(zscale(0.5, X[i]), zscale(0.5, u[i]));
}
// Riemannian HVP of App. F for a tangent direction V: P_G(H - V grad^dag G / 2 - G grad^dag V / 2).
// tmp: 144 entries.
__device__ void riem_hvp4(const zd* G, const zd* gr, const zd* H, const zd* V, zd* out, zd* tmp) {
  zd *grd = tmp, *t1 = tmp + 16, *t2 = tmp + 32, *t3 = tmp + 48, *t4 = tmp + 64, *in = tmp + 80;
  dag4(gr, grd);
  mm4(V, grd, t1);
  mm4(t1, G, t2);
  mm4(G, grd, t3);
  mm4(t3, V, t4);
  for (int i = 0; i < 16; ++i) in[i] = zsub(zsub(H[i], zscale(0.5, t2[i])), zscale(0.5, t4[i]));
  project4(G, in, out, tmp + 96);
}
// Gauss-Jordan inverse with partial pivoting; false if a pivot vanishes.  tmp: 32 entries (the
// augmented matrix [a | I], row r at tmp[8 r]).
__device__ bool inv4(const zd* a, zd* out, zd* m) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 8; ++j) m[8 * i + j] = j < 4 ? a[4 * i + j] : zmk(j - 4 == i ? 1.0 : 0.0, 0.0);
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (znorm(m[8 * r + c]) > znorm(m[8 * piv + c])) piv = r;
    if (!(znorm(m[8 * piv + c]) > 1e-300)) return false;
    if (piv != c)
      for (int j = 0; j < 8; ++j) { const zd t = m[8 * c + j]; m[8 * c + j] = m[8 * piv + j]; m[8 * piv + j] = t; }
    const zd d = m[8 * c + c];
    for (int j = 0; j < 8; ++j) m[8 * c + j] = zdiv(m[8 * c + j], d);
    for (int r = 0; r < 4; ++r)
      if (r != c) {
        const zd f = m[8 * r + c];
        for (int j = 0; j < 8; ++j) m[8 * r + j] = zsub(m[8 * r + j], zmul(f, m[8 * c + j]));
      }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) out[4 * i + j] = m[8 * i + j + 4];
  return true;
}
__device__ double fro4(const zd* a) {
  double s = 0;
  for (int i = 0; i < 16; ++i) s += znorm(a[i]);
  return sqrt(s);
}
// |G^dag G - I|_F; tmp: 32 entries
__device__ double unitarity_err4(const zd* G, zd* tmp) {
  zd *Gd = tmp, *P = tmp + 16;
  dag4(G, Gd);
  mm4(Gd, G, P);
  double e = 0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) e += znorm(zsub(P[4 * i + j], zmk(i == j ? 1.0 : 0.0, 0.0)));
  return sqrt(e);
}
__device__ void load4(const double* p, zd* m) {
  for (int i = 0; i < 16; ++i) m[i] = zmk(p[2 * i], p[2 * i + 1]);
}
__device__ void store4(const zd* m, double* p) {
  for (int i = 0; i < 16; ++i) { p[2 * i] = m[i].x; p[2 * i + 1] = m[i].y; }
}
__device__ bool finite16(const double* p) {
  bool ok = true;
  for (int i = 0; i < 32; ++i) ok = ok && isfinite(p[i]);
  return ok;
}
__device__ void store_prec(const zd* m, void* dst, int prec) {
  if (prec == P_C64) {
    float2* d = (float2*)dst;
    for (int i = 0; i < 16; ++i) d[i] = make_float2((float)m[i].x, (float)m[i].y);
  } else {
    double2* d = (double2*)dst;
    for (int i = 0; i < 16; ++i) d[i] = m[i];
  }
}

__global__ void __launch_bounds__(kPostThreads) k_prep(PrepArgs a) {
  __shared__ zd slab[kPostThreads][kSlab];
  __shared__ int sBad;
  const int tid = threadIdx.x;
  zd* G = slab[tid];
  zd* V = G + 16;
  zd* Gi = G + 32;
  zd* P = G + 48;
  zd* tmp = G + 64;   // 48 (projection), 32 (inverse, unitarity), 32 (t, Y)
  const size_t amp = a.prec == P_C64 ? 8 : 16;
  int bad = 0, inv_ok = 1, same = 1;
  if (tid == 0) sBad = 0;
  for (int k = tid; k < a.K; k += kPostThreads) {
    const double* gk = a.G_in + 32 * (size_t)k;
    if (!finite16(gk)) bad |= kStatNonFinite;
    load4(gk, G);
    if (a.tangent) {
      const double* vk = a.V_in + 32 * (size_t)k;
      if (!finite16(vk)) bad |= kStatNonFinite;
      load4(vk, V);
      if (a.riem) {
        project4(G, V, P, tmp);
        for (int i = 0; i < 16; ++i) V[i] = P[i];
      }
    } else {
      for (int i = 0; i < 16; ++i) V[i] = zmk(0, 0);
    }
    if (a.riem && !(unitarity_err4(G, tmp) <= 1e-10)) bad |= kStatNotUnitary;
    store_prec(G, (char*)a.gates + 16 * amp * (size_t)k, a.prec);
    if (a.tangent) store_prec(V, (char*)a.dirs + 16 * amp * (size_t)k, a.prec);
    store4(G, a.g64 + 32 * (size_t)k);
    store4(V, a.v64 + 32 * (size_t)k);
    if (a.with_inverse) {
      const bool ok = inv4(G, Gi, tmp) && fro4(G) * fro4(Gi) <= (a.rebuild ? kRebuildCond : kInverseCond);
      if (ok) {
        zd *t = tmp + 32, *Y = tmp + 48;
        mm4(Gi, V, t);
        mm4(t, Gi, Y);
        for (int i = 0; i < 16; ++i) Y[i] = zscale(-1.0, Y[i]);
        store4(Gi, a.gi64 + 32 * (size_t)k);
        store_prec(Gi, (char*)a.igates + 32 * amp * (size_t)k, a.prec);
        store_prec(Y, (char*)a.igates + 32 * amp * (size_t)k + 16 * amp, a.prec);
      } else {
        inv_ok = 0;
      }
    }
    if (a.keep_mode) {
      const double* kg = a.kept_g + 32 * (size_t)k;
      for (int i = 0; i < 32; ++i) same = same && __double_as_longlong(kg[i]) == __double_as_longlong(gk[i]);
    }
  }
  // one decision for the whole call (every thread has compared its gates before any copy below)
  const int any_bad = __syncthreads_or(bad);
  const int all_inv = __syncthreads_and(inv_ok);
  const int all_same = __syncthreads_and(same);
  if (bad) atomicOr(&sBad, bad);
  __syncthreads();
  if (a.keep_mode) {
    for (int k = tid; k < a.K; k += kPostThreads)
      for (int i = 0; i < 32; ++i) a.kept_g[32 * (size_t)k + i] = a.G_in[32 * (size_t)k + i];
  }
  if (tid == 0) {
    a.flags[kFlagInverse] = (a.with_inverse && all_inv) ? 1 : 0;
    a.flags[kFlagStatus] = (any_bad ? sBad : 0) | ((a.rebuild && !all_inv) ? kStatNotInvertible : 0);
    if (a.keep_mode) {
      a.flags[kFlagKeep] = (!a.invalidate_kept && a.flags[kFlagKeptValid] && all_same) ? 1 : 0;
      a.flags[kFlagKeptValid] = any_bad ? 0 : 1;
    }
  }
}

// Alg. 2 over samples (Eq. costHS): F = mean |T_s|^2, C = 1 - F.  With the folded backward boundary
// the environment sums are Ehat_k = sum_s conj(T_s) dT_s/dG_k and Dhat_k = sum_s conj(Omega_s)
// dT_s/dG_k + conj(T_s) D(dT_s/dG_k)[V], so grad C = -(2/N_s) conj(Ehat) and H(C)[V] =
// -(2/N_s) conj(Dhat) (the derivatives of the returned cost 1 - F).  Sums taken against pass-output
// states (backward from pass outputs) are first mapped back: E = Et G^-T, D = (Dt - E V^T) G^-T.
__global__ void __launch_bounds__(kPostThreads) k_post(PostArgs a) {
  __shared__ zd slab[kPostThreads][kSlab];
  __shared__ double red[kPostThreads];
  const int tid = threadIdx.x;
  if (a.flags[kFlagStatus] != 0) return;   // invalid inputs: every output is left as it was
  if (a.mode & kPostCost) {
    double f = 0;
    for (int s = tid; s < a.Ns; s += kPostThreads) f += a.tov[4 * s] * a.tov[4 * s] + a.tov[4 * s + 1] * a.tov[4 * s + 1];
    red[tid] = f;
    __syncthreads();
    for (int w = kPostThreads / 2; w >= 1; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) {
      const double F = red[0] / a.Ns;
      if (a.fidelity) *a.fidelity = F;
      if (a.cost) *a.cost = 1.0 - F;
    }
  }
  if (!(a.mode & kPostDeriv)) return;
  const bool mapped = a.flags[kFlagInverse] != 0;
  const double f = -2.0 / a.Ns;
  zd* E = slab[tid];      // then the gradient, in place
  zd* D = E + 16;         // then the HVP, in place
  zd* gi = E + 32;
  zd* v = E + 48;
  zd* Et = E + 64;
  zd* W = E + 80;
  zd* G = E + 32;         // Riemannian outputs (after the mapping is done with gi)
  zd* out = E + 64;
  zd* tmp = E + 96;       // 144
  for (int k = tid; k < a.K; k += kPostThreads) {
    const double* e = a.env + (size_t)k * kEnvVals;
    for (int i = 0; i < 16; ++i) {
      E[i] = zmk(e[2 * i], e[2 * i + 1]);
      D[i] = zmk(e[32 + 2 * i], e[32 + 2 * i + 1]);
    }
    if (mapped) {
      load4(a.gi64 + 32 * (size_t)k, gi);
      load4(a.v64 + 32 * (size_t)k, v);
      for (int i = 0; i < 16; ++i) Et[i] = E[i];
      for (int x = 0; x < 4; ++x)
        for (int y = 0; y < 4; ++y) {
          zd s = zmk(0, 0);
          for (int z = 0; z < 4; ++z) s = zadd(s, zmul(Et[4 * x + z], gi[4 * y + z]));
          E[4 * x + y] = s;
        }
      for (int x = 0; x < 4; ++x)
        for (int z = 0; z < 4; ++z) {
          zd w = D[4 * x + z];
          if (a.tangent)
            for (int u = 0; u < 4; ++u) w = zsub(w, zmul(E[4 * x + u], v[4 * z + u]));
          W[4 * x + z] = w;
        }
      for (int x = 0; x < 4; ++x)
        for (int y = 0; y < 4; ++y) {
          zd s = zmk(0, 0);
          for (int z = 0; z < 4; ++z) s = zadd(s, zmul(W[4 * x + z], gi[4 * y + z]));
          D[4 * x + y] = s;
        }
    }
    for (int i = 0; i < 16; ++i) {
      E[i] = zmk(f * E[i].x, -f * E[i].y);
      D[i] = zmk(f * D[i].x, -f * D[i].y);
    }
    if (a.riem) {
      load4(a.g64 + 32 * (size_t)k, G);
      if (a.grad) {
        project4(G, E, out, tmp);
        store4(out, a.grad + 32 * (size_t)k);
      }
      if (a.hvp && a.tangent) {
        load4(a.v64 + 32 * (size_t)k, v);
        riem_hvp4(G, E, D, v, out, tmp);
        store4(out, a.hvp + 32 * (size_t)k);
      }
    } else {
      if (a.grad) store4(E, a.grad + 32 * (size_t)k);
      if (a.hvp && a.tangent) store4(D, a.hvp + 32 * (size_t)k);
    }
  }
}

__global__ void k_convert(const double* __restrict__ src, void* dst, long long n_complex, int prec) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n_complex;
       i += (long long)gridDim.x * blockDim.x) {
    if (prec == P_C64) ((float2*)dst)[i] = make_float2((float)src[2 * i], (float)src[2 * i + 1]);
    else ((double2*)dst)[i] = make_double2(src[2 * i], src[2 * i + 1]);
  }
}

// Translationally invariant brickwalls (App. E): expansion of the layer gates and the per-layer sums.
__global__ void k_ti_expand(const double* __restrict__ layers, int n, int K, double* __restrict__ gates) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < K * 32; i += gridDim.x * blockDim.x)
    gates[i] = layers[32 * ti_layer_of(i >> 5, n) + (i & 31)];
}

// The derivative with respect to a layer gate is the sum of the derivatives with respect to the
// gates it stands for; one thread per real entry, the layer's gates added in increasing order.
__global__ void k_ti_reduce(const double* __restrict__ per_gate, int n, int L, const int* __restrict__ flags,
                            double* __restrict__ out) {
  if (flags[kFlagStatus] != 0) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < L * 32; i += gridDim.x * blockDim.x) {
    const int l = i >> 5, e = i & 31, k0 = ti_first_gate(l, n), cnt = ti_gate_count(l, n);
    double s = 0;
    for (int c = 0; c < cnt; ++c) s += per_gate[32 * (k0 + c) + e];
    out[i] = s;
  }
}

// The scratch of the entry point that allocates nothing: every problem evaluated through it lives
// here (labels, states, partial sums, flags).  Each device that loads the library holds its own copy
// of this array until the process ends; host code uses only the address looked up per device below,
// never the array's name.
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

}  // namespace

int noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return (int)hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return (int)e;
  g_scratch[device] = ptr;
  return (int)hipSuccess;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch[device];
}

int launch_convert(const double* src, void* dst, long long n_complex, int prec, void* stream) {
  if (n_complex <= 0) return (int)hipSuccess;
  const long long blocks = std::min<long long>((n_complex + 255) / 256, 1024);
  hipLaunchKernelGGL(k_convert, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, src, dst, n_complex, prec);
  return (int)hipGetLastError();
}

int launch_ti_expand(const double* layers, int n, int K, double* gates, void* stream) {
  if (K <= 0) return (int)hipSuccess;
  hipLaunchKernelGGL(k_ti_expand, dim3((unsigned)((K * 32 + 255) / 256)), dim3(256), 0, (hipStream_t)stream, layers, n, K,
                     gates);
  return (int)hipGetLastError();
}
int launch_ti_reduce(const double* per_gate, int n, int L, const int* flags, double* out, void* stream) {
  if (L <= 0) return (int)hipSuccess;
  hipLaunchKernelGGL(k_ti_reduce, dim3((unsigned)((L * 32 + 255) / 256)), dim3(256), 0, (hipStream_t)stream, per_gate, n, L,
                     flags, out);
  return (int)hipGetLastError();
}

int launch_prep(const PrepArgs& a, void* stream) {
  hipLaunchKernelGGL(k_prep, dim3(1), dim3(kPostThreads), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}
int launch_post(const PostArgs& a, void* stream) {
  hipLaunchKernelGGL(k_post, dim3(1), dim3(kPostThreads), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

}  // namespace qhvp
