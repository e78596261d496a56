// Per-call FP64 work on the device around the sweeps of one cost / gradient / HVP evaluation
// (arXiv 2604.20384): preparing the gates of a call (device precision, inverses, the tangent
// projection of App. F, the fixed-G check) and the post-processing of Alg. 2 (fidelity and cost over
// the samples, Eq. costHS; gradient and HVP from the environment sums, Eq. grad-costHS and Eq.
// hvp-costHS; the Riemannian projections of App. F).  Everything here is 4x4 arithmetic per gate or
// one sum over samples: one workgroup, fixed summation orders, so results are bitwise repeatable.
#include <hip/hip_runtime.h>

#include "qhvp_internal.h"

namespace qhvp {
namespace {

constexpr int kPostThreads = 256;

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

// 4x4 complex matrices, row-major: M[4 i + j]
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
// P_G(X) = X/2 - G X^dag G / 2, the projection onto the tangent space of U(4) at G (App. F)
__device__ void project4(const zd* G, const zd* X, zd* out) {
  zd Xd[16], t[16], u[16];
  dag4(X, Xd);
  mm4(G, Xd, t);
  mm4(t, G, u);
  for (int i = 0; i < 16; ++i) out[i] = zsub(zscale(0.5, X[i]), zscale(0.5, u[i]));
}
// Riemannian HVP of App. F for a tangent direction V: P_G(H - V grad^dag G / 2 - G grad^dag V / 2)
__device__ void riem_hvp4(const zd* G, const zd* gr, const zd* H, const zd* V, zd* out) {
  zd grd[16], t1[16], t2[16], t3[16], t4[16], in[16];
  dag4(gr, grd);
  mm4(V, grd, t1);
  mm4(t1, G, t2);
  mm4(G, grd, t3);
  mm4(t3, V, t4);
  for (int i = 0; i < 16; ++i) in[i] = zsub(zsub(H[i], zscale(0.5, t2[i])), zscale(0.5, t4[i]));
  project4(G, in, out);
}
// Gauss-Jordan inverse with partial pivoting; false if a pivot vanishes.
__device__ bool inv4(const zd* a, zd* out) {
  zd m[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 8; ++j) m[i][j] = j < 4 ? a[4 * i + j] : zmk(j - 4 == i ? 1.0 : 0.0, 0.0);
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (znorm(m[r][c]) > znorm(m[piv][c])) piv = r;
    if (!(znorm(m[piv][c]) > 1e-300)) return false;
    if (piv != c)
      for (int j = 0; j < 8; ++j) { const zd t = m[c][j]; m[c][j] = m[piv][j]; m[piv][j] = t; }
    const zd d = m[c][c];
    for (int j = 0; j < 8; ++j) m[c][j] = zdiv(m[c][j], d);
    for (int r = 0; r < 4; ++r)
      if (r != c) {
        const zd f = m[r][c];
        for (int j = 0; j < 8; ++j) m[r][j] = zsub(m[r][j], zmul(f, m[c][j]));
      }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) out[4 * i + j] = m[i][j + 4];
  return true;
}
__device__ double fro4(const zd* a) {
  double s = 0;
  for (int i = 0; i < 16; ++i) s += znorm(a[i]);
  return sqrt(s);
}
__device__ double unitarity_err4(const zd* G) {
  zd Gd[16], P[16];
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
  const int tid = threadIdx.x;
  const size_t amp = a.prec == P_C64 ? 8 : 16;
  int bad = 0, inv_ok = 1, same = 1;
  for (int k = tid; k < a.K; k += kPostThreads) {
    const double* gk = a.G_in + 32 * (size_t)k;
    zd G[16], V[16], Gi[16];
    if (!finite16(gk)) bad |= kStatNonFinite;
    load4(gk, G);
    if (a.tangent) {
      const double* vk = a.V_in + 32 * (size_t)k;
      if (!finite16(vk)) bad |= kStatNonFinite;
      load4(vk, V);
      if (a.riem) {
        zd P[16];
        project4(G, V, P);
        for (int i = 0; i < 16; ++i) V[i] = P[i];
      }
    } else {
      for (int i = 0; i < 16; ++i) V[i] = zmk(0, 0);
    }
    if (a.riem && !(unitarity_err4(G) <= 1e-10)) bad |= kStatNotUnitary;
    store_prec(G, (char*)a.gates + 16 * amp * (size_t)k, a.prec);
    if (a.tangent) store_prec(V, (char*)a.dirs + 16 * amp * (size_t)k, a.prec);
    store4(G, a.g64 + 32 * (size_t)k);
    store4(V, a.v64 + 32 * (size_t)k);
    if (a.with_inverse) {
      const bool ok = inv4(G, Gi) && fro4(G) * fro4(Gi) <= kInverseCond;
      if (ok) {
        zd t[16], Y[16];
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
  __shared__ int sBad;
  if (tid == 0) sBad = 0;
  __syncthreads();
  if (bad) atomicOr(&sBad, bad);
  __syncthreads();
  if (a.keep_mode) {
    for (int k = tid; k < a.K; k += kPostThreads)
      for (int i = 0; i < 32; ++i) a.kept_g[32 * (size_t)k + i] = a.G_in[32 * (size_t)k + i];
  }
  if (tid == 0) {
    a.flags[kFlagInverse] = (a.with_inverse && all_inv) ? 1 : 0;
    a.flags[kFlagStatus] = any_bad ? sBad : 0;
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
  const int tid = threadIdx.x;
  if (a.flags[kFlagStatus] != 0) return;   // invalid inputs: every output is left as it was
  if (a.mode & kPostCost) {
    __shared__ double red[kPostThreads];
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
  for (int k = tid; k < a.K; k += kPostThreads) {
    const double* e = a.env + (size_t)k * kEnvVals;
    zd E[16], D[16], gr[16], H[16];
    for (int i = 0; i < 16; ++i) {
      E[i] = zmk(e[2 * i], e[2 * i + 1]);
      D[i] = zmk(e[32 + 2 * i], e[32 + 2 * i + 1]);
    }
    if (mapped) {
      zd gi[16], v[16], Et[16], W[16];
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
      gr[i] = zmk(f * E[i].x, -f * E[i].y);
      H[i] = zmk(f * D[i].x, -f * D[i].y);
    }
    if (a.riem) {
      zd G[16], out[16];
      load4(a.g64 + 32 * (size_t)k, G);
      if (a.grad) {
        project4(G, gr, out);
        store4(out, a.grad + 32 * (size_t)k);
      }
      if (a.hvp && a.tangent) {
        zd v[16];
        load4(a.v64 + 32 * (size_t)k, v);
        riem_hvp4(G, gr, H, v, out);
        store4(out, a.hvp + 32 * (size_t)k);
      }
    } else {
      if (a.grad) store4(gr, a.grad + 32 * (size_t)k);
      if (a.hvp && a.tangent) store4(H, a.hvp + 32 * (size_t)k);
    }
  }
}

}  // namespace

int launch_prep(const PrepArgs& a, void* stream) {
  hipLaunchKernelGGL(k_prep, dim3(1), dim3(kPostThreads), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}
int launch_post(const PostArgs& a, void* stream) {
  hipLaunchKernelGGL(k_post, dim3(1), dim3(kPostThreads), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

}  // namespace qhvp
