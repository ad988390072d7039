// Learned coarse correction of the FGMRES preconditioner.  The paper's outer
// solver is flexible GMRES (Sec. 4.2), which accepts a preconditioner that
// changes between steps; this stage adds to the plain multi-level
// preconditioner z_p = P(v) a coarse correction P_c f(R_c v), where
//   R_c  restricts a trace vector to the multilinear functions of each macro
//        face (discrete L2 projection, per face and component),
//   f    is a two-layer network applied per macro to its 2d faces' coarse
//        coefficients, normalised to unit length on input and scaled back on
//        output (homogeneous of degree one), trained to map R_c v to
//        R_c (A-hat^{-1} v - z_p),
//   P_c  evaluates the coarse functions at the face nodes, averaged over the
//        macros that own a face.
// Training (FP32): forward, mean-squared loss in normalised units, backward
// and Adam, all in the kernels below.  Inference inside FGMRES uses a BF16
// copy of the weights with FP32 accumulation.
#include "context.h"
#include <algorithm>

namespace {

constexpr int DT = 32;  // output tile of the dense kernel (DT x DT per workgroup)

__device__ __forceinline__ unsigned short f2bf(float f) {  // round to nearest even
  unsigned int u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned int)b << 16); }

__device__ __forceinline__ float wave_sumf(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// C[i][j] = sum_k A(i, k) B(k, j) (+ bias[j], then tanh if act == 1) for an
// M x N output; A(i, k) = A[i * a_i + k * a_k], B(k, j) = B[k * b_k + j * b_j];
// C row-major with leading dimension N.  act: 0 plain, 1 bias + tanh, 2 bias.
__global__ void __launch_bounds__(256) k_dense(int M, int N, int K, const float* __restrict__ A, long long a_i,
                                               long long a_k, const float* __restrict__ B, long long b_k,
                                               long long b_j, const float* __restrict__ bias, int act,
                                               float* __restrict__ C) {
  __shared__ float sA[DT][DT + 1];
  __shared__ float sB[DT][DT + 1];
  const int i0 = blockIdx.y * DT, j0 = blockIdx.x * DT;
  const int tx = threadIdx.x % DT, ty = threadIdx.x / DT;  // ty in [0, 8): rows ty + 8 r
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += DT) {
    for (int e = threadIdx.x; e < DT * DT; e += 256) {
      const int r = e / DT, c = e % DT;
      sA[r][c] = (i0 + r < M && k0 + c < K) ? A[(i0 + r) * a_i + (long long)(k0 + c) * a_k] : 0.f;
      sB[r][c] = (k0 + r < K && j0 + c < N) ? B[(long long)(k0 + r) * b_k + (j0 + c) * b_j] : 0.f;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < DT; ++k) {
      const float b = sB[k][tx];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] += sA[ty + 8 * r][k] * b;
    }
    __syncthreads();
  }
  const int j = j0 + tx;
  if (j >= N) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + ty + 8 * r;
    if (i >= M) continue;
    float v = acc[r];
    if (act >= 1) v += bias[j];
    if (act == 1) v = tanhf(v);
    C[(size_t)i * N + j] = v;
  }
}

// Row b of the batch (source row idx[b] or b): s = ||X||, Xn = X / s (0 if s = 0),
// Tn = T / s when T is given.
__global__ void k_mlp_prep(int batch, int n_in, int n_out, const float* __restrict__ X, const float* __restrict__ T,
                           const int* __restrict__ idx, float* __restrict__ Xn, float* __restrict__ Tn,
                           float* __restrict__ S) {
  const int b = blockIdx.x;
  if (b >= batch) return;
  const long long r = idx ? idx[b] : b;
  __shared__ float red[4];
  float ss = 0.f;
  for (int k = threadIdx.x; k < n_in; k += blockDim.x) {
    const float v = X[r * n_in + k];
    ss += v * v;
  }
  ss = wave_sumf(ss);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
  __syncthreads();
  const float s = sqrtf(red[0] + red[1] + red[2] + red[3]);
  const float inv = s > 0.f ? 1.f / s : 0.f;
  for (int k = threadIdx.x; k < n_in; k += blockDim.x) Xn[(size_t)b * n_in + k] = X[r * n_in + k] * inv;
  if (T)
    for (int k = threadIdx.x; k < n_out; k += blockDim.x) Tn[(size_t)b * n_out + k] = T[r * n_out + k] * inv;
  if (threadIdx.x == 0) S[b] = s;
}

// R = Y - Tn; dY = 2 R / (batch n_out); per-block partial sums of R^2.
__global__ void k_mlp_loss(long long n, float scale, const float* __restrict__ Y, const float* __restrict__ Tn,
                           float* __restrict__ dY, float* __restrict__ partial) {
  __shared__ float red[4];
  float ss = 0.f;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float r = Y[i] - Tn[i];
    dY[i] = 2.f * scale * r;
    ss += r * r;
  }
  ss = wave_sumf(ss);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_mlp_loss_final(int nblk, float scale, const float* __restrict__ partial, float* __restrict__ loss) {
  float s = 0.f;
  for (int b = threadIdx.x; b < nblk; b += 64) s += partial[b];
  s = wave_sumf(s);
  if (threadIdx.x == 0) loss[0] = s * scale;
}

// dZ = dH (1 - H^2)
__global__ void k_tanh_back(long long n, const float* __restrict__ H, float* __restrict__ dH) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dH[i] *= 1.f - H[i] * H[i];
}

// out[j] = sum_b M[b][j]
__global__ void k_colsum(int rows, int cols, const float* __restrict__ Mt, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int b = 0; b < rows; ++b) s += Mt[(size_t)b * cols + j];
  out[j] = s;
}

// Y[b] = S[b] * Yn[b] (physical units)
__global__ void k_rescale(int batch, int n_out, const float* __restrict__ Yn, const float* __restrict__ S,
                          float* __restrict__ Y) {
  const long long n = (long long)batch * n_out;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    Y[i] = Yn[i] * S[i / n_out];
}

__global__ void k_adam(long long n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ void k_to_bf16(long long n, const float* __restrict__ p, unsigned short* __restrict__ q) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    q[i] = f2bf(p[i]);
}

// Per macro: X[macro][(lf ns + c) cq + a] = sum_j cR[k][a][j] v[face(lf)][c][j].
__global__ void k_coarse_restrict(MeshDev md, const double* __restrict__ v, float* __restrict__ X) {
  const int macro = blockIdx.x;
  const ClassDev& cd = class_of(md, macro);
  const int d = cd.dim, ns = cd.ns, cq = cd.cq;
  for (int f = threadIdx.x; f < cd.cF; f += blockDim.x) {
    const int lf = f / (ns * cq), c = (f / cq) % ns, a = f % cq;
    const int k = lf / 2;
    const int F = md.macro_face[(size_t)macro * 2 * d + lf];
    const int nn = cd.nf_nodes[lf];
    const double* seg = v + md.face_off[F] + (size_t)c * nn;
    const double* R = cd.cR + ((size_t)k * cq + a) * cd.cmaxf;
    double s = 0.0;
    for (int j = 0; j < nn; ++j) s += R[j] * seg[j];
    X[(size_t)macro * cd.cF + f] = (float)s;
  }
}

// z[g] += alpha * mean over the owning macros of sum_a cPhi[k][j][a] Y[macro][(lf ns + c) cq + a]
__global__ void k_coarse_prolong(MeshDev md, const float* __restrict__ Y, double alpha, double* __restrict__ z) {
  const int d = md.dim, ns = md.ns;
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < md.n_glob;
       g += (long long)gridDim.x * blockDim.x) {
    int lo = 0, hi = md.n_faces - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (md.face_off[mid] <= g) lo = mid; else hi = mid - 1;
    }
    const int F = lo;
    const int r = (int)(g - md.face_off[F]);
    const int mm = md.face_minus[F], mp = md.face_plus[F];
    const int m0 = mm >= 0 ? mm : mp;
    int k = 0;
    for (int lf = 0; lf < 2 * d; ++lf)
      if (md.macro_face[(size_t)m0 * 2 * d + lf] == F) { k = lf / 2; break; }
    const ClassDev& cd = class_of(md, m0);  // both sides see the same face grid
    const int cq = cd.cq;
    const int nn = cd.nf_nodes[2 * k];
    const int c = r / nn, j = r % nn;
    const double* phi = cd.cPhi + ((size_t)k * cd.cmaxf + j) * cq;
    double s = 0.0;
    int cnt = 0;
    if (mm >= 0) {
      const float* y = Y + (size_t)mm * cd.cF + ((2 * k + 1) * ns + c) * cq;
      for (int a = 0; a < cq; ++a) s += phi[a] * (double)y[a];
      ++cnt;
    }
    if (mp >= 0) {
      const float* y = Y + (size_t)mp * cd.cF + ((2 * k) * ns + c) * cq;
      for (int a = 0; a < cq; ++a) s += phi[a] * (double)y[a];
      ++cnt;
    }
    z[g] += alpha * s / cnt;
  }
}

// Xe[macro] = [X[macro] | X[macro across local face lf] for lf = 0 .. 2d-1],
// zeros across a face on the domain boundary.
__global__ void k_coarse_neighbours(MeshDev md, int F, const float* __restrict__ X, float* __restrict__ Xe) {
  const int macro = blockIdx.x, d = md.dim, nin = (1 + 2 * d) * F;
  for (int x = threadIdx.x; x < nin; x += blockDim.x) {
    const int blk = x / F, f = x % F;
    int src = macro;
    if (blk > 0) {
      const int lf = blk - 1;
      const int Fc = md.macro_face[(size_t)macro * 2 * d + lf];
      src = (lf % 2 == 1) ? md.face_plus[Fc] : md.face_minus[Fc];
    }
    Xe[(size_t)macro * nin + x] = src >= 0 ? X[(size_t)src * F + f] : 0.f;
  }
}

// Inference with BF16 weights, one workgroup per macro (row of X):
// y = ||x|| (W2 tanh(W1 x / ||x|| + b1) + b2).
__global__ void __launch_bounds__(256) k_learned_infer(int n_in, int n_hidden, int n_out,
                                                       const unsigned short* __restrict__ Wq, const float* __restrict__ X,
                                                       float* __restrict__ Y) {
  extern __shared__ float sh[];
  float* xs = sh;              // n_in
  float* hs = sh + n_in;       // n_hidden
  __shared__ float red[4];
  const int row = blockIdx.x;
  const unsigned short* W1 = Wq;
  const unsigned short* b1 = W1 + (size_t)n_hidden * n_in;
  const unsigned short* W2 = b1 + n_hidden;
  const unsigned short* b2 = W2 + (size_t)n_out * n_hidden;
  float ss = 0.f;
  for (int k = threadIdx.x; k < n_in; k += blockDim.x) {
    const float v = X[(size_t)row * n_in + k];
    xs[k] = v;
    ss += v * v;
  }
  ss = wave_sumf(ss);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
  __syncthreads();
  const float s = sqrtf(red[0] + red[1] + red[2] + red[3]);
  const float inv = s > 0.f ? 1.f / s : 0.f;
  for (int h = threadIdx.x; h < n_hidden; h += blockDim.x) {
    float a = bf2f(b1[h]);
    for (int k = 0; k < n_in; ++k) a += bf2f(W1[(size_t)h * n_in + k]) * xs[k] * inv;
    hs[h] = tanhf(a);
  }
  __syncthreads();
  for (int o = threadIdx.x; o < n_out; o += blockDim.x) {
    float a = bf2f(b2[o]);
    for (int h = 0; h < n_hidden; ++h) a += bf2f(W2[(size_t)o * n_hidden + h]) * hs[h];
    Y[(size_t)row * n_out + o] = a * s;
  }
}

inline unsigned grid1(long long n) { return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 2048)); }

void dense(hipStream_t s, int M, int N, int K, const float* A, long long a_i, long long a_k, const float* B,
           long long b_k, long long b_j, const float* bias, int act, float* C) {
  dim3 grid((N + DT - 1) / DT, (M + DT - 1) / DT);
  hipLaunchKernelGGL(k_dense, grid, dim3(256), 0, s, M, N, K, A, a_i, a_k, B, b_k, b_j, bias, act, C);
}

}  // namespace

// ---- launchers --------------------------------------------------------------

size_t mlp_param_count(int n_in, int n_hidden, int n_out) {
  return (size_t)n_hidden * n_in + n_hidden + (size_t)n_out * n_hidden + n_out;
}

size_t mlp_work_floats(int n_in, int n_hidden, int n_out, int max_batch) {
  return (size_t)max_batch * (n_in + 3 * n_out + 2 * n_hidden + 1) + 4096;
}

hipError_t launch_coarse_restrict(HdgContext& c, const double* v, float* X) {
  hipLaunchKernelGGL(k_coarse_restrict, dim3(c.hm.n_macros), dim3(128), 0, c.stream, c.md, v, X);
  return hipGetLastError();
}

hipError_t launch_coarse_neighbours(HdgContext& c, const float* X, float* Xe) {
  hipLaunchKernelGGL(k_coarse_neighbours, dim3(c.hm.n_macros), dim3(128), 0, c.stream, c.md, c.cd.cF, X, Xe);
  return hipGetLastError();
}

hipError_t launch_coarse_prolong(HdgContext& c, const float* Y, double alpha, double* z) {
  hipLaunchKernelGGL(k_coarse_prolong, dim3(grid1(c.md.n_glob)), dim3(256), 0, c.stream, c.md, Y, alpha, z);
  return hipGetLastError();
}

// Work layout for a batch of B rows: Xn [B][n_in] | Tn [B][n_out] | H [B][n_hidden] |
// Yn [B][n_out] | dY [B][n_out] | dH [B][n_hidden] | S [B] | partial [4096].
struct MlpWork {
  float *Xn, *Tn, *H, *Yn, *dY, *dH, *S, *partial;
};
static MlpWork carve(float* w, int n_in, int n_hidden, int n_out, int B) {
  MlpWork m;
  m.Xn = w; w += (size_t)B * n_in;
  m.Tn = w; w += (size_t)B * n_out;
  m.H = w; w += (size_t)B * n_hidden;
  m.Yn = w; w += (size_t)B * n_out;
  m.dY = w; w += (size_t)B * n_out;
  m.dH = w; w += (size_t)B * n_hidden;
  m.S = w; w += B;
  m.partial = w;
  return m;
}

hipError_t launch_mlp_forward(hipStream_t s, int n_in, int n_hidden, int n_out, const float* params, float* work,
                              const float* X, const int* idx, int batch, float* Y) {
  MlpWork m = carve(work, n_in, n_hidden, n_out, batch);
  const float* W1 = params;
  const float* b1 = W1 + (size_t)n_hidden * n_in;
  const float* W2 = b1 + n_hidden;
  const float* b2 = W2 + (size_t)n_out * n_hidden;
  hipLaunchKernelGGL(k_mlp_prep, dim3(batch), dim3(256), 0, s, batch, n_in, n_out, X, nullptr, idx, m.Xn, m.Tn, m.S);
  dense(s, batch, n_hidden, n_in, m.Xn, n_in, 1, W1, 1, n_in, b1, 1, m.H);
  dense(s, batch, n_out, n_hidden, m.H, n_hidden, 1, W2, 1, n_hidden, b2, 2, m.Yn);
  hipLaunchKernelGGL(k_rescale, dim3(grid1((long long)batch * n_out)), dim3(256), 0, s, batch, n_out, m.Yn, m.S, Y);
  return hipGetLastError();
}

hipError_t launch_mlp_loss_grad(hipStream_t s, int n_in, int n_hidden, int n_out, const float* params, float* grads,
                                float* work, const float* X, const float* T, const int* idx, int batch, float* loss) {
  MlpWork m = carve(work, n_in, n_hidden, n_out, batch);
  const float* W1 = params;
  const float* b1 = W1 + (size_t)n_hidden * n_in;
  const float* W2 = b1 + n_hidden;
  const float* b2 = W2 + (size_t)n_out * n_hidden;
  float* gW1 = grads;
  float* gb1 = gW1 + (size_t)n_hidden * n_in;
  float* gW2 = gb1 + n_hidden;
  float* gb2 = gW2 + (size_t)n_out * n_hidden;
  hipLaunchKernelGGL(k_mlp_prep, dim3(batch), dim3(256), 0, s, batch, n_in, n_out, X, T, idx, m.Xn, m.Tn, m.S);
  dense(s, batch, n_hidden, n_in, m.Xn, n_in, 1, W1, 1, n_in, b1, 1, m.H);         // H = tanh(Xn W1^T + b1)
  dense(s, batch, n_out, n_hidden, m.H, n_hidden, 1, W2, 1, n_hidden, b2, 2, m.Yn);  // Yn = H W2^T + b2
  const long long ny = (long long)batch * n_out;
  const float scale = 1.f / (float)ny;
  const unsigned nblk = std::min<unsigned>(grid1(ny), 1024);
  hipLaunchKernelGGL(k_mlp_loss, dim3(nblk), dim3(256), 0, s, ny, scale, m.Yn, m.Tn, m.dY, m.partial);
  if (loss) hipLaunchKernelGGL(k_mlp_loss_final, dim3(1), dim3(64), 0, s, (int)nblk, scale, m.partial, loss);
  dense(s, n_out, n_hidden, batch, m.dY, 1, n_out, m.H, n_hidden, 1, nullptr, 0, gW2);  // dW2 = dY^T H
  hipLaunchKernelGGL(k_colsum, dim3((n_out + 255) / 256), dim3(256), 0, s, batch, n_out, m.dY, gb2);
  dense(s, batch, n_hidden, n_out, m.dY, n_out, 1, W2, n_hidden, 1, nullptr, 0, m.dH);  // dH = dY W2
  hipLaunchKernelGGL(k_tanh_back, dim3(grid1((long long)batch * n_hidden)), dim3(256), 0, s,
                     (long long)batch * n_hidden, m.H, m.dH);
  dense(s, n_hidden, n_in, batch, m.dH, 1, n_hidden, m.Xn, n_in, 1, nullptr, 0, gW1);  // dW1 = dZ^T Xn
  hipLaunchKernelGGL(k_colsum, dim3((n_hidden + 255) / 256), dim3(256), 0, s, batch, n_hidden, m.dH, gb1);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(hipStream_t s, long long n, float* p, const float* g, float* m, float* v, float lr,
                           float b1, float b2, float eps, int t) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(grid1(n)), dim3(256), 0, s, n, p, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_to_bf16(hipStream_t s, long long n, const float* p, unsigned short* q) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1(n)), dim3(256), 0, s, n, p, q);
  return hipGetLastError();
}

// BF16 network of the learned stage inside the workspace: after X, Y and Xe
const unsigned short* learned_weights(const HdgContext& c) {
  const size_t F = (size_t)c.cd.cF, nm = (size_t)c.hm.n_macros;
  return reinterpret_cast<const unsigned short*>(c.ws.lrn + (2 + 1 + 2 * (size_t)c.cd.dim) * nm * F);
}

// z += P_c f(R_c v) with the bound BF16 network; X, Y: [n_macros][cF] and
// Xe: [n_macros][(1 + 2d) cF] scratch (the neighbour features, when the
// network takes them).
hipError_t launch_learned_correction(HdgContext& c, const double* v, double* z) {
  const int F = c.cd.cF;
  float* X = c.ws.lrn;
  float* Y = X + (size_t)c.hm.n_macros * F;
  float* Xe = Y + (size_t)c.hm.n_macros * F;
  hipError_t e = launch_coarse_restrict(c, v, X);
  if (e != hipSuccess) return e;
  const float* in = X;
  if (c.lrn_in != F) {
    if ((e = launch_coarse_neighbours(c, X, Xe)) != hipSuccess) return e;
    in = Xe;
  }
  const size_t shm = sizeof(float) * (c.lrn_in + c.lrn_hidden);
  hipLaunchKernelGGL(k_learned_infer, dim3(c.hm.n_macros), dim3(256), shm, c.stream, c.lrn_in, c.lrn_hidden, F,
                     learned_weights(c), in, Y);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_coarse_prolong(c, Y, 1.0, z);
}
