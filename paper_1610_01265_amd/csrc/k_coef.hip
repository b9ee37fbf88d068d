// Coefficient setup: lagged Spitzer diffusivity, face / edge weights,
// Dirichlet face weights, the operator diagonal and Gershgorin row sums.
#include "k_common.h"

namespace sts {

namespace {

constexpr int TX = 64, TY = 4;

__device__ __forceinline__ double spitzer_kappa(double T, double kappa0) {
  // kappa0 T^{5/2}: the lagged conduction coefficient (Eq. mhd:e1)
  return kappa0 * T * T * sqrt(T);
}

template <class TI>
struct SpitzerIn {
  const TI *T, *b0, *b1, *b2;
  double kappa0;
  __device__ __forceinline__ void D(int c, double &d00, double &d11, double &d22, double &d01,
                                    double &d02, double &d12) const {
    const double kap = spitzer_kappa((double)T[c], kappa0);
    const double x = (double)b0[c], y = (double)b1[c], z = (double)b2[c];
    d00 = kap * x * x;
    d11 = kap * y * y;
    d22 = kap * z * z;
    d01 = kap * x * y;
    d02 = kap * x * z;
    d12 = kap * y * z;
  }
  __device__ __forceinline__ double Dab(int c, int a, int b) const {
    const double kap = spitzer_kappa((double)T[c], kappa0);
    const TI *p[3] = {b0, b1, b2};
    return kap * (double)p[a][c] * (double)p[b][c];
  }
};

// w_a(c) = A_a Dbar_aa / dl_a on the +a face; K_ab(c) = W_e Dbar_ab on the
// edge with origin c (W_e, Dbar_ab: means over the edge's four cells).
template <class TI>
__global__ void __launch_bounds__(TX *TY) k_spitzer_coef(Grid g, SpitzerIn<TI> in, double *w0,
                                                         double *w1, double *w2, double *k01,
                                                         double *k02, double *k12) {
  const int k = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int i = blockIdx.z;
  if (k >= g.n2 || j >= g.n1) return;
  const Nb A = nbr(i, g.n0, g.per0), B = nbr(j, g.n1, g.per1), Cn = nbr(k, g.n2, g.per2);
  const int c = lin(g, i, j, k);
  const int cp0 = lin(g, A.p, j, k), cp1 = lin(g, i, B.p, k), cp2 = lin(g, i, j, Cn.p);
  double d00, d11, d22, d01, d02, d12;
  in.D(c, d00, d11, d22, d01, d02, d12);
  // faces (il* are zero where the + face does not exist)
  w0[c] = area0(g, i, j, k) * 0.5 * (d00 + in.Dab(cp0, 0, 0)) * il0(g, i);
  w1[c] = area1(g, i, j, k) * 0.5 * (d11 + in.Dab(cp1, 1, 1)) * il1(g, i, j);
  w2[c] = area2(g, i, j, k) * 0.5 * (d22 + in.Dab(cp2, 2, 2)) * il2(g, i, j, k);
  const double v = vol(g, i, j, k);
  // edge (0, 1)
  {
    double K = 0.0;
    if (A.hp && B.hp) {
      const int c11 = lin(g, A.p, B.p, k);
      const double W =
          0.25 * (v + vol(g, A.p, j, k) + vol(g, i, B.p, k) + vol(g, A.p, B.p, k));
      const double Db =
          0.25 * (d01 + in.Dab(cp0, 0, 1) + in.Dab(cp1, 0, 1) + in.Dab(c11, 0, 1));
      K = W * Db;
    }
    k01[c] = K;
  }
  // edge (0, 2)
  {
    double K = 0.0;
    if (A.hp && Cn.hp) {
      const int c11 = lin(g, A.p, j, Cn.p);
      const double W =
          0.25 * (v + vol(g, A.p, j, k) + vol(g, i, j, Cn.p) + vol(g, A.p, j, Cn.p));
      const double Db =
          0.25 * (d02 + in.Dab(cp0, 0, 2) + in.Dab(cp2, 0, 2) + in.Dab(c11, 0, 2));
      K = W * Db;
    }
    k02[c] = K;
  }
  // edge (1, 2)
  {
    double K = 0.0;
    if (B.hp && Cn.hp) {
      const int c11 = lin(g, i, B.p, Cn.p);
      const double W =
          0.25 * (v + vol(g, i, B.p, k) + vol(g, i, j, Cn.p) + vol(g, i, B.p, Cn.p));
      const double Db =
          0.25 * (d12 + in.Dab(cp1, 1, 2) + in.Dab(cp2, 1, 2) + in.Dab(c11, 1, 2));
      K = W * Db;
    }
    k12[c] = K;
  }
}

// Dirichlet face weight w_b = A_b D_00(c) / (distance centre -> face) on the
// axis-0 boundary layers; D_00 = kappa b_0^2 (conduction) or nu (isotropic).
template <class TI>
__global__ void k_dirichlet_w(Grid g, int op, const TI *T, const TI *b0, double kappa0,
                              double nu, double *wb_lo, double *wb_hi) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= g.n1 * g.n2) return;
  const int j = t / g.n2, k = t % g.n2;
  const double a = T1(g, T_A01, j) * T2(g, T_A02, k);
  for (int side = 0; side < 2; ++side) {
    const int i = side ? g.n0 - 1 : 0;
    double d = nu;
    if (op == OP_SPITZER) {
      const int c = lin(g, i, j, k);
      d = spitzer_kappa((double)T[c], kappa0) * (double)b0[c] * (double)b0[c];
    }
    const double w = (side ? g.ab_hi : g.ab_lo) * a * d / (side ? g.db_hi : g.db_lo);
    (side ? wb_hi : wb_lo)[t] = w;
  }
}

template <int OP>
__global__ void __launch_bounds__(TX *TY) k_sdiag(Grid g, Coef C, double *sdiag) {
  const int k = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int i = blockIdx.z;
  if (k >= g.n2 || j >= g.n1) return;
  double row[27];
  row27<OP>(g, C, i, j, k, row);
  sdiag[lin(g, i, j, k)] = row[13];
}

// Per-workgroup maximum of sum_j |S_cj| / V_c.
template <int OP>
__global__ void __launch_bounds__(TX *TY) k_gershgorin(Grid g, Coef C, double *part) {
  const int k = blockIdx.x * TX + threadIdx.x;
  const int j = blockIdx.y * TY + threadIdx.y;
  const int i = blockIdx.z;
  double s = 0.0;
  if (k < g.n2 && j < g.n1) {
    double row[27];
    row27<OP>(g, C, i, j, k, row);
#pragma unroll
    for (int t = 0; t < 27; ++t) s += fabs(row[t]);
    s /= vol(g, i, j, k);
  }
  __shared__ double red[TX * TY];
  const int tid = threadIdx.y * TX + threadIdx.x;
  red[tid] = s;
  __syncthreads();
  for (int h = TX * TY / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  if (tid == 0)
    part[(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_fill(double *p, long long n, double v) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

__global__ void k_to_f32(const double *__restrict__ a, float *__restrict__ b, long long n) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) b[t] = (float)a[t];
}

// flag |= 1 if any T is not finite and positive or any b is not finite
template <class TI>
__global__ void k_check_spitzer(long long n, const TI *T, const TI *b0, const TI *b1,
                                const TI *b2, int *flag) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double x = (double)T[t];
  const bool ok = isfinite(x) && x > 0.0 && isfinite((double)b0[t]) && isfinite((double)b1[t]) &&
                  isfinite((double)b2[t]);
  if (!ok) atomicOr(flag, 1);
}

dim3 grid3(const sts_ctx *c) {
  return dim3((c->n2 + TX - 1) / TX, (c->n1 + TY - 1) / TY, c->n0);
}

}  // namespace

template <class TI>
void spitzer_coef(const sts_ctx *c, const TI *T, double kappa0, const TI *b0, const TI *b1,
                  const TI *b2) {
  const long long n = c->ncell;
  SpitzerIn<TI> in{T, b0, b1, b2, kappa0};
  double *w = c->d_w;
  hipLaunchKernelGGL(k_spitzer_coef<TI>, grid3(c), dim3(TX, TY), 0, c->stream, c->grid(), in, w,
                     w + n, w + 2 * n, w + 3 * n, w + 4 * n, w + 5 * n);
  const int nb = c->n1 * c->n2;
  hipLaunchKernelGGL(k_dirichlet_w<TI>, dim3((nb + 255) / 256), dim3(256), 0, c->stream,
                     c->grid(), (int)OP_SPITZER, T, b0, kappa0, 0.0, c->d_bnd, c->d_bnd + nb);
}

void launch_spitzer_coef(const sts_ctx *c, const double *T, double kappa0, const double *b0,
                         const double *b1, const double *b2) {
  STS_PROF(c, "launch_spitzer_coef");
  spitzer_coef<double>(c, T, kappa0, b0, b1, b2);
}

void launch_spitzer_coef_f32(const sts_ctx *c, const float *T, double kappa0, const float *b0,
                             const float *b1, const float *b2) {
  STS_PROF(c, "launch_spitzer_coef_f32");
  spitzer_coef<float>(c, T, kappa0, b0, b1, b2);
  const long long n = 6 * c->ncell;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, c->d_w,
                     c->d_wf, n);
}

void launch_dirichlet_weights(const sts_ctx *c) {
  STS_PROF(c, "launch_dirichlet_weights");
  // isotropic operator: weights from geometry and nu only
  const int nb = c->n1 * c->n2;
  hipLaunchKernelGGL(k_dirichlet_w<double>, dim3((nb + 255) / 256), dim3(256), 0, c->stream,
                     c->grid(), (int)OP_ISOTROPIC, (const double *)nullptr,
                     (const double *)nullptr, 0.0, c->nu, c->d_bnd, c->d_bnd + nb);
}

void launch_sdiag(const sts_ctx *c) {
  STS_PROF(c, "launch_sdiag");
  if (c->op == OP_SPITZER)
    hipLaunchKernelGGL(k_sdiag<OP_SPITZER>, grid3(c), dim3(TX, TY), 0, c->stream, c->grid(),
                       c->coef(), c->d_sdiag);
  else
    hipLaunchKernelGGL(k_sdiag<OP_ISOTROPIC>, grid3(c), dim3(TX, TY), 0, c->stream, c->grid(),
                       c->coef(), c->d_sdiag);
}

void launch_fill(const sts_ctx *c, double *p, long long n, double v) {
  STS_PROF(c, "launch_fill");
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, p, n, v);
}

void launch_check_spitzer(const sts_ctx *c, const double *T, const double *b0, const double *b1,
                          const double *b2, int *flag) {
  STS_PROF(c, "launch_check_spitzer");
  const long long n = c->ncell;
  hipLaunchKernelGGL(k_check_spitzer<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     c->stream, n, T, b0, b1, b2, flag);
}

void launch_check_spitzer_f32(const sts_ctx *c, const float *T, const float *b0, const float *b1,
                              const float *b2, int *flag) {
  STS_PROF(c, "launch_check_spitzer_f32");
  const long long n = c->ncell;
  hipLaunchKernelGGL(k_check_spitzer<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     c->stream, n, T, b0, b1, b2, flag);
}

int gershgorin_parts(const sts_ctx *c) {
  const dim3 g = grid3(c);
  return (int)(g.x * g.y * g.z);
}

void launch_gershgorin(const sts_ctx *c, double *partials, int) {
  STS_PROF(c, "launch_gershgorin");
  if (c->op == OP_SPITZER)
    hipLaunchKernelGGL(k_gershgorin<OP_SPITZER>, grid3(c), dim3(TX, TY), 0, c->stream,
                       c->grid(), c->coef(), partials);
  else
    hipLaunchKernelGGL(k_gershgorin<OP_ISOTROPIC>, grid3(c), dim3(TX, TY), 0, c->stream,
                       c->grid(), c->coef(), partials);
}

}  // namespace sts
