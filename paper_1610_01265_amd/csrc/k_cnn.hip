// Small 3D CNN for the learned PCG initial guess: BF16 implicit-GEMM
// convolutions on MFMA (FP32 accumulate), their input / weight gradients,
// and the element-wise pieces of training (input packing, loss, Adam).
//
// Layout: activations and gradients are channel-last BF16 [cells][16]
// (2-channel inputs and the 1-channel output are padded to 16 channels with
// zero weights).  A 3x3x3 convolution with "same" padding (zero along r and
// theta, circular along phi) is the GEMM
//   out[cell][co] = sum_{tap, ci} W[co][ci][tap] in[cell + off(tap)][ci],
// M = cells, N = 16, K = 27 * 16.  Each MFMA v_mfma_f32_16x16x32_bf16
// computes C^T (16 channels x 16 cells) over K = 32 = two taps x 16 input
// channels:  A = weights (lane l: co = l%16, K = 8(l/16)..+7),
// B = activations (lane l: cell l%16, K = 8(l/16)..+7, i.e. 8 contiguous
// channels of one cell), C: lane l holds co = 4(l/16)..+3 of cell l%16.
// The input gradient is the same convolution with the tap-flipped,
// channel-transposed weights (zero / circular padding are self-adjoint).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "k_common.h"
#include "k_reduce.h"
#include "cnn_internal.h"

namespace sts {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));  // 16-byte staging chunk

namespace {

constexpr int CC = 16;           // channels
constexpr int NTAP = 27;
constexpr int NSTEP = 14;        // K steps of two taps (tap 27 = zero padding)
constexpr int TKC = 64, TJC = 4; // output tile per workgroup plane: 4 rows x 64 cells
constexpr int HKC = TKC + 2, HJC = TJC + 2;
constexpr int PLC = HKC * HJC;   // cells per LDS plane (tile + halo)

// epilogues of k_conv (numbers are the cnn_conv kinds of the C ABI)
enum { CV_RELU = 0, CV_LAST = 1, CV_MASK = 2, CV_F32 = 3, CV_OUT4 = 5 };

// target number of workgroups of the plane-marching kernels, and the output
// planes the convolution computes per iteration (between two waits for
// input planes; its LDS ring holds CNN_PPI + 2 planes)
#ifndef CNN_WG_TARGET
#define CNN_WG_TARGET 2048
#endif
#ifndef CNN_PPI
#define CNN_PPI 1
#endif

struct CnnGrid {
  int n0, n1, n2;  // phi (axis 2) is circular; r, theta zero-padded
};

__device__ __forceinline__ int tap_a(int t) { return t / 9 - 1; }
__device__ __forceinline__ int tap_b(int t) { return (t / 3) % 3 - 1; }
__device__ __forceinline__ int tap_c(int t) { return t % 3 - 1; }

// Forward-type convolution (also used for the input gradient).
//   wfrag[s][lane][8]: A fragments, s = K step
//   mode CV_RELU: out_bf = bf16(max(acc + bias, 0))
//   mode CV_LAST: outf[cell] = acc(co 0) + bias[0]     (FP32, one channel)
//   mode CV_MASK: out_bf = bf16(acc * (mask[cell][co] > 0))   (no mask: acc)
//   mode CV_F32 : outf[cell][co] = acc + bias           (FP32; bias optional)
//   mode CV_OUT4: outf[cell][co] = acc + bias, co < 4   (FP32, four channels)
template <int MODE>
__global__ void __launch_bounds__(256)
    k_conv(CnnGrid g, const __bf16 *__restrict__ in, const __bf16 *__restrict__ wfrag,
           const float *__restrict__ bias, const __bf16 *__restrict__ mask,
           __bf16 *__restrict__ out_bf, float *__restrict__ outf, int CI, int nchunk, int rev) {
  constexpr int PP = CNN_PPI, RS = CNN_PPI + 2;  // planes per iteration, ring slots
  __shared__ __attribute__((aligned(16))) __bf16 s_in[RS][PLC * CC];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int ntk = (g.n2 + TKC - 1) / TKC, ntj = (g.n1 + TJC - 1) / TJC;
  const int w = wg_index(rev);
  const int bx = w % ntk, by = (w / ntk) % ntj, bz = w / (ntk * ntj);
  const int k0 = bx * TKC, j0 = by * TJC;
  const int i0 = bz * CI, i1 = min(i0 + CI, g.n0);
  (void)nchunk;
  const long long n12 = (long long)g.n1 * g.n2;

  // A fragments (weights) for all K steps: 14 x 8 bf16 per lane
  bf16x8 wa[NSTEP];
#pragma unroll
  for (int s = 0; s < NSTEP; ++s)
    wa[s] = *reinterpret_cast<const bf16x8 *>(wfrag + ((size_t)s * 64 + lane) * 8);

  // halo-tile loads: PLC cells x 32 B = 2 x 16 B chunks per cell
  constexpr int NCH = PLC * 2;                 // 16-byte chunks per plane
  constexpr int NLD = (NCH + 255) / 256;       // per thread
  int src[NLD];     // cell offset inside a plane (or -1 for zero padding)
  int dst[NLD];
#pragma unroll
  for (int q = 0; q < NLD; ++q) {
    const int ch = t + q * 256;
    const int cell = ch >> 1, half = ch & 1;
    const int hj = cell / HKC, hk = cell - hj * HKC;
    const int jj = j0 - 1 + hj;
    int kk = (k0 - 1 + hk) % g.n2;
    if (kk < 0) kk += g.n2;
    const bool ok = ch < NCH && jj >= 0 && jj < g.n1;
    src[q] = ok ? ((jj * g.n2 + kk) * 2 + half) : -1;
    dst[q] = ch < NCH ? ch : -1;
  }
  auto load_plane = [&](int ip, u32x4 *v) {
    const bool pin = ip >= 0 && ip < g.n0;
    const u32x4 *base = reinterpret_cast<const u32x4 *>(in + (long long)(pin ? ip : 0) * n12 * CC);
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      v[q] = (pin && src[q] >= 0) ? base[src[q]] : u32x4(0u);
    }
  };
  auto store_plane = [&](int ip, const u32x4 *v) {
    u32x4 *s = reinterpret_cast<u32x4 *>(s_in[(ip + RS) % RS]);
#pragma unroll
    for (int q = 0; q < NLD; ++q)
      if (dst[q] >= 0) s[dst[q]] = v[q];
  };
  u32x4 v[PP][NLD];
  for (int ip = i0 - 1; ip <= i0 + PP; ++ip) {
    load_plane(ip, v[0]);
    store_plane(ip, v[0]);
  }
  __syncthreads();

  const int grp = lane >> 4, cl = lane & 15;
  const int j = j0 + wv;
  // CV_MASK: the mask entries of output plane i (this lane's 4 channels of
  // its 4 cells; 1 where there is no mask or no cell), loaded before the
  // plane's MFMAs so that their latency runs under them
  auto load_mask = [&](int i, uint2 *mv) {
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int k = k0 + 16 * nb + cl;
      const long long cell = (long long)i * n12 + (long long)j * g.n2 + k;
      mv[nb] = (mask && j < g.n1 && k < g.n2)
                   ? *reinterpret_cast<const uint2 *>(mask + cell * CC + 4 * grp)
                   : make_uint2(0x3F803F80u, 0x3F803F80u);  // bf16 1.0 x 4
    }
  };
  // output plane i from input planes i-1, i, i+1 of the ring
  auto compute = [&](int i, const uint2 *mv) {
    f32x4 acc[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    auto load_b = [&](int s, bf16x8 *bv) {
      const int tap = min(2 * s + (grp >> 1), NTAP - 1);  // tap 27 has zero weights
      const int a = tap_a(tap), b = tap_b(tap), c = tap_c(tap);
      const bf16x8 *pl = reinterpret_cast<const bf16x8 *>(s_in[(i + a + RS) % RS]);
      const int rowb = (wv + 1 + b) * HKC + 1 + c + cl;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) bv[nb] = pl[(rowb + 16 * nb) * 2 + (grp & 1)];
    };
#pragma unroll
    for (int s = 0; s < NSTEP; ++s) {
      bf16x8 bv[4];
      load_b(s, bv);
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
        acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[s], bv[nb], acc[nb], 0, 0, 0);
    }
    if (j < g.n1) {
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const int k = k0 + 16 * nb + cl;
        if (k >= g.n2) continue;
        const long long cell = (long long)i * n12 + (long long)j * g.n2 + k;
        const int co0 = 4 * grp;
        if (MODE == CV_LAST) {
          if (grp == 0) outf[cell] = acc[nb][0] + bias[0];
        } else if (MODE == CV_OUT4) {
          if (grp == 0)
            *reinterpret_cast<float4 *>(outf + cell * 4) =
                make_float4(acc[nb][0] + bias[0], acc[nb][1] + bias[1], acc[nb][2] + bias[2],
                            acc[nb][3] + bias[3]);
        } else if (MODE == CV_F32) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            outf[cell * CC + co0 + e] = acc[nb][e] + (bias ? bias[co0 + e] : 0.0f);
        } else {
          __bf16 o[4];
          if (MODE == CV_RELU) {
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = (__bf16)fmaxf(acc[nb][e] + bias[co0 + e], 0.0f);
          } else {  // CV_MASK
            __bf16 mk[4];
            __builtin_memcpy(mk, &mv[nb], 8);
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = (__bf16)((float)mk[e] > 0.0f ? acc[nb][e] : 0.0f);
          }
          uint2 pk;
          __builtin_memcpy(&pk, o, 8);
          *reinterpret_cast<uint2 *>(out_bf + cell * CC + co0) = pk;
        }
      }
    }
  };
  // each iteration: outputs i .. i+PP-1 (inputs i-1 .. i+PP in the ring),
  // meanwhile the inputs of the next iteration, i+PP+1 .. i+2PP, are loaded
  // into registers and staged over the planes i-1 .. i+PP-2 afterwards
  for (int i = i0; i < i1; i += PP) {
    uint2 mv[PP][4];
    if (MODE == CV_MASK) {
#pragma unroll
      for (int q = 0; q < PP; ++q)
        if (i + q < i1) load_mask(i + q, mv[q]);
    }
#pragma unroll
    for (int q = 0; q < PP; ++q)
      if (i + PP + 1 + q <= i1) load_plane(i + PP + 1 + q, v[q]);
#pragma unroll
    for (int q = 0; q < PP; ++q)
      if (i + q < i1) compute(i + q, mv[q]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PP; ++q)
      if (i + PP + 1 + q <= i1) store_plane(i + PP + 1 + q, v[q]);
    __syncthreads();
  }
}

// Weight and bias gradients of one layer:
//   dW[tap][co][ci] = sum_cells dout[cell][co] act[cell + off(tap)][ci]
//   db[co]          = sum_cells dout[cell][co]
// As an MFMA product with K = cells: A = dout (lane: co = l%16, 8 cells),
// B = act shifted by the tap (lane: ci = l%16, the same 8 cells), C[co][ci];
// the bias is a 28th product with B = ones.  Workgroups take work items
// (a 4 x 64 tile and a chunk of r-planes, grid-stride) and march the
// activation planes p of the chunk and its two halo planes: act plane p is
// the tap-a operand of output plane x = p - a, so each B fragment gathered
// from LDS feeds the products of the three output planes p + 1, p, p - 1
// (a = -1, 0, +1), whose dout fragments stay in registers; every (x, tap)
// pair meets once.  The activation plane and the dout tile are double
// buffered in LDS (one barrier per plane); all 28 products accumulate in
// registers, and each workgroup writes its partial sums, reduced in a fixed
// order by k_wgrad_reduce.  LDS cells are 32 B (16 channels) with a 32-B
// gap after every 8 cells, so the 2-byte operand reads of the four 16-lane
// groups fall in disjoint banks.
__device__ __forceinline__ int lds_cell(int x) { return (x + (x >> 3)) * CC; }

constexpr int PLCP = PLC + (PLC + 7) / 8;        // padded cells of one ring plane
constexpr int TCP = TJC * TKC + TJC * TKC / 8;   // padded cells of the dout tile

__global__ void __launch_bounds__(256, 2)
    k_wgrad(CnnGrid g, const __bf16 *__restrict__ act, const __bf16 *__restrict__ dout,
            float *__restrict__ part, int CI, int nitems, int rev) {
  __shared__ __attribute__((aligned(16))) __bf16 s_in[2][PLCP * CC];
  __shared__ __attribute__((aligned(16))) __bf16 s_d[2][TCP * CC];
  const int t = threadIdx.x, lane = t & 63;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int grp = lane >> 4, cl = lane & 15;
  // operand reads: cell u + 8 grp + e of a padded plane sits at
  // lds_cell(u + e) + 9 grp CC (u a multiple of 8 plus a wave-uniform
  // shift), so every read is one per-lane base plus a uniform offset
  const int lane_off = grp * 9 * CC + cl;
  const int ntk = (g.n2 + TKC - 1) / TKC, ntj = (g.n1 + TJC - 1) / TJC;
  const long long n12 = (long long)g.n1 * g.n2;
  f32x4 acc[NTAP + 1];
#pragma unroll
  for (int q = 0; q <= NTAP; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
  bf16x8 ones, zero8;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    ones[e] = (__bf16)1.0f;
    zero8[e] = (__bf16)0.0f;
  }
  constexpr int NCH = PLC * 2;
  constexpr int NLD = (NCH + 255) / 256;

  const int w = wg_index(rev);
  for (int item = w; item < nitems; item += gridDim.x) {
    const int bx = item % ntk, by = (item / ntk) % ntj, bz = item / (ntk * ntj);
    const int k0 = bx * TKC, j0 = by * TJC;
    const int i0 = bz * CI, i1 = min(i0 + CI, g.n0);
    int src[NLD], dst[NLD];
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int ch = t + q * 256;
      const int cell = ch >> 1, half = ch & 1;
      const int hj = cell / HKC, hk = cell - hj * HKC;
      const int jj = j0 - 1 + hj;
      int kk = (k0 - 1 + hk) % g.n2;
      if (kk < 0) kk += g.n2;
      const bool ok = ch < NCH && jj >= 0 && jj < g.n1;
      src[q] = ok ? ((jj * g.n2 + kk) * 2 + half) : -1;
      dst[q] = ch < NCH ? lds_cell(cell) / 8 + half : -1;  // in 16-byte units
    }
    // this thread's share of the dout tile: cell t, both halves
    const int dj = t >> 6, dk = t & 63;
    const bool din = j0 + dj < g.n1 && k0 + dk < g.n2;
    const int doff = ((j0 + dj) * g.n2 + (k0 + dk)) * 2;
    auto load_act = [&](int ip, u32x4 *v) {
      const bool pin = ip >= 0 && ip < g.n0;
      const u32x4 *base =
          reinterpret_cast<const u32x4 *>(act + (long long)(pin ? ip : 0) * n12 * CC);
#pragma unroll
      for (int q = 0; q < NLD; ++q) v[q] = (pin && src[q] >= 0) ? base[src[q]] : u32x4(0u);
    };
    auto store_act = [&](int ip, const u32x4 *v) {
      u32x4 *sp = reinterpret_cast<u32x4 *>(s_in[ip & 1]);
#pragma unroll
      for (int q = 0; q < NLD; ++q)
        if (dst[q] >= 0) sp[dst[q]] = v[q];
    };
    auto load_dout = [&](int ip, u32x4 *d) {
      d[0] = d[1] = u32x4(0u);
      if (din && ip < i1) {
        const u32x4 *dp = reinterpret_cast<const u32x4 *>(dout + (long long)ip * n12 * CC);
        d[0] = dp[doff];
        d[1] = dp[doff + 1];
      }
    };
    auto store_dout = [&](int ip, const u32x4 *d) {
      u32x4 *sd = reinterpret_cast<u32x4 *>(s_d[ip & 1]);
      sd[lds_cell(t) / 8] = d[0];
      sd[lds_cell(t) / 8 + 1] = d[1];
    };
    // A fragments of output plane x (its dout tile staged in s_d[x & 1])
    auto gather_a = [&](int x, bf16x8 *a) {
      const __bf16 *sd = s_d[x & 1] + lane_off;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const int u = wv * TKC + ks * 32;
#pragma unroll
        for (int e = 0; e < 8; ++e) a[ks][e] = sd[lds_cell(u + e)];
      }
    };
    // act plane p + 1 and dout plane p + 2 are staged while plane p is used
    __syncthreads();  // the previous item's reads of the buffers are done
    {
      u32x4 v[NLD], d[2];
      load_act(i0 - 1, v);
      load_dout(i0, d);
      store_act(i0 - 1, v);
      store_dout(i0, d);
    }
    __syncthreads();
    bf16x8 am[2] = {zero8, zero8}, a0[2] = {zero8, zero8}, ap[2];
    for (int p = i0 - 1; p <= i1; ++p) {
      // dout of output plane p + 1 (zero outside the chunk)
      if (p + 1 < i1) {
        gather_a(p + 1, ap);
      } else {
        ap[0] = ap[1] = zero8;
      }
      u32x4 v[NLD], d[2];
      const bool nxt_act = p + 1 <= i1, nxt_d = p + 2 < i1;
      if (nxt_act) load_act(p + 1, v);
      if (nxt_d) load_dout(p + 2, d);
      if (p >= 0 && p < g.n0) {
        const __bf16 *pl = s_in[p & 1] + lane_off;
        // B fragment q = 9 ks + bc of this plane: (b, c) = (bc / 3 - 1, bc % 3 - 1)
        auto gather_b = [&](int q, bf16x8 &bv) {
          const int ks = q / 9, bc = q % 9;
          const int u = (wv + 1 + bc / 3 - 1) * HKC + bc % 3 + ks * 32;
#pragma unroll
          for (int e = 0; e < 8; ++e) bv[e] = pl[lds_cell(u + e)];
        };
        // software pipeline: fragment q + 1 is read while q's products issue
        bf16x8 bq[2];
        gather_b(0, bq[0]);
#pragma unroll
        for (int q = 0; q < 18; ++q) {
          const int ks = q / 9, bc = q % 9;
          if (q + 1 < 18) gather_b(q + 1, bq[(q + 1) & 1]);
          __builtin_amdgcn_sched_barrier(0);
          const bf16x8 bv = bq[q & 1];
          // tap (a, b, c) = 9 (a + 1) + 3 (b + 1) + (c + 1); output plane p - a
          // (a zero fragment outside the chunk adds exact zeros)
          acc[18 + bc] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[ks], bv, acc[18 + bc], 0, 0, 0);
          acc[9 + bc] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0[ks], bv, acc[9 + bc], 0, 0, 0);
          acc[bc] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap[ks], bv, acc[bc], 0, 0, 0);
          if (bc == 0)
            acc[NTAP] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0[ks], ones, acc[NTAP], 0, 0, 0);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
      if (nxt_act) store_act(p + 1, v);
      if (nxt_d) store_dout(p + 2, d);
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        am[ks] = a0[ks];
        a0[ks] = ap[ks];
      }
    }
  }
  // sum the four wavefronts in a fixed order (ring memory reused)
  __syncthreads();
  float *red = reinterpret_cast<float *>(&s_in[0][0]);  // 4 x 256 floats per product
  for (int q = 0; q <= NTAP; ++q) {
#pragma unroll
    for (int e = 0; e < 4; ++e) red[wv * 256 + (4 * grp + e) * 16 + cl] = acc[q][e];
    __syncthreads();
    const float s4 = red[t] + red[256 + t] + red[512 + t] + red[768 + t];
    part[((size_t)w * (NTAP + 1) + q) * 256 + t] = s4;
    __syncthreads();
  }
}

// g[co][ci][tap] (the master-weight layout) and g_bias[co] = sums over the
// workgroups' partials part[w][q][co][ci].  Coalesced: a workgroup owns 32
// consecutive entries of the partial layout and splits the workgroup range
// into 32 slices; each thread sums its slice in order with four running sums
// (partials w, w + 4, ... in the first), which are then added in order, and
// the slices are added in order (a fixed summation order: deterministic).
// 1024 threads and short slices keep enough loads in flight: with 8 slices
// of 256 threads the sum was latency-bound (19.8 us for 512 partials).
constexpr int WR_OUT = 32, WR_SLICES = 32;
__global__ void __launch_bounds__(WR_OUT *WR_SLICES)
    k_wgrad_reduce(const float *__restrict__ part, int nwg, float *__restrict__ g) {
  __shared__ float red[WR_SLICES][WR_OUT];
  const int o = threadIdx.x % WR_OUT, sl = threadIdx.x / WR_OUT;
  const int idx = blockIdx.x * WR_OUT + o;  // = q * 256 + cc
  const size_t stride = (size_t)(NTAP + 1) * 256;
  const int per = (nwg + WR_SLICES - 1) / WR_SLICES;
  const int w0 = min(nwg, sl * per), w1 = min(nwg, w0 + per);
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  int w = w0;
  for (; w + 3 < w1; w += 4) {
    s0 += part[w * stride + idx];
    s1 += part[(w + 1) * stride + idx];
    s2 += part[(w + 2) * stride + idx];
    s3 += part[(w + 3) * stride + idx];
  }
  for (; w < w1; ++w) s0 += part[w * stride + idx];
  red[sl][o] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (sl == 0) {
    float t = red[0][o];
    for (int q = 1; q < WR_SLICES; ++q) t += red[q][o];
    const int q = idx >> 8, cc = idx & 255;
    if (q < NTAP)
      g[cc * NTAP + q] = t;
    else if ((cc & 15) == 0)
      g[NTAP * 256 + (cc >> 4)] = t;  // bias: column ci = 0
  }
}

// Network input: channel 0 = rhs * rs, channel 1 = (T - ts) * tsc, others 0.
__global__ void k_pack_input(long long n, const double *__restrict__ rhs,
                             const double *__restrict__ T, double rs, double tsh, double tsc,
                             __bf16 *__restrict__ x) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  __bf16 o[16];
  o[0] = (__bf16)(float)(rhs[c] * rs);
  o[1] = (__bf16)(float)((T[c] - tsh) * tsc);
  for (int q = 2; q < 16; ++q) o[q] = (__bf16)0.0f;
  uint4 p0, p1;
  __builtin_memcpy(&p0, o, 16);
  __builtin_memcpy(&p1, o + 8, 16);
  reinterpret_cast<uint4 *>(x + c * CC)[0] = p0;
  reinterpret_cast<uint4 *>(x + c * CC)[1] = p1;
}

// MSE loss on the normalised increment and its gradient (channel 0).
//   target = (x_star - T) * inv_sd;  d = pred - target;  loss = mean d^2
__global__ void __launch_bounds__(256)
    k_loss(long long n, const float *__restrict__ pred, const double *__restrict__ xs,
           const double *__restrict__ T, double inv_sd, __bf16 *__restrict__ g,
           double *__restrict__ part) {
  double s = 0.0;
  const float scale = (float)(2.0 / (double)n);
  const long long stride = (long long)gridDim.x * 256;
  for (long long c = (long long)blockIdx.x * 256 + threadIdx.x; c < n; c += stride) {
    const double tg = (xs[c] - T[c]) * inv_sd;
    const double d = (double)pred[c] - tg;
    s += d * d;
    __bf16 o[16];
    o[0] = (__bf16)(scale * (float)d);
    for (int q = 1; q < 16; ++q) o[q] = (__bf16)0.0f;
    uint4 p0, p1;
    __builtin_memcpy(&p0, o, 16);
    __builtin_memcpy(&p1, o + 8, 16);
    reinterpret_cast<uint4 *>(g + c * CC)[0] = p0;
    reinterpret_cast<uint4 *>(g + c * CC)[1] = p1;
  }
  wg_sum2<256>(s, 0.0, threadIdx.x, part + blockIdx.x, nullptr);
}

// x0 = T + sd * pred
__global__ void k_guess(long long n, const double *__restrict__ T, const float *__restrict__ pred,
                        double sd, double *__restrict__ x0) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) x0[c] = T[c] + sd * (double)pred[c];
}

// Adam on FP32 master parameters (gradients masked where the padded network
// has no parameter: mask[q] = 0).
__global__ void k_adam(int n, float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, const float *__restrict__ mask, float lr,
                       float b1, float b2, float c1, float c2, float eps) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float gq = g[q] * mask[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  p[q] = p[q] - lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// BF16 A fragments from the FP32 master weights W[co][ci][tap] of one layer:
//   forward: frag[s][l][e] = W[co = l%16][ci = 8((l/16)%2) + e][tap = 2s + (l/16)/2]
//   input gradient (transposed, tap-flipped):
//            frag[s][l][e] = W[co = 8((l/16)%2) + e][ci = l%16][26 - tap]
__global__ void k_make_frags(const float *__restrict__ W, __bf16 *__restrict__ ffwd,
                             __bf16 *__restrict__ fbwd) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // s * 512 + l * 8 + e
  if (idx >= NSTEP * 64 * 8) return;
  const int s = idx / 512, l = (idx / 8) % 64, e = idx % 8;
  const int g4 = l >> 4, tap = 2 * s + (g4 >> 1);
  const int r16 = l & 15, c8 = 8 * (g4 & 1) + e;
  float wf = 0.f, wb = 0.f;
  if (tap < NTAP) {
    wf = W[(r16 * CC + c8) * NTAP + tap];
    wb = W[(c8 * CC + r16) * NTAP + (NTAP - 1 - tap)];
  }
  ffwd[idx] = (__bf16)wf;
  fbwd[idx] = (__bf16)wb;
}

// Mean and root-mean-square of scale * (x - y) (y optional): partial sums
// per workgroup, then one workgroup sums them in a fixed order.
__global__ void __launch_bounds__(256)
    k_moments(long long n, const double *__restrict__ x, const double *__restrict__ y, double sc,
              double *__restrict__ part) {
  double s1 = 0.0, s2 = 0.0;
  const long long stride = (long long)gridDim.x * 256;
  for (long long c = (long long)blockIdx.x * 256 + threadIdx.x; c < n; c += stride) {
    const double d = sc * (y ? x[c] - y[c] : x[c]);
    s1 += d;
    s2 += d * d;
  }
  wg_sum2<256>(s1, s2, threadIdx.x, part + blockIdx.x, part + gridDim.x + blockIdx.x);
}

__global__ void __launch_bounds__(256)
    k_sum_parts(const double *__restrict__ part, int n, int two, double *__restrict__ out) {
  block_sum_parts(part, n, n, out, two ? out + 1 : nullptr);
}

int conv_chunk(int n0, int ntiles) {
  long long ci = (long long)ntiles * n0 / CNN_WG_TARGET;
  if (ci < 1) ci = 1;
  if (ci > 16) ci = 16;
  return (int)ci;
}

}  // namespace

// ---------------------------------------------------------------- launchers
void launch_cnn_conv(const CnnLaunch &L, int mode, const void *in, const void *wfrag, const float *bias,
              const void *mask, void *out_bf, float *outf) {
  CnnGrid g{L.n0, L.n1, L.n2};
  const int ntk = (L.n2 + TKC - 1) / TKC, ntj = (L.n1 + TJC - 1) / TJC;
  const int CI = conv_chunk(L.n0, ntk * ntj);
  const int nchunk = (L.n0 + CI - 1) / CI;
  const dim3 grid(ntk * ntj * nchunk), blk(256);
  const __bf16 *pin = (const __bf16 *)in, *pw = (const __bf16 *)wfrag, *pm = (const __bf16 *)mask;
  __bf16 *pob = (__bf16 *)out_bf;
  switch (mode) {
    case CV_RELU:
      hipLaunchKernelGGL(k_conv<CV_RELU>, grid, blk, 0, L.stream, g, pin, pw, bias, pm, pob, outf, CI, nchunk, L.rev);
      break;
    case CV_LAST:
      hipLaunchKernelGGL(k_conv<CV_LAST>, grid, blk, 0, L.stream, g, pin, pw, bias, pm, pob, outf, CI, nchunk, L.rev);
      break;
    case CV_MASK:
      hipLaunchKernelGGL(k_conv<CV_MASK>, grid, blk, 0, L.stream, g, pin, pw, bias, pm, pob, outf, CI, nchunk, L.rev);
      break;
    case CV_OUT4:
      hipLaunchKernelGGL(k_conv<CV_OUT4>, grid, blk, 0, L.stream, g, pin, pw, bias, pm, pob, outf, CI, nchunk, L.rev);
      break;
    default:
      hipLaunchKernelGGL(k_conv<CV_F32>, grid, blk, 0, L.stream, g, pin, pw, bias, pm, pob, outf, CI, nchunk, L.rev);
  }
}

int cnn_wgrad_parts() { return 512; }

void launch_cnn_wgrad(const CnnLaunch &L, const void *act, const void *dout, float *part,
                      float *g) {
  CnnGrid gr{L.n0, L.n1, L.n2};
  const int ntk = (L.n2 + TKC - 1) / TKC, ntj = (L.n1 + TJC - 1) / TJC;
  const int CI = conv_chunk(L.n0, ntk * ntj);
  const int nitems = ntk * ntj * ((L.n0 + CI - 1) / CI);
  const int nwg = std::min(nitems, cnn_wgrad_parts());
  hipLaunchKernelGGL(k_wgrad, dim3(nwg), dim3(256), 0, L.stream, gr, (const __bf16 *)act,
                     (const __bf16 *)dout, part, CI, nitems, L.rev);
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((NTAP + 1) * 256 / WR_OUT), dim3(WR_OUT * WR_SLICES), 0,
                     L.stream, part, nwg, g);
}

void launch_cnn_pack_input(const CnnLaunch &L, const double *rhs, const double *T, double rs, double tsh,
                    double tsc, void *x) {
  const long long n = (long long)L.n0 * L.n1 * L.n2;
  hipLaunchKernelGGL(k_pack_input, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.stream, n,
                     rhs, T, rs, tsh, tsc, (__bf16 *)x);
}

int cnn_loss_parts() { return 1024; }

void launch_cnn_loss(const CnnLaunch &L, const float *pred, const double *xs, const double *T,
              double inv_sd, void *g, double *part) {
  const long long n = (long long)L.n0 * L.n1 * L.n2;
  hipLaunchKernelGGL(k_loss, dim3(cnn_loss_parts()), dim3(256), 0, L.stream, n, pred, xs, T,
                     inv_sd, (__bf16 *)g, part);
}

void launch_cnn_guess(const CnnLaunch &L, const double *T, const float *pred, double sd, double *x0) {
  const long long n = (long long)L.n0 * L.n1 * L.n2;
  hipLaunchKernelGGL(k_guess, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L.stream, n, T, pred,
                     sd, x0);
}

void launch_cnn_adam(const CnnLaunch &L, int n, float *p, float *m, float *v, const float *g,
                     const float *mask, float lr, int step, float b1, float b2, float eps) {
  // bias corrections 1 - beta^t of this step t
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, L.stream, n, p, m, v, g, mask,
                     lr, b1, b2, c1, c2, eps);
}

void launch_cnn_make_frags(const CnnLaunch &L, const float *W, void *ffwd, void *fbwd) {
  hipLaunchKernelGGL(k_make_frags, dim3((NSTEP * 64 * 8 + 255) / 256), dim3(256), 0, L.stream, W,
                     (__bf16 *)ffwd, (__bf16 *)fbwd);
}

int cnn_moment_parts() { return 512; }

void launch_cnn_moments(const CnnLaunch &L, const double *x, const double *y, double sc, double *part,
                 double *out2) {
  const long long n = (long long)L.n0 * L.n1 * L.n2;
  const int np = cnn_moment_parts();
  hipLaunchKernelGGL(k_moments, dim3(np), dim3(256), 0, L.stream, n, x, y, sc, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, L.stream, part, np, 1, out2);
}

void launch_cnn_sum_parts(const CnnLaunch &L, const double *part, int n, double *out) {
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, L.stream, part, n, 0, out);
}

}  // namespace sts
