// Local H*psi of the compensated single-precision form with exact digit
// products on the int8 matrix cores (the engine of wvl_oz.h), for uniform
// batches with a shared potential and line lengths that are multiples of 16.
//
// Three kernels, one plane per workgroup and step, the plane's digits in LDS:
//   z:      u = W_z c                         over (orbital, y) xz-planes
//   planes: psi = W_y W_x u, rho, e_pot, y = pot_scale V psi,
//           t = W_y^T W_x^T y, kxy = (K_x + K_y) c   over z-planes, the
//           orbitals of a density group in turn (the group's partial in
//           orbital order, as in the other in-plane kernels)
//   final:  Hc = W_z^T t + kin_scale k (K_z c + kxy), e_kin   over xz-planes
// with W = CW, W^T = CWT, K = CK the combined filters (Sec. 2.4, last
// paragraph; Sec. 3.1 for the separable form) and k = -1/(2 h^2).  t, u and
// kxy are compact float pairs in the workspace (hi float, lo as an int16
// fraction of ulp(hi): 6 bytes a value); every plane enters a kernel as
// float pairs, is split into digits with its own exponent, and leaves as
// float pairs (t, u, kxy, Hc) or float64 sums (rho, energies).
#include <algorithm>

#include "wvl_oz.h"

namespace wvl {

namespace {

constexpr int kOzZWaves = 8;     // z kernels: 512 threads, two workgroups per CU
constexpr int kOzXyWaves = 12;   // in-plane kernel: 768 threads, 3 tiles per wave at 96 x 96

__device__ __forceinline__ double oz_pair_d(f2 v) { return (double)v.hi + (double)v.lo; }

// ---------------------------------------------------------------------------
// the potential as float pairs, and the exponent of every z-plane's max |V|
__global__ __launch_bounds__(256) void k_oz_vprep(const double* V, int npl, float* vhl, int64_t M,
                                                  int* vexp) {
  const int z = blockIdx.x;
  float m = 0.0f;
  for (int i = threadIdx.x; i < npl; i += 256) {
    const int64_t e = (int64_t)z * npl + i;
    const double v = V[e];
    const float h = (float)v;
    vhl[e] = h;
    vhl[M + e] = (float)(v - (double)h);
    m = fmaxf(m, fabsf(h));
  }
  __shared__ float red[4];
  #pragma unroll
  for (int s = 32; s > 0; s >>= 1) m = fmaxf(m, __shfl_xor(m, s, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) vexp[z] = oz_exp_of(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
}

// ---------------------------------------------------------------------------
// z step: u = W_z c over the xz-plane (b, y): lines x, contracted z
__global__ __launch_bounds__(64 * kOzZWaves) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_oz_z(OzArgs a) {
  extern __shared__ __align__(16) uint8_t oz_lds[];
  const int b = blockIdx.x / a.m2, y = blockIdx.x - b * a.m2;
  const int m1 = a.m1, m3 = a.m3;
  const int64_t zs = (int64_t)m1 * a.m2;
  const int64_t gp = a.orbs[b].off + (int64_t)y * m1;
  const OzGeo gz{m3, m1, oz_pitch(m3), a.dz};
  const int e = oz_load<false, kOzZWaves>(a.c, a.plane, gp, zs, gz, oz_lds, -2000);
  __syncthreads();
  const int E = e + OzK<OP_CW>::EF - 54;
  const int lane = threadIdx.x & 63, n = lane & 15, gq = lane >> 4;
  float* u = a.u;
  oz_pass<OP_CW, true, kOzZWaves>(oz_lds, gz, 0, [&](int, int k0, int o0, const int64_t (&T)[4]) {
    // elements (x = o0 + 4 g + v, z = k0 + n)
    const int64_t at = gp + (int64_t)(k0 + n) * zs + o0 + 4 * gq;
    const f2 r[4] = {oz_tof(T[0], E), oz_tof(T[1], E), oz_tof(T[2], E), oz_tof(T[3], E)};
    oz_store4_cp(u, a.plane, at, r);
  });
}

// ---------------------------------------------------------------------------
// planes
// one (orbital, z-plane); the group's density plane accumulates in LDS
// (rho_l; bi == 0: first orbital of the group)
__device__ __forceinline__ void oz_xy_plane(const OzArgs& a, int b, int z, int bi, uint8_t* lds,
                                            double* rho_l) {
  constexpr int NW = kOzXyWaves;
  const int m1 = a.m1, m2 = a.m2;
  const int npl = m1 * m2;
  const OzGeo gx{m1, m2, oz_pitch(m1), a.dxy};    // [y][x]: lines y, contracted x
  const OzGeo gy{m2, m1, oz_pitch(m2), a.dxy};    // [x][y]: lines x, contracted y
  const OrbDev& od = a.orbs[b];
  const int64_t gp = od.off + (int64_t)z * npl;
  const int lane = threadIdx.x & 63, n = lane & 15, gq = lane >> 4;

  // ---- psi = W_y W_x u
  int e = oz_load<true, NW, true>(a.u, a.plane, gp, m1, gx, lds, -2000);
  __syncthreads();
  oz_pass_to_digits<OP_CW, NW>(lds, gx, gy);
  e += OzK<OP_CW>::GF;
  // ---- the y pass gives psi; pointwise: rho (group partial), e_pot and the
  //      digits of y = pot_scale V psi (exponent ey)
  const int Epsi = e + OzK<OP_CW>::EF - 54;
  const int ey = e + OzK<OP_CW>::GF + a.vexp[z] + a.pexp;
  const float* vh = a.vhl + (int64_t)z * npl;
  const float* vl = vh + a.M;
  const double occ = od.occ;
  const f2 ps{a.ps_hi, a.ps_lo};
  double ep = 0.0;
  {
    OzPacked<NW> pk;
    pk.n = 0;
    oz_pass<OP_CW, true, NW>(lds, gy, 0, [&](int t, int k0, int o0, const int64_t (&T)[4]) {
      // elements (x = o0 + 4 g + v, y = k0 + n): four consecutive x of row y
      const int pe = (k0 + n) * m1 + o0 + 4 * gq;
      const int pr = (k0 + n) * oz_rho_pitch(m1) + o0 + 4 * gq;   // in the LDS density plane
      const float4 h4 = *reinterpret_cast<const float4*>(vh + pe);
      const float4 l4 = *reinterpret_cast<const float4*>(vl + pe);
      const float hv[4] = {h4.x, h4.y, h4.z, h4.w}, lv[4] = {l4.x, l4.y, l4.z, l4.w};
      double r4[4] = {0.0, 0.0, 0.0, 0.0};
      if (bi != 0) {
        const double4 q = *reinterpret_cast<const double4*>(rho_l + pr);
        r4[0] = q.x; r4[1] = q.y; r4[2] = q.z; r4[3] = q.w;
      }
      OzZ zz[4];
      #pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double pd = oz_tod(T[v], Epsi);
        const double p2 = pd * pd;
        r4[v] = __builtin_fma(occ, p2, r4[v]);
        ep = __builtin_fma((double)hv[v] + (double)lv[v], p2, ep);
        f2 yv = oz_mul(f2{hv[v], lv[v]}, oz_tof(T[v], Epsi));
        if (a.ps_scaled) yv = oz_mul(yv, ps);
        zz[v] = oz_digits(oz_fix(yv.hi, yv.lo, 47 - ey));
      }
      *reinterpret_cast<double4*>(rho_l + pr) = make_double4(r4[0], r4[1], r4[2], r4[3]);
      oz_pack(zz, pk.d[t]);
      pk.n = t + 1;
    });
    __syncthreads();
    oz_store_packed<NW>(pk, gy, 0, lds, gx);   // y in [y][x]: line y = k0 + n, index x
    __syncthreads();
  }
  e = ey;
  // ---- t = W_y^T W_x^T y
  oz_pass_to_digits<OP_CWT, NW>(lds, gx, gy);
  e += OzK<OP_CWT>::GF;
  {
    const int Et = e + OzK<OP_CWT>::EF - 54;
    float* tp = a.t;
    oz_pass<OP_CWT, true, NW>(lds, gy, 0, [&](int, int k0, int o0, const int64_t (&T)[4]) {
      const int64_t at = gp + (int64_t)(k0 + n) * m1 + o0 + 4 * gq;
      const f2 r[4] = {oz_tof(T[0], Et), oz_tof(T[1], Et), oz_tof(T[2], Et), oz_tof(T[3], Et)};
      oz_store4_cp(tp, a.plane, at, r);
    });
    __syncthreads();
  }
  // ---- kxy = (K_x + K_y) c (without the factor -1/(2 h^2)): the x pass on c
  //      in [y][x], its sums kept; the y pass on c in [x][y] (data as the B
  //      operand, so that a lane holds the same elements), the two added
  //      exactly
  const int ec = oz_load<true, NW>(a.c, a.plane, gp, m1, gx, lds, -2000);
  __syncthreads();
  int64_t Tx[oz_mt(NW)][4];
  oz_pass<OP_CK, true, NW, false>(lds, gx, 1, [&](int t, int, int, const int64_t (&T)[4]) {
    #pragma unroll
    for (int v = 0; v < 4; ++v) Tx[t][v] = T[v];
  });
  __syncthreads();
  oz_transpose<NW>(lds, gx, gy);      // c's digits in [x][y] for the y pass
  {
    const int Ek = ec + OzK<OP_CK>::EF - 54;
    float* kp = a.kxy;
    oz_pass<OP_CK, false, NW, false>(lds, gy, 2, [&](int t, int k0, int o0, const int64_t (&T)[4]) {
      // elements (y = k0 + 4 g + v, x = o0 + n)
      #pragma unroll
      for (int v = 0; v < 4; ++v) {
        const f2 r = oz_tof(T[v] + Tx[t][v], Ek);
        const int64_t at = gp + (int64_t)(k0 + 4 * gq + v) * m1 + o0 + n;
        kp[at] = r.hi;
        oz_lo_plane(kp, a.plane)[at] = oz_lo16(r.hi, r.lo);
      }
    });
  }
  const double sp = oz_block_sum<NW>(ep);
  if (threadIdx.x == 0) a.epot[a.pq[b] + z] = sp;
}

template <int WPE>
__global__ __launch_bounds__(64 * kOzXyWaves) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void k_oz_xy(OzArgs a) {
  extern __shared__ __align__(16) uint8_t oz_lds[];
  double* rho_l = reinterpret_cast<double*>(oz_lds + kOzDig * a.dxy);
  const int g = blockIdx.x % a.ngroups;
  const int z = blockIdx.x / a.ngroups;
  #pragma nounroll
  for (int slot = 0; slot < a.G; ++slot) {
    const int b = g * a.G + slot;
    if (b >= a.norb) break;
    oz_xy_plane(a, b, z, slot, oz_lds, rho_l);
  }
  // the group's density partial of this plane, once
  __syncthreads();
  const int npl = a.m1 * a.m2, rpitch = oz_rho_pitch(a.m1), half = a.m1 >> 1;
  double* rp = a.rho_part + (int64_t)g * a.M + (int64_t)z * npl;
  for (int e = threadIdx.x; e < (npl >> 1); e += 64 * kOzXyWaves) {
    const int y = e / half, x = (e - y * half) << 1;
    *reinterpret_cast<double2*>(rp + y * a.m1 + x) =
        *reinterpret_cast<const double2*>(rho_l + y * rpitch + x);
  }
}

// ---------------------------------------------------------------------------
// final z step over the xz-plane (b, y):
//   Hc = W_z^T t + kin_scale k (K_z c + kxy),  e_kin = <c, k (K_z c + kxy)>
template <int WPE>
__global__ __launch_bounds__(64 * kOzZWaves) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void k_oz_zfinal(OzArgs a) {
  extern __shared__ __align__(16) uint8_t oz_lds[];
  const int b = blockIdx.x / a.m2, y = blockIdx.x - b * a.m2;
  const int m1 = a.m1, m3 = a.m3;
  const int64_t zs = (int64_t)m1 * a.m2;
  const OrbDev& od = a.orbs[b];
  const int64_t gp = od.off + (int64_t)y * m1;
  const OzGeo gz{m3, m1, oz_pitch(m3), a.dz};
  const int lane = threadIdx.x & 63, n = lane & 15, gq = lane >> 4;
  constexpr int NW = kOzZWaves;
  const int et = oz_load<false, NW, true>(a.t, a.plane, gp, zs, gz, oz_lds, -2000);
  __syncthreads();
  // both passes with the data as the B operand: a lane holds four
  // consecutive z of one line x, so that c's digits of its elements are one
  // word per digit plane in LDS (the kinetic energy needs c there)
  int64_t Tt[oz_mt(NW)][4];
  oz_pass<OP_CWT, false, NW>(oz_lds, gz, 0, [&](int t, int, int, const int64_t (&T)[4]) {
    #pragma unroll
    for (int v = 0; v < 4; ++v) Tt[t][v] = T[v];
  });
  __syncthreads();
  const int ec = oz_load<false, NW>(a.c, a.plane, gp, zs, gz, oz_lds, -2000);
  __syncthreads();
  const int Et = et + OzK<OP_CWT>::EF - 54;
  const int Ek = ec + OzK<OP_CK>::EF - 54;
  // K c = K_z c + kxy (without k) as a float pair (kxy may exceed this
  // xz-plane's own bound: K_y reaches rows up to 29 away); e_kin = k <c, K c>;
  // Hc = W_z^T t + kd K c with kd = k kin_scale, a power of two in the usual
  // case (exact scaling of the pair)
  const double ks = od.kscale[0];
  const double kd = ks * a.kin_mul;
  int kx2 = 0;
  const double kf = frexp(kd, &kx2);
  const bool pow2 = kf == 0.5 || kf == -0.5;
  const float ksign = kf < 0 ? -1.0f : 1.0f;
  const float kh = (float)kd;
  const f2 kp{kh, (float)(kd - (double)kh)};
  double ek = 0.0;
  const float* kxy = a.kxy;
  const int16_t* kxy_lo = oz_lo_plane(kxy, a.plane);
  float* out = a.out;
  oz_pass<OP_CK, false, NW, false>(oz_lds, gz, 0, [&](int t, int k0, int o0, const int64_t (&T)[4]) {
    // elements (z = k0 + 4 g + v, x = o0 + n)
    const int x = o0 + n, z0 = k0 + 4 * gq;
    // c there, from its digits (one word of four z per digit plane)
    uint32_t dw[kOzDig];
    #pragma unroll
    for (int q = 0; q < kOzDig; ++q)
      dw[q] = *reinterpret_cast<const uint32_t*>(oz_lds + q * gz.dstride + x * gz.pitch + z0);
    #pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t at = gp + (int64_t)(z0 + v) * zs + x;
      const float khi = kxy[at];
      const f2 kc = oz_add(oz_tof(T[v], Ek), f2{khi, oz_lo_of(khi, kxy_lo[at])});
      ek = __builtin_fma(oz_tod(oz_undigits(dw, v), ec - 47), oz_pair_d(kc), ek);
      const f2 sc = pow2 ? f2{ksign * ldexpf(kc.hi, kx2 - 1), ksign * ldexpf(kc.lo, kx2 - 1)}
                         : oz_mul(kc, kp);
      const f2 o = oz_add(oz_tof(Tt[t][v], Et), sc);
      out[at] = o.hi;
      out[a.plane + at] = o.lo;
    }
  });
  const double sk2 = oz_block_sum<NW>(ek);
  if (threadIdx.x == 0) a.ekin[(int64_t)b * a.m2 + y] = ks * sk2;
}

// ---------------------------------------------------------------------------
// The preconditioner's operator (Sec. 2, Eq. "precon", the shift applied by
// the CG update): q = k (K_x + K_y + K_z) p for the compensated form, with
// <p, q> per plane for the step length.
//   z:  q = k K_z p over xz-planes, <p, k K_z p> per xz-plane
//   xy: q += k (K_x + K_y) p over z-planes, <p, k (K_x + K_y) p> per plane
// k = -1/(2 h^2) multiplies the exact sums (a power of two: exact scaling).

__device__ __forceinline__ f2 oz_kscale(f2 r, bool pow2, int kx2, float ksign, f2 kp) {
  return pow2 ? f2{ksign * ldexpf(r.hi, kx2 - 1), ksign * ldexpf(r.lo, kx2 - 1)} : oz_mul(r, kp);
}

__global__ __launch_bounds__(64 * kOzZWaves) __attribute__((amdgpu_waves_per_eu(4, 4)))
void k_oz_helm_z(OzHelmArgs a) {
  extern __shared__ __align__(16) uint8_t oz_lds[];
  constexpr int NW = kOzZWaves;
  const int b = blockIdx.x / a.m2, y = blockIdx.x - b * a.m2;
  const int m1 = a.m1, m3 = a.m3;
  const int64_t zs = (int64_t)m1 * a.m2;
  const OrbDev& od = a.orbs[b];
  const int64_t gp = od.off + (int64_t)y * m1;
  const OzGeo gz{m3, m1, oz_pitch(m3), a.dz};
  const int lane = threadIdx.x & 63, n = lane & 15, gq = lane >> 4;
  const int ep = oz_load<false, NW>(a.p, a.plane, gp, zs, gz, oz_lds, -2000);
  __syncthreads();
  const int Ek = ep + OzK<OP_CK>::EF - 54;
  const double kd = od.kscale[0];
  int kx2 = 0;
  const double kf = frexp(kd, &kx2);
  const bool pow2 = kf == 0.5 || kf == -0.5;
  const float ksign = kf < 0 ? -1.0f : 1.0f;
  const float kh = (float)kd;
  const f2 kp{kh, (float)(kd - (double)kh)};
  double e = 0.0;
  float* q = a.q;
  oz_pass<OP_CK, false, NW, false>(oz_lds, gz, 0, [&](int, int k0, int o0, const int64_t (&T)[4]) {
    // elements (z = k0 + 4 g + v, x = o0 + n); p there from its digits
    const int x = o0 + n, z0 = k0 + 4 * gq;
    uint32_t dw[kOzDig];
    #pragma unroll
    for (int d = 0; d < kOzDig; ++d)
      dw[d] = *reinterpret_cast<const uint32_t*>(oz_lds + d * gz.dstride + x * gz.pitch + z0);
    #pragma unroll
    for (int v = 0; v < 4; ++v) {
      const f2 r = oz_tof(T[v], Ek);
      e = __builtin_fma(oz_tod(oz_undigits(dw, v), ep - 47), oz_pair_d(r), e);
      const f2 o = oz_kscale(r, pow2, kx2, ksign, kp);
      const int64_t at = gp + (int64_t)(z0 + v) * zs + x;
      q[at] = o.hi;
      q[a.plane + at] = o.lo;
    }
  });
  const double sk = oz_block_sum<NW>(e);
  if (threadIdx.x == 0) a.ez[(int64_t)b * a.m2 + y] = kd * sk;
}

template <int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 8 ? 4 : 3, NW == 8 ? 4 : 3)))
void k_oz_helm_xy(OzHelmArgs a) {
  extern __shared__ __align__(16) uint8_t oz_lds[];
  const int b = blockIdx.x / a.m3, z = blockIdx.x - b * a.m3;
  const int m1 = a.m1, m2 = a.m2;
  const OzGeo gx{m1, m2, oz_pitch(m1), a.dxy};
  const OzGeo gy{m2, m1, oz_pitch(m2), a.dxy};
  const OrbDev& od = a.orbs[b];
  const int64_t gp = od.off + (int64_t)z * m1 * m2;
  const int lane = threadIdx.x & 63, n = lane & 15, gq = lane >> 4;
  const int ep = oz_load<true, NW>(a.p, a.plane, gp, m1, gx, oz_lds, -2000);
  __syncthreads();
  int64_t Tx[oz_mt(NW)][4];
  oz_pass<OP_CK, true, NW, false>(oz_lds, gx, 1, [&](int t, int, int, const int64_t (&T)[4]) {
    #pragma unroll
    for (int v = 0; v < 4; ++v) Tx[t][v] = T[v];
  });
  oz_transpose<NW>(oz_lds, gx, gy);
  const int Ek = ep + OzK<OP_CK>::EF - 54;
  const double kd = od.kscale[0];
  int kx2 = 0;
  const double kf = frexp(kd, &kx2);
  const bool pow2 = kf == 0.5 || kf == -0.5;
  const float ksign = kf < 0 ? -1.0f : 1.0f;
  const float kh = (float)kd;
  const f2 kp{kh, (float)(kd - (double)kh)};
  double e = 0.0;
  float* q = a.q;
  oz_pass<OP_CK, false, NW, false>(oz_lds, gy, 2, [&](int t, int k0, int o0, const int64_t (&T)[4]) {
    // elements (y = k0 + 4 g + v, x = o0 + n); p there from its digits ([x][y])
    const int x = o0 + n, y0 = k0 + 4 * gq;
    uint32_t dw[kOzDig];
    #pragma unroll
    for (int d = 0; d < kOzDig; ++d)
      dw[d] = *reinterpret_cast<const uint32_t*>(oz_lds + d * gy.dstride + x * gy.pitch + y0);
    #pragma unroll
    for (int v = 0; v < 4; ++v) {
      const f2 r = oz_tof(T[v] + Tx[t][v], Ek);
      e = __builtin_fma(oz_tod(oz_undigits(dw, v), ep - 47), oz_pair_d(r), e);
      const int64_t at = gp + (int64_t)(y0 + v) * m1 + x;
      const f2 o = oz_add(f2{q[at], q[a.plane + at]}, oz_kscale(r, pow2, kx2, ksign, kp));
      q[at] = o.hi;
      q[a.plane + at] = o.lo;
    }
  });
  const double sk = oz_block_sum<NW>(e);
  if (threadIdx.x == 0) a.exy[(int64_t)b * a.m3 + z] = kd * sk;
}

}  // namespace

hipError_t launch_oz_helm(const OzHelmArgs& a, hipStream_t st) {
  const OzLds l = oz_lds(a.m1, a.m2, a.m3);
  hipLaunchKernelGGL(k_oz_helm_z, dim3(a.norb * a.m2), dim3(64 * kOzZWaves), l.z_bytes, st, a);
  const size_t xy = (size_t)kOzDig * l.dxy;       // digits only (no density plane)
  hipLaunchKernelGGL(k_oz_helm_xy<kOzZWaves>, dim3(a.norb * a.m3), dim3(64 * kOzZWaves), xy, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// host side

OzLds oz_lds(int m1, int m2, int m3) {
  OzLds r;
  const int axy = std::max(m2 * oz_pitch(m1), m1 * oz_pitch(m2));
  r.dxy = (axy + 15) & ~15;
  r.dz = (m1 * oz_pitch(m3) + 15) & ~15;
  r.xy_bytes = (size_t)kOzDig * r.dxy + sizeof(double) * (size_t)oz_rho_pitch(m1) * m2;   // + rho
  r.z_bytes = (size_t)kOzDig * r.dz;
  return r;
}

bool oz_supported(int m1, int m2, int m3) {
  for (int m : {m1, m2, m3})
    if (m < 16 || (m & 15) != 0) return false;
  // tiles per wave and pass, value quads per thread when loading a plane
  const int txy = (m1 >> 4) * (m2 >> 4), txz = (m1 >> 4) * (m3 >> 4);
  if (txy > kOzMaxTiles || txz > kOzMaxTiles) return false;
  if (m1 * m2 / 4 > kOzMaxQuads || m1 * m3 / 4 > kOzMaxQuads) return false;
  // the in-LDS transpose of c: one 8 x 8 block tile (32 x 32 values) per wave
  if (((m1 + 31) / 32) * ((m2 + 31) / 32) > kOzXyWaves) return false;
  const OzLds l = oz_lds(m1, m2, m3);
  return l.xy_bytes <= 160 * 1024 && l.z_bytes <= 160 * 1024;
}

hipError_t launch_oz_vprep(const double* V, int npl, int m3, float* vhl, int64_t M, int* vexp,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_oz_vprep, dim3(m3), dim3(256), 0, st, V, npl, vhl, M, vexp);
  return hipGetLastError();
}

hipError_t launch_oz_z(const OzArgs& a, hipStream_t st) {
  const OzLds l = oz_lds(a.m1, a.m2, a.m3);
  hipLaunchKernelGGL(k_oz_z, dim3(a.norb * a.m2), dim3(64 * kOzZWaves), l.z_bytes, st, a);
  return hipGetLastError();
}

// one workgroup of 12 waves per CU (3 waves per SIMD)
hipError_t launch_oz_xy(const OzArgs& a, hipStream_t st) {
  const OzLds l = oz_lds(a.m1, a.m2, a.m3);
  hipLaunchKernelGGL(k_oz_xy<3>, dim3(a.m3 * a.ngroups), dim3(64 * kOzXyWaves), l.xy_bytes, st, a);
  return hipGetLastError();
}

hipError_t launch_oz_zfinal(const OzArgs& a, int occ, hipStream_t st) {
  const OzLds l = oz_lds(a.m1, a.m2, a.m3);
  const dim3 g(a.norb * a.m2), b(64 * kOzZWaves);
  if (occ == 4) hipLaunchKernelGGL(k_oz_zfinal<4>, g, b, l.z_bytes, st, a);
  else hipLaunchKernelGGL(k_oz_zfinal<2>, g, b, l.z_bytes, st, a);
  return hipGetLastError();
}

}  // namespace wvl
