// Frequency-domain layout of the two-pass (four-step) 256^3 transform.
//
// The y axis is split as ky = n1 + 16 n2.  The frequency side of the 3D
// transform works on tiles (kxb, n1) of 16384 values: four x frequencies
// kx = 4 kxb + kxx, the sixteen ky with ky mod 16 = n1, and all 256 kz.
// Inside a tile the order is [kz / 16][n2][kz mod 16][kxx], so that the
// kernels that read or write the frequency side move whole tiles with fully
// contiguous 8 KiB rows.  F, the bank rows, M and the orientation sum X all
// use this order; natural order appears only at the C ABI's export calls.
#pragma once
#include <hip/hip_runtime.h>

namespace os3d {

constexpr int kLayoutNatural = 0;
constexpr int kLayoutFour256 = 1;

__host__ __device__ inline void l4_to_k(long long p, int& kz, int& ky, int& kx) {
  const int tile = (int)(p >> 14), in = (int)(p & 16383);
  const int kxb = tile >> 4, n1 = tile & 15;
  const int kxx = in & 3, kzl = (in >> 2) & 15, n2 = (in >> 6) & 15, kzh = in >> 10;
  kz = kzh * 16 + kzl;
  ky = n1 + 16 * n2;
  kx = 4 * kxb + kxx;
}

__host__ __device__ inline long long k_to_l4(int kz, int ky, int kx) {
  const int kxb = kx >> 2, kxx = kx & 3, n1 = ky & 15, n2 = ky >> 4;
  return ((long long)(kxb * 16 + n1) << 14) + ((((kz >> 4) * 16 + n2)) << 6) + ((kz & 15) << 2) + kxx;
}

// Frequency indices of storage position p under `layout` for dims (Nz, Ny, Nx).
__host__ __device__ inline void pos_to_k(int layout, long long p, int Nz, int Ny, int Nx, int& kz, int& ky, int& kx) {
  if (layout == kLayoutFour256) {
    l4_to_k(p, kz, ky, kx);
    return;
  }
  kx = (int)(p % Nx);
  ky = (int)((p / Nx) % Ny);
  kz = (int)(p / ((long long)Nx * Ny));
}

__host__ __device__ inline long long k_to_pos(int layout, int kz, int ky, int kx, int Ny, int Nx) {
  if (layout == kLayoutFour256) return k_to_l4(kz, ky, kx);
  return ((long long)kz * Ny + ky) * Nx + kx;
}

}  // namespace os3d
