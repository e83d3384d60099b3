// Lower-order field pipeline (float64).
//
// The linear part of the effective field, exchange + periodic demagnetization
// + uniaxial anisotropy, is one symmetric 3x3 Fourier multiplier (FieldArgs in
// pipeline.h): the anisotropy matrix 2K e e^T is constant in space, so it
// commutes with the DFT.  Unlike the scalar multipliers of the Krylov
// operators it couples the three components, so it is applied by its own
// kernel between complete forward and inverse transforms:
//   2D: x-forward, y-forward, k_field3, y-inverse, x-inverse
//   3D: x-forward, y-forward, z-forward, k_field3, z-inverse, y-inverse, x-inverse
// The pipeline runs once per Picard iteration (right-hand side), per energy
// or diagnostic evaluation, and per adjoint Krylov iteration when the
// lower-order field is present; the forward Krylov operators do not use it.
#include "pipeline_run.h"

namespace llg {

// One thread per (kx, y, z) spectral point: read the three half-spectrum
// values, apply M(xi) / N_g, write them back.
__global__ __launch_bounds__(256) void k_field3(cx<double>* __restrict__ spec, SpecGeom g, FieldArgs fa) {
  const long long npts = (long long)(g.nh + 1) * g.ny * g.nz;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= npts) return;
  const int kx = int(t % (g.nh + 1));
  const long long row = t / (g.nh + 1);
  const int y = int(row % g.ny), z = int(row / g.ny);
  const int ky = y < g.ny / 2 ? y : y - g.ny;
  const int kz = (g.nz == 1 || z < g.nz / 2) ? z : z - g.nz;
  const double xx = fa.cx * kx, yy = fa.cy * ky, zz = fa.cz * kz;
  const double s2 = xx * xx + yy * yy + zz * zz;
  // derivative wave vector: Nyquist entries (kx = nx/2, ky = -ny/2, kz = -nz/2) are zero
  const double dx = kx == g.nh ? 0.0 : xx;
  const double dy = (g.ny > 1 && ky == -g.ny / 2) ? 0.0 : yy;
  const double dz = (g.nz > 1 && kz == -g.nz / 2) ? 0.0 : zz;
  const double q = s2 > 0.0 ? fa.s_dm / s2 : 0.0;
  const double d = fa.s_id + fa.s_ex * s2;
  const double e[3] = {fa.e0, fa.e1, fa.e2};
  const double w[3] = {dx, dy, dz};
  cx<double>* p = spec + row * g.rs + kx;
  const int stride = g.nh + 1;
  const cx<double> u[3] = {p[0], p[stride], p[2 * stride]};
  const double wu_r = w[0] * u[0].x + w[1] * u[1].x + w[2] * u[2].x;
  const double wu_i = w[0] * u[0].y + w[1] * u[1].y + w[2] * u[2].y;
  const double eu_r = e[0] * u[0].x + e[1] * u[1].x + e[2] * u[2].x;
  const double eu_i = e[0] * u[0].y + e[1] * u[1].y + e[2] * u[2].y;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double re = d * u[c].x + q * w[c] * wu_r + fa.s_an * e[c] * eu_r;
    const double im = d * u[c].y + q * w[c] * wu_i + fa.s_an * e[c] * eu_i;
    p[c * stride] = cx<double>{re * fa.inv_ng, im * fa.inv_ng};
  }
}

template <int NH>
static hipError_t field_nh(const Ctx& c, const FieldArgs& fa, int epi, const NodalArgs& na,
                           const PipeIO<double, double, double>& io, hipStream_t st) {
  using T = double;
  launch_xfwd<T, T, T, NH, PRO_COPY3>(c, na, io, st);
  cx<T>* spec = reinterpret_cast<cx<T>*>(c.spec);
  const SymArgs none{};
  hipError_t e;
  if ((e = launch_axis<T>(c, 1, 0, none, spec, st)) != hipSuccess) return e;
  if (c.dim == 3 && (e = launch_axis<T>(c, 2, 0, none, spec, st)) != hipSuccess) return e;
  {
    const long long npts = (long long)(c.geom.nh + 1) * c.ny * c.nz;
    ProfScope ps(c.prof, st, KK_FIELD3, double(npts) * 3 * 2 * sizeof(cx<T>));
    hipLaunchKernelGGL(k_field3, dim3(unsigned((npts + 255) / 256)), dim3(256), 0, st, spec, c.geom, fa);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (c.dim == 3 && (e = launch_axis<T>(c, 2, 1, none, spec, st)) != hipSuccess) return e;
  if ((e = launch_axis<T>(c, 1, 1, none, spec, st)) != hipSuccess) return e;
  switch (epi) {
    case EPI_STORE3: launch_xinv<T, T, T, NH, EPI_STORE3>(c, na, io, st); break;
    case EPI_RHS: launch_xinv<T, T, T, NH, EPI_RHS>(c, na, io, st); break;
    case EPI_ADDF: launch_xinv<T, T, T, NH, EPI_ADDF>(c, na, io, st); break;
    case EPI_JT: launch_xinv<T, T, T, NH, EPI_JT>(c, na, io, st); break;
    case EPI_ENERGY: launch_xinv<T, T, T, NH, EPI_ENERGY>(c, na, io, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t run_field(const Ctx& c, const FieldArgs& fa, int epi, const NodalArgs& na,
                     const PipeIO<double, double, double>& io, hipStream_t st) {
  switch (c.geom.nh) {
#define LLG_CASE(n) \
  case n: return field_nh<n>(c, fa, epi, na, io, st);
    LLG_FOR_NH(LLG_CASE)
#undef LLG_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace llg
