// Per-mode standard PSATD update on the staggered grid (Sec. 4.2, eqs.
// eq_update_B_with_rho_standard and eq_update_E_with_rho_standard), c = eps0 = 1:
//   B' = C B - i (S/w) [k]_s x E + i X1 [k]_s x J
//   E' = C E + i (S/w) [k]_s x B + X4 J + i (X3 rho^n - X2 rho^{n+1}) [k]_s,   X4 = -S/w.
// The paper states the update in the Fourier convention of App. A, where every
// component is transformed at its own Yee position.  The spectra handled here are
// plain index-space DFTs; multiplying the paper's equations through by the
// components' half-cell phase factors turns each i[k^d]_s into
//   D+_d = i [k^d]_s exp(+i k^d dx_d / 2)   (derivative from nodes to centres, App. A
//                                            eq. staggered_finite_difference_nodal),
//   D-_d = i [k^d]_s exp(-i k^d dx_d / 2)   (centres to nodes, the inverse shift),
// so the update needs no extra phase:
//   bx' = C bx - Sw (D+y ez - D+z ey) + X1 (D+y jz - D+z jy)            (and cyclic)
//   ex' = C ex + Sw (D-y bz - D-z by) - Sw jx + (X3 ro - X2 rn) D+x      (and cyclic)
// One thread per half-spectrum mode; every array is read and written once.
// Optionally (spectral centering) the nodal current is centred to the Yee grid and the
// updated fields back to the nodes inside the same pass, by the centering's Fourier
// symbol: on a periodic grid the finite-order stencil of Sec. 3 is exactly that
// multiplication (App. C), so the result equals real-space centering up to rounding.
#include "kernels.h"

namespace pic {

namespace {

// SPECTRAL: the currents arrive on the nodes and are centred by Tc (Sec. 3 centering as
// its exact Fourier symbol on the periodic grid, App. C), and the updated E, B are also
// written centred back to the nodes (conj Tc along the same axes as in real space).
// GAL: the standard Galilean update of Sec. 4.3 (eqs. eq_update_B/E_with_rho_galilean) with
// its complex per-mode coefficients in place of the real ones:
//   bx' = TC bx - TS (D+y ez - D+z ey) + X1 (D+y jz - D+z jy)
//   ex' = TC ex + TS (D-y bz - D-z by) + X4 jx + (TX3 ro - X2 rn) D+x,
// TC = theta^2 C, TS = theta^2 S/w_s, TX3 = theta^2 X3 (theta = exp(i v_gal . [k]_c dt / 2)).
// AVG (with GAL): also the averaged fields of Sec. 4.4 (eqs. eq_update_B/E_with_rho_averaged)
// from the start values, into NOD (Yee-grid spectra), [k]_s = -i D+ for the charge term:
//   <bx> = Psi1 bx + Psi2 (D+y ez - D+z ey) + Y1 (D+y jz - D+z jy)
//   <ex> = Psi1 ex - Psi2 (D-y bz - D-z by) + Y4 jx - i (Y3 ro + Y2 rn) D+x.
// CC (standard update): the current is first projected onto the Fourier-space continuity
// equation of App. A, (rho^{n+1} - rho^n)/dt + i [k]_s . J = 0, with the update's own [k]_s.
// In the paper's convention J' = J - [k]_s ([k]_s . J - i (rn - ro)/dt) / |[k]_s|^2; with the
// index-space operators (D-_d D+_d = -[k_d]_s^2, |D+_d| = |[k_d]_s|) that is
//   R = D-x jx + D-y jy + D-z jz + (rn - ro)/dt,   j_d' = j_d + D+_d R / |D+|^2,
// and modes with |D+| = 0 (k = 0, the nodal solver's Nyquist planes) keep J.
template <typename T, bool SPECTRAL, bool GAL, bool AVG = false, bool CC = false>
__global__ void __launch_bounds__(256) k_psatd_update(PsatdTables<T> t, Batch<cplx<T>*> F, Batch<const cplx<T>*> S,
                                                      Batch<cplx<T>*> NOD, int nx, int ny, int nzh, int pz) {
  const long long total = (long long)nx * ny * nzh;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int kz = (int)(idx % nzh);
  const long long r = idx / nzh;
  const int j = (int)(r % ny);
  const int i = (int)(r / ny);
  const size_t a = (size_t)r * pz + kz;

  const cplx<T> px = t.Dp[0][i], py = t.Dp[1][j], pzd = t.Dp[2][kz];
  const cplx<T> mx = t.Dm[0][i], my = t.Dm[1][j], mz = t.Dm[2][kz];
  // coefficients as complex numbers (imaginary parts zero for standard PSATD)
  cplx<T> gC, gS, g1, g2, g3, g4;
  if (GAL) {
    gC = t.G[0][idx];
    gS = t.G[1][idx];
    g1 = t.G[2][idx];
    g2 = t.G[3][idx];
    g3 = t.G[4][idx];
    g4 = t.G[5][idx];
  } else {
    const T Sw = t.Sw[idx];
    gC = cmake(t.C[idx], (T)0);
    gS = cmake(Sw, (T)0);
    g1 = cmake(t.X1[idx], (T)0);
    g2 = cmake(t.X2[idx], (T)0);
    g3 = cmake(t.X3[idx], (T)0);
    g4 = cmake(-Sw, (T)0);
  }
  // a * z for a coefficient a of the mode: a real scale in the standard update
  auto mul = [&](cplx<T> c, cplx<T> z) { return GAL ? cmul(c, z) : cscale(z, c.x); };

  const cplx<T> ex = F.p[0][a], ey = F.p[1][a], ez = F.p[2][a];
  const cplx<T> bx = F.p[3][a], by = F.p[4][a], bz = F.p[5][a];
  cplx<T> jx = S.p[0][a], jy = S.p[1][a], jz = S.p[2][a];
  cplx<T> tcx, tcy, tcz;
  if (SPECTRAL) {
    tcx = t.Tc[0][i];
    tcy = t.Tc[1][j];
    tcz = t.Tc[2][kz];
    jx = cmul(jx, tcx);
    jy = cmul(jy, tcy);
    jz = cmul(jz, tcz);
  }
  const cplx<T> ro = S.p[3][a], rn = S.p[4][a];
  if (CC) {
    const T k2 = px.x * px.x + px.y * px.y + py.x * py.x + py.y * py.y + pzd.x * pzd.x + pzd.y * pzd.y;
    if (k2 > (T)0) {
      const cplx<T> R =
          cadd(cadd(cadd(cmul(mx, jx), cmul(my, jy)), cmul(mz, jz)), cscale(csub(rn, ro), t.inv_dt));
      const cplx<T> f = cscale(R, (T)1 / k2);
      jx = cadd(jx, cmul(px, f));
      jy = cadd(jy, cmul(py, f));
      jz = cadd(jz, cmul(pzd, f));
    }
  }

  // B update: curl terms with D+ (E, J live on edges; B on faces)
  const cplx<T> cEx = csub(cmul(py, ez), cmul(pzd, ey));
  const cplx<T> cEy = csub(cmul(pzd, ex), cmul(px, ez));
  const cplx<T> cEz = csub(cmul(px, ey), cmul(py, ex));
  const cplx<T> cJx = csub(cmul(py, jz), cmul(pzd, jy));
  const cplx<T> cJy = csub(cmul(pzd, jx), cmul(px, jz));
  const cplx<T> cJz = csub(cmul(px, jy), cmul(py, jx));
  if (AVG) {  // from the start values (E, B are overwritten below)
    const cplx<T> P1 = t.Av[0][idx], P2 = t.Av[1][idx], Y1 = t.Av[2][idx], Y2 = t.Av[3][idx], Y3 = t.Av[4][idx],
                  Y4 = t.Av[5][idx];
    const cplx<T> cBx = csub(cmul(my, bz), cmul(mz, by));
    const cplx<T> cBy = csub(cmul(mz, bx), cmul(mx, bz));
    const cplx<T> cBz = csub(cmul(mx, by), cmul(my, bx));
    const cplx<T> r2 = cadd(cmul(Y3, ro), cmul(Y2, rn));
    const cplx<T> mr = cmake(r2.y, -r2.x);  // -i (Y3 ro + Y2 rn)
    NOD.p[0][a] = cadd(cadd(csub(cmul(P1, ex), cmul(P2, cBx)), cmul(Y4, jx)), cmul(mr, px));
    NOD.p[1][a] = cadd(cadd(csub(cmul(P1, ey), cmul(P2, cBy)), cmul(Y4, jy)), cmul(mr, py));
    NOD.p[2][a] = cadd(cadd(csub(cmul(P1, ez), cmul(P2, cBz)), cmul(Y4, jz)), cmul(mr, pzd));
    NOD.p[3][a] = cadd(cadd(cmul(P1, bx), cmul(P2, cEx)), cmul(Y1, cJx));
    NOD.p[4][a] = cadd(cadd(cmul(P1, by), cmul(P2, cEy)), cmul(Y1, cJy));
    NOD.p[5][a] = cadd(cadd(cmul(P1, bz), cmul(P2, cEz)), cmul(Y1, cJz));
  }
  const cplx<T> nbx = cadd(csub(mul(gC, bx), mul(gS, cEx)), mul(g1, cJx));
  const cplx<T> nby = cadd(csub(mul(gC, by), mul(gS, cEy)), mul(g1, cJy));
  const cplx<T> nbz = cadd(csub(mul(gC, bz), mul(gS, cEz)), mul(g1, cJz));
  F.p[3][a] = nbx;
  F.p[4][a] = nby;
  F.p[5][a] = nbz;

  // E update: curl of B with D-, source terms
  const cplx<T> cBx = csub(cmul(my, bz), cmul(mz, by));
  const cplx<T> cBy = csub(cmul(mz, bx), cmul(mx, bz));
  const cplx<T> cBz = csub(cmul(mx, by), cmul(my, bx));
  const cplx<T> rr = csub(mul(g3, ro), mul(g2, rn));
  const cplx<T> nex = cadd(cadd(cadd(mul(gC, ex), mul(gS, cBx)), mul(g4, jx)), cmul(rr, px));
  const cplx<T> ney = cadd(cadd(cadd(mul(gC, ey), mul(gS, cBy)), mul(g4, jy)), cmul(rr, py));
  const cplx<T> nez = cadd(cadd(cadd(mul(gC, ez), mul(gS, cBz)), mul(g4, jz)), cmul(rr, pzd));
  F.p[0][a] = nex;
  F.p[1][a] = ney;
  F.p[2][a] = nez;
  if (SPECTRAL) {  // centres -> nodes: E^d along d, B^d along the two other axes
    const cplx<T> sx = cconj(tcx), sy = cconj(tcy), sz = cconj(tcz);
    NOD.p[0][a] = cmul(nex, sx);
    NOD.p[1][a] = cmul(ney, sy);
    NOD.p[2][a] = cmul(nez, sz);
    NOD.p[3][a] = cmul(cmul(nbx, sy), sz);
    NOD.p[4][a] = cmul(cmul(nby, sx), sz);
    NOD.p[5][a] = cmul(cmul(nbz, sx), sy);
  }
}

// Adjoint (conjugate transpose per mode) of the update above, for reverse-mode
// differentiation.  F holds the adjoints of the updated E (0..2) and B (3..5) and is
// overwritten with those of the old E, B; A receives the adjoints of J (0..2), rho^n (3)
// and rho^{n+1} (4).  With a x v = A_a v, (A_a)^H w = -(conj a) x w, so
//   lE = C lE' + Sw (conj D+ x lB'),   lB = C lB' - Sw (conj D- x lE'),
//   lJ = -X1 (conj D+ x lB') - Sw lE',  lro = X3 conj D+ . lE',  lrn = -X2 conj D+ . lE'.
// CC: then the transpose of the current correction j' = j + D+ (D- . j + (rn - ro)/dt)/|D+|^2:
//   s = conj D+ . lJ / |D+|^2,  lJ += conj D- s,  lrn += s/dt,  lro -= s/dt.
template <typename T, bool CC = false>
__global__ void __launch_bounds__(256) k_psatd_adjoint(PsatdTables<T> t, Batch<cplx<T>*> F, Batch<cplx<T>*> A, int nx,
                                                       int ny, int nzh, int pz) {
  const long long total = (long long)nx * ny * nzh;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int kz = (int)(idx % nzh);
  const long long r = idx / nzh;
  const int j = (int)(r % ny);
  const int i = (int)(r / ny);
  const size_t a = (size_t)r * pz + kz;
  const T C = t.C[idx], Sw = t.Sw[idx], X1 = t.X1[idx], X2 = t.X2[idx], X3 = t.X3[idx];
  const cplx<T> px = cconj(t.Dp[0][i]), py = cconj(t.Dp[1][j]), pzd = cconj(t.Dp[2][kz]);
  const cplx<T> mx = cconj(t.Dm[0][i]), my = cconj(t.Dm[1][j]), mz = cconj(t.Dm[2][kz]);
  const cplx<T> ex = F.p[0][a], ey = F.p[1][a], ez = F.p[2][a];
  const cplx<T> bx = F.p[3][a], by = F.p[4][a], bz = F.p[5][a];
  // conj(D+) x lB' and conj(D-) x lE'
  const cplx<T> pBx = csub(cmul(py, bz), cmul(pzd, by));
  const cplx<T> pBy = csub(cmul(pzd, bx), cmul(px, bz));
  const cplx<T> pBz = csub(cmul(px, by), cmul(py, bx));
  const cplx<T> mEx = csub(cmul(my, ez), cmul(mz, ey));
  const cplx<T> mEy = csub(cmul(mz, ex), cmul(mx, ez));
  const cplx<T> mEz = csub(cmul(mx, ey), cmul(my, ex));
  const cplx<T> dE = cadd(cadd(cmul(px, ex), cmul(py, ey)), cmul(pzd, ez));
  F.p[0][a] = cadd(cscale(ex, C), cscale(pBx, Sw));
  F.p[1][a] = cadd(cscale(ey, C), cscale(pBy, Sw));
  F.p[2][a] = cadd(cscale(ez, C), cscale(pBz, Sw));
  F.p[3][a] = csub(cscale(bx, C), cscale(mEx, Sw));
  F.p[4][a] = csub(cscale(by, C), cscale(mEy, Sw));
  F.p[5][a] = csub(cscale(bz, C), cscale(mEz, Sw));
  cplx<T> lj[3] = {csub(cscale(pBx, -X1), cscale(ex, Sw)), csub(cscale(pBy, -X1), cscale(ey, Sw)),
                   csub(cscale(pBz, -X1), cscale(ez, Sw))};
  cplx<T> lro = cscale(dE, X3), lrn = cscale(dE, -X2);
  if (CC) {
    const T k2 = px.x * px.x + px.y * px.y + py.x * py.x + py.y * py.y + pzd.x * pzd.x + pzd.y * pzd.y;
    if (k2 > (T)0) {
      const cplx<T> sj = cscale(cadd(cadd(cmul(px, lj[0]), cmul(py, lj[1])), cmul(pzd, lj[2])), (T)1 / k2);
      lj[0] = cadd(lj[0], cmul(mx, sj));
      lj[1] = cadd(lj[1], cmul(my, sj));
      lj[2] = cadd(lj[2], cmul(mz, sj));
      const cplx<T> sd = cscale(sj, t.inv_dt);
      lrn = cadd(lrn, sd);
      lro = csub(lro, sd);
    }
  }
  A.p[0][a] = lj[0];
  A.p[1][a] = lj[1];
  A.p[2][a] = lj[2];
  A.p[3][a] = lro;
  A.p[4][a] = lrn;
}

}  // namespace

template <typename T>
void psatd_adjoint(const PsatdTables<T>& t, cplx<T>* const E[3], cplx<T>* const B[3], cplx<T>* const J[3],
                   cplx<T>* rho_old, cplx<T>* rho_new, int nx, int ny, int nzh, int pz, hipStream_t s) {
  Batch<cplx<T>*> F{}, A{};
  for (int d = 0; d < 3; ++d) {
    F.p[d] = E[d];
    F.p[3 + d] = B[d];
    A.p[d] = J[d];
  }
  A.p[3] = rho_old;
  A.p[4] = rho_new;
  const long long total = (long long)nx * ny * nzh;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (t.cc)
    hipLaunchKernelGGL((k_psatd_adjoint<T, true>), grid, dim3(256), 0, s, t, F, A, nx, ny, nzh, pz);
  else
    hipLaunchKernelGGL((k_psatd_adjoint<T, false>), grid, dim3(256), 0, s, t, F, A, nx, ny, nzh, pz);
}

template <typename T>
void psatd_update(const PsatdTables<T>& t, cplx<T>* const E[3], cplx<T>* const B[3], const cplx<T>* const J[3],
                  const cplx<T>* rho_old, const cplx<T>* rho_new, int nx, int ny, int nzh, int pz,
                  cplx<T>* const* nodal, hipStream_t s) {
  Batch<cplx<T>*> F{};
  Batch<const cplx<T>*> S{};
  for (int d = 0; d < 3; ++d) {
    F.p[d] = E[d];
    F.p[3 + d] = B[d];
    S.p[d] = J[d];
  }
  S.p[3] = rho_old;
  S.p[4] = rho_new;
  Batch<cplx<T>*> N{};
  if (nodal)
    for (int q = 0; q < 6; ++q) N.p[q] = nodal[q];
  const long long total = (long long)nx * ny * nzh;
  const dim3 grid((unsigned)((total + 255) / 256));
  if (nodal && !t.Av[0] && t.cc)  // spectral centering (standard PSATD only), current correction
    hipLaunchKernelGGL((k_psatd_update<T, true, false, false, true>), grid, dim3(256), 0, s, t, F, S, N, nx, ny, nzh,
                       pz);
  else if (nodal && !t.Av[0])  // spectral centering (standard PSATD only)
    hipLaunchKernelGGL((k_psatd_update<T, true, false>), grid, dim3(256), 0, s, t, F, S, N, nx, ny, nzh, pz);
  else if (t.Av[0])
    hipLaunchKernelGGL((k_psatd_update<T, false, true, true>), grid, dim3(256), 0, s, t, F, S, N, nx, ny, nzh, pz);
  else if (t.G[0])
    hipLaunchKernelGGL((k_psatd_update<T, false, true>), grid, dim3(256), 0, s, t, F, S, N, nx, ny, nzh, pz);
  else if (t.cc)
    hipLaunchKernelGGL((k_psatd_update<T, false, false, false, true>), grid, dim3(256), 0, s, t, F, S, N, nx, ny, nzh,
                       pz);
  else
    hipLaunchKernelGGL((k_psatd_update<T, false, false>), grid, dim3(256), 0, s, t, F, S, N, nx, ny, nzh, pz);
}

template void psatd_update<float>(const PsatdTables<float>&, cplx<float>* const*, cplx<float>* const*,
                                  const cplx<float>* const*, const cplx<float>*, const cplx<float>*, int, int, int,
                                  int, cplx<float>* const*, hipStream_t);
template void psatd_update<double>(const PsatdTables<double>&, cplx<double>* const*, cplx<double>* const*,
                                   const cplx<double>* const*, const cplx<double>*, const cplx<double>*, int, int,
                                   int, int, cplx<double>* const*, hipStream_t);

}  // namespace pic

namespace pic {
template void psatd_adjoint<float>(const PsatdTables<float>&, cplx<float>* const*, cplx<float>* const*,
                                   cplx<float>* const*, cplx<float>*, cplx<float>*, int, int, int, int, hipStream_t);
template void psatd_adjoint<double>(const PsatdTables<double>&, cplx<double>* const*, cplx<double>* const*,
                                    cplx<double>* const*, cplx<double>*, cplx<double>*, int, int, int, int,
                                    hipStream_t);
}  // namespace pic
