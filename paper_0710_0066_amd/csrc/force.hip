// Force and molecular-dynamics kernels (FP64) for gfx950.
//
// Convention: F^a(x,mu) = dS/dw along U_mu(x) -> exp(i w T^a) U_mu(x), T^a = lambda^a/2;
// the momentum kick p <- p - dt F is applied by passing F = p and coef = -dt.
//
// pair force: F += coef * 2 Re <a, (d_{x,mu,a} W) b> for the hop operator W = M (eq. 2)
// or its x0-block restriction (links between blocks are absent: zero). With the two
// entries of W that contain U_mu(x), and (1 -/+ gamma) = 2 x (Hermitian projector),
//   F^a = -kappa Im tr( lambda^a Q ),   Q = Y U^+ - U X,
//   X = sum_k hb_k (x) ha_k^*   (half spinors of (1 - gamma_mu) b(x+mu) and of a(x)),
//   Y = sum_k hb'_k (x) ha'_k^* (half spinors of (1 + gamma_mu) b(x) and of a(x+mu)),
// with the x0 wrap phase -1 on the link at x0 = L0-1.
// gauge force (Wilson plaquette action, Sec. 1): F^a = (beta/6) Im tr(lambda^a U A),
// A = sum of the six staples of U_mu(x).
// T_U (Sec. 2, eq. 3): U <- exp(i dt P) U, exponential by scaling and squaring of a
// degree-16 Taylor polynomial, then Gram-Schmidt reunitarisation with the third row the
// conjugate cross product of the first two (exactly unitary, det 1 up to rounding).
#include "force.h"

namespace sap {

typedef cx<double> C;

struct M3 { C m[9]; };

__device__ __forceinline__ M3 mmul(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      C t = cmul(a.m[3 * i], b.m[k]);
      t = cfma(t, a.m[3 * i + 1], b.m[3 + k]);
      t = cfma(t, a.m[3 * i + 2], b.m[6 + k]);
      r.m[3 * i + k] = t;
    }
  return r;
}
// a * b^dagger
__device__ __forceinline__ M3 mmul_nd(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      C t = cmulj(a.m[3 * i], b.m[3 * k]);
      t = t + cmulj(a.m[3 * i + 1], b.m[3 * k + 1]);
      t = t + cmulj(a.m[3 * i + 2], b.m[3 * k + 2]);
      r.m[3 * i + k] = t;
    }
  return r;
}
// a^dagger * b
__device__ __forceinline__ M3 mmul_dn(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      C t = cjmul(a.m[i], b.m[k]);
      t = cjfma(t, a.m[3 + i], b.m[3 + k]);
      t = cjfma(t, a.m[6 + i], b.m[6 + k]);
      r.m[3 * i + k] = t;
    }
  return r;
}

__device__ __forceinline__ M3 load_U(const double2* U, long long Vhp, int par, long long j, int mu) {
  M3 r;
  const double2* p = U + par * 36 * Vhp + tiled(j, 9 * mu, 36);
#pragma unroll
  for (int e = 0; e < 9; ++e) r.m[e] = ld<double>(p + e * TILE);
  return r;
}
__device__ __forceinline__ void store_U(double2* U, long long Vhp, int par, long long j, int mu, const M3& r) {
  double2* p = U + par * 36 * Vhp + tiled(j, 9 * mu, 36);
#pragma unroll
  for (int e = 0; e < 9; ++e) st<double>(p + e * TILE, r.m[e]);
}

__device__ __forceinline__ void load_sp(const double2* f, long long j, C s[4][3]) {
  const double2* q = f + tiled(j, 0, 12);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) s[sp][c] = ld<double>(q + (sp * 3 + c) * TILE);
}
__device__ __forceinline__ void store_sp(double2* f, long long j, const C s[4][3]) {
  double2* q = f + tiled(j, 0, 12);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) st<double>(q + (sp * 3 + c) * TILE, s[sp][c]);
}

// Im tr(lambda^a Q) for a = 1..8 into out[0..7] (Q row-major, Q_ij = m[3i+j])
__device__ __forceinline__ void im_tr_lambda(const M3& Q, double out[8]) {
  const C* q = Q.m;
  out[0] = q[3].i + q[1].i;                 // lambda1: Q10 + Q01
  out[1] = -q[3].r + q[1].r;                // lambda2: -i Q10 + i Q01
  out[2] = q[0].i - q[4].i;                 // lambda3: Q00 - Q11
  out[3] = q[6].i + q[2].i;                 // lambda4: Q20 + Q02
  out[4] = -q[6].r + q[2].r;                // lambda5: -i Q20 + i Q02
  out[5] = q[7].i + q[5].i;                 // lambda6: Q21 + Q12
  out[6] = -q[7].r + q[5].r;                // lambda7: -i Q21 + i Q12
  out[7] = (q[0].i + q[4].i - 2.0 * q[8].i) * 0.57735026918962576451;  // lambda8
}

__device__ __forceinline__ void add_force(double* F, long long Vhp, int par, long long j, int mu, double c,
                                          const double v[8]) {
  double* p = F + par * 32 * Vhp + tiled(j, 8 * mu, 32);
#pragma unroll
  for (int a = 0; a < 8; ++a) p[a * TILE] += c * v[a];
}

// sum_k h1_k (x) conj(h2_k) as a colour matrix
__device__ __forceinline__ M3 outer2(const C h1[2][3], const C h2[2][3]) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) r.m[3 * i + k] = cmulj(h1[0][i], h2[0][k]) + cmulj(h1[1][i], h2[1][k]);
  return r;
}

// One work-item per link: a workgroup holds 64 sites of one parity (blockIdx.y) and one
// wavefront per direction mu (the four wavefronts read the same site spinors through L2).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void k_pair_force(Geo g, double* F, double c, const double2* a, const double2* b, const double2* U, int lb,
                  const double* sx) {
  const int mu = threadIdx.x >> 6;
  const int p = blockIdx.y;
  const long long j = (long long)blockIdx.x * 64 + (threadIdx.x & 63);
  if (j >= g.Vh) return;
  const long long Vhp = g.Vhp;
  const Site s = decode(g, j, p);
  if (lb && mu == 0 && (s.x0 % lb) == lb - 1) return;    // link absent from W
  const long long jn = nbr(g, s, j, mu, +1);
  const double2* ap = a + p * 12 * Vhp;
  const double2* bp = b + p * 12 * Vhp;
  const double2* aq = a + (1 - p) * 12 * Vhp;
  const double2* bq = b + (1 - p) * 12 * Vhp;
  C sp[4][3], hb[2][3], ha[2][3];
  // X = sum_k hb_k (x) ha_k^*: (1 - gamma_mu) b(x + mu) and a(x)
  load_sp(bq, jn, sp);
  project<double>(mu, false, sp, hb);
  load_sp(ap, j, sp);
  project<double>(mu, false, sp, ha);
  const M3 X = outer2(hb, ha);
  // Y: (1 + gamma_mu) b(x) and a(x + mu)
  load_sp(bp, j, sp);
  project<double>(mu, true, sp, hb);
  load_sp(aq, jn, sp);
  project<double>(mu, true, sp, ha);
  const M3 Y = outer2(hb, ha);
  const M3 Um = load_U(U, Vhp, p, j, mu);
  const M3 YU = mmul_nd(Y, Um), UX = mmul(Um, X);
  M3 Q;
#pragma unroll
  for (int e = 0; e < 9; ++e) Q.m[e] = YU.m[e] - UX.m[e];
  double v[8];
  im_tr_lambda(Q, v);
  const double sgn = (mu == 0 && s.x0 == g.L0 - 1) ? -1.0 : 1.0;
  add_force(F, Vhp, p, j, mu, c * sgn * (sx ? sx[s.x0 * 4 + mu] : 1.0), v);
}

// Staple sum of U_mu(x):
//   A = sum_{nu != mu} U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ + U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
__device__ M3 staples(const Geo& g, const double2* U, int p, long long j, const Site& s, int mu) {
  const long long Vhp = g.Vhp;
  M3 A;
#pragma unroll
  for (int e = 0; e < 9; ++e) A.m[e] = {0.0, 0.0};
  const long long jpm = nbr(g, s, j, mu, +1);                 // x+mu, parity 1-p
  const Site spm = decode(g, jpm, 1 - p);
  // one direction at a time: unrolling would keep the links of all six staples live
#pragma unroll 1
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    const long long jpn = nbr(g, s, j, nu, +1);               // x+nu, parity 1-p
    const long long jmn = nbr(g, s, j, nu, -1);               // x-nu, parity 1-p
    const long long jpmmn = nbr(g, spm, jpm, nu, -1);         // x+mu-nu, parity p
    // U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+ (the memory fences keep the scheduler from
    // loading the links of both staples at once, which would cost occupancy)
    const M3 ab = mmul_nd(load_U(U, Vhp, 1 - p, jpm, nu), load_U(U, Vhp, 1 - p, jpn, mu));
    asm volatile("" ::: "memory");
    const M3 up = mmul_nd(ab, load_U(U, Vhp, p, j, nu));
#pragma unroll
    for (int e = 0; e < 9; ++e) A.m[e] = A.m[e] + up.m[e];
    asm volatile("" ::: "memory");
    // U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu) = (U_mu(x-nu) U_nu(x+mu-nu))^+ U_nu(x-nu)
    const M3 t = mmul(load_U(U, Vhp, 1 - p, jmn, mu), load_U(U, Vhp, p, jpmmn, nu));
    asm volatile("" ::: "memory");
    const M3 lo = mmul_dn(t, load_U(U, Vhp, 1 - p, jmn, nu));
#pragma unroll
    for (int e = 0; e < 9; ++e) A.m[e] = A.m[e] + lo.m[e];
    asm volatile("" ::: "memory");
  }
  return A;
}

// One work-item per link: a workgroup holds 64 sites of one parity (blockIdx.y) and one
// wavefront per direction mu, so that the staple sums of the four links of a site run in
// parallel and the registers of one staple sum decide the occupancy.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void k_gauge_force(Geo g, double* F, double c, const double2* U, const double* sx) {
  const int mu = threadIdx.x >> 6;
  const int p = blockIdx.y;
  const long long j = (long long)blockIdx.x * 64 + (threadIdx.x & 63);
  if (j >= g.Vh) return;
  const Site s = decode(g, j, p);
  const M3 W = mmul(load_U(U, g.Vhp, p, j, mu), staples(g, U, p, j, s, mu));
  double v[8];
  im_tr_lambda(W, v);
  add_force(F, g.Vhp, p, j, mu, c * (sx ? sx[s.x0 * 4 + mu] : 1.0), v);
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
__device__ __forceinline__ double bsum256(double v) {
  __shared__ double sh[4];
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return (threadIdx.x == 0) ? (sh[0] + sh[1]) + (sh[2] + sh[3]) : 0.0;
}

// Per-workgroup partial of sum_x sum_{mu>nu} Re tr U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
__global__ __launch_bounds__(256) void k_plaq(Geo g, const double2* U, double* part) {
  const int p = threadIdx.x >> 7;
  const long long j = (long long)blockIdx.x * 128 + (threadIdx.x & 127);
  double acc = 0.0;
  if (j < g.Vh) {
    const Site s = decode(g, j, p);
    for (int mu = 1; mu < 4; ++mu)
      for (int nu = 0; nu < mu; ++nu) {
        const long long jpm = nbr(g, s, j, mu, +1), jpn = nbr(g, s, j, nu, +1);
        const M3 a = mmul(load_U(U, g.Vhp, p, j, mu), load_U(U, g.Vhp, 1 - p, jpm, nu));
        const M3 b = mmul(load_U(U, g.Vhp, p, j, nu), load_U(U, g.Vhp, 1 - p, jpn, mu));
        const M3 P = mmul_nd(a, b);
        acc += P.m[0].r + P.m[4].r + P.m[8].r;
      }
  }
  const double t = bsum256(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Per-workgroup maximum over the links of the largest deviation from SU(3): the largest
// entry modulus of U U^+ - 1 and |det U - 1|. A NaN entry gives a NaN maximum (kept by
// the comparisons below), so a non-finite field fails the check as well.
__device__ __forceinline__ double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }
__global__ __launch_bounds__(256) void k_su3_dev(Geo g, const double2* U, double* part) {
  __shared__ double sh[4];
  const int p = threadIdx.x >> 7;
  const long long j = (long long)blockIdx.x * 128 + (threadIdx.x & 127);
  double dev = 0.0;
  if (j < g.Vh) {
    for (int mu = 0; mu < 4; ++mu) {
      const M3 u = load_U(U, g.Vhp, p, j, mu);
      const M3 uu = mmul_nd(u, u);
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        const double re = uu.m[e].r - ((e % 4 == 0) ? 1.0 : 0.0);
        dev = nanmax(dev, sqrt(re * re + uu.m[e].i * uu.m[e].i));
      }
      // det = row 0 . (row 1 x row 2)
      const C c0 = cmul(u.m[4], u.m[8]) - cmul(u.m[5], u.m[7]);
      const C c1 = cmul(u.m[5], u.m[6]) - cmul(u.m[3], u.m[8]);
      const C c2 = cmul(u.m[3], u.m[7]) - cmul(u.m[4], u.m[6]);
      const C det = cmul(u.m[0], c0) + cmul(u.m[1], c1) + cmul(u.m[2], c2);
      dev = nanmax(dev, sqrt((det.r - 1.0) * (det.r - 1.0) + det.i * det.i));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) dev = nanmax(dev, __shfl_down(dev, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = dev;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = nanmax(nanmax(sh[0], sh[1]), nanmax(sh[2], sh[3]));
}

// one wavefront of 64 lanes: lane l takes part[l], part[l + 64], ... in order, then a
// fixed shuffle tree combines the lanes (the result does not depend on timing)
__global__ void k_max_parts(int n, const double* part, double* out) {
  const int l = threadIdx.x;
  double m = 0.0;
  for (int i = l; i < n; i += 64) m = nanmax(m, part[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = nanmax(m, __shfl_down(m, off, 64));
  if (l == 0) out[0] = m;
}

// Per-workgroup partial of 1/2 sum p^2 over valid sites
__global__ __launch_bounds__(256) void k_kinetic(Geo g, const double* P, double* part) {
  const int p = threadIdx.x >> 7;
  const long long j = (long long)blockIdx.x * 128 + (threadIdx.x & 127);
  double acc = 0.0;
  if (j < g.Vh) {
    const double* q = P + p * 32 * g.Vhp + tiled(j, 0, 32);
    for (int k = 0; k < 32; ++k) {
      const double v = q[k * TILE];
      acc += v * v;
    }
  }
  const double t = bsum256(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = 0.5 * t;
}

// one wavefront, as k_max_parts: a fixed order of additions, so the sum is bitwise
// reproducible
__global__ void k_sum_parts(int n, const double* part, double* out) {
  const int l = threadIdx.x;
  double s = 0.0;
  for (int i = l; i < n; i += 64) s += part[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (l == 0) out[0] = s;
}

// exp(A) for anti-Hermitian 3x3 A (Taylor degree 16 after scaling by 2^-k, |A/2^k| <= 1/2)
__device__ M3 expm_ah(const M3& A) {
  double nrm = 0.0;
#pragma unroll
  for (int e = 0; e < 9; ++e) nrm += A.m[e].r * A.m[e].r + A.m[e].i * A.m[e].i;
  nrm = sqrt(nrm);
  int k = 0;
  while (nrm > 0.5 && k < 60) { nrm *= 0.5; ++k; }
  const double sc = ldexp(1.0, -k);
  M3 B;
#pragma unroll
  for (int e = 0; e < 9; ++e) B.m[e] = sc * A.m[e];
  // Horner: E = I + B(I + B/2(I + B/3(... (I + B/16))))
  M3 E;
#pragma unroll
  for (int e = 0; e < 9; ++e) E.m[e] = {0.0, 0.0};
  E.m[0] = E.m[4] = E.m[8] = {1.0, 0.0};
  for (int n = 16; n >= 1; --n) {
    M3 T = mmul(B, E);
    const double inv = 1.0 / n;
#pragma unroll
    for (int e = 0; e < 9; ++e) E.m[e] = inv * T.m[e];
    E.m[0].r += 1.0; E.m[4].r += 1.0; E.m[8].r += 1.0;
  }
  for (int i = 0; i < k; ++i) E = mmul(E, E);
  return E;
}

__device__ M3 reunitarize(const M3& U) {
  M3 R;
  C r0[3] = {U.m[0], U.m[1], U.m[2]}, r1[3] = {U.m[3], U.m[4], U.m[5]};
  double n0 = 0.0;
  for (int c = 0; c < 3; ++c) n0 += r0[c].r * r0[c].r + r0[c].i * r0[c].i;
  n0 = 1.0 / sqrt(n0);
  for (int c = 0; c < 3; ++c) r0[c] = n0 * r0[c];
  C d = {0.0, 0.0};   // <r0, r1>
  for (int c = 0; c < 3; ++c) d = cjfma(d, r0[c], r1[c]);
  for (int c = 0; c < 3; ++c) r1[c] = r1[c] - cmul(d, r0[c]);
  double n1 = 0.0;
  for (int c = 0; c < 3; ++c) n1 += r1[c].r * r1[c].r + r1[c].i * r1[c].i;
  n1 = 1.0 / sqrt(n1);
  for (int c = 0; c < 3; ++c) r1[c] = n1 * r1[c];
  // r2 = conj(r0 x r1)
  C x0 = cmul(r0[1], r1[2]) - cmul(r0[2], r1[1]);
  C x1 = cmul(r0[2], r1[0]) - cmul(r0[0], r1[2]);
  C x2 = cmul(r0[0], r1[1]) - cmul(r0[1], r1[0]);
  R.m[0] = r0[0]; R.m[1] = r0[1]; R.m[2] = r0[2];
  R.m[3] = r1[0]; R.m[4] = r1[1]; R.m[5] = r1[2];
  R.m[6] = {x0.r, -x0.i}; R.m[7] = {x1.r, -x1.i}; R.m[8] = {x2.r, -x2.i};
  return R;
}

// U_mu(x) <- exp(i dt P_mu(x)) U_mu(x), P = sum_a p^a lambda^a / 2
__global__ __launch_bounds__(256) void k_update_links(Geo g, double2* U, LinkCopies lc, const double* Pm, double dt0,
                                                      const double* sx) {
  const int p = threadIdx.x >> 7;
  const long long j = (long long)blockIdx.x * 128 + (threadIdx.x & 127);
  if (j >= g.Vh) return;
  const int x0 = (int)(j / g.V3h);
  for (int mu = 0; mu < 4; ++mu) {
    const double dt = dt0 * (sx ? sx[x0 * 4 + mu] : 1.0);
    if (dt == 0.0) continue;                   // inactive link: stays as it is
    const double* q = Pm + p * 32 * g.Vhp + tiled(j, 8 * mu, 32);
    double a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = q[k * TILE];
    const double r3 = 0.57735026918962576451;
    // P (Hermitian), then A = i dt P
    C P[9];
    P[0] = {0.5 * (a[2] + r3 * a[7]), 0.0};
    P[4] = {0.5 * (-a[2] + r3 * a[7]), 0.0};
    P[8] = {-r3 * a[7], 0.0};
    P[1] = {0.5 * a[0], -0.5 * a[1]}; P[3] = {0.5 * a[0], 0.5 * a[1]};
    P[2] = {0.5 * a[3], -0.5 * a[4]}; P[6] = {0.5 * a[3], 0.5 * a[4]};
    P[5] = {0.5 * a[5], -0.5 * a[6]}; P[7] = {0.5 * a[5], 0.5 * a[6]};
    M3 A;
#pragma unroll
    for (int e = 0; e < 9; ++e) A.m[e] = {-dt * P[e].i, dt * P[e].r};
    const M3 E = expm_ah(A);
    const M3 Un = reunitarize(mmul(E, load_U(U, g.Vhp, p, j, mu)));
    store_U(U, g.Vhp, p, j, mu, Un);
    // the reduced copies of the hop kernels, from the new link in registers
    double2 e[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) e[k] = make_double2(Un.m[k].r, Un.m[k].i);
    write_link_copies(lc, g.Vhp, p, j, mu, e);
  }
}

// U'(x0, ...) = U(x0 + n, ...): translation of the gauge field by n slices in x0
__global__ __launch_bounds__(256) void k_shift_links(Geo g, double2* out, const double2* in, int n) {
  const int p = threadIdx.x >> 7;
  const long long j = (long long)blockIdx.x * 128 + (threadIdx.x & 127);
  if (j >= g.Vh) return;
  const int x0 = (int)(j / g.V3h);
  const long long sidx = j - (long long)x0 * g.V3h;
  int y0 = (x0 + n) % g.L0;
  if (y0 < 0) y0 += g.L0;
  const int py = (p + n) & 1;
  const long long jy = (long long)y0 * g.V3h + sidx;
  for (int mu = 0; mu < 4; ++mu) store_U(out, g.Vhp, p, j, mu, load_U(in, g.Vhp, py, jy, mu));
}

// elementwise helpers on full FP64 spinor fields (both parities, valid sites only)
// mode 0: out = gamma5 in;  1: out = Pi in (black-block boundary projector);
// mode 2: out = in on white blocks, 0 on black;  3: out = a - Pi b
__global__ __launch_bounds__(256) void k_spin_op(Geo g, int mode, int l0, int outer, double2* out,
                                                 const double2* in, const double2* in2) {
  const int p = threadIdx.x >> 7;
  const long long j = (long long)blockIdx.x * 128 + (threadIdx.x & 127);
  if (j >= g.Vh) return;
  const Site s = decode(g, j, p);
  const long long off = p * 12 * g.Vhp;
  C v[4][3];
  load_sp((mode == 3 ? in2 : in) + off, j, v);
  const int blk = s.x0 / l0, r = s.x0 % l0;
  const bool black = (blk & 1) == 1;
  if (mode == 0) {
    for (int c = 0; c < 3; ++c) { v[2][c] = -v[2][c]; v[3][c] = -v[3][c]; }
  } else if (mode == 1 || mode == 3) {
    // first slice of a black block: (1 - g0)/2 -> h = (u + d)/2, (h, h)
    // last slice of a black block:  (1 + g0)/2 -> h = (u - d)/2, (h, -h)
    // with an outer block length, only the slices whose crossing hop exists in W_outer
    const bool first = black && r == 0 && !(outer && s.x0 % outer == 0);
    const bool last = black && r == l0 - 1 && !(outer && s.x0 % outer == outer - 1);
    for (int c = 0; c < 3; ++c)
      for (int k = 0; k < 2; ++k) {
        C h = {0.0, 0.0};
        if (first) h = 0.5 * (v[k][c] + v[k + 2][c]);
        if (last) h = 0.5 * (v[k][c] - v[k + 2][c]);
        v[k][c] = h;
        v[k + 2][c] = last ? -h : h;
      }
    if (mode == 3) {
      C a[4][3];
      load_sp(in + off, j, a);
      for (int sp = 0; sp < 4; ++sp)
        for (int c = 0; c < 3; ++c) v[sp][c] = a[sp][c] - v[sp][c];
    }
  } else if (mode == 2) {
    if (black)
      for (int sp = 0; sp < 4; ++sp)
        for (int c = 0; c < 3; ++c) v[sp][c] = {0.0, 0.0};
  }
  store_sp(out + off, j, v);
}

// partial sums of |f|^2 over both parities (deterministic per-workgroup partials)
__global__ __launch_bounds__(256) void k_norm2_full(Geo g, const double2* f, double* part) {
  const int p = threadIdx.x >> 7;
  const long long j = (long long)blockIdx.x * 128 + (threadIdx.x & 127);
  double acc = 0.0;
  if (j < g.Vh) {
    C v[4][3];
    load_sp(f + p * 12 * g.Vhp, j, v);
    for (int sp = 0; sp < 4; ++sp)
      for (int c = 0; c < 3; ++c) acc += v[sp][c].r * v[sp][c].r + v[sp][c].i * v[sp][c].i;
  }
  const double t = bsum256(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Per-(slice, chunk) partial sums of |F(x, mu)| = (sum_a F^a(x, mu)^2)^(1/2) over 128 slice
// sites of each parity: spatial directions (mu = 1, 2, 3) and time direction (mu = 0).
// part[2 * blockIdx.x + {0, 1}]; blockIdx.x = x0 * nck + chunk.
__global__ __launch_bounds__(256) void k_force_profile(Geo g, const double* F, int nck, double* part) {
  __shared__ double sh[2][4];
  const int x0 = blockIdx.x / nck, ck = blockIdx.x - x0 * nck;
  const int p = threadIdx.x >> 7;
  const int s = ck * 128 + (threadIdx.x & 127);
  double vs = 0.0, vt = 0.0;
  if (s < g.V3h) {
    const long long j = (long long)x0 * g.V3h + s;
    const double* q = F + p * 32 * g.Vhp + tiled(j, 0, 32);
    for (int mu = 0; mu < 4; ++mu) {
      double n2 = 0.0;
      for (int a = 0; a < 8; ++a) {
        const double v = q[(8 * mu + a) * TILE];
        n2 += v * v;
      }
      if (mu == 0) vt = sqrt(n2);
      else vs += sqrt(n2);
    }
  }
  vs = wsum(vs);
  vt = wsum(vt);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = vs;
    sh[1][threadIdx.x >> 6] = vt;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int k = threadIdx.x;
    part[2 * blockIdx.x + k] = (sh[k][0] + sh[k][1]) + (sh[k][2] + sh[k][3]);
  }
}

// out[x0] = spatial mean, out[L0 + x0] = time mean; partials summed in chunk order
__global__ void k_force_profile_fin(Geo g, int nck, const double* part, double* out) {
  const int x0 = blockIdx.x * blockDim.x + threadIdx.x;
  if (x0 >= g.L0) return;
  double vs = 0.0, vt = 0.0;
  for (int ck = 0; ck < nck; ++ck) {
    vs += part[2 * (x0 * nck + ck)];
    vt += part[2 * (x0 * nck + ck) + 1];
  }
  const double V3 = 2.0 * g.V3h;
  out[x0] = vs / (3.0 * V3);
  out[g.L0 + x0] = vt / V3;
}

// out = a x + b y over a whole FP64 spinor field (both parities, padding included)
__global__ void k_lincomb(long long n, double2* out, double a, const double2* x, double b, const double2* y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double2 u = x[i], v = y[i];
    double2 w;
    w.x = a * u.x + b * v.x;
    w.y = a * u.y + b * v.y;
    out[i] = w;
  }
}

// p += c * F over the whole momentum buffer
__global__ void k_axpy_mom(long long n, double* p, double c, const double* F) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] += c * F[i];
}

// ---------------------------------------------------------------------------------
static inline unsigned site_blocks(const Geo& g) { return (unsigned)((g.Vh + 127) / 128); }

void launch_pair_force(const Geo& g, double* F, double coef_times_minus_kappa, const double2* a, const double2* b,
                       const double2* U, int lb, hipStream_t s, const double* sx) {
  hipLaunchKernelGGL(k_pair_force, dim3((unsigned)((g.Vh + 63) / 64), 2), dim3(256), 0, s, g, F,
                     coef_times_minus_kappa, a, b, U, lb, sx);
}
void launch_gauge_force(const Geo& g, double* F, double c, const double2* U, hipStream_t s, const double* sx) {
  hipLaunchKernelGGL(k_gauge_force, dim3((unsigned)((g.Vh + 63) / 64), 2), dim3(256), 0, s, g, F, c, U, sx);
}
void launch_shift_links(const Geo& g, double2* out, const double2* in, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_shift_links, dim3(site_blocks(g)), dim3(256), 0, s, g, out, in, n);
}
void launch_plaq_sum(const Geo& g, const double2* U, double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_plaq, dim3(site_blocks(g)), dim3(256), 0, s, g, U, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, (int)site_blocks(g), part, out);
}
void launch_su3_dev(const Geo& g, const double2* U, double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_su3_dev, dim3(site_blocks(g)), dim3(256), 0, s, g, U, part);
  hipLaunchKernelGGL(k_max_parts, dim3(1), dim3(64), 0, s, (int)site_blocks(g), part, out);
}
void launch_kinetic(const Geo& g, const double* P, double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_kinetic, dim3(site_blocks(g)), dim3(256), 0, s, g, P, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, (int)site_blocks(g), part, out);
}
void launch_norm2_full(const Geo& g, const double2* f, double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_norm2_full, dim3(site_blocks(g)), dim3(256), 0, s, g, f, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, (int)site_blocks(g), part, out);
}
void launch_update_links(const Geo& g, double2* U, const LinkCopies& lc, const double* P, double dt, hipStream_t s,
                         const double* sx) {
  hipLaunchKernelGGL(k_update_links, dim3(site_blocks(g)), dim3(256), 0, s, g, U, lc, P, dt, sx);
}
void launch_spin_op(const Geo& g, int mode, int l0, double2* out, const double2* in, const double2* in2,
                    hipStream_t s, int outer) {
  hipLaunchKernelGGL(k_spin_op, dim3(site_blocks(g)), dim3(256), 0, s, g, mode, l0, outer, out, in, in2);
}
void launch_lincomb(const Geo& g, double2* out, double a, const double2* x, double b, const double2* y,
                    hipStream_t s) {
  const long long n = 24 * g.Vhp;
  hipLaunchKernelGGL(k_lincomb, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, out, a, x, b, y);
}
int force_profile_nck(const Geo& g) { return (g.V3h + 127) / 128; }
void launch_force_profile(const Geo& g, const double* F, double* part, double* out, hipStream_t s) {
  const int nck = force_profile_nck(g);
  hipLaunchKernelGGL(k_force_profile, dim3((unsigned)(g.L0 * nck)), dim3(256), 0, s, g, F, nck, part);
  hipLaunchKernelGGL(k_force_profile_fin, dim3((unsigned)((g.L0 + 63) / 64)), dim3(64), 0, s, g, nck, part, out);
}
void launch_axpy_mom(const Geo& g, double* p, double c, const double* F, hipStream_t s) {
  const long long n = 64 * g.Vhp;
  hipLaunchKernelGGL(k_axpy_mom, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, p, c, F);
}

}  // namespace sap
