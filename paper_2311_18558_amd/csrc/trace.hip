// Per-path field computation (trace_fields) and its adjoint.
//
// One lane per path.  Path data is read from the interaction-major
// structure of arrays, so for every interaction slot consecutive lanes read
// consecutive addresses.  Per-material permittivity and specular amplitude
// are staged in LDS once per workgroup (per-id mode) or read per
// interaction (neural-material mode).  The transfer chain of Sec. II-C is
// kept in registers: a 2-vector of complex field components and, for the
// adjoint, the per-interaction basis changes, incoming fields and Fresnel
// coefficients of the path (the depth bound is a template parameter so
// these arrays stay in registers).
//
// A path may end in a diffuse reflection (kind 1 at its last interaction,
// Sec. II-D-2, Eq. scattered_field with the Lambertian pattern
// f_s = cos(theta_s)/pi, K_x = 0 and chi = 0):
//   |E_s| = S |diag(r_perp, r_par) y| sqrt(cos(theta_i) dA f_s),
// y the incoming field in the incidence basis; the scattered field is
// (|E_s|, 0) in the basis (k_s x n, e_perp x k_s) and spreads as
// 1/(rho d) with rho the unfolded length to the diffuse point and d the
// distance to the Rx.  Elsewhere the kind is ignored (specular).
//
// Optional trainable patterns (rtc_patterns):
//  * Tx gain (Sec. III-A) G(k) = 4 pi eta sum_i (w_i/a_i) e^{lam_i mu_i.k}
//    = eta sum_i w_i c_i e^{lam_i (mu_i.k - 1)}, c_i = 2 lam_i/(1 - e^{-2 lam_i}),
//    the Tx field sqrt(G) (cos zeta, sin zeta) (Eq. polarization_model);
//  * per material K_x and the trainable scattering pattern of Eq.
//    trainable_scattering_pattern at a diffuse reflection:
//      f_s = w1 cos(theta_s)/pi + w2 e^{lam2 (k_s.k_b - 1)}/a(lam2)
//            + w3 e^{lam3 (k_s.k_r - 1)}/a(lam3),
//    k_b = -k_in, k_r the specular direction, a(lam) the hemispherical
//    integral of the shifted lobe by Meder's interpolation for an axis at
//    cos(beta) = cos(theta_i) (both axes make that angle with the normal);
//    the scattered field is |E_s| (sqrt(1 - K_x), sqrt(K_x)).
#include <cmath>

#include "api_common.h"
#include "utd.h"
#include "dev_common.h"

namespace rtc {

constexpr int kTraceBlock = 256;
constexpr int kTraceAdjMaxBlocks = 1024;
constexpr double kC0 = 299792458.0;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kPi = 3.14159265358979323846;
constexpr float kInvPi = 0.318309886183790671538f;

struct TraceArgs {
  int n_links, n_paths, n_mat;
  int max_depth;  // interaction slots per path in the store (<= the template bound)
  int64_t DP;  // max_depth * n_paths: row stride of per-interaction rows
  const int64_t* link_off;
  const float* tx_pos;
  const float* rx_pos;
  const uint8_t* depth;
  const float *px, *py, *pz, *nx, *ny, *nz;
  const uint8_t* kind;  // interaction kinds or null (all specular)
  const float* dA;      // diffuse area elements (read where kind is 1)
  const uint16_t* mat;
  const double* tau;
  const float* raw;        // per-id raw parameters [n_mat*3] or null
  const float* per_inter;  // [3*RS] or null
  const int32_t* inter_idx;  // slot -> row of per_inter (compact rows), or null (row = slot)
  int64_t RS;              // row length of per_inter and dLd_inter
  int n_vmf;               // Tx gain mixtures (0: isotropic)
  const float* tx_raw;     // [1 + 5 n_vmf] or null
  const float* pat_raw;    // [n_mat_pat * 6] per material K_x and pattern, or null
  int n_mat_pat;           // materials of pat_raw
  const float* edge;       // [4 * n_paths] edge direction and wedge n of diffraction paths, or null
  const uint16_t* mat_n;   // [n_paths] material of face n, or null
  double k0;               // carrier wavenumber 2 pi / lambda_c
  float inv_eps0w;         // 1/(eps0 * omega_c)
  double lam4pi;           // lambda_c / (4 pi)
  float cz_tx, sz_tx, cz_rx, sz_rx;
  float ux, uy, uz;  // ULA axis
  int lane_acc;      // adjoint, per id: per-thread material sums in LDS (else a wave walk)
};

RTC_DEV int find_link(const int64_t* off, int n_links, int64_t p) {
  int lo = 0, hi = n_links - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= p)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Material at one interaction: complex permittivity, S and R = sqrt(1-S^2).
struct MatVal {
  float2 eta;
  float S, R;
};

RTC_DEV MatVal make_mat(float eps, float sig, float S, float inv_eps0w) {
  MatVal v;
  v.eta = make_float2(eps, -sig * inv_eps0w);
  v.S = S;
  v.R = sqrtf(fmaxf(fmaf(-S, S, 1.0f), 0.0f));
  return v;
}

// Sec. III-C transforms with one-dimensional embeddings and unit read-out.
RTC_DEV MatVal material_from_raw(const float* raw, int m, float inv_eps0w) {
  float u0 = raw[3 * m + 0], u1 = raw[3 * m + 1], u2 = raw[3 * m + 2];
  return make_mat(1.0f + expf(u0), expf(u1), 1.0f / (1.0f + expf(-u2)), inv_eps0w);
}

// Stage the per-id material table in LDS (all threads of the block call).
RTC_DEV void stage_materials(const TraceArgs& A, MatVal* tab) {
  if (A.raw) {
    for (int m = threadIdx.x; m < A.n_mat; m += blockDim.x)
      tab[m] = material_from_raw(A.raw, m, A.inv_eps0w);
  }
  __syncthreads();
}

RTC_DEV MatVal interaction_material(const TraceArgs& A, const MatVal* tab, int64_t slot) {
  if (A.per_inter) {
    const int64_t r = A.inter_idx ? (int64_t)A.inter_idx[slot] : slot;
    return make_mat(A.per_inter[r], A.per_inter[A.RS + r], A.per_inter[2 * A.RS + r],
                    A.inv_eps0w);
  }
  int m = A.mat[slot];
  m = m < A.n_mat ? m : A.n_mat - 1;
  return tab[m];
}

// ------------------------------------------------------------- patterns
constexpr int kMaxVmf = 8;
constexpr int kTxGrad = 1 + 5 * kMaxVmf;  // eta, w, lam, mu (3 each)
constexpr int kPatGrad = 6;               // K_x (raw), w1..w3, lam2, lam3

struct VmfTab {
  int M;
  float eta;
  float w[kMaxVmf], lam[kMaxVmf], c[kMaxVmf], mu[kMaxVmf][3];
};

struct PatVal {
  float kx, w1, w2, w3, lam2, lam3;
};

RTC_DEV float logistic(float u) { return 1.0f / (1.0f + expf(-u)); }

// Raw Tx parameters -> table (one thread): eta = logistic, w = softmax,
// lam = exp, mu = normalised.
RTC_DEV void vmf_from_raw(const float* r, int M, VmfTab* t) {
  t->M = M;
  t->eta = logistic(r[0]);
  float mx = -INFINITY;
  for (int i = 0; i < M; ++i) mx = fmaxf(mx, r[1 + i]);
  float sum = 0.0f;
  for (int i = 0; i < M; ++i) sum += expf(r[1 + i] - mx);
  for (int i = 0; i < M; ++i) {
    t->w[i] = expf(r[1 + i] - mx) / sum;
    const float lam = expf(r[1 + M + i]);
    t->lam[i] = lam;
    t->c[i] = (float)(2.0 * (double)lam / -expm1(-2.0 * (double)lam));
    const float m0 = r[1 + 2 * M + 3 * i], m1 = r[2 + 2 * M + 3 * i], m2 = r[3 + 2 * M + 3 * i];
    const float inv = 1.0f / sqrtf(m0 * m0 + m1 * m1 + m2 * m2);
    t->mu[i][0] = m0 * inv;
    t->mu[i][1] = m1 * inv;
    t->mu[i][2] = m2 * inv;
  }
}

RTC_DEV float vmf_gain(const VmfTab& t, v3 k) {
  float g = 0.0f;
  for (int i = 0; i < t.M; ++i) {
    const float cmu = t.mu[i][0] * k.x + t.mu[i][1] * k.y + t.mu[i][2] * k.z;
    g = fmaf(t.w[i] * t.c[i], expf(t.lam[i] * (cmu - 1.0f)), g);
  }
  return t.eta * g;
}

RTC_DEV PatVal pattern_from_raw(const float* r, int m) {
  const float* q = r + 6 * m;
  PatVal v;
  v.kx = logistic(q[0]);
  const float mx = fmaxf(q[1], fmaxf(q[2], q[3]));
  const float e1 = expf(q[1] - mx), e2 = expf(q[2] - mx), e3 = expf(q[3] - mx);
  const float inv = 1.0f / (e1 + e2 + e3);
  v.w1 = e1 * inv;
  v.w2 = e2 * inv;
  v.w3 = e3 * inv;
  v.lam2 = expf(q[4]);
  v.lam3 = expf(q[5]);
  return v;
}

// Meder's hemispherical integral of e^{lam (v.axis - 1)} for an axis at
// cos(beta) = x from the normal, and d ln(a)/d lam:
//   a = (2 pi/lam)(1 - E)(E + s (1 - E)),  E = e^{-lam},
//   s = (1 - e^{-t(1+x)}) / ((1 - e^{-t})(1 + e^{-t x})),
//   t = sqrt(lam)(1.6988 lam^2 + 10.8438 lam)/(lam^2 + 6.2201 lam + 10.2415).
RTC_DEV double hemi_norm(double lam, double x, double* dlog) {
  const double P = 1.6988 * lam * lam + 10.8438 * lam;
  const double Qd = lam * lam + 6.2201 * lam + 10.2415;
  const double t = sqrt(lam) * P / Qd;
  const double a1 = -expm1(-t * (1.0 + x)), b1 = -expm1(-t), e1 = exp(-t * x);
  const double s = a1 / (b1 * (1.0 + e1));
  const double E = exp(-lam), omE = -expm1(-lam);
  const double inner = E + s * omE;
  const double a = (2.0 * kPi / lam) * omE * inner;
  if (dlog) {
    const double dt = t * (0.5 / lam + (3.3976 * lam + 10.8438) / P - (2.0 * lam + 6.2201) / Qd);
    const double dlns_dt = (1.0 + x) * exp(-t * (1.0 + x)) / a1 - exp(-t) / b1 + x * e1 / (1.0 + e1);
    const double ds = s * dlns_dt * dt;
    *dlog = -1.0 / lam + E / omE + (-E + ds * omE + s * E) / inner;
  }
  return a;
}

// Pattern value at a diffuse interaction and what its derivatives need.
struct PatEval {
  float f;            // f_s
  float cos_s, L2, L3;  // Lambertian factor and the two normalised lobes
  float d2, d3;       // (k_s.axis - 1) - d ln a/d lam for each lobe
};

RTC_DEV PatEval eval_pattern(const PatVal& pv, v3 k_in, v3 k_s, v3 nf, float cos_i) {
  PatEval e;
  const float cs = dot3(k_s, nf);
  const v3 k_r = add3(k_in, scl3(nf, 2.0f * cos_i));
  const float c2 = -dot3(k_s, k_in), c3 = dot3(k_s, k_r);
  double dl2, dl3;
  const double a2 = hemi_norm((double)pv.lam2, (double)cos_i, &dl2);
  const double a3 = hemi_norm((double)pv.lam3, (double)cos_i, &dl3);
  e.cos_s = cs > 0.0f ? cs * kInvPi : 0.0f;
  e.L2 = cs > 0.0f ? (float)(exp((double)pv.lam2 * ((double)c2 - 1.0)) / a2) : 0.0f;
  e.L3 = cs > 0.0f ? (float)(exp((double)pv.lam3 * ((double)c3 - 1.0)) / a3) : 0.0f;
  e.d2 = (float)((double)c2 - 1.0 - dl2);
  e.d3 = (float)((double)c3 - 1.0 - dl3);
  e.f = pv.w1 * e.cos_s + pv.w2 * e.L2 + pv.w3 * e.L3;
  return e;
}

// Stage the Tx table and the per-material pattern table (all threads call).
RTC_DEV void stage_patterns(const TraceArgs& A, VmfTab* vt, PatVal* pt) {
  if (A.n_vmf > 0 && threadIdx.x == 0) vmf_from_raw(A.tx_raw, A.n_vmf, vt);
  if (A.pat_raw) {
    for (int m = threadIdx.x; m < A.n_mat_pat; m += blockDim.x) pt[m] = pattern_from_raw(A.pat_raw, m);
  }
  __syncthreads();
}

RTC_DEV int pat_id(const TraceArgs& A, int64_t slot) {
  int m = A.mat[slot];
  return m < A.n_mat_pat ? m : A.n_mat_pat - 1;
}

// Fresnel coefficients (Eqs. fresnel-1/-2) for permittivity eta at
// incidence cosine c; also returns s = sqrt(eta - sin^2) (principal).
RTC_DEV void fresnel(float2 eta, float c, float2* rperp, float2* rpar, float2* s_out) {
  float sin2 = fmaf(-c, c, 1.0f);
  float2 s = csqrt_principal(make_float2(eta.x - sin2, eta.y));
  float2 ec = cscale(eta, c);
  *rperp = cdiv(make_float2(c - s.x, -s.y), make_float2(c + s.x, s.y));
  *rpar = cdiv(csub(ec, s), cadd(ec, s));
  *s_out = s;
}

// Geometry of one specular interaction: the basis change D (row-major; rows
// = new incoming basis (e_perp, e_par_in), columns = previous outgoing basis
// (p_out, q_out)) and the new outgoing basis (e_perp, e_par_out) with
// e_perp = k_i x n / |k_i x n|, e_par = e_perp x k.  The normal is flipped
// so that cos(theta_i) = -k_i . n > 0, which is returned.
RTC_DEV float reflect_geometry(v3 k_in, v3 n, v3 p_out, v3 q_out, float D[4], v3* np_out,
                               v3* nq_out) {
  float dn = dot3(k_in, n);
  if (dn > 0.0f) {
    n = scl3(n, -1.0f);
    dn = -dn;
  }
  v3 cr = cross3(k_in, n);
  v3 e_perp;
  if (dot3(cr, cr) > 1e-12f) {
    e_perp = sub3(cr, scl3(k_in, dot3(cr, k_in)));  // re-orthogonalised
  } else {
    // normal incidence: any transverse vector (r_par = -r_perp there)
    e_perp = sub3(p_out, scl3(k_in, dot3(p_out, k_in)));
  }
  e_perp = unit3(e_perp);
  v3 e_par_in = cross3(e_perp, k_in);
  v3 k_r = sub3(k_in, scl3(n, 2.0f * dn));
  v3 e_par_out = cross3(e_perp, k_r);
  D[0] = dot3(e_perp, p_out);
  D[1] = dot3(e_perp, q_out);
  D[2] = dot3(e_par_in, p_out);
  D[3] = dot3(e_par_in, q_out);
  *np_out = e_perp;
  *nq_out = e_par_out;
  return -dn;
}

RTC_DEV v3 load3(const float* x, const float* y, const float* z, int64_t i) {
  return v3{x[i], y[i], z[i]};
}

// Forward chain of one path.  With SAVE, the per-interaction quantities the
// adjoint needs are kept.
template <int MAXD, bool SAVE>
struct Chain {
  int Q;
  float2 E0, E1;  // field in the Rx (theta_hat, phi_hat) basis
  float Dq[4];    // final basis change into the Rx basis
  float scale;    // lambda/(4 pi c tau)
  v3 k1;
  float D[SAVE ? MAXD : 1][4];
  float2 y0[SAVE ? MAXD : 1], y1[SAVE ? MAXD : 1];
  float2 rperp[SAVE ? MAXD : 1], rpar[SAVE ? MAXD : 1], sroot[SAVE ? MAXD : 1];
  float cos_t[SAVE ? MAXD : 1];
  MatVal mv[SAVE ? MAXD : 1];
  bool dif;    // the last interaction is diffuse
  float G0;    // sqrt(cos(theta_i) dA f_s) of the diffuse interaction
  float nv;    // |diag(r_perp, r_par) y| of the diffuse interaction
  float G;     // Tx gain at k1 (1 for the isotropic Tx)
  float f;     // f_s of the diffuse interaction
  int pid;     // its pattern material
  PatVal pv;   // its pattern
  PatEval pe;
  // first-order edge diffraction (the path's only interaction)
  bool dfr;
  float2 yb, yp;   // incident field in the edge-fixed basis (beta', phi')
  float2 W2, W3;   // pre * (face-0 term), pre * (face-n term) of D
  float c0, cn;    // incidence cosines of Luebbers' face coefficients
  MatVal mvn;      // material of face n
  float dscale;    // lambda/(4 pi) / sqrt(s' s (s + s'))
};

// Diffraction at an edge point (Sec. II-E): geometry in FP64 from the
// stored FP32 points, the UTD terms of utd.h, Luebbers' face coefficients
// (Fresnel r_perp for the soft, r_par for the hard polarisation) and the
// field into the diffracted edge-fixed basis.  E0, E1: the incident field in
// (p_out, q_out); on return the diffracted one in (np, nq) = (beta_hat,
// phi_hat).
template <int MAXD, bool SAVE>
RTC_DEV void diffract(const TraceArgs& A, v3 tx, v3 q, v3 rx, v3 n0f, int64_t p, MatVal mv0,
                      MatVal mvn, v3 p_out, v3 q_out, float2& E0, float2& E1, v3* np, v3* nq,
                      Chain<MAXD, SAVE>& C) {
  const int64_t P = A.n_paths;
  double e[3] = {A.edge[p], A.edge[P + p], A.edge[2 * P + p]};
  const double nw = A.edge[3 * P + p];
  double n0[3] = {n0f.x, n0f.y, n0f.z};
  auto dotd = [](const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
  auto crossd = [](const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
  };
  auto normd = [&](double* a) {
    const double r = 1.0 / sqrt(dotd(a, a));
    a[0] *= r;
    a[1] *= r;
    a[2] *= r;
  };
  normd(e);
  normd(n0);
  double si[3] = {(double)q.x - tx.x, (double)q.y - tx.y, (double)q.z - tx.z};
  double so[3] = {(double)rx.x - q.x, (double)rx.y - q.y, (double)rx.z - q.z};
  const double sp = sqrt(dotd(si, si)), sd = sqrt(dotd(so, so));
  normd(si);
  normd(so);
  double t0[3], pi_[3], bi[3], po[3], bo[3];
  crossd(n0, e, t0);
  crossd(e, si, pi_);
  normd(pi_);
  pi_[0] = -pi_[0];
  pi_[1] = -pi_[1];
  pi_[2] = -pi_[2];
  crossd(pi_, si, bi);
  crossd(e, so, po);
  normd(po);
  crossd(po, so, bo);
  // angles about the edge from face 0 towards its normal, in [0, 2 pi)
  auto angle = [&](const double* d, double sgn) {
    const double de = sgn * dotd(d, e);
    const double x = sgn * dotd(d, t0) - de * dotd(e, t0);
    const double y = sgn * dotd(d, n0) - de * dotd(e, n0);
    double a = atan2(y, x);
    return a < 0.0 ? a + 2.0 * kUtdPi : a;
  };
  const double phip = angle(si, -1.0), phi = angle(so, 1.0);
  const double cb = dotd(so, e);
  const double sb = sqrt(fmax(1.0 - cb * cb, 0.0));
  const double L = sd * sp * sb * sb / (sd + sp);
  Cd T[4];
  utd_terms(phi, phip, nw, A.k0 * L, T);
  // pre = -e^{-j pi/4} / (2 n sqrt(2 pi k) sin beta0)
  const double pm = -kSqrtHalf / (2.0 * nw * sqrt(2.0 * kUtdPi * A.k0) * sb);
  const Cd pre = cd(pm, -pm);
  float2 W[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const Cd w = cd_mul(pre, T[i]);
    W[i] = make_float2((float)w.x, (float)w.y);
  }
  const float c0 = (float)(sb * fabs(sin(phip)));
  const float cn = (float)(sb * fabs(sin(nw * kUtdPi - phi)));
  float2 r0s, r0h, rns, rnh, sq;
  fresnel(mv0.eta, c0, &r0s, &r0h, &sq);
  fresnel(mvn.eta, cn, &rns, &rnh, &sq);
  const float2 W01 = cadd(W[0], W[1]);
  const float2 Ds = cadd(W01, cadd(cmul(r0s, W[2]), cmul(rns, W[3])));
  const float2 Dh = cadd(W01, cadd(cmul(r0h, W[2]), cmul(rnh, W[3])));
  const v3 bif = v3{(float)bi[0], (float)bi[1], (float)bi[2]};
  const v3 pif = v3{(float)pi_[0], (float)pi_[1], (float)pi_[2]};
  const float2 yb = cadd(cscale(E0, dot3(bif, p_out)), cscale(E1, dot3(bif, q_out)));
  const float2 yp = cadd(cscale(E0, dot3(pif, p_out)), cscale(E1, dot3(pif, q_out)));
  E0 = cscale(cmul(Ds, yb), -1.0f);
  E1 = cscale(cmul(Dh, yp), -1.0f);
  *np = v3{(float)bo[0], (float)bo[1], (float)bo[2]};
  *nq = v3{(float)po[0], (float)po[1], (float)po[2]};
  C.dfr = true;
  C.dscale = (float)(A.lam4pi / sqrt(sp * sd * (sp + sd)));
  if constexpr (SAVE) {
    C.yb = yb;
    C.yp = yp;
    C.W2 = W[2];
    C.W3 = W[3];
    C.c0 = c0;
    C.cn = cn;
    C.mvn = mvn;
  }
}

// PAT: the trainable Tx gain and scattering patterns are compiled in; DFR:
// edge diffraction is (the plain chain keeps its register budget without
// them; diffraction paths, depth 1, run in their own shallow instance).
template <int MAXD, bool SAVE, bool PAT, bool DFR>
RTC_DEV void run_chain(const TraceArgs& A, const MatVal* tab, const VmfTab* vt, const PatVal* ptab,
                       int64_t p, Chain<MAXD, SAVE>& C) {
  int l = find_link(A.link_off, A.n_links, p);
  v3 tx = v3{A.tx_pos[3 * l], A.tx_pos[3 * l + 1], A.tx_pos[3 * l + 2]};
  v3 rx = v3{A.rx_pos[3 * l], A.rx_pos[3 * l + 1], A.rx_pos[3 * l + 2]};
  int Q = A.depth[p];
  Q = Q < A.max_depth ? Q : A.max_depth;  // never past the store's slots
  Q = Q < MAXD ? Q : MAXD;
  C.Q = Q;
  v3 first = Q > 0 ? load3(A.px, A.py, A.pz, p) : rx;
  v3 k1 = unit3(sub3(first, tx));
  C.k1 = k1;
  v3 p_out, q_out;
  sph_basis(k1, &p_out, &q_out);
  // Tx pattern: sqrt(G) (cos zeta, sin zeta) (Sec. II-B), G = 1 isotropic
  float2 E0 = make_float2(A.cz_tx, 0.0f);
  float2 E1 = make_float2(A.sz_tx, 0.0f);
  C.G = 1.0f;
  if (PAT && A.n_vmf > 0) {
    C.G = vmf_gain(*vt, k1);
    const float sg = sqrtf(fmaxf(C.G, 0.0f));
    E0.x *= sg;
    E1.x *= sg;
  }
  C.f = 0.0f;
  C.pid = 0;
  v3 prev = tx;
  float rho = 0.0f;  // unfolded length from the Tx
  C.dif = false;
  C.dfr = false;
  C.G0 = C.nv = 0.0f;
#pragma unroll
  for (int j = 0; j < MAXD; ++j) {
    if (j < Q) {
      int64_t slot = (int64_t)j * A.n_paths + p;
      v3 s = load3(A.px, A.py, A.pz, slot);
      v3 n = load3(A.nx, A.ny, A.nz, slot);
      v3 seg = sub3(s, prev);
      rho += sqrtf(dot3(seg, seg));
      v3 k_in = unit3(seg);
      float D[4];
      v3 np, nq;
      float c = reflect_geometry(k_in, n, p_out, q_out, D, &np, &nq);
      float2 y0 = cadd(cscale(E0, D[0]), cscale(E1, D[1]));
      float2 y1 = cadd(cscale(E0, D[2]), cscale(E1, D[3]));
      MatVal mv = interaction_material(A, tab, slot);
      float2 rp, rl, sr;
      fresnel(mv.eta, c, &rp, &rl, &sr);
      const bool dif = A.kind != nullptr && j == Q - 1 && A.kind[slot] == 1;
      const bool dfr = DFR && A.edge != nullptr && A.kind != nullptr && j == 0 && Q == 1 &&
                       A.kind[slot] == 2;
      if (dfr) {
        MatVal mvn = mv;
        if (A.raw) {
          int mn = A.mat_n[p];
          mvn = tab[mn < A.n_mat ? mn : A.n_mat - 1];
        }
        diffract<MAXD, SAVE>(A, tx, s, rx, n, p, mv, mvn, p_out, q_out, E0, E1, &np, &nq, C);
      } else if (dif) {
        v3 nf = dot3(k_in, n) > 0.0f ? scl3(n, -1.0f) : n;  // towards the incidence side
        v3 k_s = unit3(sub3(rx, s));
        float f = fmaxf(dot3(k_s, nf), 0.0f) * kInvPi;  // Lambertian
        float kx = 0.0f;
        if (PAT && A.pat_raw) {
          C.pid = pat_id(A, slot);
          C.pv = ptab[C.pid];
          C.pe = eval_pattern(C.pv, k_in, k_s, nf, c);
          f = C.pe.f;
          kx = C.pv.kx;
        }
        C.f = f;
        float geo = c * A.dA[slot] * f;
        float G0 = sqrtf(fmaxf(geo, 0.0f));
        float nv = sqrtf(cabs2(cmul(rp, y0)) + cabs2(cmul(rl, y1)));
        const float As = mv.S * nv * G0;
        E0 = make_float2(As * sqrtf(1.0f - kx), 0.0f);
        E1 = make_float2(As * sqrtf(kx), 0.0f);
        v3 cr = cross3(k_s, nf);
        v3 e_perp = dot3(cr, cr) > 1e-12f ? cr : np;  // k_s along n: incidence e_perp
        e_perp = unit3(sub3(e_perp, scl3(k_s, dot3(e_perp, k_s))));
        np = e_perp;
        nq = cross3(e_perp, k_s);
        C.dif = true;
        C.G0 = G0;
        C.nv = nv;
      } else {
        E0 = cscale(cmul(rp, y0), mv.R);
        E1 = cscale(cmul(rl, y1), mv.R);
      }
      if constexpr (SAVE) {
        C.D[j][0] = D[0];
        C.D[j][1] = D[1];
        C.D[j][2] = D[2];
        C.D[j][3] = D[3];
        C.y0[j] = y0;
        C.y1[j] = y1;
        C.rperp[j] = rp;
        C.rpar[j] = rl;
        C.sroot[j] = sr;
        C.cos_t[j] = c;
        C.mv[j] = mv;
      }
      p_out = np;
      q_out = nq;
      prev = s;
    }
  }
  v3 k_last = unit3(sub3(rx, prev));
  v3 th, ph;
  sph_basis(scl3(k_last, -1.0f), &th, &ph);
  C.Dq[0] = dot3(th, p_out);
  C.Dq[1] = dot3(th, q_out);
  C.Dq[2] = dot3(ph, p_out);
  C.Dq[3] = dot3(ph, q_out);
  C.E0 = cadd(cscale(E0, C.Dq[0]), cscale(E1, C.Dq[1]));
  C.E1 = cadd(cscale(E0, C.Dq[2]), cscale(E1, C.Dq[3]));
  // spreading of planar reflections with a point source: 1/(total length);
  // after a diffuse reflection 1/(rho d)
  if (C.dif) {
    v3 seg = sub3(rx, prev);
    C.scale = (float)(A.lam4pi / ((double)rho * (double)sqrtf(dot3(seg, seg))));
  } else if (C.dfr) {
    C.scale = C.dscale;
  } else {
    C.scale = (float)(A.lam4pi / (kC0 * A.tau[p]));
  }
}

// Dynamic LDS of the trace kernels: material table | Tx table | pattern
// table | (adjoint) per-wave accumulators, each 16-byte aligned.
struct TraceLds {
  MatVal* tab;
  VmfTab* vt;
  PatVal* pt;
  double* acc;
};
RTC_DEV size_t align16(size_t n) { return (n + 15) / 16 * 16; }
inline size_t align16h(size_t n) { return (n + 15) / 16 * 16; }
inline size_t trace_lds_fixed(const TraceArgs& A) {
  return align16h((A.raw ? A.n_mat : 0) * sizeof(MatVal)) + align16h(sizeof(VmfTab)) +
         align16h((A.pat_raw ? A.n_mat_pat : 0) * sizeof(PatVal));
}
RTC_DEV TraceLds trace_lds(const TraceArgs& A, unsigned char* smem) {
  TraceLds L;
  size_t o = 0;
  L.tab = reinterpret_cast<MatVal*>(smem + o);
  o += align16((A.raw ? A.n_mat : 0) * sizeof(MatVal));
  L.vt = reinterpret_cast<VmfTab*>(smem + o);
  o += align16(sizeof(VmfTab));
  L.pt = reinterpret_cast<PatVal*>(smem + o);
  o += align16((A.pat_raw ? A.n_mat_pat : 0) * sizeof(PatVal));
  L.acc = reinterpret_cast<double*>(smem + o);
  return L;
}

// A first-order diffraction path: depth 1 with kind 2 in its only slot.
RTC_DEV bool is_dfr_path(const TraceArgs& A, int64_t p) {
  return A.edge != nullptr && A.kind != nullptr && A.depth[p] == 1 && A.kind[p] == 2;
}

// Forward.  With diffraction paths in the store (A.edge), the DFR instance
// handles exactly those and the others skip them.
template <int MAXD, bool PAT, bool DFR>
__global__ void __launch_bounds__(kTraceBlock) trace_fields_kernel(TraceArgs A, float2* a,
                                                                    float* psi) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_f[];
  const TraceLds Ls = trace_lds(A, smem_f);
  stage_materials(A, Ls.tab);
  if constexpr (PAT) stage_patterns(A, Ls.vt, Ls.pt);
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= A.n_paths) return;
  if (A.edge != nullptr && is_dfr_path(A, p) != DFR) return;
  Chain<MAXD, false> C;
  run_chain<MAXD, false, PAT, DFR>(A, Ls.tab, Ls.vt, Ls.pt, p, C);
  // C_R^H E with a real (isotropic, slant zeta) Rx pattern
  float2 recv = cadd(cscale(C.E0, A.cz_rx), cscale(C.E1, A.sz_rx));
  if (a) a[p] = cscale(recv, C.scale);
  if (psi) psi[p] = (float)kPi * (C.k1.x * A.ux + C.k1.y * A.uy + C.k1.z * A.uz);
}

// Adjoint.  For a path, a = w_j^T x_j at every interaction j, where x_j is
// the outgoing field after the Fresnel map F_j = diag(R r_perp, R r_par) and
// w_j^T = K c_R^T D_{Q+1} F_Q D_Q ... F_{j+1} D_{j+1}.  Hence
//   da/d(R r_perp)_j = w_j[0] y_j[0],  da/d(R r_par)_j = w_j[1] y_j[1]
// with y_j the incoming field in the interaction basis.  With the
// holomorphic chain rule dL/deta = conj(da/deta) dL/da, and for real
// parameters dL/dx = Re(conj(da/dx) dL/da).
// Layout of the reduced gradients (per-wave LDS rows, per-block partials):
// [3 n_mat] materials (per-id mode) | [6 n_mat_pat] patterns | [kTxGrad] Tx,
// sections present as requested (GradLayout).
struct GradLayout {
  int mat, pat, tx, stride;  // offsets of the sections (-1 absent), row length
};

template <int MAXD, bool PER_ID, bool PAT, bool DFR>
__global__ void __launch_bounds__(kTraceBlock)
    trace_fields_adjoint_kernel(TraceArgs A, const float2* dLda, float* dLd_inter,
                                double* block_part, GradLayout GL) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const TraceLds Ls = trace_lds(A, smem);
  MatVal* tab = Ls.tab;
  double* acc = Ls.acc;
  stage_materials(A, tab);
  if constexpr (PAT) stage_patterns(A, Ls.vt, Ls.pt);
  // per-thread material sums [3 n_mat][blockDim] (FP32, each thread's paths
  // in order), after the per-wave rows
  float* lacc = (PER_ID && A.lane_acc && GL.mat >= 0)
                    ? reinterpret_cast<float*>(acc + GL.stride * (int)(blockDim.x >> 6))
                    : nullptr;
  if (GL.stride > 0) {
    for (int i = threadIdx.x; i < GL.stride * (int)(blockDim.x >> 6); i += blockDim.x) acc[i] = 0.0;
    if (lacc)
      for (int i = threadIdx.x; i < 3 * A.n_mat * (int)blockDim.x; i += blockDim.x) lacc[i] = 0.0f;
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n_waves = blockDim.x >> 6;
  const double eps0w_inv = (double)A.inv_eps0w;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < A.n_paths;
       base += (int64_t)gridDim.x * blockDim.x) {
    int64_t p = base + threadIdx.x;
    bool valid = p < A.n_paths;
    // with diffraction paths in the store the DFR instance takes exactly those
    if (valid && A.edge != nullptr) valid = is_dfr_path(A, p) == DFR;
    float g_eps[MAXD], g_sig[MAXD], g_S[MAXD];
    int ids[MAXD];
    int Q = 0;
    bool dfr_path = false;
    // pattern gradients of the path's diffuse interaction (at most one):
    // raw K_x, then w1..w3, lam2, lam3 in natural coordinates
    float g_pat[kPatGrad];
    int pat_m = 0x7fffffff;
#pragma unroll
    for (int k = 0; k < kPatGrad; ++k) g_pat[k] = 0.0f;
    float gG = 0.0f;  // dL/dG of the Tx gain
    v3 k1 = v3{0.0f, 0.0f, 1.0f};
#pragma unroll
    for (int j = 0; j < MAXD; ++j) {
      g_eps[j] = g_sig[j] = g_S[j] = 0.0f;
      ids[j] = 0x7fffffff;
    }
    if (valid) {
      Chain<MAXD, true> C;
      run_chain<MAXD, true, PAT, DFR>(A, tab, Ls.vt, Ls.pt, p, C);
      Q = C.Q;
      float2 Ga = dLda[p];
      dfr_path = C.dfr;
      k1 = C.k1;
      if (PAT && GL.tx >= 0 && C.G > 0.0f) {
        // a is proportional to sqrt(G): dL/dG = Re(conj(a) dL/da) / (2 G)
        const float2 recv = cadd(cscale(C.E0, A.cz_rx), cscale(C.E1, A.sz_rx));
        const float2 av = cscale(recv, C.scale);
        gG = (av.x * Ga.x + av.y * Ga.y) / (2.0f * C.G);
      }
      // w^T = K c_R^T D_{Q+1}  (real at the start)
      float K = C.scale;
      float2 w0 = make_float2(K * (A.cz_rx * C.Dq[0] + A.sz_rx * C.Dq[2]), 0.0f);
      float2 w1 = make_float2(K * (A.cz_rx * C.Dq[1] + A.sz_rx * C.Dq[3]), 0.0f);
#pragma unroll
      for (int j = MAXD - 1; j >= 0; --j) {
        if (DFR && j == 0 && C.dfr) {
          // a = w0 (-D_s yb) + w1 (-D_h yp) with D = W01 + R0 W2 + Rn W3:
          // da/deta_0 = -(w0 yb dR0s/deta + w1 yp dR0h/deta) W2, likewise
          // face n with W3 (the covector w is real here: Q = 1)
          float2 r_s, r_h, sq;
          float2 dts, dth, dns, dnh;
          {
            const float c = C.c0;
            const float2 eta = C.mv[0].eta;
            fresnel(eta, c, &r_s, &r_h, &sq);
            const float2 cps = make_float2(c + sq.x, sq.y);
            dts = cdiv(make_float2(-c, 0.0f), cmul(sq, cmul(cps, cps)));
            const float2 ecs = cadd(cscale(eta, c), sq);
            dth = cdiv(cscale(make_float2(eta.x - 2.0f * fmaf(-c, c, 1.0f), eta.y), c),
                       cmul(sq, cmul(ecs, ecs)));
          }
          {
            const float c = C.cn;
            const float2 eta = C.mvn.eta;
            fresnel(eta, c, &r_s, &r_h, &sq);
            const float2 cps = make_float2(c + sq.x, sq.y);
            dns = cdiv(make_float2(-c, 0.0f), cmul(sq, cmul(cps, cps)));
            const float2 ecs = cadd(cscale(eta, c), sq);
            dnh = cdiv(cscale(make_float2(eta.x - 2.0f * fmaf(-c, c, 1.0f), eta.y), c),
                       cmul(sq, cmul(ecs, ecs)));
          }
          const float2 ub = cscale(C.yb, -w0.x), up = cscale(C.yp, -w1.x);
          const float2 da0 = cmul(cadd(cmul(ub, dts), cmul(up, dth)), C.W2);
          const float2 dan = cmul(cadd(cmul(ub, dns), cmul(up, dnh)), C.W3);
          const float2 G0 = cmulc(da0, Ga);  // conj(da/deta) dL/da
          const float2 Gn = cmulc(dan, Ga);
          g_eps[0] = G0.x;
          g_sig[0] = -G0.y * A.inv_eps0w;
          g_S[0] = 0.0f;
          ids[0] = PER_ID ? (int)min((int)A.mat[p], A.n_mat - 1) : 0;
          if constexpr (PER_ID && MAXD >= 2) {
            g_eps[1] = Gn.x;
            g_sig[1] = -Gn.y * A.inv_eps0w;
            g_S[1] = 0.0f;
            ids[1] = (int)min((int)A.mat_n[p], A.n_mat - 1);
          } else {
            // per-interaction materials: both faces take the interaction's
            g_eps[0] += Gn.x;
            g_sig[0] += -Gn.y * A.inv_eps0w;
          }
        } else if (j < Q && C.dif && j == Q - 1) {
          // a = K q_R |E_s| is real, so dL/dx = Re(dL/da) da/dx.  With
          // |E_s| = S G0 nv, nv = |v|, v = (r_perp y0, r_par y1):
          //   d nv/d eta_re = Re(Z)/nv, d nv/d eta_im = -Im(Z)/nv,
          //   Z = conj(r_perp) dr_perp/deta |y0|^2 + conj(r_par) dr_par/deta |y1|^2
          // and d nv = Re(c^T dy) with c = (conj(v0) r_perp, conj(v1) r_par)/nv,
          // which continues the sweep through the preceding interactions.
          // the scattered field is |E_s| (sqrt(1 - K_x), sqrt(K_x)) and a =
          // K (qR0 sqrt(1 - K_x) + qR1 sqrt(K_x)) |E_s|
          const float qR0 = A.cz_rx * C.Dq[0] + A.sz_rx * C.Dq[2];
          const float qR1 = A.cz_rx * C.Dq[1] + A.sz_rx * C.Dq[3];
          const float kx = (PAT && A.pat_raw) ? C.pv.kx : 0.0f;
          const float sk0 = sqrtf(1.0f - kx), sk1 = sqrtf(kx);
          const float qR = qR0 * sk0 + qR1 * sk1;
          const float gam = Ga.x * K * qR;
          if (PAT && GL.pat >= 0) {
            // d a/du_kx with K_x = logistic(u): K |E_s| K_x (1 - K_x)
            //   (-qR0 / (2 sqrt(1 - K_x)) + qR1 / (2 sqrt(K_x)))
            const float As = C.mv[j].S * C.G0 * C.nv;
            g_pat[0] = Ga.x * K * As * 0.5f * (-qR0 * kx * sk0 + qR1 * (1.0f - kx) * sk1);
            // |E_s| grows as sqrt(f_s): dL/df = gam |E_s| / (2 f)
            const float dLdf = C.f > 0.0f ? gam * As / (2.0f * C.f) : 0.0f;
            g_pat[1] = dLdf * C.pe.cos_s;
            g_pat[2] = dLdf * C.pe.L2;
            g_pat[3] = dLdf * C.pe.L3;
            g_pat[4] = dLdf * C.pv.w2 * C.pe.L2 * C.pe.d2;
            g_pat[5] = dLdf * C.pv.w3 * C.pe.L3 * C.pe.d3;
            pat_m = C.pid;
          }
          const float2 rp = C.rperp[j], rl = C.rpar[j], sq = C.sroot[j];
          const float c = C.cos_t[j];
          const float2 eta = C.mv[j].eta;
          const float S = C.mv[j].S;
          float2 cps = make_float2(c + sq.x, sq.y);
          float2 d_perp = cdiv(make_float2(-c, 0.0f), cmul(sq, cmul(cps, cps)));
          float sin2 = fmaf(-c, c, 1.0f);
          float2 ecs = cadd(cscale(eta, c), sq);
          float2 d_par = cdiv(cscale(make_float2(eta.x - 2.0f * sin2, eta.y), c),
                              cmul(sq, cmul(ecs, ecs)));
          const float2 Z = cadd(cscale(cmulc(rp, d_perp), cabs2(C.y0[j])),
                                cscale(cmulc(rl, d_par), cabs2(C.y1[j])));
          const float coef = C.nv > 0.0f ? gam * S * C.G0 / C.nv : 0.0f;
          g_eps[j] = coef * Z.x;
          g_sig[j] = coef * Z.y * A.inv_eps0w;
          g_S[j] = gam * C.G0 * C.nv;
          ids[j] = PER_ID ? (int)min((int)A.mat[(int64_t)j * A.n_paths + p], A.n_mat - 1) : 0;
          const float inv_nv = C.nv > 0.0f ? 1.0f / C.nv : 0.0f;
          const float2 c0 = cscale(cmul(cconj(cmul(rp, C.y0[j])), rp), inv_nv);
          const float2 c1 = cscale(cmul(cconj(cmul(rl, C.y1[j])), rl), inv_nv);
          w0 = cadd(cscale(c0, C.D[j][0]), cscale(c1, C.D[j][2]));
          w1 = cadd(cscale(c0, C.D[j][1]), cscale(c1, C.D[j][3]));
          Ga = make_float2(gam * S * C.G0, 0.0f);
        } else if (j < Q) {
          float2 Aperp = cmul(w0, C.y0[j]);
          float2 Apar = cmul(w1, C.y1[j]);
          float2 rp = C.rperp[j], rl = C.rpar[j], s = C.sroot[j];
          float c = C.cos_t[j];
          float2 eta = C.mv[j].eta;
          float R = C.mv[j].R;
          // dr_perp/deta = -c / (s (c+s)^2)
          float2 cps = make_float2(c + s.x, s.y);
          float2 d_perp = cdiv(make_float2(-c, 0.0f), cmul(s, cmul(cps, cps)));
          // dr_par/deta = c (eta - 2 sin^2) / (s (eta c + s)^2)
          float sin2 = fmaf(-c, c, 1.0f);
          float2 ecs = cadd(cscale(eta, c), s);
          float2 d_par = cdiv(cscale(make_float2(eta.x - 2.0f * sin2, eta.y), c),
                              cmul(s, cmul(ecs, ecs)));
          float2 da_deta = cscale(cadd(cmul(Aperp, d_perp), cmul(Apar, d_par)), R);
          float2 da_dR = cadd(cmul(Aperp, rp), cmul(Apar, rl));
          float2 Geta = cmulc(da_deta, Ga);  // conj(da/deta) * dL/da
          float GR = da_dR.x * Ga.x + da_dR.y * Ga.y;  // Re(conj(da/dR) dL/da)
          g_eps[j] = Geta.x;
          g_sig[j] = -Geta.y * A.inv_eps0w;
          float S = C.mv[j].S;
          g_S[j] = R > 0.0f ? -GR * S / R : 0.0f;
          ids[j] = PER_ID ? (int)min((int)A.mat[(int64_t)j * A.n_paths + p], A.n_mat - 1) : 0;
          // w^T <- w^T F_j D_j
          float2 f0 = cmul(w0, cscale(rp, R));
          float2 f1 = cmul(w1, cscale(rl, R));
          w0 = cadd(cscale(f0, C.D[j][0]), cscale(f1, C.D[j][2]));
          w1 = cadd(cscale(f0, C.D[j][1]), cscale(f1, C.D[j][3]));
        }
      }
    }
    if constexpr (!PER_ID) {
      if (valid) {
#pragma unroll
        for (int j = 0; j < MAXD; ++j) {
          if (j >= A.max_depth) break;  // the template bound may exceed the store's
          int64_t slot = (int64_t)j * A.n_paths + p;
          // compact rows: used slots only; otherwise slots past the depth get zeros
          if (A.inter_idx && j >= Q) continue;
          const int64_t r = A.inter_idx ? (int64_t)A.inter_idx[slot] : slot;
          dLd_inter[r] = g_eps[j];
          dLd_inter[A.RS + r] = g_sig[j];
          dLd_inter[2 * A.RS + r] = g_S[j];
        }
        if constexpr (DFR) {
          // the shallow instance's slots end at MAXD: the rest of the rows get zeros
          if (!A.inter_idx)
            for (int j = MAXD; j < A.max_depth; ++j) {
              const int64_t slot = (int64_t)j * A.n_paths + p;
              dLd_inter[slot] = 0.0f;
              dLd_inter[A.RS + slot] = 0.0f;
              dLd_inter[2 * A.RS + slot] = 0.0f;
            }
        }
      }
    } else {
      // a diffraction path carries its face-n gradient in slot 1
      if (DFR && dfr_path) Q = 2;
      // Per-id sums, deterministic.  With per-thread sums (lacc) each
      // thread adds its interactions' gradients to its own column of the
      // material table (the workgroup sums the columns in order at the end);
      // otherwise each wave walks the distinct ids present in it in
      // increasing order, and for each id the lanes' contributions (fixed
      // order over j) are summed by a butterfly in FP64 and added to the
      // wave's own LDS table (waves are summed in order at the end).
      if (lacc) {
        if (valid) {
#pragma unroll
          for (int j = 0; j < MAXD; ++j) {
            if (j < Q) {
              float* col = lacc + 3 * ids[j] * (int)blockDim.x + threadIdx.x;
              col[0] += g_eps[j];
              col[blockDim.x] += g_sig[j];
              col[2 * blockDim.x] += g_S[j];
            }
          }
        }
      } else {
        double* wacc = acc + wave * GL.stride + GL.mat;
        {
          int done_mask = 0;  // bit j set once interaction j is accounted
          while (true) {
            int cand = 0x7fffffff;
#pragma unroll
            for (int j = 0; j < MAXD; ++j)
              if (j < Q && !(done_mask >> j & 1)) cand = min(cand, ids[j]);
            int mmin = cand;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) mmin = min(mmin, __shfl_xor(mmin, o, 64));
            if (mmin == 0x7fffffff) break;
            double se = 0.0, ss = 0.0, sS = 0.0;
#pragma unroll
            for (int j = 0; j < MAXD; ++j) {
              if (j < Q && !(done_mask >> j & 1) && ids[j] == mmin) {
                se += (double)g_eps[j];
                ss += (double)g_sig[j];
                sS += (double)g_S[j];
                done_mask |= 1 << j;
              }
            }
            se = wave_sum_f64(se);
            ss = wave_sum_f64(ss);
            sS = wave_sum_f64(sS);
            if (lane == 0) {
              wacc[3 * mmin + 0] += se;
              wacc[3 * mmin + 1] += ss;
              wacc[3 * mmin + 2] += sS;
            }
          }
        }
      }
    }
    if (PAT && GL.pat >= 0) {
      // the same deterministic walk over the pattern ids of the wave
      double* wacc = acc + wave * GL.stride + GL.pat;
      bool done = !valid || pat_m == 0x7fffffff;
      while (true) {
        int mmin = done ? 0x7fffffff : pat_m;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) mmin = min(mmin, __shfl_xor(mmin, o, 64));
        if (mmin == 0x7fffffff) break;
        const bool mine = !done && pat_m == mmin;
#pragma unroll
        for (int k = 0; k < kPatGrad; ++k) {
          const double v = wave_sum_f64(mine ? (double)g_pat[k] : 0.0);
          if (lane == 0) wacc[kPatGrad * mmin + k] += v;
        }
        if (mine) done = true;
      }
    }
    if (PAT && GL.tx >= 0) {
      // natural Tx gradients of this path, summed over the wave in order:
      //   eta: G/eta,  w_i: eta c_i e_i,  lam_i: eta w_i c_i e_i ((mu_i.k - 1)
      //   + d ln c_i/d lam_i),  mu_i: eta w_i c_i e_i lam_i k
      const VmfTab& vt = *Ls.vt;
      const int M = vt.M;
      double* wacc = acc + wave * GL.stride + GL.tx;
      const float eta = vt.eta;
      double t_eta = 0.0;
      for (int i = 0; i < M; ++i) {
        const float cmu = vt.mu[i][0] * k1.x + vt.mu[i][1] * k1.y + vt.mu[i][2] * k1.z;
        const float ce = vt.c[i] * expf(vt.lam[i] * (cmu - 1.0f));
        t_eta += (double)(vt.w[i] * ce);
        const double lam = (double)vt.lam[i];
        const float dlnc = (float)(1.0 / lam - 2.0 * exp(-2.0 * lam) / -expm1(-2.0 * lam));
        const float gw = gG * eta * ce;
        const float gl = gw * vt.w[i] * ((cmu - 1.0f) + dlnc);
        const float gm = gw * vt.w[i] * vt.lam[i];
        const double s_w = wave_sum_f64((double)gw);
        const double s_l = wave_sum_f64((double)gl);
        const double s_m0 = wave_sum_f64((double)(gm * k1.x));
        const double s_m1 = wave_sum_f64((double)(gm * k1.y));
        const double s_m2 = wave_sum_f64((double)(gm * k1.z));
        if (lane == 0) {
          wacc[1 + i] += s_w;
          wacc[1 + M + i] += s_l;
          wacc[1 + 2 * M + 3 * i + 0] += s_m0;
          wacc[1 + 2 * M + 3 * i + 1] += s_m1;
          wacc[1 + 2 * M + 3 * i + 2] += s_m2;
        }
      }
      const double s_eta = wave_sum_f64((double)gG * t_eta);
      if (lane == 0) wacc[0] += s_eta;
    }
  }
  if (GL.stride > 0) {
    __syncthreads();
    if (lacc) {
      // the columns of each material entry: quarter qt of the threads'
      // columns summed by one thread (FP64) in a fixed order that starts at
      // its own column t % 64 (so the lanes of a wave read 64 different
      // banks), the quarters in order
      const int n_e = 3 * A.n_mat, nq = (int)blockDim.x / 64;
      double* qsum = acc + GL.stride * n_waves + (3 * A.n_mat * blockDim.x + 1) / 2;
      for (int t = threadIdx.x; t < n_e * nq; t += blockDim.x) {
        const int e = t / nq, qt = t % nq;
        const float* src = lacc + e * (int)blockDim.x + 64 * qt;
        double v = 0.0;
        for (int k = 0; k < 64; ++k) v += (double)src[(k + t) & 63];
        qsum[t] = v;
      }
      __syncthreads();
      for (int e = threadIdx.x; e < n_e; e += blockDim.x) {
        double v = 0.0;
        for (int qt = 0; qt < nq; ++qt) v += qsum[e * nq + qt];
        acc[GL.mat + e] += v;  // wave 0's row, untouched by the walk
      }
      __syncthreads();
    }
    for (int i = threadIdx.x; i < GL.stride; i += blockDim.x) {
      double t = 0.0;
      for (int w = 0; w < n_waves; ++w) t += acc[w * GL.stride + i];
      block_part[(int64_t)blockIdx.x * GL.stride + i] = t;
    }
  }
  (void)eps0w_inv;
}

// Sum the per-block partials (FP64, fixed order: strided per thread, then a
// tree over the workgroup).  One workgroup of kTraceBlock threads per
// output.
__global__ void __launch_bounds__(kTraceBlock)
    trace_adjoint_reduce_kernel(const double* block_part, int n_blocks, int stride, double* tot) {
  __shared__ double red[kTraceBlock];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < n_blocks; b += blockDim.x) s += block_part[(int64_t)b * stride + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[i] = red[0];
}

// Raw-parameter transforms of the reduced gradients (one workgroup):
//   materials: d eps/du0 = eps - 1, d sigma/du1 = sigma, dS/du2 = S (1 - S);
//   patterns: K_x already raw; softmax weights dL/dq_j = w_j (g_j - sum_i
//   w_i g_i); lam = exp(q): dL/dq = lam g;
//   Tx: eta = logistic, softmax weights, lam = exp, mu = m/|m|:
//   dL/dm = (g - (mu.g) mu)/|m|.
__global__ void trace_adjoint_transform_kernel(const double* tot, GradLayout GL, int n_mat,
                                               const float* raw, int n_mat_pat,
                                               const float* pat_raw, int n_vmf,
                                               const float* tx_raw, float* dLd_raw,
                                               float* dLd_pat, float* dLd_tx) {
  if (GL.mat >= 0 && dLd_raw) {
    for (int i = threadIdx.x; i < 3 * n_mat; i += blockDim.x) {
      const int m = i / 3, c = i % 3;
      const double u = (double)raw[3 * m + c];
      double d;
      if (c < 2) {
        d = exp(u);
      } else {
        const double S = 1.0 / (1.0 + exp(-u));
        d = S * (1.0 - S);
      }
      dLd_raw[i] = (float)(tot[GL.mat + i] * d);
    }
  }
  if (GL.pat >= 0 && dLd_pat) {
    for (int m = threadIdx.x; m < n_mat_pat; m += blockDim.x) {
      const float* q = pat_raw + 6 * m;
      const double* g = tot + GL.pat + 6 * m;
      const double mx = fmax((double)q[1], fmax((double)q[2], (double)q[3]));
      double w[3], sw = 0.0;
      for (int j = 0; j < 3; ++j) sw += (w[j] = exp((double)q[1 + j] - mx));
      double dot = 0.0;
      for (int j = 0; j < 3; ++j) dot += (w[j] /= sw) * g[1 + j];
      dLd_pat[6 * m + 0] = (float)g[0];
      for (int j = 0; j < 3; ++j) dLd_pat[6 * m + 1 + j] = (float)(w[j] * (g[1 + j] - dot));
      dLd_pat[6 * m + 4] = (float)(exp((double)q[4]) * g[4]);
      dLd_pat[6 * m + 5] = (float)(exp((double)q[5]) * g[5]);
    }
  }
  if (GL.tx >= 0 && dLd_tx && threadIdx.x == 0) {
    const int M = n_vmf;
    const double* g = tot + GL.tx;
    const double eta = 1.0 / (1.0 + exp(-(double)tx_raw[0]));
    dLd_tx[0] = (float)(eta * (1.0 - eta) * g[0]);
    double mx = -INFINITY;
    for (int i = 0; i < M; ++i) mx = fmax(mx, (double)tx_raw[1 + i]);
    double sw = 0.0;
    for (int i = 0; i < M; ++i) sw += exp((double)tx_raw[1 + i] - mx);
    double dot = 0.0;
    for (int i = 0; i < M; ++i) dot += exp((double)tx_raw[1 + i] - mx) / sw * g[1 + i];
    for (int i = 0; i < M; ++i) {
      const double wi = exp((double)tx_raw[1 + i] - mx) / sw;
      dLd_tx[1 + i] = (float)(wi * (g[1 + i] - dot));
      dLd_tx[1 + M + i] = (float)(exp((double)tx_raw[1 + M + i]) * g[1 + M + i]);
      const double m0 = tx_raw[1 + 2 * M + 3 * i], m1 = tx_raw[2 + 2 * M + 3 * i],
                   m2 = tx_raw[3 + 2 * M + 3 * i];
      const double nm = sqrt(m0 * m0 + m1 * m1 + m2 * m2);
      const double u0 = m0 / nm, u1 = m1 / nm, u2 = m2 / nm;
      const double g0 = g[1 + 2 * M + 3 * i], g1 = g[2 + 2 * M + 3 * i], g2 = g[3 + 2 * M + 3 * i];
      const double ug = u0 * g0 + u1 * g1 + u2 * g2;
      dLd_tx[1 + 2 * M + 3 * i + 0] = (float)((g0 - ug * u0) / nm);
      dLd_tx[1 + 2 * M + 3 * i + 1] = (float)((g1 - ug * u1) / nm);
      dLd_tx[1 + 2 * M + 3 * i + 2] = (float)((g2 - ug * u2) / nm);
    }
  }
}

static TraceArgs make_args(const rtc_radio* r, const rtc_paths* P, const rtc_materials* M,
                           const rtc_patterns* pat) {
  TraceArgs A;
  A.lane_acc = 0;
  A.n_links = P->n_links;
  A.n_paths = P->n_paths;
  A.n_mat = M->raw ? M->n_mat : 1;
  A.max_depth = P->max_depth;
  A.DP = (int64_t)P->max_depth * P->n_paths;
  A.link_off = P->link_off;
  A.tx_pos = P->tx_pos;
  A.rx_pos = P->rx_pos;
  A.depth = P->depth;
  A.px = P->px;
  A.py = P->py;
  A.pz = P->pz;
  A.nx = P->nx;
  A.ny = P->ny;
  A.nz = P->nz;
  A.kind = P->kind;
  A.dA = P->dA;
  A.mat = P->mat;
  A.tau = P->tau;
  A.raw = M->raw;
  A.per_inter = M->per_inter;
  A.inter_idx = M->per_inter ? M->inter_idx : nullptr;
  A.RS = A.inter_idx ? M->n_inter : A.DP;
  A.n_vmf = (pat && pat->tx_raw) ? pat->n_vmf : 0;
  A.tx_raw = pat ? pat->tx_raw : nullptr;
  A.pat_raw = pat ? pat->mat_raw : nullptr;
  A.n_mat_pat = M->n_mat > 0 ? M->n_mat : 1;
  A.edge = P->edge;
  A.mat_n = P->mat_n;
  A.k0 = 2.0 * kPi * r->fc_hz / kC0;
  double omega = 2.0 * kPi * r->fc_hz;
  A.inv_eps0w = (float)(1.0 / (kEps0 * omega));
  A.lam4pi = (kC0 / r->fc_hz) / (4.0 * kPi);
  A.cz_tx = cosf(r->zeta_tx);
  A.sz_tx = sinf(r->zeta_tx);
  A.cz_rx = cosf(r->zeta_rx);
  A.sz_rx = sinf(r->zeta_rx);
  A.ux = r->ula_axis[0];
  A.uy = r->ula_axis[1];
  A.uz = r->ula_axis[2];
  return A;
}

static int depth_bucket(int d) {
  if (d <= 1) return 1;
  if (d <= 2) return 2;
  if (d <= 3) return 3;
  if (d <= 4) return 4;
  if (d <= 6) return 6;
  return 8;
}

static int64_t adj_blocks(int32_t n_paths) {
  int64_t blocks = ((int64_t)n_paths + kTraceBlock - 1) / kTraceBlock;
  if (blocks > kTraceAdjMaxBlocks) blocks = kTraceAdjMaxBlocks;
  return blocks < 1 ? 1 : blocks;
}

// Gradient sections: materials (per-id), patterns, Tx (sizes for the
// workspace use the largest Tx section, kTxGrad).
static GradLayout grad_layout(bool mat, int n_mat, bool pat, int n_mat_pat, bool tx) {
  GradLayout g;
  int o = 0;
  g.mat = mat ? o : -1;
  o += mat ? 3 * n_mat : 0;
  g.pat = pat ? o : -1;
  o += pat ? kPatGrad * n_mat_pat : 0;
  g.tx = tx ? o : -1;
  o += tx ? kTxGrad : 0;
  g.stride = o;
  return g;
}

static size_t ws_for(int32_t n_paths, const GradLayout& g) {
  if (g.stride == 0) return 0;
  // per-block partials of the main and the diffraction launch, then the sums
  return (size_t)(2 * adj_blocks(n_paths) + 1) * g.stride * sizeof(double);
}

size_t ws_trace_adjoint(int32_t n_paths, int32_t n_mat) {
  if (n_mat < 1) n_mat = 1;
  return ws_for(n_paths, grad_layout(true, n_mat, false, 0, false));
}

// Workspace for every gradient the pattern variant can produce.
size_t ws_trace_adjoint_pat(int32_t n_paths, int32_t n_mat) {
  if (n_mat < 1) n_mat = 1;
  return ws_for(n_paths, grad_layout(true, n_mat, true, n_mat, true));
}

static rtc_status check_patterns(const rtc_patterns* pat, const rtc_materials* m, const char* fn) {
  if (!pat) return RTC_OK;
  RTC_REQUIRE(pat->n_vmf >= 0 && pat->n_vmf <= kMaxVmf, RTC_ERR_RANGE,
              "%s: n_vmf must be in [0, %d]", fn, kMaxVmf);
  RTC_REQUIRE(pat->n_vmf == 0 || pat->tx_raw != nullptr, RTC_ERR_INVALID_ARG,
              "%s: tx_raw is required when n_vmf > 0", fn);
  RTC_REQUIRE(!pat->mat_raw || m->n_mat >= 1, RTC_ERR_SHAPE,
              "%s: mat_raw needs n_mat >= 1 materials", fn);
  return RTC_OK;
}

}  // namespace rtc

using namespace rtc;

extern "C" rtc_status rtc_trace_fields_pat(const rtc_radio* radio, const rtc_paths* paths,
                                           const rtc_materials* mats, const rtc_patterns* pats,
                                           void* a, float* psi, void* stream) {
  const char* fn = "rtc_trace_fields";
  rtc_status st;
  if ((st = check_radio(radio, fn)) != RTC_OK) return st;
  if ((st = check_paths(paths, fn, true)) != RTC_OK) return st;
  if ((st = check_mats(mats, paths, fn)) != RTC_OK) return st;
  if ((st = check_patterns(pats, mats, fn)) != RTC_OK) return st;
  if (paths->n_paths == 0 || (a == nullptr && psi == nullptr)) return RTC_OK;
  RTC_REQUIRE(paths->n_links >= 1, RTC_ERR_SHAPE, "%s: n_paths > 0 needs n_links >= 1", fn);
  TraceArgs A = make_args(radio, paths, mats, pats);
  dim3 grid((paths->n_paths + kTraceBlock - 1) / kTraceBlock);
  size_t shm = trace_lds_fixed(A);
  hipStream_t s = as_stream(stream);
  const bool pat = A.n_vmf > 0 || A.pat_raw != nullptr;
  float2* a2 = reinterpret_cast<float2*>(a);
  switch (depth_bucket(paths->max_depth)) {
#define RTC_CASE(D)                                                                          \
  case D:                                                                                    \
    if (pat)                                                                                 \
      hipLaunchKernelGGL((trace_fields_kernel<D, true, false>), grid, dim3(kTraceBlock), shm, \
                         s, A, a2, psi);                                                     \
    else                                                                                     \
      hipLaunchKernelGGL((trace_fields_kernel<D, false, false>), grid, dim3(kTraceBlock),    \
                         shm, s, A, a2, psi);                                                \
    break;
    RTC_CASE(1)
    RTC_CASE(2)
    RTC_CASE(3)
    RTC_CASE(4)
    RTC_CASE(6)
    RTC_CASE(8)
#undef RTC_CASE
  }
  if (A.edge) {
    if ((st = check_launch(fn)) != RTC_OK) return st;
    // the diffraction paths (depth 1) in their own instance
    if (pat)
      hipLaunchKernelGGL((trace_fields_kernel<2, true, true>), grid, dim3(kTraceBlock), shm, s, A,
                         a2, psi);
    else
      hipLaunchKernelGGL((trace_fields_kernel<2, false, true>), grid, dim3(kTraceBlock), shm, s,
                         A, a2, psi);
  }
  return check_launch(fn);
}

extern "C" rtc_status rtc_trace_fields(const rtc_radio* radio, const rtc_paths* paths,
                                       const rtc_materials* mats, void* a, float* psi,
                                       void* stream) {
  return rtc_trace_fields_pat(radio, paths, mats, nullptr, a, psi, stream);
}

extern "C" rtc_status rtc_trace_fields_adjoint_pat(
    const rtc_radio* radio, const rtc_paths* paths, const rtc_materials* mats,
    const rtc_patterns* pats, const void* dLda, float* dLd_raw, float* dLd_inter, float* dLd_tx,
    float* dLd_pat, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "rtc_trace_fields_adjoint";
  rtc_status st;
  if ((st = check_radio(radio, fn)) != RTC_OK) return st;
  if ((st = check_paths(paths, fn, true)) != RTC_OK) return st;
  if ((st = check_mats(mats, paths, fn)) != RTC_OK) return st;
  if ((st = check_patterns(pats, mats, fn)) != RTC_OK) return st;
  RTC_REQUIRE(dLda != nullptr || paths->n_paths == 0, RTC_ERR_INVALID_ARG, "%s: dLda is NULL", fn);
  bool per_id = mats->raw != nullptr;
  RTC_REQUIRE(per_id ? (dLd_raw != nullptr && dLd_inter == nullptr)
                     : (dLd_inter != nullptr && dLd_raw == nullptr),
              RTC_ERR_INVALID_ARG,
              "%s: per-id mode needs dLd_raw (and dLd_inter NULL); per-interaction mode the "
              "reverse",
              fn);
  const bool want_tx = dLd_tx != nullptr;
  const bool want_pat = dLd_pat != nullptr;
  RTC_REQUIRE(!want_tx || (pats && pats->n_vmf > 0), RTC_ERR_INVALID_ARG,
              "%s: dLd_tx needs a Tx gain (n_vmf > 0)", fn);
  RTC_REQUIRE(!want_pat || (pats && pats->mat_raw), RTC_ERR_INVALID_ARG,
              "%s: dLd_pat needs mat_raw", fn);
  RTC_REQUIRE(!want_pat || per_id, RTC_ERR_UNSUPPORTED,
              "%s: pattern gradients need per-id materials", fn);
  hipStream_t s = as_stream(stream);
  TraceArgs A = make_args(radio, paths, mats, pats);
  const GradLayout GL = grad_layout(per_id, A.n_mat, want_pat, A.n_mat_pat, want_tx);
  int64_t blocks = ((int64_t)paths->n_paths + kTraceBlock - 1) / kTraceBlock;
  if (GL.stride > 0) {
    size_t need = ws_for(paths->n_paths, GL);
    RTC_REQUIRE(ws != nullptr && ws_bytes >= need, RTC_ERR_WORKSPACE,
                "%s: workspace of %zu bytes required", fn, need);
    blocks = adj_blocks(paths->n_paths);
  } else if (paths->n_paths == 0) {
    return RTC_OK;
  }
  if (paths->n_paths > 0 || GL.stride > 0) {
    RTC_REQUIRE(paths->n_links >= 1 || paths->n_paths == 0, RTC_ERR_SHAPE,
                "%s: n_paths > 0 needs n_links >= 1", fn);
  }
  size_t shm = trace_lds_fixed(A) + (size_t)(kTraceBlock / 64) * GL.stride * sizeof(double);
  // per-thread material sums (and their quarter sums) where they fit beside
  // two workgroups per CU; beyond 16 materials the wave walk
  {
    const size_t lane_bytes = (size_t)3 * A.n_mat * kTraceBlock * sizeof(float);
    const size_t q_bytes = ((size_t)3 * A.n_mat * (kTraceBlock / 64) + 1) * sizeof(double);
    if (per_id && GL.mat >= 0 && lane_bytes <= 48 * 1024) {
      A.lane_acc = 1;
      shm += (lane_bytes + 7) / 8 * 8 + q_bytes;
    }
  }
  RTC_REQUIRE(shm <= 160 * 1024, RTC_ERR_RANGE,
              "%s: %zu bytes of LDS needed (too many materials for the gradients asked)", fn, shm);
  double* part = reinterpret_cast<double*>(ws);
  const float2* g_a = reinterpret_cast<const float2*>(dLda);
  // the optional physics is compiled in only when the paths or patterns use
  // it; diffraction paths (depth 1) run in their own instance, whose
  // per-block partials follow the main launch's (face n in a second slot)
  const bool pat = A.n_vmf > 0 || A.pat_raw != nullptr;
  double* part2 = part + blocks * GL.stride;
  switch (depth_bucket(paths->max_depth)) {
#define RTC_LAUNCH(D, ID, PAT, DINT)                                                          \
  hipLaunchKernelGGL((trace_fields_adjoint_kernel<D, ID, PAT, false>), dim3(blocks),          \
                     dim3(kTraceBlock), shm, s, A, g_a, DINT, part, GL)
#define RTC_CASE(D)                                                                           \
  case D:                                                                                     \
    if (per_id) {                                                                             \
      if (pat)                                                                                \
        RTC_LAUNCH(D, true, true, nullptr);                                                   \
      else                                                                                    \
        RTC_LAUNCH(D, true, false, nullptr);                                                  \
    } else {                                                                                  \
      if (pat)                                                                                \
        RTC_LAUNCH(D, false, true, dLd_inter);                                                \
      else                                                                                    \
        RTC_LAUNCH(D, false, false, dLd_inter);                                               \
    }                                                                                         \
    break;
    RTC_CASE(1)
    RTC_CASE(2)
    RTC_CASE(3)
    RTC_CASE(4)
    RTC_CASE(6)
    RTC_CASE(8)
#undef RTC_CASE
#undef RTC_LAUNCH
  }
  if ((st = check_launch(fn)) != RTC_OK) return st;
  int64_t rows = blocks;
  if (A.edge) {
#define RTC_DLAUNCH(ID, PAT, DINT)                                                            \
  hipLaunchKernelGGL((trace_fields_adjoint_kernel<2, ID, PAT, true>), dim3(blocks),           \
                     dim3(kTraceBlock), shm, s, A, g_a, DINT, part2, GL)
    if (per_id) {
      if (pat)
        RTC_DLAUNCH(true, true, nullptr);
      else
        RTC_DLAUNCH(true, false, nullptr);
    } else {
      if (pat)
        RTC_DLAUNCH(false, true, dLd_inter);
      else
        RTC_DLAUNCH(false, false, dLd_inter);
    }
#undef RTC_DLAUNCH
    if ((st = check_launch(fn)) != RTC_OK) return st;
    rows = 2 * blocks;
  }
  if (GL.stride > 0) {
    double* tot = part + rows * GL.stride;
    hipLaunchKernelGGL(trace_adjoint_reduce_kernel, dim3(GL.stride), dim3(kTraceBlock), 0, s, part,
                       (int)rows, GL.stride, tot);
    if ((st = check_launch(fn)) != RTC_OK) return st;
    hipLaunchKernelGGL(trace_adjoint_transform_kernel, dim3(1), dim3(kTraceBlock), 0, s, tot, GL,
                       A.n_mat, mats->raw, A.n_mat_pat, A.pat_raw, A.n_vmf, A.tx_raw, dLd_raw,
                       dLd_pat, dLd_tx);
    return check_launch(fn);
  }
  return RTC_OK;
}

extern "C" rtc_status rtc_trace_fields_adjoint(const rtc_radio* radio, const rtc_paths* paths,
                                               const rtc_materials* mats, const void* dLda,
                                               float* dLd_raw, float* dLd_inter, void* ws,
                                               size_t ws_bytes, void* stream) {
  return rtc_trace_fields_adjoint_pat(radio, paths, mats, nullptr, dLda, dLd_raw, dLd_inter,
                                      nullptr, nullptr, ws, ws_bytes, stream);
}
