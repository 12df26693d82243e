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
#include <cmath>

#include "api_common.h"
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
  const float* per_inter;  // [3*DP] or null
  float inv_eps0w;         // 1/(eps0 * omega_c)
  double lam4pi;           // lambda_c / (4 pi)
  float cz_tx, sz_tx, cz_rx, sz_rx;
  float ux, uy, uz;  // ULA axis
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
    return make_mat(A.per_inter[slot], A.per_inter[A.DP + slot], A.per_inter[2 * A.DP + slot],
                    A.inv_eps0w);
  }
  int m = A.mat[slot];
  m = m < A.n_mat ? m : A.n_mat - 1;
  return tab[m];
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
};

template <int MAXD, bool SAVE>
RTC_DEV void run_chain(const TraceArgs& A, const MatVal* tab, int64_t p, Chain<MAXD, SAVE>& C) {
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
  // Tx pattern: isotropic, slant angle zeta (Sec. II-B)
  float2 E0 = make_float2(A.cz_tx, 0.0f);
  float2 E1 = make_float2(A.sz_tx, 0.0f);
  v3 prev = tx;
  float rho = 0.0f;  // unfolded length from the Tx
  C.dif = false;
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
      if (dif) {
        v3 nf = dot3(k_in, n) > 0.0f ? scl3(n, -1.0f) : n;  // towards the incidence side
        v3 k_s = unit3(sub3(rx, s));
        float geo = c * A.dA[slot] * fmaxf(dot3(k_s, nf), 0.0f) * kInvPi;
        float G0 = sqrtf(fmaxf(geo, 0.0f));
        float nv = sqrtf(cabs2(cmul(rp, y0)) + cabs2(cmul(rl, y1)));
        E0 = make_float2(mv.S * nv * G0, 0.0f);
        E1 = make_float2(0.0f, 0.0f);
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
  } else {
    C.scale = (float)(A.lam4pi / (kC0 * A.tau[p]));
  }
}

template <int MAXD>
__global__ void __launch_bounds__(kTraceBlock) trace_fields_kernel(TraceArgs A, float2* a,
                                                                    float* psi) {
  extern __shared__ MatVal tab[];
  stage_materials(A, tab);
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= A.n_paths) return;
  Chain<MAXD, false> C;
  run_chain<MAXD, false>(A, tab, p, C);
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
template <int MAXD, bool PER_ID>
__global__ void __launch_bounds__(kTraceBlock)
    trace_fields_adjoint_kernel(TraceArgs A, const float2* dLda, float* dLd_inter,
                                double* block_part) {
  extern __shared__ unsigned char smem[];
  MatVal* tab = reinterpret_cast<MatVal*>(smem);
  double* acc = reinterpret_cast<double*>(smem + ((A.raw ? A.n_mat : 0) * sizeof(MatVal) + 15) / 16 * 16);
  stage_materials(A, tab);
  if constexpr (PER_ID) {
    for (int i = threadIdx.x; i < 3 * A.n_mat * (int)(blockDim.x >> 6); i += blockDim.x)
      acc[i] = 0.0;
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
    float g_eps[MAXD], g_sig[MAXD], g_S[MAXD];
    int ids[MAXD];
    int Q = 0;
#pragma unroll
    for (int j = 0; j < MAXD; ++j) {
      g_eps[j] = g_sig[j] = g_S[j] = 0.0f;
      ids[j] = 0x7fffffff;
    }
    if (valid) {
      Chain<MAXD, true> C;
      run_chain<MAXD, true>(A, tab, p, C);
      Q = C.Q;
      float2 Ga = dLda[p];
      // w^T = K c_R^T D_{Q+1}  (real at the start)
      float K = C.scale;
      float2 w0 = make_float2(K * (A.cz_rx * C.Dq[0] + A.sz_rx * C.Dq[2]), 0.0f);
      float2 w1 = make_float2(K * (A.cz_rx * C.Dq[1] + A.sz_rx * C.Dq[3]), 0.0f);
#pragma unroll
      for (int j = MAXD - 1; j >= 0; --j) {
        if (j < Q && C.dif && j == Q - 1) {
          // a = K q_R |E_s| is real, so dL/dx = Re(dL/da) da/dx.  With
          // |E_s| = S G0 nv, nv = |v|, v = (r_perp y0, r_par y1):
          //   d nv/d eta_re = Re(Z)/nv, d nv/d eta_im = -Im(Z)/nv,
          //   Z = conj(r_perp) dr_perp/deta |y0|^2 + conj(r_par) dr_par/deta |y1|^2
          // and d nv = Re(c^T dy) with c = (conj(v0) r_perp, conj(v1) r_par)/nv,
          // which continues the sweep through the preceding interactions.
          const float qR = A.cz_rx * C.Dq[0] + A.sz_rx * C.Dq[2];
          const float gam = Ga.x * K * qR;
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
          // slots past the depth get zeros
          dLd_inter[slot] = g_eps[j];
          dLd_inter[A.DP + slot] = g_sig[j];
          dLd_inter[2 * A.DP + slot] = g_S[j];
        }
      }
    } else {
      // Segmented reduction by material id, deterministic: each wave walks
      // the distinct ids present in it in increasing order; for each id the
      // lanes' contributions (fixed order over j) are summed by a butterfly
      // in FP64 and added to the wave's own LDS table (waves are summed in
      // order at the end).
      {
        double* wacc = acc + wave * 3 * A.n_mat;
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
  }
  if constexpr (PER_ID) {
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * A.n_mat; i += blockDim.x) {
      double t = 0.0;
      for (int w = 0; w < n_waves; ++w) t += acc[w * 3 * A.n_mat + i];
      block_part[(int64_t)blockIdx.x * 3 * A.n_mat + i] = t;
    }
  }
  (void)eps0w_inv;
}

// Sum the per-block partials (FP64, fixed order: strided per thread, then a
// tree over the workgroup) and apply the raw parameter transforms:
// d eps/du0 = eps - 1, d sigma/du1 = sigma, dS/du2 = S (1 - S).
// One workgroup of kTraceBlock threads per output.
__global__ void __launch_bounds__(kTraceBlock)
    trace_adjoint_finish_kernel(const double* block_part, int n_blocks, int n_mat,
                                const float* raw, float* dLd_raw) {
  __shared__ double red[kTraceBlock];
  const int i = blockIdx.x;  // output index < 3 n_mat
  double s = 0.0;
  for (int b = threadIdx.x; b < n_blocks; b += blockDim.x) s += block_part[(int64_t)b * 3 * n_mat + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  s = red[0];
  int m = i / 3, c = i % 3;
  double u = (double)raw[3 * m + c];
  double d;
  if (c == 0)
    d = exp(u);
  else if (c == 1)
    d = exp(u);
  else {
    double S = 1.0 / (1.0 + exp(-u));
    d = S * (1.0 - S);
  }
  dLd_raw[i] = (float)(s * d);
}

static TraceArgs make_args(const rtc_radio* r, const rtc_paths* P, const rtc_materials* M) {
  TraceArgs A;
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

size_t ws_trace_adjoint(int32_t n_paths, int32_t n_mat) {
  if (n_mat < 1) n_mat = 1;
  int64_t blocks = ((int64_t)n_paths + kTraceBlock - 1) / kTraceBlock;
  if (blocks > kTraceAdjMaxBlocks) blocks = kTraceAdjMaxBlocks;
  if (blocks < 1) blocks = 1;
  return (size_t)blocks * 3 * n_mat * sizeof(double);
}

}  // namespace rtc

using namespace rtc;

extern "C" rtc_status rtc_trace_fields(const rtc_radio* radio, const rtc_paths* paths,
                                       const rtc_materials* mats, void* a, float* psi,
                                       void* stream) {
  const char* fn = "rtc_trace_fields";
  rtc_status st;
  if ((st = check_radio(radio, fn)) != RTC_OK) return st;
  if ((st = check_paths(paths, fn, true)) != RTC_OK) return st;
  if ((st = check_mats(mats, paths, fn)) != RTC_OK) return st;
  if (paths->n_paths == 0 || (a == nullptr && psi == nullptr)) return RTC_OK;
  RTC_REQUIRE(paths->n_links >= 1, RTC_ERR_SHAPE, "%s: n_paths > 0 needs n_links >= 1", fn);
  TraceArgs A = make_args(radio, paths, mats);
  dim3 grid((paths->n_paths + kTraceBlock - 1) / kTraceBlock);
  size_t shm = (mats->raw ? mats->n_mat : 0) * sizeof(MatVal);
  hipStream_t s = as_stream(stream);
  switch (depth_bucket(paths->max_depth)) {
#define RTC_CASE(D)                                                                          \
  case D:                                                                                    \
    hipLaunchKernelGGL(trace_fields_kernel<D>, grid, dim3(kTraceBlock), shm, s, A,           \
                       reinterpret_cast<float2*>(a), psi);                                   \
    break;
    RTC_CASE(1)
    RTC_CASE(2)
    RTC_CASE(3)
    RTC_CASE(4)
    RTC_CASE(6)
    RTC_CASE(8)
#undef RTC_CASE
  }
  return check_launch(fn);
}

extern "C" rtc_status rtc_trace_fields_adjoint(const rtc_radio* radio, const rtc_paths* paths,
                                               const rtc_materials* mats, const void* dLda,
                                               float* dLd_raw, float* dLd_inter, void* ws,
                                               size_t ws_bytes, void* stream) {
  const char* fn = "rtc_trace_fields_adjoint";
  rtc_status st;
  if ((st = check_radio(radio, fn)) != RTC_OK) return st;
  if ((st = check_paths(paths, fn, true)) != RTC_OK) return st;
  if ((st = check_mats(mats, paths, fn)) != RTC_OK) return st;
  RTC_REQUIRE(dLda != nullptr || paths->n_paths == 0, RTC_ERR_INVALID_ARG, "%s: dLda is NULL", fn);
  bool per_id = mats->raw != nullptr;
  RTC_REQUIRE(per_id ? (dLd_raw != nullptr && dLd_inter == nullptr)
                     : (dLd_inter != nullptr && dLd_raw == nullptr),
              RTC_ERR_INVALID_ARG,
              "%s: per-id mode needs dLd_raw (and dLd_inter NULL); per-interaction mode the "
              "reverse",
              fn);
  hipStream_t s = as_stream(stream);
  TraceArgs A = make_args(radio, paths, mats);
  int64_t blocks = ((int64_t)paths->n_paths + kTraceBlock - 1) / kTraceBlock;
  if (per_id) {
    size_t need = ws_trace_adjoint(paths->n_paths, mats->n_mat);
    RTC_REQUIRE(ws != nullptr && ws_bytes >= need, RTC_ERR_WORKSPACE,
                "%s: workspace of %zu bytes required", fn, need);
    if (blocks > kTraceAdjMaxBlocks) blocks = kTraceAdjMaxBlocks;
    if (blocks < 1) blocks = 1;
  } else if (paths->n_paths == 0) {
    return RTC_OK;
  }
  if (paths->n_paths > 0 || per_id) {
    RTC_REQUIRE(paths->n_links >= 1 || paths->n_paths == 0, RTC_ERR_SHAPE,
                "%s: n_paths > 0 needs n_links >= 1", fn);
  }
  size_t tab_bytes = ((per_id ? mats->n_mat : 0) * sizeof(MatVal) + 15) / 16 * 16;
  size_t shm = tab_bytes + (per_id ? (kTraceBlock / 64) * 3 * mats->n_mat * sizeof(double) : 0);
  double* part = reinterpret_cast<double*>(ws);
  switch (depth_bucket(paths->max_depth)) {
#define RTC_CASE(D)                                                                            \
  case D:                                                                                      \
    if (per_id)                                                                                \
      hipLaunchKernelGGL((trace_fields_adjoint_kernel<D, true>), dim3(blocks), dim3(kTraceBlock), \
                         shm, s, A, reinterpret_cast<const float2*>(dLda), nullptr, part);     \
    else                                                                                       \
      hipLaunchKernelGGL((trace_fields_adjoint_kernel<D, false>), dim3(blocks),                \
                         dim3(kTraceBlock), shm, s, A, reinterpret_cast<const float2*>(dLda),  \
                         dLd_inter, nullptr);                                                  \
    break;
    RTC_CASE(1)
    RTC_CASE(2)
    RTC_CASE(3)
    RTC_CASE(4)
    RTC_CASE(6)
    RTC_CASE(8)
#undef RTC_CASE
  }
  if ((st = check_launch(fn)) != RTC_OK) return st;
  if (per_id) {
    int n = 3 * mats->n_mat;
    hipLaunchKernelGGL(trace_adjoint_finish_kernel, dim3(n), dim3(kTraceBlock), 0, s, part,
                       (int)blocks, mats->n_mat, mats->raw, dLd_raw);
    return check_launch(fn);
  }
  return RTC_OK;
}
