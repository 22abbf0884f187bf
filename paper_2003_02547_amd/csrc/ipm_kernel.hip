// Batched OCP-QP primal-dual interior-point method on gfx950.
//
// One 64-lane workgroup solves one instance end to end (the whole IPM loop
// runs inside the launch).  Stage blocks are compile-time sized (NX, NU, NG)
// and staged through LDS; per-stage data is streamed from HBM in the stage
// order of each sweep.
//
// Method (paper: "HPIPM: a high-performance quadratic programming framework
// for model predictive control"):
//   * residual function and Newton system of eq:alg:pdipm:delta, delta
//     formulation (Section 3.2; mode "speed" of Section 4.2);
//   * elimination of dt then dlam into the reduced system eq:alg:kkt
//     (Section 3.3);
//   * square-root Riccati recursion, variant (b) of Section 3.3: with
//     L_{n+1} L_{n+1}' = P_{n+1} and U = L_{n+1}' [B_n A_n], the stage matrix
//     M_n = Phi_n + U'U is Cholesky-factorized, M_n = [[L_uu, 0], [L_xu, L_xx]]
//     (u first), and L_n = L_xx;
//   * infeasible-start Mehrotra predictor-corrector with the conditional
//     corrector, primal regularization and lower clamps (Section 4.2).
//
// Riccati equations (derived from eq:alg:kkt by dynamic programming):
//   m_n  = gt_n + F_n'(L_{n+1} L_{n+1}' rb_n + p_{n+1})
//   y_n  = L_uu^{-1} m_u,   p_n = m_x - L_xu y_n
//   dx_0 = -(L_0 L_0')^{-1} p_0
//   du_n = -L_uu^{-T} (y_n + L_xu' dx_n),   dx_{n+1} = F_n dz_n + rb_n
//   dpi_{n+1} = L_{n+1} L_{n+1}' dx_{n+1} + p_{n+1}
// with gt = r_g - C'(W r_d - T^{-1} r_m), dt = C dy - r_d,
// dlam = -T^{-1}(r_m + Lam dt), C = [G; -G] the stacked two-sided rows.
#include <hip/hip_runtime.h>

#include "layout.h"

namespace oqp {

constexpr int WAVE = 64;

__device__ __forceinline__ double nmax(double a, double b) { return (a > b || a != a) ? a : b; }

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = nmax(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Value of v held by lane `src` (src is wave-uniform).
__device__ __forceinline__ double bcast(double v, int src)
{
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Right-hand-side variants of the complementarity row r_m.
enum { RM_SHIFT = 0,      // r_m = lam.*t - shift
       RM_CORRECTOR = 1,  // r_m = lam.*t + dlam_aff.*dt_aff - shift
       RM_IR = 2 };       // r_m taken from the refinement residual arrays

template <int NX, int NU, int NG>
struct Ipm {
    static constexpr Layout Lo = make_layout(NX, NU, NG);
    static constexpr int NZ = NX + NU;
    static constexpr int NC = NZ + NG;
    static constexpr int NV = NX + NG;
    static constexpr int LDZ = NZ | 1;
    static constexpr int LDX = NX | 1;
    static constexpr int LDV = NV | 1;
    static constexpr int LDG = NG > 0 ? (NG | 1) : 1;
    static constexpr int NCP = NC > WAVE ? 2 * WAVE : WAVE;  // LDS vector length for slot vectors
    static_assert(NZ <= WAVE && NX <= WAVE && NG <= WAVE, "stage block must fit one wave");

    struct Smem {
        double M[LDZ * NZ];      // stage matrix / factor (column-major)
        double Lx[2][LDX * NX];  // L_{n+1} (lower, zero strict upper), by stage parity
        double F[LDX * NZ];      // [B A] of the stage
        double V[LDV * NZ];      // [U; sqrt(w) G]
        double G[LDG * NZ];      // general rows of the stage
        double col[2][WAVE];     // Cholesky column broadcast
        double z[WAVE];          // z_n (or dz_n)
        double t0[WAVE], t1[WAVE], t2[WAVE];
        double e[NCP];           // reduced-gradient terms per constraint slot
        double ws[NCP];          // barrier weights per constraint slot
        double xn[2][WAVE];      // x_{n+1} / dx_{n+1}, by parity
        double pin[2][WAVE];     // pi_{n+1}, by parity
        double pn[2][WAVE];      // p_{n+1}, by parity
    };

    const double* __restrict__ dat;
    double* __restrict__ itr;
    double* __restrict__ wk;
    int N, nc, lane;
    const KParams& P;

    // The workgroup's LDS block (one instance per workgroup).
    __device__ __forceinline__ static Smem& S()
    {
        __shared__ Smem smem;
        return smem;
    }

    __device__ __forceinline__ Ipm(const double* d, double* i, double* w, int N_, int nc_, const KParams& P_)
        : dat(d), itr(i), wk(w), N(N_), nc(nc_), lane((int)threadIdx.x), P(P_) {}

    __device__ __forceinline__ const double* Dp(int n) const { return dat + (size_t)n * Lo.SREC; }
    __device__ __forceinline__ double* Ip(int n) const { return itr + (size_t)n * Lo.IREC; }
    __device__ __forceinline__ double* Wp(int n) const { return wk + (size_t)n * Lo.WREC; }

    // global (ld = R) -> LDS (ld = LD), R x C column-major
    template <int R, int C, int LD>
    __device__ __forceinline__ void load_mat(double* dst, const double* __restrict__ src) const
    {
        Smem& s = S();
        (void)s;
#pragma unroll
        for (int e0 = 0; e0 < R * C; e0 += WAVE) {
            int e = e0 + lane;
            if (e < R * C) {
                int i = e % R, j = e / R;
                dst[i + j * LD] = src[e];
            }
        }
    }

    __device__ __forceinline__ static double slot_mask(const double* d, int c)
    {
        return c < NZ ? d[Lo.D_bm + c] : d[Lo.D_gm + (c - NZ)];
    }

    // r_m for slot c of stage record (ir, w), lower and upper.
    __device__ __forceinline__ void rm_of(int rmode, double shift, const double* ir, const double* w, int c, double& rml,
                          double& rmu) const
    {
        Smem& s = S();
        (void)s;
        if (rmode == RM_IR) {
            rml = w[Lo.W_irml + c];
            rmu = w[Lo.W_irmu + c];
            return;
        }
        double ll = ir[Lo.I_ll + c], lu = ir[Lo.I_lu + c], tl = ir[Lo.I_tl + c], tu = ir[Lo.I_tu + c];
        rml = ll * tl - shift;
        rmu = lu * tu - shift;
        if (rmode == RM_CORRECTOR) {
            rml += w[Lo.W_all + c] * w[Lo.W_atl + c];
            rmu += w[Lo.W_alu + c] * w[Lo.W_atu + c];
        }
    }

    // ------------------------------------------------------------------
    // Right-looking Cholesky of s.M (NZ x NZ), one row per lane, rows held in
    // registers.  On return lane i < NZ holds row i of L in r[0..i] and 1/L_ii.
    // ------------------------------------------------------------------
    __device__ __forceinline__ void cholesky(double (&r)[NZ], double& dinv) const
    {
        Smem& s = S();
        (void)s;
#pragma unroll
        for (int k = 0; k < NZ; ++k) r[k] = lane < NZ ? s.M[lane + k * LDZ] : 0.0;
        dinv = 0.0;
#pragma unroll
        for (int j = 0; j < NZ; ++j) {
            double piv = bcast(r[j], j);
            double ljj = sqrt(piv);
            double inv = 1.0 / ljj;
            double lij = r[j] * inv;
            if (lane == j) {
                r[j] = ljj;
                dinv = inv;
            } else if (lane > j) {
                r[j] = lij;
            }
            if (j + 1 < NZ) {
                s.col[j & 1][lane] = lij;
                __syncthreads();
#pragma unroll
                for (int k = j + 1; k < NZ; ++k) {
                    double lkj = s.col[j & 1][k];
                    if (lane >= k) r[k] -= lij * lkj;
                }
            }
        }
    }

    // Forward substitution with the (u, u) block, fused with the x rows:
    // lanes i < NU end with y = L_uu^{-1} m_u, lanes NU <= i < NZ with
    // p = m_x - L_xu y.  rowL[j] = L[i][j] for j < NU; dinv is 1/L_ii.
    template <int CNT>
    __device__ __forceinline__ double fwd_subst_u(double m, const double (&rowL)[CNT], double dinv) const
    {
        Smem& s = S();
        (void)s;
#pragma unroll
        for (int j = 0; j < NU; ++j) {
            double y = bcast(m, j) * bcast(dinv, j);
            if (lane == j) m = y;
            else if (lane > j) m -= rowL[j] * y;
        }
        return m;
    }

    // ------------------------------------------------------------------
    // Backward pass: residuals at the iterate, barrier terms, square-root
    // Riccati factorization and the right-hand-side sweep for r_m = lam.*t -
    // shift.  Returns per-wave residual norms and lam't.
    // ------------------------------------------------------------------
    __device__ __forceinline__ void backward_factor(double shift, bool factor, double& n_g, double& n_b, double& n_d, double& n_m,
                                    double& s_lt)
    {
        Smem& s = S();
        (void)s;
        double mg = 0.0, mb = 0.0, md = 0.0, mm = 0.0, slt = 0.0;
        for (int n = N; n >= 0; --n) {
            const int cur = n & 1, nxt = (n + 1) & 1;
            const double* d = Dp(n);
            double* ir = Ip(n);
            double* w = Wp(n);
            load_mat<NZ, NZ, LDZ>(s.M, d + Lo.D_H);
            if (n < N) load_mat<NX, NZ, LDX>(s.F, d + Lo.D_F);
            if constexpr (NG > 0) load_mat<NG, NZ, LDG>(s.G, d + Lo.D_G);
            double zj = 0.0;
            if (lane < NZ) {
                zj = ir[Lo.I_z + lane];
                s.z[lane] = zj;
            }
            if (lane < NX) s.t0[lane] = ir[Lo.I_pi + lane];  // pi_n
            if constexpr (NG > 0) {
                if (lane < NG)
                    s.t1[lane] = d[Lo.D_gm + lane] * (ir[Lo.I_ll + NZ + lane] - ir[Lo.I_lu + NZ + lane]);
            }
            if (n == N) {
                if (lane < NX) {
                    s.xn[nxt][lane] = 0.0;
                    s.pin[nxt][lane] = 0.0;
                    s.pn[nxt][lane] = 0.0;
                }
            }
            __syncthreads();

            // r_g = H z + g + F' pi_{n+1} - [0; pi_n] - C' lam
            double rg = 0.0;
            if (lane < NZ) {
                const int j = lane;
                double acc = d[Lo.D_g + j];
#pragma unroll
                for (int k = 0; k < NZ; ++k) acc += s.M[j + k * LDZ] * s.z[k];
                if (n < N) {
#pragma unroll
                    for (int i = 0; i < NX; ++i) acc += s.F[i + j * LDX] * s.pin[nxt][i];
                }
                if (j >= NU) acc -= s.t0[j - NU];
                acc -= d[Lo.D_bm + j] * (ir[Lo.I_ll + j] - ir[Lo.I_lu + j]);
                if constexpr (NG > 0) {
#pragma unroll
                    for (int r = 0; r < NG; ++r) acc -= s.G[r + j * LDG] * s.t1[r];
                }
                rg = acc;
                w[Lo.W_rg + j] = rg;
                mg = nmax(mg, fabs(rg));
            }
            // r_b = F z + b - x_{n+1}
            double rb = 0.0;
            if (n < N && lane < NX) {
                const int i = lane;
                double acc = d[Lo.D_b + i];
#pragma unroll
                for (int k = 0; k < NZ; ++k) acc += s.F[i + k * LDX] * s.z[k];
                acc -= s.xn[nxt][i];
                rb = acc;
                w[Lo.W_rb + i] = rb;
                mb = nmax(mb, fabs(rb));
            }
            // r_d, complementarity, weights and reduced-gradient terms per slot
            for (int c = lane; c < NC; c += WAVE) {
                double m, lo, hi, gz;
                if (c < NZ) {
                    m = d[Lo.D_bm + c];
                    lo = d[Lo.D_blo + c];
                    hi = d[Lo.D_bhi + c];
                    gz = s.z[c];
                } else {
                    const int r = c - NZ;
                    m = d[Lo.D_gm + r];
                    lo = d[Lo.D_glo + r];
                    hi = d[Lo.D_ghi + r];
                    gz = 0.0;
#pragma unroll
                    for (int k = 0; k < NZ; ++k) gz += s.G[r + k * LDG] * s.z[k];
                }
                double rdl = 0.0, rdu = 0.0, e = 0.0, wsum = 0.0;
                if (m != 0.0) {
                    const double ll = ir[Lo.I_ll + c], lu = ir[Lo.I_lu + c];
                    const double tl = ir[Lo.I_tl + c], tu = ir[Lo.I_tu + c];
                    rdl = -gz + tl + lo;
                    rdu = gz + tu - hi;
                    md = nmax(md, nmax(fabs(rdl), fabs(rdu)));
                    const double a = ll * tl, b = lu * tu;
                    mm = nmax(mm, nmax(a, b));
                    slt += a + b;
                    const double wl = ll / tl, wu = lu / tu;
                    wsum = wl + wu;
                    const double rml = a - shift, rmu = b - shift;
                    e = (wl * rdl - rml / tl) - (wu * rdu - rmu / tu);
                }
                w[Lo.W_rdl + c] = rdl;
                w[Lo.W_rdu + c] = rdu;
                s.e[c] = e;
                s.ws[c] = wsum;
            }
            if (!factor) {
                // residual-only pass: carry x_n and pi_n to stage n-1
                __syncthreads();
                if (lane >= NU && lane < NZ) s.xn[cur][lane - NU] = zj;
                if (lane < NX) s.pin[cur][lane] = s.t0[lane];
                __syncthreads();
                continue;
            }
            if (lane < NX) s.t2[lane] = rb;
            __syncthreads();

            // Phi = H + diag(box weights) + reg I ; V = [L_{n+1}' F ; sqrt(w_g) G]
            if (lane < NZ) s.M[lane + lane * LDZ] += s.ws[lane] + P.reg_prim;
            if constexpr (NG > 0) {
#pragma unroll
                for (int e0 = 0; e0 < NG * NZ; e0 += WAVE) {
                    int e = e0 + lane;
                    if (e < NG * NZ) {
                        int r = e % NG, k = e / NG;
                        s.V[NX + r + k * LDV] = sqrt(s.ws[NZ + r]) * s.G[r + k * LDG];
                    }
                }
            }
            if (n < N) {
                // trmm: V[i][k] = sum_l L[l][i] F[l][k]  (L lower, zero strict upper)
                const double* Lx = s.Lx[nxt];
#pragma unroll
                for (int e0 = 0; e0 < NX * NZ; e0 += WAVE) {
                    int e = e0 + lane;
                    if (e < NX * NZ) {
                        int i = e % NX, k = e / NX;
                        double acc = 0.0;
#pragma unroll
                        for (int l = 0; l < NX; ++l) acc += Lx[l + i * LDX] * s.F[l + k * LDX];
                        s.V[i + k * LDV] = acc;
                    }
                }
            }
            __syncthreads();
            // syrk: M += V'V over the rows present at this stage
            {
                constexpr int R0 = 0;
                const int r_begin = (n < N) ? R0 : NX;
                if (r_begin < NV) {
#pragma unroll
                    for (int e0 = 0; e0 < NZ * NZ; e0 += WAVE) {
                        int e = e0 + lane;
                        if (e < NZ * NZ) {
                            int i = e % NZ, k = e / NZ;
                            double acc = 0.0;
                            for (int r = r_begin; r < NV; ++r) acc += s.V[r + i * LDV] * s.V[r + k * LDV];
                            s.M[i + k * LDZ] += acc;
                        }
                    }
                }
            }
            __syncthreads();

            double rowL[NZ];
            double dinv;
            cholesky(rowL, dinv);
            if (lane < NZ) {
#pragma unroll
                for (int k = 0; k < NZ; ++k) w[Lo.W_L + lane + k * NZ] = (k <= lane) ? rowL[k] : 0.0;
                w[Lo.W_dinv + lane] = dinv;
            }

            // reduced gradient gt = r_g - C'(e)
            double m = 0.0;
            if (lane < NZ) {
                double acc = rg - s.e[lane];
                if constexpr (NG > 0) {
#pragma unroll
                    for (int r = 0; r < NG; ++r) acc -= s.G[r + lane * LDG] * s.e[NZ + r];
                }
                m = acc;
            }
            if (n < N) {
                const double* Lx = s.Lx[nxt];
                // t1 = L' rb
                if (lane < NX) {
                    double acc = 0.0;
#pragma unroll
                    for (int l = 0; l < NX; ++l) acc += Lx[l + lane * LDX] * s.t2[l];
                    s.t1[lane] = acc;
                }
                __syncthreads();
                // t0 = L t1 + p_{n+1}
                if (lane < NX) {
                    double acc = s.pn[nxt][lane];
#pragma unroll
                    for (int l = 0; l < NX; ++l) acc += Lx[lane + l * LDX] * s.t1[l];
                    s.t2[lane] = acc;
                }
                __syncthreads();
                if (lane < NZ) {
                    double acc = 0.0;
#pragma unroll
                    for (int i = 0; i < NX; ++i) acc += s.F[i + lane * LDX] * s.t2[i];
                    m += acc;
                }
            }
            m = fwd_subst_u<NZ>(m, rowL, dinv);
            if (lane < NU) w[Lo.W_yu + lane] = m;
            if (lane >= NU && lane < NZ) {
                w[Lo.W_pv + lane - NU] = m;
                s.pn[cur][lane - NU] = m;
                s.xn[cur][lane - NU] = zj;
                const int i = lane - NU;
#pragma unroll
                for (int k = 0; k < NX; ++k) s.Lx[cur][i + k * LDX] = (k <= i) ? rowL[NU + k] : 0.0;
            }
            if (lane < NX) s.pin[cur][lane] = s.t0[lane];
            __syncthreads();
        }
        n_g = wave_max(mg);
        n_b = wave_max(mb);
        n_d = wave_max(md);
        n_m = wave_max(mm);
        s_lt = wave_sum(slt);
    }

    // ------------------------------------------------------------------
    // Backward right-hand-side sweep with stored factors.
    // RHS: r_g / r_b / r_d from offsets og, ob, odl, odu; r_m per rmode.
    // ------------------------------------------------------------------
    __device__ __forceinline__ void backward_vec(int rmode, double shift, int og, int ob, int odl, int odu)
    {
        Smem& s = S();
        (void)s;
        for (int n = N; n >= 0; --n) {
            const int cur = n & 1, nxt = (n + 1) & 1;
            const double* d = Dp(n);
            double* ir = Ip(n);
            double* w = Wp(n);
            if (n < N) load_mat<NX, NZ, LDX>(s.F, d + Lo.D_F);
            if constexpr (NG > 0) load_mat<NG, NZ, LDG>(s.G, d + Lo.D_G);
            if (n == N && lane < NX) s.pn[nxt][lane] = 0.0;
            // factor rows (first NU columns) in registers; (x, x) block to LDS
            double rowL[NU > 0 ? NU : 1];
#pragma unroll
            for (int k = 0; k < (NU > 0 ? NU : 1); ++k) rowL[k] = 0.0;
            double dinv = 0.0;
            if (lane < NZ) {
#pragma unroll
                for (int k = 0; k < NU; ++k) rowL[k] = w[Lo.W_L + lane + k * NZ];
                dinv = w[Lo.W_dinv + lane];
            }
            if (lane >= NU && lane < NZ) {
                const int i = lane - NU;
#pragma unroll
                for (int k = 0; k < NX; ++k) s.Lx[cur][i + k * LDX] = w[Lo.W_L + lane + (NU + k) * NZ];
            }
            for (int c = lane; c < NC; c += WAVE) {
                double e = 0.0;
                if (slot_mask(d, c) != 0.0) {
                    double rml, rmu;
                    rm_of(rmode, shift, ir, w, c, rml, rmu);
                    const double ll = ir[Lo.I_ll + c], lu = ir[Lo.I_lu + c];
                    const double tl = ir[Lo.I_tl + c], tu = ir[Lo.I_tu + c];
                    e = ((ll / tl) * w[odl + c] - rml / tl) - ((lu / tu) * w[odu + c] - rmu / tu);
                }
                s.e[c] = e;
            }
            if (n < N && lane < NX) s.t2[lane] = w[ob + lane];
            __syncthreads();
            double m = 0.0;
            if (lane < NZ) {
                double acc = w[og + lane] - s.e[lane];
                if constexpr (NG > 0) {
#pragma unroll
                    for (int r = 0; r < NG; ++r) acc -= s.G[r + lane * LDG] * s.e[NZ + r];
                }
                m = acc;
            }
            if (n < N) {
                const double* Lx = s.Lx[nxt];
                if (lane < NX) {
                    double acc = 0.0;
#pragma unroll
                    for (int l = 0; l < NX; ++l) acc += Lx[l + lane * LDX] * s.t2[l];
                    s.t1[lane] = acc;
                }
                __syncthreads();
                if (lane < NX) {
                    double acc = s.pn[nxt][lane];
#pragma unroll
                    for (int l = 0; l < NX; ++l) acc += Lx[lane + l * LDX] * s.t1[l];
                    s.t2[lane] = acc;
                }
                __syncthreads();
                if (lane < NZ) {
                    double acc = 0.0;
#pragma unroll
                    for (int i = 0; i < NX; ++i) acc += s.F[i + lane * LDX] * s.t2[i];
                    m += acc;
                }
            }
            m = fwd_subst_u<NU>(m, rowL, dinv);
            if (lane < NU) w[Lo.W_yu + lane] = m;
            if (lane >= NU && lane < NZ) {
                w[Lo.W_pv + lane - NU] = m;
                s.pn[cur][lane - NU] = m;
            }
            __syncthreads();
        }
    }

    // ------------------------------------------------------------------
    // Forward substitution and recovery of dt, dlam.  Writes the step into
    // the (oz, opi, oll, olu, otl, otu) workspace offsets and returns the
    // largest alpha keeping lam, t >= 0 (uncapped; HUGE_VAL if unblocked).
    // ------------------------------------------------------------------
    __device__ __forceinline__ double forward(int rmode, double shift, int odl, int odu, int ob, int oz, int opi, int oll, int olu,
                              int otl, int otu)
    {
        Smem& s = S();
        (void)s;
        double amin = HUGE_VAL;
        // dx_0 = -(L0 L0')^{-1} p_0 with L0 the (x, x) block of stage 0
        {
            double* w0 = Wp(0);
            if (lane < NX) {
#pragma unroll
                for (int k = 0; k < NX; ++k) s.Lx[0][lane + k * LDX] = w0[Lo.W_L + (NU + lane) + (NU + k) * NZ];
            }
            double v = (lane < NX) ? -w0[Lo.W_pv + lane] : 0.0;
            double di = (lane < NX) ? w0[Lo.W_dinv + NU + lane] : 0.0;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < NX; ++j) {
                double y = bcast(v, j) * bcast(di, j);
                if (lane == j) v = y;
                else if (lane > j && lane < NX) v -= s.Lx[0][lane + j * LDX] * y;
            }
#pragma unroll
            for (int j = NX - 1; j >= 0; --j) {
                double x = bcast(v, j) * bcast(di, j);
                if (lane == j) v = x;
                else if (lane < j) v -= s.Lx[0][j + lane * LDX] * x;
            }
            if (lane < NX) s.xn[0][lane] = v;
            if (lane < NX) w0[opi + lane] = 0.0;
            __syncthreads();
        }
        for (int n = 0; n <= N; ++n) {
            const int cur = n & 1, nxt = (n + 1) & 1;
            const double* d = Dp(n);
            double* ir = Ip(n);
            double* w = Wp(n);
            // factor columns 0..NU-1 of stage n into s.M (column-major)
#pragma unroll
            for (int e0 = 0; e0 < NZ * NU; e0 += WAVE) {
                int e = e0 + lane;
                if (e < NZ * NU) {
                    int i = e % NZ, j = e / NZ;
                    s.M[i + j * LDZ] = w[Lo.W_L + i + j * NZ];
                }
            }
            if (lane < NU) s.t0[lane] = w[Lo.W_dinv + lane];
            if (n < N) {
                double* w1 = Wp(n + 1);
                load_mat<NX, NZ, LDX>(s.F, d + Lo.D_F);
                if (lane < NX) {
#pragma unroll
                    for (int k = 0; k < NX; ++k)
                        s.Lx[nxt][lane + k * LDX] = w1[Lo.W_L + (NU + lane) + (NU + k) * NZ];
                    s.pn[nxt][lane] = w1[Lo.W_pv + lane];
                }
            }
            if constexpr (NG > 0) load_mat<NG, NZ, LDG>(s.G, d + Lo.D_G);
            __syncthreads();
            // v = y_u + L_xu' dx ; back-substitution with L_uu'
            double v = 0.0;
            if (lane < NU) {
                double acc = w[Lo.W_yu + lane];
#pragma unroll
                for (int i = 0; i < NX; ++i) acc += s.M[(NU + i) + lane * LDZ] * s.xn[cur][i];
                v = acc;
            }
            const double dv = (lane < NU) ? s.t0[lane] : 0.0;
#pragma unroll
            for (int j = NU - 1; j >= 0; --j) {
                double x = bcast(v, j) * bcast(dv, j);
                if (lane == j) v = x;
                else if (lane < j) v -= s.M[j + lane * LDZ] * x;
            }
            // dz = [-w; dx]
            double dzj = 0.0;
            if (lane < NU) dzj = -v;
            else if (lane < NZ) dzj = s.xn[cur][lane - NU];
            if (lane < NZ) {
                s.z[lane] = dzj;
                w[oz + lane] = dzj;
            }
            __syncthreads();
            if (n < N) {
                // dx_{n+1} = F dz + rb
                double* w1 = Wp(n + 1);
                const double* Lx = s.Lx[nxt];
                if (lane < NX) {
                    double acc = w[ob + lane];
#pragma unroll
                    for (int k = 0; k < NZ; ++k) acc += s.F[lane + k * LDX] * s.z[k];
                    s.xn[nxt][lane] = acc;
                }
                __syncthreads();
                if (lane < NX) {
                    double acc = 0.0;
#pragma unroll
                    for (int l = 0; l < NX; ++l) acc += Lx[l + lane * LDX] * s.xn[nxt][l];
                    s.t1[lane] = acc;
                }
                __syncthreads();
                if (lane < NX) {
                    double acc = s.pn[nxt][lane];
#pragma unroll
                    for (int l = 0; l < NX; ++l) acc += Lx[lane + l * LDX] * s.t1[l];
                    w1[opi + lane] = acc;
                }
            }
            // constraint steps
            for (int c = lane; c < NC; c += WAVE) {
                double dll = 0.0, dlu = 0.0, dtl = 0.0, dtu = 0.0;
                if (slot_mask(d, c) != 0.0) {
                    double gdz;
                    if (c < NZ) {
                        gdz = s.z[c];
                    } else {
                        const int r = c - NZ;
                        gdz = 0.0;
#pragma unroll
                        for (int k = 0; k < NZ; ++k) gdz += s.G[r + k * LDG] * s.z[k];
                    }
                    double rml, rmu;
                    rm_of(rmode, shift, ir, w, c, rml, rmu);
                    const double ll = ir[Lo.I_ll + c], lu = ir[Lo.I_lu + c];
                    const double tl = ir[Lo.I_tl + c], tu = ir[Lo.I_tu + c];
                    dtl = gdz - w[odl + c];
                    dtu = -gdz - w[odu + c];
                    dll = -(rml + ll * dtl) / tl;
                    dlu = -(rmu + lu * dtu) / tu;
                    if (dll < 0.0) amin = fmin(amin, -ll / dll);
                    if (dlu < 0.0) amin = fmin(amin, -lu / dlu);
                    if (dtl < 0.0) amin = fmin(amin, -tl / dtl);
                    if (dtu < 0.0) amin = fmin(amin, -tu / dtu);
                }
                w[oll + c] = dll;
                w[olu + c] = dlu;
                w[otl + c] = dtl;
                w[otu + c] = dtu;
            }
            __syncthreads();
        }
        return wave_min(amin);
    }

    // mean complementarity after a step of length alpha along (oll, olu, otl, otu)
    __device__ __forceinline__ double mu_after(double alpha, int oll, int olu, int otl, int otu) const
    {
        Smem& s = S();
        (void)s;
        double acc = 0.0;
        for (int n = 0; n <= N; ++n) {
            const double* d = Dp(n);
            const double* ir = Ip(n);
            const double* w = Wp(n);
            for (int c = lane; c < NC; c += WAVE) {
                if (slot_mask(d, c) != 0.0) {
                    acc += (ir[Lo.I_ll + c] + alpha * w[oll + c]) * (ir[Lo.I_tl + c] + alpha * w[otl + c]);
                    acc += (ir[Lo.I_lu + c] + alpha * w[olu + c]) * (ir[Lo.I_tu + c] + alpha * w[otu + c]);
                }
            }
        }
        return wave_sum(acc) / (2.0 * nc);
    }

    __device__ __forceinline__ void update(double alpha)
    {
        Smem& s = S();
        (void)s;
        for (int n = 0; n <= N; ++n) {
            const double* d = Dp(n);
            double* ir = Ip(n);
            const double* w = Wp(n);
            if (lane < NZ) ir[Lo.I_z + lane] += alpha * w[Lo.W_dz + lane];
            if (n > 0 && lane < NX) ir[Lo.I_pi + lane] += alpha * w[Lo.W_dpi + lane];
            for (int c = lane; c < NC; c += WAVE) {
                if (slot_mask(d, c) != 0.0) {
                    ir[Lo.I_ll + c] = fmax(ir[Lo.I_ll + c] + alpha * w[Lo.W_dll + c], P.lam_min);
                    ir[Lo.I_lu + c] = fmax(ir[Lo.I_lu + c] + alpha * w[Lo.W_dlu + c], P.lam_min);
                    ir[Lo.I_tl + c] = fmax(ir[Lo.I_tl + c] + alpha * w[Lo.W_dtl + c], P.t_min);
                    ir[Lo.I_tu + c] = fmax(ir[Lo.I_tu + c] + alpha * w[Lo.W_dtu + c], P.t_min);
                }
            }
        }
        __syncthreads();
    }

    // cold start: y = 0, pi = 0, t = max(C y - d, 1), lam = 1 (masked slots 0)
    __device__ __forceinline__ void init()
    {
        Smem& s = S();
        (void)s;
        for (int n = 0; n <= N; ++n) {
            const double* d = Dp(n);
            double* ir = Ip(n);
            if (lane < NZ) ir[Lo.I_z + lane] = 0.0;
            if (lane < NX) ir[Lo.I_pi + lane] = 0.0;
            for (int c = lane; c < NC; c += WAVE) {
                double m, lo, hi;
                if (c < NZ) {
                    m = d[Lo.D_bm + c]; lo = d[Lo.D_blo + c]; hi = d[Lo.D_bhi + c];
                } else {
                    m = d[Lo.D_gm + c - NZ]; lo = d[Lo.D_glo + c - NZ]; hi = d[Lo.D_ghi + c - NZ];
                }
                const bool on = m != 0.0;
                ir[Lo.I_ll + c] = on ? 1.0 : 0.0;
                ir[Lo.I_lu + c] = on ? 1.0 : 0.0;
                ir[Lo.I_tl + c] = on ? fmax(-lo, 1.0) : 0.0;
                ir[Lo.I_tu + c] = on ? fmax(hi, 1.0) : 0.0;
            }
        }
        __syncthreads();
    }

    __device__ __forceinline__ void copy_step_out(double* out) const
    {
        Smem& s = S();
        (void)s;
        for (int n = 0; n <= N; ++n) {
            double* o = out + (size_t)n * Lo.IREC;
            const double* w = Wp(n);
            if (lane < NZ) o[Lo.I_z + lane] = w[Lo.W_dz + lane];
            if (lane < NX) o[Lo.I_pi + lane] = w[Lo.W_dpi + lane];
            for (int c = lane; c < NC; c += WAVE) {
                o[Lo.I_ll + c] = w[Lo.W_dll + c];
                o[Lo.I_lu + c] = w[Lo.W_dlu + c];
                o[Lo.I_tl + c] = w[Lo.W_dtl + c];
                o[Lo.I_tu + c] = w[Lo.W_dtu + c];
            }
        }
    }

    // ------------------------------------------------------------------
    __device__ __forceinline__ void solve(DevStat* st)
    {
        Smem& s = S();
        (void)s;
        init();
        int status = ST_MAX_ITER, k = 0;
        double ng = 0, nb = 0, nd = 0, nm = 0, mu = 0.0;
        const double inv2nc = nc > 0 ? 1.0 / (2.0 * nc) : 0.0;
        for (k = 0;; ++k) {
            double slt;
            backward_factor(0.0, true, ng, nb, nd, nm, slt);
            mu = slt * inv2nc;
            if (ng != ng || nb != nb || nd != nd || nm != nm || mu != mu) { status = ST_NAN; break; }
            if (ng <= P.tol_stat && nb <= P.tol_eq && nd <= P.tol_ineq && nm <= P.tol_comp) {
                status = ST_SUCCESS;
                break;
            }
            if (k >= P.iter_max) { status = ST_MAX_ITER; break; }
            // predictor: dlam/dt into the affine slots, dz/dpi into the step slots
            double amax = forward(RM_SHIFT, 0.0, Lo.W_rdl, Lo.W_rdu, Lo.W_rb, Lo.W_dz, Lo.W_dpi, Lo.W_all, Lo.W_alu,
                                  Lo.W_atl, Lo.W_atu);
            int oll = Lo.W_all, olu = Lo.W_alu, otl = Lo.W_atl, otu = Lo.W_atu;
            if (nc > 0) {
                const double a_aff = fmin(amax, 1.0);
                const double mu_aff = mu_after(a_aff, Lo.W_all, Lo.W_alu, Lo.W_atl, Lo.W_atu);
                const double ratio = mu > 0.0 ? mu_aff / mu : 0.0;
                const double smu = ratio * ratio * ratio * mu;
                backward_vec(RM_CORRECTOR, smu, Lo.W_rg, Lo.W_rb, Lo.W_rdl, Lo.W_rdu);
                amax = forward(RM_CORRECTOR, smu, Lo.W_rdl, Lo.W_rdu, Lo.W_rb, Lo.W_dz, Lo.W_dpi, Lo.W_dll,
                               Lo.W_dlu, Lo.W_dtl, Lo.W_dtu);
                const double mu_c = mu_after(fmin(amax, 1.0), Lo.W_dll, Lo.W_dlu, Lo.W_dtl, Lo.W_dtu);
                if (mu_c > P.corr_ratio * mu_aff) {
                    backward_vec(RM_SHIFT, smu, Lo.W_rg, Lo.W_rb, Lo.W_rdl, Lo.W_rdu);
                    amax = forward(RM_SHIFT, smu, Lo.W_rdl, Lo.W_rdu, Lo.W_rb, Lo.W_dz, Lo.W_dpi, Lo.W_dll, Lo.W_dlu,
                                   Lo.W_dtl, Lo.W_dtu);
                }
                oll = Lo.W_dll; olu = Lo.W_dlu; otl = Lo.W_dtl; otu = Lo.W_dtu;
            }
            (void)oll; (void)olu; (void)otl; (void)otu;
            const double alpha = fmin(1.0, P.gamma * amax);
            update(alpha);
            if (alpha < P.alpha_min) {
                double slt2;
                backward_factor(0.0, false, ng, nb, nd, nm, slt2);
                mu = slt2 * inv2nc;
                status = ST_MIN_STEP;
                ++k;
                break;
            }
        }
        if (lane == 0) {
            st->status = status;
            st->iters = k;
            st->ir_steps = 0;
            st->mu = mu;
            st->res[0] = ng; st->res[1] = nb; st->res[2] = nd; st->res[3] = nm;
        }
    }

    __device__ __forceinline__ void newton(DevStat* st, double* step_out)
    {
        Smem& s = S();
        (void)s;
        double ng, nb, nd, nm, slt;
        backward_factor(P.tau, true, ng, nb, nd, nm, slt);
        forward(RM_SHIFT, P.tau, Lo.W_rdl, Lo.W_rdu, Lo.W_rb, Lo.W_dz, Lo.W_dpi, Lo.W_dll, Lo.W_dlu, Lo.W_dtl,
                Lo.W_dtu);
        __syncthreads();
        copy_step_out(step_out);
        if (lane == 0) {
            st->status = ST_SUCCESS;
            st->iters = 0;
            st->ir_steps = 0;
            st->mu = nc > 0 ? slt / (2.0 * nc) : 0.0;
            st->res[0] = ng; st->res[1] = nb; st->res[2] = nd; st->res[3] = nm;
        }
    }
};

template <int NX, int NU, int NG>
__global__ __launch_bounds__(WAVE) void ipm_kernel(const InstDesc* __restrict__ desc, int count,
                                                    const double* __restrict__ data, double* __restrict__ iter,
                                                    double* __restrict__ work, double* __restrict__ step_out,
                                                    DevStat* __restrict__ stat, KParams P)
{
    using S = Ipm<NX, NU, NG>;
    const int b = blockIdx.x;
    if (b >= count) return;
    const InstDesc ds = desc[b];
    S ipm(data + ds.data, iter + ds.iter, work + ds.work, ds.N, ds.nc, P);
    if (P.mode == KMODE_NEWTON)
        ipm.newton(stat + ds.index, step_out + ds.iter);
    else
        ipm.solve(stat + ds.index);
}

// ---------------------------------------------------------------------------
// Variant table
// ---------------------------------------------------------------------------

typedef void (*launch_fn)(const InstDesc*, int, const double*, double*, double*, double*, DevStat*, KParams,
                          hipStream_t);

template <int NX, int NU, int NG>
static void launch(const InstDesc* desc, int count, const double* data, double* iter, double* work, double* step,
                   DevStat* stat, KParams P, hipStream_t stream)
{
    hipLaunchKernelGGL((ipm_kernel<NX, NU, NG>), dim3(count), dim3(WAVE), 0, stream, desc, count, data, iter, work,
                       step, stat, P);
}

struct Variant {
    int NX, NU, NG;
    launch_fn fn;
};

#define OQP_VARIANT(x, u, g) {x, u, g, &launch<x, u, g>}
static const Variant kVariants[] = {
    OQP_VARIANT(4, 4, 0),  OQP_VARIANT(4, 4, 4),  OQP_VARIANT(8, 4, 0),  OQP_VARIANT(8, 8, 0),
    OQP_VARIANT(16, 8, 0), OQP_VARIANT(16, 16, 0), OQP_VARIANT(24, 8, 0), OQP_VARIANT(32, 16, 0),
};
#undef OQP_VARIANT

}  // namespace oqp

// Host-side access to the variant table (used by the C-ABI implementation).
namespace oqp {
int variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
void variant_dims(int v, int* nx, int* nu, int* ng)
{
    *nx = kVariants[v].NX;
    *nu = kVariants[v].NU;
    *ng = kVariants[v].NG;
}
int variant_launch(int v, const InstDesc* desc, int count, const double* data, double* iter, double* work,
                   double* step, DevStat* stat, const KParams& P, void* stream)
{
    if (count <= 0) return 0;
    kVariants[v].fn(desc, count, data, iter, work, step, stat, P, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}
}  // namespace oqp
