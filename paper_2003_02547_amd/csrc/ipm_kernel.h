// Batched OCP-QP primal-dual interior-point method on gfx950.
//
// One 64-lane workgroup (one wave) solves one instance end to end: the whole
// IPM loop runs inside the launch.  Stage blocks are compile-time sized
// (NX, NU, NG) and staged through LDS; each sweep streams its stage records
// from HBM one stage ahead (register prefetch), so the global-memory latency
// of the next stage overlaps the arithmetic of the current one.
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
//
// Passes per IPM iteration: A (backward: apply the previous step, residuals,
// barrier terms, factorization, predictor right-hand side), B (forward:
// predictor step, step length, affine duality measure), C (backward:
// corrector right-hand side), B again (corrector step); C and B once more
// only when the conditional corrector is rejected.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "dev_common.h"
#include "ipm_launch.h"
#include "layout.h"

namespace oqp {

template <int NX, int NU, int NG, int KM>
struct Ipm {
    static constexpr bool MIXED = KM == KM_MIXED;
    static constexpr bool ABS = KM == KM_ABS;  // absolute formulation (Section 3.2)
    // factorization by an array algorithm (QR) instead of the Cholesky factor
    // of the normal matrix (Section 4.2, mode robust)
    static constexpr bool ROBUST = KM == KM_ROBUST;
    // soft constraints (Section 2.2): slack pairs on the soft layout
    static constexpr bool SOFT = KM == KM_SOFT;
    // Cholesky factors checked each iteration by the refinement residual of
    // the predictor step, the array algorithm when they are not accurate
    // enough (Section 4.2, mode balance)
    static constexpr bool BALANCE = KM == KM_BALANCE;
    // FP64 refinement of the prediction-centering-correction direction
    // (mixed path; modes balance and robust, Section 4.2; the FP64 build when
    // asked for by a positive ir_max, Section 3.4)
    static constexpr bool REFINE = MIXED || ROBUST || BALANCE || KM == KM_F64;
    // arithmetic type of the factorization and of the right-hand-side sweeps
    // (FP32 in the mixed path; pivots, residuals and refinement stay FP64)
    using TS = typename std::conditional<MIXED, float, double>::type;
    static constexpr Layout Lo = make_layout(NX, NU, NG, SOFT);
    static constexpr int NZ = NX + NU;
    static constexpr int NC = NZ + NG;
    static constexpr int NV = NX + NG;
    static constexpr int NZP = ru8(NZ);
    static constexpr int NXP = ru8(NX);
    static constexpr int NVP = ru8(NV);
    static constexpr int LDZ = NZP + 1;
    static constexpr int LDX = NXP + 1;
    static constexpr int LDV = NVP + 1;
    static constexpr int LDG = NG > 0 ? (NG | 1) : 1;
    static constexpr int NCT = cdiv(NC, WAVE);                   // constraint slots per lane
    static constexpr int EH = cdiv(NZ * NZ, WAVE);               // H elements per lane
    static constexpr int EF = cdiv(NX * NZ, WAVE);               // F elements per lane
    static constexpr int EG = NG > 0 ? cdiv(NG * NZ, WAVE) : 1;
    static constexpr int EL = NU > 0 ? cdiv(NZ * NU, WAVE) : 1;  // factor u-columns per lane
    static constexpr int EX = cdiv(NX * NX, WAVE);               // factor (x, x) block per lane
    static constexpr int NU1 = NU > 0 ? NU : 1;
    // Stage matrices go through registers (prefetched one stage ahead) only
    // for small stage blocks; larger ones are loaded into LDS at stage start.
    static constexpr bool PM = NZ <= 32;
    static constexpr int EHr = PM ? EH : 1, EFr = PM ? EF : 1, EGr = PM ? EG : 1, EXr = PM ? EX : 1;
    static constexpr int TZ = NZP / 8;                           // register tile extents
    static constexpr int TX = NXP / 8;
    static_assert(NZ <= WAVE && NG <= WAVE, "stage block must fit one wave");
    static_assert(NV < WAVE, "reflector broadcast buffer");

    struct Smem {
        // vectors read with wave-uniform addresses first: their offsets fit
        // the short offset fields of paired LDS reads
        alignas(16) double col[2 * WAVE];  // Cholesky column pair (interleaved) / reflector broadcast
        double z[WAVE];           // z_n or dz_n
        double t1[WAVE], t2[WAVE];
        double rb[WAVE];          // r_b of the stage
        double xn[2][NXP];        // x_{n+1} / dx_{n+1}, by parity
        double pin[2][NXP];       // pi_{n+1}, by parity
        double pn[2][NXP];        // p_{n+1}, by parity
        double e[NCT * WAVE];     // reduced-gradient terms per constraint slot
        double ws[NCT * WAVE];    // barrier weights per constraint slot
        double M[LDZ * NZP];      // stage matrix / factor (column-major)
        double Lx[2][LDX * NXP];  // L_{n+1} (lower, zero strict upper), by stage parity
        double F[LDX * NZP];      // [B A] of the stage
        double V[LDV * NZP];      // [U; sqrt(w) G]
        double G[LDG * NZP];      // general rows of the stage
    };

    const double* __restrict__ dat;
    double* __restrict__ itr;
    double* __restrict__ wk;
    int N, nc, lane;
    const KParams& P;

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

    __device__ __forceinline__ int slot(int t) const { return lane + WAVE * t; }

    // per-lane loads of an R x C column-major block (element e = lane + 64 t);
    // with PM off only the source is remembered and commit reads it directly
    template <int R, int C, int E>
    __device__ __forceinline__ void fetch(double (&r)[E], const double* __restrict__ src, const double*& keep) const
    {
        keep = src;
        if constexpr (PM) {
#pragma unroll
            for (int t = 0; t < E; ++t) {
                const int e = lane + WAVE * t;
                r[t] = (e < R * C) ? src[e] : 0.0;
            }
        }
    }
    template <int R, int C, int E>
    __device__ __forceinline__ void commit(double* dst, int ld, const double (&r)[E], const double* src) const
    {
        if constexpr (PM) {
#pragma unroll
            for (int t = 0; t < E; ++t) {
                const int e = lane + WAVE * t;
                if (e < R * C) dst[(e % R) + (e / R) * ld] = r[t];
            }
        } else {
#pragma unroll 4
            for (int e = lane; e < R * C; e += WAVE) dst[(e % R) + (e / R) * ld] = src[e];
        }
    }
    // small blocks that always go through registers
    template <int R, int C, int E>
    __device__ __forceinline__ void fetch_r(double (&r)[E], const double* __restrict__ src) const
    {
#pragma unroll
        for (int t = 0; t < E; ++t) {
            const int e = lane + WAVE * t;
            r[t] = (e < R * C) ? src[e] : 0.0;
        }
    }
    template <int R, int C, int E>
    __device__ __forceinline__ void commit_r(double* dst, int ld, const double (&r)[E]) const
    {
#pragma unroll
        for (int t = 0; t < E; ++t) {
            const int e = lane + WAVE * t;
            if (e < R * C) dst[(e % R) + (e / R) * ld] = r[t];
        }
    }
    // (x, x) block of a stage factor (rows/cols NU.., column-major NZ x NZ)
    // into an NX x NX LDS block, optionally with the strict upper part zeroed
    __device__ __forceinline__ void fetch_lxx(double (&r)[EXr], const double* __restrict__ wl, const double*& keep) const
    {
        keep = wl;
        if constexpr (PM) {
#pragma unroll
            for (int t = 0; t < EX; ++t) {
                const int e = lane + WAVE * t;
                r[t] = (e < NX * NX) ? wl[(NU + e % NX) + (NU + e / NX) * NZ] : 0.0;
            }
        }
    }
    __device__ __forceinline__ void commit_lxx(double* dst, const double (&r)[EXr], const double* wl, bool lower) const
    {
        if constexpr (PM) {
#pragma unroll
            for (int t = 0; t < EX; ++t) {
                const int e = lane + WAVE * t;
                if (e < NX * NX) {
                    const int i = e % NX, k = e / NX;
                    dst[i + k * LDX] = (!lower || k <= i) ? r[t] : 0.0;
                }
            }
        } else {
#pragma unroll 4
            for (int e = lane; e < NX * NX; e += WAVE) {
                const int i = e % NX, k = e / NX;
                dst[i + k * LDX] = (!lower || k <= i) ? wl[(NU + i) + (NU + k) * NZ] : 0.0;
            }
        }
    }

    // constraint slot data: mask, lower, upper
    __device__ __forceinline__ void slot_bounds(const double* d, int c, double& m, double& lo, double& hi) const
    {
        if (c < NZ) {
            m = d[Lo.D_bm + c];
            lo = d[Lo.D_blo + c];
            hi = d[Lo.D_bhi + c];
        } else if (c < NC) {
            m = d[Lo.D_gm + (c - NZ)];
            lo = d[Lo.D_glo + (c - NZ)];
            hi = d[Lo.D_ghi + (c - NZ)];
        } else {
            m = 0.0;
            lo = 0.0;
            hi = 0.0;
        }
    }

    // ------------------------------------------------------------------
    // Soft constraints (soft build).  A soft slot holds a slack pair
    // (s^l, s^u): the lower row reads G z + s^l, the upper row -G z + s^u,
    // each with a bound row s >= ls (multiplier lam_s, slack t_s).  The pair
    // is eliminated from the Newton system per slot: with D = Z + w + w_s and
    // g_s = r_s - e - e_s (e_s = (lam_s rd_s - rm_s) / t_s), the slot enters
    // the Riccati recursion with weight w (Z + w_s) / D and term e + w g_s /
    // D, and pass B recovers ds^l = -(g_s^l + w_l G dz) / D_l, ds^u =
    // -(g_s^u - w_u G dz) / D_u.  The slot values travel in the prefetch
    // records of the passes like the rows' (NCS = 1 placeholder otherwise).
    // ------------------------------------------------------------------
    static constexpr int NCS = SOFT ? NCT : 1;
    struct SoftA {  // pass A: data, iterate and last step of a slot
        double sm, Zl, Zu, zl, zu, lls, lus, sl, su, lsl, lsu, tsl, tsu, dsl, dsu, dlsl, dlsu, dtsl, dtsu;
    };
    struct SoftOutA {  // pass A outputs: updated iterate and slack residuals
        double sm, sl, su, lsl, lsu, tsl, tsu, rsl, rsu, rdsl, rdsu;
    };
    struct SoftR {  // passes B, C: what the elimination of a right-hand side reads
        double sm, Zl, Zu, lsl, lsu, tsl, tsu, rsl, rsu, rdsl, rdsu, alsl, alsu, atsl, atsu;
    };
    struct SoftOutB {  // pass B outputs: slack steps and bound-row steps
        double sm, dsl, dsu, dlsl, dlsu, dtsl, dtsu;
    };

    __device__ __forceinline__ void load_softA(SoftA& q, const double* d, const double* ir, const double* w, int c,
                                               bool upd) const
    {
        q = SoftA{};
        if (c >= NC) return;
        q.sm = d[Lo.D_sm + c];
        if (q.sm == 0.0) return;
        q.Zl = d[Lo.D_Zl + c];
        q.Zu = d[Lo.D_Zu + c];
        q.zl = d[Lo.D_zl + c];
        q.zu = d[Lo.D_zu + c];
        q.lls = d[Lo.D_lls + c];
        q.lus = d[Lo.D_lus + c];
        q.sl = ir[Lo.I_sl + c];
        q.su = ir[Lo.I_su + c];
        q.lsl = ir[Lo.I_lsl + c];
        q.lsu = ir[Lo.I_lsu + c];
        q.tsl = ir[Lo.I_tsl + c];
        q.tsu = ir[Lo.I_tsu + c];
        if (upd) {
            q.dsl = w[Lo.W_dsl + c];
            q.dsu = w[Lo.W_dsu + c];
            q.dlsl = w[Lo.W_dlsl + c];
            q.dlsu = w[Lo.W_dlsu + c];
            q.dtsl = w[Lo.W_dtsl + c];
            q.dtsu = w[Lo.W_dtsu + c];
        }
    }

    __device__ __forceinline__ void load_softR(SoftR& q, int rmode, const double* d, const double* ir,
                                               const double* w, int c) const
    {
        q = SoftR{};
        if (c >= NC) return;
        q.sm = d[Lo.D_sm + c];
        if (q.sm == 0.0) return;
        q.Zl = d[Lo.D_Zl + c];
        q.Zu = d[Lo.D_Zu + c];
        q.lsl = ir[Lo.I_lsl + c];
        q.lsu = ir[Lo.I_lsu + c];
        q.tsl = ir[Lo.I_tsl + c];
        q.tsu = ir[Lo.I_tsu + c];
        q.rsl = w[Lo.W_rsl + c];
        q.rsu = w[Lo.W_rsu + c];
        q.rdsl = w[Lo.W_rdsl + c];
        q.rdsu = w[Lo.W_rdsu + c];
        if (rmode == RM_CORRECTOR) {
            q.alsl = w[Lo.W_alsl + c];
            q.alsu = w[Lo.W_alsu + c];
            q.atsl = w[Lo.W_atsl + c];
            q.atsu = w[Lo.W_atsu + c];
        }
    }

    // Elimination of a soft slot for a right-hand side: turns the row terms
    // el, eu into el + wl g_l / D_l, eu + wu g_u / D_u and returns D, g_s
    // and the bound rows' r_m (per rmode, as rm_value for the rows).
    __device__ __forceinline__ void soft_rhs(const SoftR& q, int rmode, double shift, double wl, double wu,
                                             double& el, double& eu, double& Dl, double& gl, double& Du,
                                             double& gu, double& rmsl, double& rmsu) const
    {
        rmsl = q.lsl * q.tsl - shift;
        rmsu = q.lsu * q.tsu - shift;
        if (rmode == RM_CORRECTOR) {
            rmsl += q.alsl * q.atsl;
            rmsu += q.alsu * q.atsu;
        }
        const double itsl = rcp_nr(q.tsl), itsu = rcp_nr(q.tsu);
        const double esl = (q.lsl * q.rdsl - rmsl) * itsl;
        const double esu = (q.lsu * q.rdsu - rmsu) * itsu;
        Dl = q.Zl + wl + q.lsl * itsl;
        Du = q.Zu + wu + q.lsu * itsu;
        gl = q.rsl - el - esl;
        gu = q.rsu - eu - esu;
        el += wl * gl * rcp_nr(Dl);
        eu += wu * gu * rcp_nr(Du);
    }

    // ------------------------------------------------------------------
    // Register-blocked products on LDS blocks (lanes as an 8 x 8 grid)
    // ------------------------------------------------------------------

    // V[i][k] = sum_l L[l][i] F[l][k], i < NX, k < NZP (L lower, zero strict upper)
    __device__ __forceinline__ void trmm_LtF(const double* __restrict__ Lx) const
    {
        Smem& s = S();
        const int a = lane & 7, b = lane >> 3;
        TS acc[TX][TZ];
#pragma unroll
        for (int p = 0; p < TX; ++p)
#pragma unroll
            for (int q = 0; q < TZ; ++q) acc[p][q] = 0;
#pragma unroll 4
        for (int l = 0; l < NX; ++l) {
            TS lv[TX], fv[TZ];
#pragma unroll
            for (int p = 0; p < TX; ++p) lv[p] = (TS)Lx[l + (a + 8 * p) * LDX];
#pragma unroll
            for (int q = 0; q < TZ; ++q) fv[q] = (TS)s.F[l + (b + 8 * q) * LDX];
#pragma unroll
            for (int p = 0; p < TX; ++p)
#pragma unroll
                for (int q = 0; q < TZ; ++q) acc[p][q] += lv[p] * fv[q];
        }
#pragma unroll
        for (int p = 0; p < TX; ++p)
#pragma unroll
            for (int q = 0; q < TZ; ++q)
                if (a + 8 * p < NX) s.V[(a + 8 * p) + (b + 8 * q) * LDV] = (double)acc[p][q];
    }

    // M[i][k] += sum_{r0 <= r < NV} V[r][i] V[r][k] for i, k < NZP
    __device__ __forceinline__ void syrk_VtV(int r0) const
    {
        Smem& s = S();
        const int a = lane & 7, b = lane >> 3;
        TS acc[TZ][TZ];
#pragma unroll
        for (int p = 0; p < TZ; ++p)
#pragma unroll
            for (int q = 0; q < TZ; ++q) acc[p][q] = 0;
#pragma unroll 4
        for (int r = r0; r < NV; ++r) {
            TS vi[TZ], vk[TZ];
#pragma unroll
            for (int p = 0; p < TZ; ++p) vi[p] = (TS)s.V[r + (a + 8 * p) * LDV];
#pragma unroll
            for (int q = 0; q < TZ; ++q) vk[q] = (TS)s.V[r + (b + 8 * q) * LDV];
#pragma unroll
            for (int p = 0; p < TZ; ++p)
#pragma unroll
                for (int q = 0; q < TZ; ++q) acc[p][q] += vi[p] * vk[q];
        }
#pragma unroll
        for (int p = 0; p < TZ; ++p)
#pragma unroll
            for (int q = 0; q < TZ; ++q) s.M[(a + 8 * p) + (b + 8 * q) * LDZ] += (double)acc[p][q];
    }

    // ------------------------------------------------------------------
    // Right-looking Cholesky of s.M (NZ x NZ), one row per lane, rows held in
    // registers.  On return lane i < NZ holds row i of L in r[0..i] and 1/L_ii.
    // ------------------------------------------------------------------
    // rounding to the sweep type
    __device__ __forceinline__ static double rnd(double x) { return (double)(TS)x; }

    // Returns false when a pivot is not positive (or NaN).
    __device__ __forceinline__ bool cholesky(double (&r)[NZ], double& dinv) const
    {
        Smem& s = S();
        // lanes past the block repeat its last row (no predicated loads; their
        // values are never read)
#pragma unroll
        for (int k = 0; k < NZ; ++k) r[k] = s.M[(lane < NZ ? lane : NZ - 1) + k * LDZ];
        dinv = 0.0;
        // Mixed path: off-diagonal entries and their updates in FP32, the
        // diagonal of every row accumulated in FP64 (FP64 pivots).
        double dd = 0.0;
        if constexpr (MIXED) {
            dd = lane < NZ ? s.M[lane + lane * LDZ] : 1.0;
#pragma unroll
            for (int k = 0; k < NZ; ++k) r[k] = rnd(r[k]);
        }
        bool ok = true;
        // Updates are not masked: lane i only ever needs r[k] for k <= i, and
        // the entries above the diagonal absorb harmless garbage.  Columns are
        // taken two at a time: column j + 1 is factored as soon as column j
        // has updated it, and the rest of the trailing block receives both
        // columns' updates in column order (the same operations as one column
        // at a time), with one LDS exchange of the pair.
#pragma unroll
        for (int j = 0; j < NZ; j += 2) {
            double piv = MIXED ? bcast(dd, j) : bcast(r[j], j);
            ok = ok && (piv > 0.0);
            double inv = rsqrt_nr(piv);
            const double l0 = MIXED ? rnd(r[j] * inv) : r[j] * inv;
            if (lane == j) {
                dinv = inv;
                r[j] = piv * inv;  // sqrt(pivot)
            } else if (lane > j) {
                r[j] = l0;
                if constexpr (MIXED) dd -= l0 * l0;
            }
            if (j + 1 == NZ) break;
            // the entries needed by the next columns go through the scalar
            // unit (critical path), the rest through LDS
            r[j + 1] = (double)((TS)r[j + 1] - (TS)l0 * (TS)bcast(l0, j + 1));
            piv = MIXED ? bcast(dd, j + 1) : bcast(r[j + 1], j + 1);
            ok = ok && (piv > 0.0);
            inv = rsqrt_nr(piv);
            const double l1 = MIXED ? rnd(r[j + 1] * inv) : r[j + 1] * inv;
            if (lane == j + 1) {
                dinv = inv;
                r[j + 1] = piv * inv;
            } else if (lane > j + 1) {
                r[j + 1] = l1;
                if constexpr (MIXED) dd -= l1 * l1;
            }
            if (j + 2 < NZ) {
                s.col[2 * lane] = l0;
                s.col[2 * lane + 1] = l1;
                r[j + 2] = (double)((TS)r[j + 2] - (TS)l0 * (TS)bcast(l0, j + 2));
                r[j + 2] = (double)((TS)r[j + 2] - (TS)l1 * (TS)bcast(l1, j + 2));
                wsync();
#pragma unroll
                for (int k = j + 3; k < NZ; ++k) {
                    r[k] = (double)((TS)r[k] - (TS)l0 * (TS)s.col[2 * k]);
                    r[k] = (double)((TS)r[k] - (TS)l1 * (TS)s.col[2 * k + 1]);
                }
                wsync();
            }
        }
        return ok;
    }

    // Array-algorithm factorization (Section 4.2, mode robust): with R_0 the
    // upper Cholesky factor of Phi (R_0' = the factor in rowL) and V = [U;
    // sqrt(w) G] (rows r0.. of s.V), the upper triangular R of the QR
    // decomposition of [R_0; V] satisfies R'R = Phi + V'V = M, so L = R'
    // without forming the normal matrix V'V.  Householder reflections, one
    // per column; lane k holds column k of [R; V]: R(j, k) = rowL[j] (j <= k,
    // the layout of a row of L) and V(:, k) in registers.  Reflector of
    // column j: beta = |[a; x]|, v0 = a - beta (in the cancellation-free form
    // -|x|^2 / (a + beta) for a > 0), u = [1; x / v0], tau = 2 v0^2 / (|x|^2 +
    // v0^2); beta > 0 keeps the diagonal of R positive.  On return rowL, dinv
    // hold the factor of M as the Cholesky routine leaves it.
    __device__ __forceinline__ void qr_update(double (&rowL)[NZ], double& dinv, int r0) const
    {
        Smem& s = S();
        double vr[NV];
#pragma unroll
        for (int r = 0; r < NV; ++r) vr[r] = (lane < NZ && r >= r0) ? s.V[r + lane * LDV] : 0.0;
        wsync();
#pragma unroll
        for (int j = 0; j < NZ; ++j) {
            if (lane == j) {
                const double a = rowL[j];
                double sg = 0.0;
#pragma unroll
                for (int r = 0; r < NV; ++r) sg += vr[r] * vr[r];
                const double beta = sqrt(a * a + sg);
                const double v0 = a <= 0.0 ? a - beta : -sg / (a + beta);
                const double tau = sg == 0.0 ? 0.0 : 2.0 * v0 * v0 / (sg + v0 * v0);
                const double iv0 = sg == 0.0 ? 0.0 : 1.0 / v0;
#pragma unroll
                for (int r = 0; r < NV; ++r) s.col[r] = vr[r] * iv0;
                s.col[NV] = tau;
                rowL[j] = beta;
#pragma unroll
                for (int r = 0; r < NV; ++r) vr[r] = 0.0;
            }
            wsync();
            if (lane > j && lane < NZ) {
                const double tau = s.col[NV];
                double sd = rowL[j];
#pragma unroll
                for (int r = 0; r < NV; ++r) sd += s.col[r] * vr[r];
                const double ts = tau * sd;
                rowL[j] -= ts;
#pragma unroll
                for (int r = 0; r < NV; ++r) vr[r] -= ts * s.col[r];
            }
            wsync();
        }
        dinv = 0.0;
#pragma unroll
        for (int j = 0; j < NZ; ++j)
            if (lane == j) dinv = 1.0 / rowL[j];
    }

    // Forward substitution with the (u, u) block, fused with the x rows:
    // lanes i < NU end with y = L_uu^{-1} m_u, lanes NU <= i < NZ with
    // p = m_x - L_xu y.  rowL[j] = L[i][j] for j < NU; dinv is 1/L_ii (FP64).
    template <int CNT>
    __device__ __forceinline__ double fwd_subst_u(double m, const double (&rowL)[CNT], double dinv) const
    {
        m = rnd(m);
#pragma unroll
        for (int j = 0; j < NU; ++j) {
            const double y = rnd(bcast(m, j) * bcast(dinv, j));
            if (lane == j) m = y;
            else if (lane > j) m = (double)((TS)m - (TS)rowL[j] * (TS)y);
        }
        return m;
    }

    // m += F'(Lx (Lx' rb) + p_{n+1}) with rb in s.rb and Lx = L_{n+1}.
    __device__ __forceinline__ double add_cost_to_go(double m, const double* __restrict__ Lx,
                                                     const double* __restrict__ pnext) const
    {
        Smem& s = S();
        if (lane < NX) {
            TS acc = 0;
#pragma unroll
            for (int l = 0; l < NX; ++l) acc += (TS)Lx[l + lane * LDX] * (TS)s.rb[l];
            s.t1[lane] = (double)acc;
        }
        wsync();
        if (lane < NX) {
            TS acc = (TS)pnext[lane];
#pragma unroll
            for (int l = 0; l < NX; ++l) acc += (TS)Lx[lane + l * LDX] * (TS)s.t1[l];
            s.t2[lane] = (double)acc;
        }
        wsync();
        if (lane < NZ) {
            TS acc = (TS)m;
#pragma unroll
            for (int i = 0; i < NX; ++i) acc += (TS)s.F[i + lane * LDX] * (TS)s.t2[i];
            m = (double)acc;
        }
        return m;
    }

    // ==================================================================
    // Pass A: apply the previous step (optional), residuals at the iterate,
    // barrier terms, factorization, right-hand-side sweep for r_m = lam.*t -
    // shift.  Returns the residual norms and lam't of the (updated) iterate.
    // ==================================================================
    struct PreA {
        double H[EHr], F[EFr], G[EGr];
        const double *sH, *sF, *sG;
        double g, z, dz, b, pi, dpi;
        double m[NCT], lo[NCT], hi[NCT], ll[NCT], lu[NCT], tl[NCT], tu[NCT];
        double dll[NCT], dlu[NCT], dtl[NCT], dtu[NCT];
        SoftA sf[NCS];
    };

    __device__ __forceinline__ void loadA(PreA& p, int n, bool upd) const
    {
        const double* d = Dp(n);
        const double* ir = Ip(n);
        const double* w = Wp(n);
        fetch<NZ, NZ, EHr>(p.H, d + Lo.D_H, p.sH);
        if (n < N) fetch<NX, NZ, EFr>(p.F, d + Lo.D_F, p.sF);
        if constexpr (NG > 0) fetch<NG, NZ, EGr>(p.G, d + Lo.D_G, p.sG);
        p.g = p.z = p.dz = p.b = p.pi = p.dpi = 0.0;
        if (lane < NZ) {
            p.g = d[Lo.D_g + lane];
            p.z = ir[Lo.I_z + lane];
            if (upd) p.dz = w[Lo.W_dz + lane];
        }
        if (lane < NX) {
            if (n < N) p.b = d[Lo.D_b + lane];
            p.pi = ir[Lo.I_pi + lane];
            if (upd) p.dpi = w[Lo.W_dpi + lane];
        }
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
            const int c = slot(t);
            slot_bounds(d, c, p.m[t], p.lo[t], p.hi[t]);
            p.ll[t] = p.lu[t] = p.tl[t] = p.tu[t] = 0.0;
            p.dll[t] = p.dlu[t] = p.dtl[t] = p.dtu[t] = 0.0;
            if (c < NC) {
                p.ll[t] = ir[Lo.I_ll + c];
                p.lu[t] = ir[Lo.I_lu + c];
                p.tl[t] = ir[Lo.I_tl + c];
                p.tu[t] = ir[Lo.I_tu + c];
                if (upd) {
                    p.dll[t] = w[Lo.W_dll + c];
                    p.dlu[t] = w[Lo.W_dlu + c];
                    p.dtl[t] = w[Lo.W_dtl + c];
                    p.dtu[t] = w[Lo.W_dtu + c];
                }
            }
            if constexpr (SOFT) load_softA(p.sf[t], d, ir, w, c, upd);
        }
    }

    // Outputs of one stage of pass A, written to global memory at the top of
    // the next stage (before that stage's prefetch is issued), so that the
    // loop body itself holds no global memory operation: the single wait per
    // stage then covers loads and stores issued a whole stage earlier.
    struct OutA {
        double z, pi, rg, rb, dinv, mv;
        double ll[NCT], lu[NCT], tl[NCT], tu[NCT], rdl[NCT], rdu[NCT], m[NCT];
        SoftOutA so[NCS];
    };

    __device__ __forceinline__ void flushA(int n, bool upd, bool factor, const OutA& o) const
    {
        Smem& s = S();
        double* ir = Ip(n);
        double* w = Wp(n);
        if (upd) {
            if (lane < NZ) ir[Lo.I_z + lane] = o.z;
            if (lane < NX && n > 0) ir[Lo.I_pi + lane] = o.pi;
        }
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
            const int c = slot(t);
            if (c < NC) {
                if (upd && o.m[t] != 0.0) {
                    ir[Lo.I_ll + c] = o.ll[t];
                    ir[Lo.I_lu + c] = o.lu[t];
                    ir[Lo.I_tl + c] = o.tl[t];
                    ir[Lo.I_tu + c] = o.tu[t];
                }
                w[Lo.W_rdl + c] = o.rdl[t];
                w[Lo.W_rdu + c] = o.rdu[t];
                if constexpr (SOFT) {
                    if (o.so[t].sm != 0.0) {
                        if (upd) {
                            ir[Lo.I_sl + c] = o.so[t].sl;
                            ir[Lo.I_su + c] = o.so[t].su;
                            ir[Lo.I_lsl + c] = o.so[t].lsl;
                            ir[Lo.I_lsu + c] = o.so[t].lsu;
                            ir[Lo.I_tsl + c] = o.so[t].tsl;
                            ir[Lo.I_tsu + c] = o.so[t].tsu;
                        }
                        w[Lo.W_rsl + c] = o.so[t].rsl;
                        w[Lo.W_rsu + c] = o.so[t].rsu;
                        w[Lo.W_rdsl + c] = o.so[t].rdsl;
                        w[Lo.W_rdsu + c] = o.so[t].rdsu;
                    }
                }
            }
        }
        if (lane < NZ) w[Lo.W_rg + lane] = o.rg;
        if (n < N && lane < NX) w[Lo.W_rb + lane] = o.rb;
        if (factor) {
            if (lane < NZ) w[Lo.W_dinv + lane] = o.dinv;
            if (lane < NU) w[Lo.W_yu + lane] = o.mv;
            else if (lane < NZ) w[Lo.W_pv + lane - NU] = o.mv;
        }
    }

    // With absf (absolute formulation, Section 3.2) the right-hand side is
    // built from the data alone, -[g; b; d; r_m - 2 Lam T e]: the residual
    // matrix-vector products are skipped and their norms are not formed.
    __device__ __forceinline__ bool passA(bool upd, double alpha, double shift, bool factor, bool absf, bool qr,
                                          double& o_g,
                                          double& o_b, double& o_d, double& o_m, double& o_lt) const
    {
        Smem& s = S();
        double mg = 0.0, mb = 0.0, md = 0.0, mm = 0.0, slt = 0.0;
        bool fact_ok = true;
        PreA p;
        OutA o;
        loadA(p, N, upd);
        for (int n = N; n >= 0; --n) {
            const int cur = n & 1, nxt = cur ^ 1;
            commit<NZ, NZ, EHr>(s.M, LDZ, p.H, p.sH);
            if (n < N) commit<NX, NZ, EFr>(s.F, LDX, p.F, p.sF);
            if constexpr (NG > 0) commit<NG, NZ, EGr>(s.G, LDG, p.G, p.sG);
            const double g = p.g, b = p.b, dz = p.dz, dpi = p.dpi;
            double z = p.z, pi = p.pi;
            double m[NCT], lo[NCT], hi[NCT], ll[NCT], lu[NCT], tl[NCT], tu[NCT];
#pragma unroll
            for (int t = 0; t < NCT; ++t) {
                m[t] = p.m[t];
                lo[t] = p.lo[t];
                hi[t] = p.hi[t];
                ll[t] = p.ll[t];
                lu[t] = p.lu[t];
                tl[t] = p.tl[t];
                tu[t] = p.tu[t];
                if (upd && m[t] != 0.0) {
                    ll[t] = fmax(ll[t] + alpha * p.dll[t], P.lam_min);
                    lu[t] = fmax(lu[t] + alpha * p.dlu[t], P.lam_min);
                    tl[t] = fmax(tl[t] + alpha * p.dtl[t], P.t_min);
                    tu[t] = fmax(tu[t] + alpha * p.dtu[t], P.t_min);
                }
            }
            // slack pairs after the step (clamped like the rows)
            SoftA sa[NCS];
            if constexpr (SOFT) {
#pragma unroll
                for (int t = 0; t < NCT; ++t) {
                    sa[t] = p.sf[t];
                    if (upd && sa[t].sm != 0.0) {
                        sa[t].sl += alpha * sa[t].dsl;
                        sa[t].su += alpha * sa[t].dsu;
                        sa[t].lsl = fmax(sa[t].lsl + alpha * sa[t].dlsl, P.lam_min);
                        sa[t].lsu = fmax(sa[t].lsu + alpha * sa[t].dlsu, P.lam_min);
                        sa[t].tsl = fmax(sa[t].tsl + alpha * sa[t].dtsl, P.t_min);
                        sa[t].tsu = fmax(sa[t].tsu + alpha * sa[t].dtsu, P.t_min);
                    }
                }
            }
            if (n < N) flushA(n + 1, upd, factor, o);  // outputs of the previous stage
            if (n > 0) loadA(p, n - 1, upd);           // prefetch the next stage of the sweep

            if (upd) {
                z += alpha * dz;
                if (n > 0) pi += alpha * dpi;
            }
            if (n == N && lane < NX) {
                s.xn[nxt][lane] = 0.0;
                s.pin[nxt][lane] = 0.0;
                s.pn[nxt][lane] = 0.0;
            }
            if (lane < NZ) s.z[lane] = z;
            if (lane < NX) s.t2[lane] = pi;
            if constexpr (NG > 0) {
#pragma unroll
                for (int t = 0; t < NCT; ++t) {
                    const int c = slot(t);
                    if (c >= NZ && c < NC) s.t1[c - NZ] = m[t] * (ll[t] - lu[t]);
                }
            }
            wsync();

            // r_g = H z + g + F' pi_{n+1} - [0; pi_n] - C' lam
            double rg = 0.0;
            if (absf) {
                if (lane < NZ) rg = g;
            } else if (lane < NZ) {
                const int j = lane;
                double acc = g;
#pragma unroll
                for (int k = 0; k < NZ; ++k) acc += s.M[j + k * LDZ] * s.z[k];
                if (n < N) {
#pragma unroll
                    for (int i = 0; i < NX; ++i) acc += s.F[i + j * LDX] * s.pin[nxt][i];
                }
                if (j >= NU) acc -= s.t2[j - NU];
                acc -= m[0] * (ll[0] - lu[0]);
                if constexpr (NG > 0) {
#pragma unroll
                    for (int r = 0; r < NG; ++r) acc -= s.G[r + j * LDG] * s.t1[r];
                }
                rg = acc;
                mg = nmax(mg, fabs(rg));
            }
            // r_b = F z + b - x_{n+1}
            double rb = 0.0;
            if (absf) {
                if (n < N && lane < NX) rb = b;
            } else if (n < N && lane < NX) {
                double acc = b;
#pragma unroll
                for (int k = 0; k < NZ; ++k) acc += s.F[lane + k * LDX] * s.z[k];
                rb = acc - s.xn[nxt][lane];
                mb = nmax(mb, fabs(rb));
            }
            // r_d, complementarity, barrier weights, reduced-gradient terms
            double e0 = 0.0, ws0 = 0.0;
#pragma unroll
            for (int t = 0; t < NCT; ++t) {
                const int c = slot(t);
                double e = 0.0, wsum = 0.0, rdl = 0.0, rdu = 0.0;
                if constexpr (SOFT) o.so[t] = SoftOutA{};
                if (c < NC) {
                    if (m[t] != 0.0) {
                        if (absf) {
                            rdl = lo[t];
                            rdu = -hi[t];
                        } else {
                            double gz;
                            if (c < NZ) {
                                gz = z;
                            } else {
                                const int r = c - NZ;
                                gz = 0.0;
#pragma unroll
                                for (int k = 0; k < NZ; ++k) gz += s.G[r + k * LDG] * s.z[k];
                            }
                            rdl = -gz + tl[t] + lo[t];
                            rdu = gz + tu[t] - hi[t];
                            if constexpr (SOFT) {
                                // a soft row holds its slack: G z + s^l, -G z + s^u
                                rdl -= sa[t].sl;
                                rdu -= sa[t].su;
                            }
                            md = nmax(md, nmax(fabs(rdl), fabs(rdu)));
                        }
                        const double a1 = ll[t] * tl[t], a2 = lu[t] * tu[t];
                        mm = nmax(mm, nmax(a1, a2));
                        slt += a1 + a2;
                        const double itl = rcp_nr(tl[t]), itu = rcp_nr(tu[t]);
                        const double wl = ll[t] * itl, wu = lu[t] * itu;
                        wsum = wl + wu;
                        // r_m / t, with r_m = lam t - shift (delta) or -lam t - shift (absolute)
                        const double ml = absf ? -ll[t] - shift * itl : ll[t] - shift * itl;
                        const double mu_ = absf ? -lu[t] - shift * itu : lu[t] - shift * itu;
                        e = (wl * rdl - ml) - (wu * rdu - mu_);
                        if constexpr (SOFT) {
                            const SoftA& q = sa[t];
                            SoftOutA& so = o.so[t];
                            if (q.sm != 0.0) {
                                // slack rows: stationarity r_s = Z s + z - lam_row -
                                // lam_s, bound rows rd_s = -s + t_s + ls and their
                                // complementarity; then the elimination
                                so.sm = 1.0;
                                so.rsl = q.Zl * q.sl + q.zl - ll[t] - q.lsl;
                                so.rsu = q.Zu * q.su + q.zu - lu[t] - q.lsu;
                                so.rdsl = -q.sl + q.tsl + q.lls;
                                so.rdsu = -q.su + q.tsu + q.lus;
                                mg = nmax(mg, nmax(fabs(so.rsl), fabs(so.rsu)));
                                md = nmax(md, nmax(fabs(so.rdsl), fabs(so.rdsu)));
                                const double a3 = q.lsl * q.tsl, a4 = q.lsu * q.tsu;
                                mm = nmax(mm, nmax(a3, a4));
                                slt += a3 + a4;
                                const double itsl = rcp_nr(q.tsl), itsu = rcp_nr(q.tsu);
                                const double wsl = q.lsl * itsl, wsu = q.lsu * itsu;
                                const double esl = wsl * so.rdsl - (q.lsl - shift * itsl);
                                const double esu = wsu * so.rdsu - (q.lsu - shift * itsu);
                                const double iDl = rcp_nr(q.Zl + wl + wsl), iDu = rcp_nr(q.Zu + wu + wsu);
                                const double el = wl * rdl - ml, eu = wu * rdu - mu_;
                                const double gl = so.rsl - el - esl, gu = so.rsu - eu - esu;
                                e = (el + wl * gl * iDl) - (eu + wu * gu * iDu);
                                wsum = wl * (q.Zl + wsl) * iDl + wu * (q.Zu + wsu) * iDu;
                                so.sl = q.sl;
                                so.su = q.su;
                                so.lsl = q.lsl;
                                so.lsu = q.lsu;
                                so.tsl = q.tsl;
                                so.tsu = q.tsu;
                            }
                        }
                    }
                    s.e[c] = e;
                    s.ws[c] = wsum;
                }
                o.rdl[t] = rdl;
                o.rdu[t] = rdu;
                o.ll[t] = ll[t];
                o.lu[t] = lu[t];
                o.tl[t] = tl[t];
                o.tu[t] = tu[t];
                o.m[t] = m[t];
                if (t == 0) {
                    e0 = e;
                    ws0 = wsum;
                }
            }
            if (lane < NX) s.rb[lane] = rb;
            o.z = z;
            o.pi = pi;
            o.rg = rg;
            o.rb = rb;

            if (factor) {
                // Phi = H + diag(box weights) + reg I ; V = [L_{n+1}' F ; sqrt(w_g) G]
                if (lane < NZ) s.M[lane + lane * LDZ] += ws0 + P.reg_prim;
                wsync();
                if constexpr (NG > 0) {
#pragma unroll
                    for (int t = 0; t < EG; ++t) {
                        const int e = lane + WAVE * t;
                        if (e < NG * NZ) {
                            const int r = e % NG, k = e / NG;
                            s.V[NX + r + k * LDV] = sqrt(s.ws[NZ + r]) * s.G[r + k * LDG];
                        }
                    }
                }
                if (n < N) trmm_LtF(s.Lx[nxt]);
                wsync();
                // the array algorithm (robust build; balance build when this
                // iteration's Cholesky factors were not accurate enough)
                // factors M = Phi + V'V without forming V'V
                if constexpr (BALANCE) {
                    if (!qr) {
                        if (n < N || NG > 0) syrk_VtV(n < N ? 0 : NX);
                        wsync();
                    }
                } else if constexpr (!ROBUST) {
                    if (n < N || NG > 0) syrk_VtV(n < N ? 0 : NX);
                    wsync();
                }

                double rowL[NZ];
                double dinv;
                fact_ok = cholesky(rowL, dinv) && fact_ok;
                if constexpr (ROBUST) {
                    if (n < N || NG > 0) qr_update(rowL, dinv, n < N ? 0 : NX);
                } else if constexpr (BALANCE) {
                    if (qr && (n < N || NG > 0)) qr_update(rowL, dinv, n < N ? 0 : NX);
                }
                // the factor goes to its record straight from the rows in
                // registers: lane j stores row j, so every column is one
                // coalesced store (no LDS staging: the LDS block of an
                // instance stays small enough for seven instances per CU)
                if (lane < NZ) {
                    double* wl = Wp(n) + Lo.W_L + lane;
#pragma unroll
                    for (int k = 0; k < NZ; ++k) wl[k * NZ] = (k <= lane) ? rowL[k] : 0.0;
                }
                o.dinv = dinv;

                // reduced gradient and cost-to-go terms, then forward substitution
                double mv = 0.0;
                if (lane < NZ) {
                    double acc = rg - e0;
                    if constexpr (NG > 0) {
#pragma unroll
                        for (int r = 0; r < NG; ++r) acc -= s.G[r + lane * LDG] * s.e[NZ + r];
                    }
                    mv = acc;
                }
                if (n < N) mv = add_cost_to_go(mv, s.Lx[nxt], s.pn[nxt]);
                mv = fwd_subst_u<NZ>(mv, rowL, dinv);
                o.mv = mv;
                if (lane >= NU && lane < NZ) {
                    const int i = lane - NU;
                    s.pn[cur][i] = mv;
#pragma unroll
                    for (int k = 0; k < NX; ++k) s.Lx[cur][i + k * LDX] = (k <= i) ? rowL[NU + k] : 0.0;
                }
            }
            if (lane >= NU && lane < NZ) s.xn[cur][lane - NU] = z;
            if (lane < NX) s.pin[cur][lane] = pi;
            wsync();
        }
        flushA(0, upd, factor, o);
        o_g = wave_max(mg);
        o_b = wave_max(mb);
        o_d = wave_max(md);
        o_m = wave_max(mm);
        o_lt = wave_sum(slt);
        return fact_ok;
    }

    // slot values used by the right-hand-side sweeps
    __device__ __forceinline__ void load_slots_rm(int rmode, const double* d, const double* ir, const double* w,
                                                  int odl, int odu, double (&m)[NCT], double (&rdl)[NCT],
                                                  double (&rdu)[NCT], double (&ll)[NCT], double (&lu)[NCT],
                                                  double (&tl)[NCT], double (&tu)[NCT], double (&a1)[NCT],
                                                  double (&a2)[NCT], double (&a3)[NCT], double (&a4)[NCT]) const
    {
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
            const int c = slot(t);
            double lo_, hi_;
            slot_bounds(d, c, m[t], lo_, hi_);
            rdl[t] = rdu[t] = ll[t] = lu[t] = tl[t] = tu[t] = 0.0;
            a1[t] = a2[t] = a3[t] = a4[t] = 0.0;
            if (c < NC) {
                rdl[t] = w[odl + c];
                rdu[t] = w[odu + c];
                ll[t] = ir[Lo.I_ll + c];
                lu[t] = ir[Lo.I_lu + c];
                tl[t] = ir[Lo.I_tl + c];
                tu[t] = ir[Lo.I_tu + c];
                if (rmode == RM_CORRECTOR) {
                    a1[t] = w[Lo.W_all + c];
                    a2[t] = w[Lo.W_alu + c];
                    a3[t] = w[Lo.W_atl + c];
                    a4[t] = w[Lo.W_atu + c];
                } else if (rmode == RM_IR) {
                    a1[t] = w[Lo.W_irml + c];
                    a2[t] = w[Lo.W_irmu + c];
                }
            }
        }
    }

    // r_m (lower, upper) of a slot from the loaded values
    // (absolute formulation: r_m - 2 lam t, the right-hand side of the full-step iterate)
    __device__ __forceinline__ void rm_value(int rmode, double shift, double ll, double lu, double tl, double tu,
                                             double a1, double a2, double a3, double a4, double& rml,
                                             double& rmu) const
    {
        if (rmode == RM_IR) {
            rml = a1;
            rmu = a2;
            return;
        }
        rml = ll * tl - shift;
        rmu = lu * tu - shift;
        if (rmode == RM_CORRECTOR) {
            rml += a1 * a3;
            rmu += a2 * a4;
        }
        if (ABS) {
            rml -= 2.0 * ll * tl;
            rmu -= 2.0 * lu * tu;
        }
    }

    // ==================================================================
    // Pass C: backward right-hand-side sweep with the stored factors for
    // the RHS (r_g, r_b, r_d) at offsets og, ob, odl, odu and r_m per rmode.
    // ==================================================================
    struct PreC {
        double Lxx[EXr], F[EFr], G[EGr];
        const double *sLxx, *sF, *sG;
        double rowL[NU1];
        double dinv, rg, rb;
        double m[NCT], rdl[NCT], rdu[NCT], ll[NCT], lu[NCT], tl[NCT], tu[NCT];
        double a1[NCT], a2[NCT], a3[NCT], a4[NCT];
        SoftR sr[NCS];
    };

    __device__ __forceinline__ void loadC(PreC& p, int n, int rmode, int og, int ob, int odl, int odu) const
    {
        const double* d = Dp(n);
        const double* ir = Ip(n);
        const double* w = Wp(n);
        fetch_lxx(p.Lxx, w + Lo.W_L, p.sLxx);
        if (n < N) fetch<NX, NZ, EFr>(p.F, d + Lo.D_F, p.sF);
        if constexpr (NG > 0) fetch<NG, NZ, EGr>(p.G, d + Lo.D_G, p.sG);
#pragma unroll
        for (int k = 0; k < NU1; ++k) p.rowL[k] = (lane < NZ && k < NU) ? w[Lo.W_L + lane + k * NZ] : 0.0;
        p.dinv = lane < NZ ? w[Lo.W_dinv + lane] : 0.0;
        p.rg = lane < NZ ? w[og + lane] : 0.0;
        p.rb = (n < N && lane < NX) ? w[ob + lane] : 0.0;
        load_slots_rm(rmode, d, ir, w, odl, odu, p.m, p.rdl, p.rdu, p.ll, p.lu, p.tl, p.tu, p.a1, p.a2, p.a3, p.a4);
        if constexpr (SOFT) {
#pragma unroll
            for (int t = 0; t < NCT; ++t) load_softR(p.sr[t], rmode, d, ir, w, slot(t));
        }
    }

    __device__ __forceinline__ void flushC(int n, double mv) const
    {
        double* w = Wp(n);
        if (lane < NU) w[Lo.W_yu + lane] = mv;
        else if (lane < NZ) w[Lo.W_pv + lane - NU] = mv;
    }

    __device__ __forceinline__ void passC(int rmode, double shift, int og, int ob, int odl, int odu) const
    {
        Smem& s = S();
        PreC p;
        double out_mv = 0.0;
        loadC(p, N, rmode, og, ob, odl, odu);
        for (int n = N; n >= 0; --n) {
            const int cur = n & 1, nxt = cur ^ 1;
            // (x, x) block of this stage's factor becomes L_{n+1} of stage n-1
            commit_lxx(s.Lx[cur], p.Lxx, p.sLxx, true);
            if (n < N) commit<NX, NZ, EFr>(s.F, LDX, p.F, p.sF);
            if constexpr (NG > 0) commit<NG, NZ, EGr>(s.G, LDG, p.G, p.sG);
            double rowL[NU1];
#pragma unroll
            for (int k = 0; k < NU1; ++k) rowL[k] = p.rowL[k];
            const double dinv = p.dinv, rg = p.rg, rb = p.rb;
            double e0 = 0.0;
#pragma unroll
            for (int t = 0; t < NCT; ++t) {
                const int c = slot(t);
                double e = 0.0;
                if (c < NC && p.m[t] != 0.0) {
                    double rml, rmu;
                    rm_value(rmode, shift, p.ll[t], p.lu[t], p.tl[t], p.tu[t], p.a1[t], p.a2[t], p.a3[t], p.a4[t],
                             rml, rmu);
                    const double itl = rcp_nr(p.tl[t]), itu = rcp_nr(p.tu[t]);
                    e = (p.ll[t] * p.rdl[t] - rml) * itl - (p.lu[t] * p.rdu[t] - rmu) * itu;
                    if constexpr (SOFT) {
                        if (p.sr[t].sm != 0.0) {
                            double el = (p.ll[t] * p.rdl[t] - rml) * itl, eu = (p.lu[t] * p.rdu[t] - rmu) * itu;
                            double Dl, gl, Du, gu, rmsl, rmsu;
                            soft_rhs(p.sr[t], rmode, shift, p.ll[t] * itl, p.lu[t] * itu, el, eu, Dl, gl, Du, gu, rmsl,
                                     rmsu);
                            e = el - eu;
                        }
                    }
                }
                if (c < NC) s.e[c] = e;
                if (t == 0) e0 = e;
            }
            if (n == N && lane < NX) s.pn[nxt][lane] = 0.0;
            if (lane < NX) s.rb[lane] = rb;
            if (n < N) flushC(n + 1, out_mv);
            if (n > 0) loadC(p, n - 1, rmode, og, ob, odl, odu);
            wsync();
            double mv = 0.0;
            if (lane < NZ) {
                double acc = rg - e0;
                if constexpr (NG > 0) {
#pragma unroll
                    for (int r = 0; r < NG; ++r) acc -= s.G[r + lane * LDG] * s.e[NZ + r];
                }
                mv = acc;
            }
            if (n < N) mv = add_cost_to_go(mv, s.Lx[nxt], s.pn[nxt]);
            mv = fwd_subst_u<NU1>(mv, rowL, dinv);
            out_mv = mv;
            if (lane >= NU && lane < NZ) s.pn[cur][lane - NU] = mv;
            wsync();
        }
        flushC(0, out_mv);
    }

    // ==================================================================
    // Pass B: forward substitution and recovery of dt, dlam for the RHS of
    // pass A / C.  Writes dz, dpi to (oz, opi) and dlam, dt to (oll, olu,
    // otl, otu).  Returns the largest alpha keeping lam, t >= 0 (uncapped;
    // HUGE_VAL if unblocked) and the sums s1 = sum(lam dt + dlam t), s2 =
    // sum(dlam dt), so that the duality measure after a step of length a is
    // (lam't + a s1 + a^2 s2) / n_c.
    // ==================================================================
    struct PreB {
        double L[EL], Lxx[EXr], F[EFr], G[EGr];
        const double *sLxx, *sF, *sG;
        double dinv, yu, rb, pn;
        double zc, pic;  // current z_n, pi_{n+1} (absolute formulation: step = solution - iterate)
        double m[NCT], rdl[NCT], rdu[NCT], ll[NCT], lu[NCT], tl[NCT], tu[NCT];
        double a1[NCT], a2[NCT], a3[NCT], a4[NCT];
        SoftR sr[NCS];
    };

    __device__ __forceinline__ void loadB(PreB& p, int n, int rmode, int ob, int odl, int odu) const
    {
        const double* d = Dp(n);
        const double* ir = Ip(n);
        const double* w = Wp(n);
        if constexpr (NU > 0) fetch_r<NZ, NU, EL>(p.L, w + Lo.W_L);
        p.dinv = lane < NU ? w[Lo.W_dinv + lane] : 0.0;
        p.yu = lane < NU ? w[Lo.W_yu + lane] : 0.0;
        p.rb = p.pn = 0.0;
        p.zc = p.pic = 0.0;
        if (ABS && lane < NZ) p.zc = ir[Lo.I_z + lane];
        if (n < N) {
            const double* w1 = Wp(n + 1);
            fetch_lxx(p.Lxx, w1 + Lo.W_L, p.sLxx);
            fetch<NX, NZ, EFr>(p.F, d + Lo.D_F, p.sF);
            if (lane < NX) {
                p.rb = w[ob + lane];
                p.pn = w1[Lo.W_pv + lane];
                if (ABS) p.pic = Ip(n + 1)[Lo.I_pi + lane];
            }
        }
        if constexpr (NG > 0) fetch<NG, NZ, EGr>(p.G, d + Lo.D_G, p.sG);
        load_slots_rm(rmode, d, ir, w, odl, odu, p.m, p.rdl, p.rdu, p.ll, p.lu, p.tl, p.tu, p.a1, p.a2, p.a3, p.a4);
        if constexpr (SOFT) {
#pragma unroll
            for (int t = 0; t < NCT; ++t) load_softR(p.sr[t], rmode, d, ir, w, slot(t));
        }
    }

    struct OutB {
        double dz, dpi;
        double dll[NCT], dlu[NCT], dtl[NCT], dtu[NCT];
        SoftOutB so[NCS];
    };

    __device__ __forceinline__ void flushB(int n, const OutB& o, int oz, int opi, int oll, int olu, int otl,
                                           int otu) const
    {
        double* w = Wp(n);
        if (lane < NZ) w[oz + lane] = o.dz;
        if (n < N && lane < NX) Wp(n + 1)[opi + lane] = o.dpi;
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
            const int c = slot(t);
            if (c < NC) {
                w[oll + c] = o.dll[t];
                w[olu + c] = o.dlu[t];
                w[otl + c] = o.dtl[t];
                w[otu + c] = o.dtu[t];
                if constexpr (SOFT) {
                    if (o.so[t].sm != 0.0) {
                        // the affine step keeps only what the corrector reads
                        const bool aff = oll == Lo.W_all;
                        if (!aff) {
                            w[Lo.W_dsl + c] = o.so[t].dsl;
                            w[Lo.W_dsu + c] = o.so[t].dsu;
                        }
                        w[(aff ? Lo.W_alsl : Lo.W_dlsl) + c] = o.so[t].dlsl;
                        w[(aff ? Lo.W_alsu : Lo.W_dlsu) + c] = o.so[t].dlsu;
                        w[(aff ? Lo.W_atsl : Lo.W_dtsl) + c] = o.so[t].dtsl;
                        w[(aff ? Lo.W_atsu : Lo.W_dtsu) + c] = o.so[t].dtsu;
                    }
                }
            }
        }
    }

    __device__ __forceinline__ double passB(int rmode, double shift, int ob, int odl, int odu, int oz, int opi,
                                            int oll, int olu, int otl, int otu, double& o_s1, double& o_s2) const
    {
        Smem& s = S();
        double amin = HUGE_VAL, s1 = 0.0, s2 = 0.0;
        PreB p;
        OutB o;
        loadB(p, 0, rmode, ob, odl, odu);
        // dx_0 = -(L0 L0')^{-1} p_0 with L0 the (x, x) block of stage 0
        {
            double* w0 = Wp(0);
#pragma unroll
            for (int t = 0; t < EX; ++t) {
                const int e = lane + WAVE * t;
                if (e < NX * NX)
                    s.Lx[0][(e % NX) + (e / NX) * LDX] = w0[Lo.W_L + (NU + e % NX) + (NU + e / NX) * NZ];
            }
            double v = (lane < NX) ? -w0[Lo.W_pv + lane] : 0.0;
            const double di = (lane < NX) ? w0[Lo.W_dinv + NU + lane] : 0.0;
            if (lane < NX) w0[opi + lane] = 0.0;
            wsync();
            v = rnd(v);
#pragma unroll
            for (int j = 0; j < NX; ++j) {
                const double y = rnd(bcast(v, j) * bcast(di, j));
                if (lane == j) v = y;
                else if (lane > j && lane < NX) v = (double)((TS)v - (TS)s.Lx[0][lane + j * LDX] * (TS)y);
            }
#pragma unroll
            for (int j = NX - 1; j >= 0; --j) {
                const double x = rnd(bcast(v, j) * bcast(di, j));
                if (lane == j) v = x;
                else if (lane < j) v = (double)((TS)v - (TS)s.Lx[0][j + lane * LDX] * (TS)x);
            }
            wsync();
            if (lane < NX) s.xn[0][lane] = v;
            wsync();
        }
        for (int n = 0; n <= N; ++n) {
            const int cur = n & 1, nxt = cur ^ 1;
            if constexpr (NU > 0) commit_r<NZ, NU, EL>(s.M, LDZ, p.L);
            if (n < N) {
                commit_lxx(s.Lx[nxt], p.Lxx, p.sLxx, false);
                commit<NX, NZ, EFr>(s.F, LDX, p.F, p.sF);
            }
            if constexpr (NG > 0) commit<NG, NZ, EGr>(s.G, LDG, p.G, p.sG);
            const double dv = p.dinv, yu = p.yu, rb = p.rb, pn = p.pn, zc = p.zc, pic = p.pic;
            double m[NCT], rdl[NCT], rdu[NCT], ll[NCT], lu[NCT], tl[NCT], tu[NCT];
            double rml[NCT], rmu[NCT];
#pragma unroll
            for (int t = 0; t < NCT; ++t) {
                m[t] = p.m[t];
                rdl[t] = p.rdl[t];
                rdu[t] = p.rdu[t];
                ll[t] = p.ll[t];
                lu[t] = p.lu[t];
                tl[t] = p.tl[t];
                tu[t] = p.tu[t];
                rm_value(rmode, shift, ll[t], lu[t], tl[t], tu[t], p.a1[t], p.a2[t], p.a3[t], p.a4[t], rml[t],
                         rmu[t]);
            }
            SoftR sq[NCS];
            if constexpr (SOFT) {
#pragma unroll
                for (int t = 0; t < NCT; ++t) sq[t] = p.sr[t];
            }
            if (n > 0) flushB(n - 1, o, oz, opi, oll, olu, otl, otu);
            if (n < N) loadB(p, n + 1, rmode, ob, odl, odu);
            wsync();
            // v = y_u + L_xu' dx ; back-substitution with L_uu'
            double v = 0.0;
            if (lane < NU) {
                TS acc = (TS)yu;
#pragma unroll
                for (int i = 0; i < NX; ++i) acc += (TS)s.M[(NU + i) + lane * LDZ] * (TS)s.xn[cur][i];
                v = (double)acc;
            }
#pragma unroll
            for (int j = NU - 1; j >= 0; --j) {
                const double x = rnd(bcast(v, j) * bcast(dv, j));
                if (lane == j) v = x;
                else if (lane < j) v = (double)((TS)v - (TS)s.M[j + lane * LDZ] * (TS)x);
            }
            double dz = 0.0;
            if (lane < NU) dz = -v;
            else if (lane < NZ) dz = s.xn[cur][lane - NU];
            if (lane < NZ) s.z[lane] = dz;
            o.dz = ABS ? dz - zc : dz;
            wsync();
            o.dpi = 0.0;
            if (n < N) {
                const double* Lx = s.Lx[nxt];
                if (lane < NX) {
                    TS acc = (TS)rb;
#pragma unroll
                    for (int k = 0; k < NZ; ++k) acc += (TS)s.F[lane + k * LDX] * (TS)s.z[k];
                    s.xn[nxt][lane] = (double)acc;
                }
                wsync();
                if (lane < NX) {
                    TS acc = 0;
#pragma unroll
                    for (int l = 0; l < NX; ++l) acc += (TS)Lx[l + lane * LDX] * (TS)s.xn[nxt][l];
                    s.t1[lane] = (double)acc;
                }
                wsync();
                if (lane < NX) {
                    TS acc = (TS)pn;
#pragma unroll
                    for (int l = 0; l < NX; ++l) acc += (TS)Lx[lane + l * LDX] * (TS)s.t1[l];
                    o.dpi = ABS ? (double)acc - pic : (double)acc;
                }
            }
            // constraint steps, step length, duality-measure sums
#pragma unroll
            for (int t = 0; t < NCT; ++t) {
                const int c = slot(t);
                double dll = 0.0, dlu = 0.0, dtl = 0.0, dtu = 0.0;
                if constexpr (SOFT) o.so[t] = SoftOutB{};
                if (c < NC && m[t] != 0.0) {
                    double gdz;
                    if (c < NZ) {
                        gdz = dz;
                    } else {
                        const int r = c - NZ;
                        gdz = 0.0;
#pragma unroll
                        for (int k = 0; k < NZ; ++k) gdz += s.G[r + k * LDG] * s.z[k];
                    }
                    if constexpr (SOFT) {
                        double dsl = 0.0, dsu = 0.0;
                        if (sq[t].sm != 0.0) {
                            // slack steps and the steps of their bound rows
                            const SoftR& q = sq[t];
                            const double itl = rcp_nr(tl[t]), itu = rcp_nr(tu[t]);
                            const double wl = ll[t] * itl, wu = lu[t] * itu;
                            double el = (ll[t] * rdl[t] - rml[t]) * itl, eu = (lu[t] * rdu[t] - rmu[t]) * itu;
                            double Dl, gl, Du, gu, rmsl, rmsu;
                            soft_rhs(q, rmode, shift, wl, wu, el, eu, Dl, gl, Du, gu, rmsl, rmsu);
                            dsl = -(gl + wl * gdz) * rcp_nr(Dl);
                            dsu = -(gu - wu * gdz) * rcp_nr(Du);
                            const double dtsl = dsl - q.rdsl, dtsu = dsu - q.rdsu;
                            const double dlsl = -(rmsl + q.lsl * dtsl) * rcp_nr(q.tsl);
                            const double dlsu = -(rmsu + q.lsu * dtsu) * rcp_nr(q.tsu);
                            if (dlsl < 0.0) amin = fmin(amin, -q.lsl * __builtin_amdgcn_rcp(dlsl));
                            if (dlsu < 0.0) amin = fmin(amin, -q.lsu * __builtin_amdgcn_rcp(dlsu));
                            if (dtsl < 0.0) amin = fmin(amin, -q.tsl * __builtin_amdgcn_rcp(dtsl));
                            if (dtsu < 0.0) amin = fmin(amin, -q.tsu * __builtin_amdgcn_rcp(dtsu));
                            s1 += q.lsl * dtsl + dlsl * q.tsl + q.lsu * dtsu + dlsu * q.tsu;
                            s2 += dlsl * dtsl + dlsu * dtsu;
                            o.so[t] = SoftOutB{1.0, dsl, dsu, dlsl, dlsu, dtsl, dtsu};
                        }
                        dtl = gdz + dsl - rdl[t];
                        dtu = -gdz + dsu - rdu[t];
                    } else {
                        dtl = gdz - rdl[t];
                        dtu = -gdz - rdu[t];
                    }
                    dll = -(rml[t] + ll[t] * dtl) * rcp_nr(tl[t]);
                    dlu = -(rmu[t] + lu[t] * dtu) * rcp_nr(tu[t]);
                    if (ABS) {
                        // absolute formulation: the step is the full-step
                        // iterate minus the current one (eq:alg:pdipm:step)
                        dtl -= tl[t];
                        dtu -= tu[t];
                        dll -= ll[t];
                        dlu -= lu[t];
                    }
                    // step to the boundary; approximate reciprocals suffice for a
                    // length that is scaled by gamma < 1 afterwards
                    if (dll < 0.0) amin = fmin(amin, -ll[t] * __builtin_amdgcn_rcp(dll));
                    if (dlu < 0.0) amin = fmin(amin, -lu[t] * __builtin_amdgcn_rcp(dlu));
                    if (dtl < 0.0) amin = fmin(amin, -tl[t] * __builtin_amdgcn_rcp(dtl));
                    if (dtu < 0.0) amin = fmin(amin, -tu[t] * __builtin_amdgcn_rcp(dtu));
                    s1 += ll[t] * dtl + dll * tl[t] + lu[t] * dtu + dlu * tu[t];
                    s2 += dll * dtl + dlu * dtu;
                }
                o.dll[t] = dll;
                o.dlu[t] = dlu;
                o.dtl[t] = dtl;
                o.dtu[t] = dtu;
            }
            wsync();
        }
        flushB(N, o, oz, opi, oll, olu, otl, otu);
        o_s1 = wave_sum(s1);
        o_s2 = wave_sum(s2);
        return wave_min(amin);
    }

    // ==================================================================
    // Pass R (mixed path): residual of the Newton system for the step at
    // offsets (oz, opi, oll, olu, otl, otu), in FP64 (Section 3.4):
    //   r_ir = K step + r,  r = (r_g, r_b, r_d, r_m) with r_m per rmode.
    // Writes r_ir to the refinement arrays and returns its inf-norm.
    // ==================================================================
    struct PreR {
        double H[EHr], F[EFr], G[EGr];
        const double *sH, *sF, *sG;
        double dz, dpi, rg, rb;
        double m[NCT], rdl[NCT], rdu[NCT], ll[NCT], lu[NCT], tl[NCT], tu[NCT];
        double a1[NCT], a2[NCT], a3[NCT], a4[NCT];
        double sll[NCT], slu[NCT], stl[NCT], stu[NCT];
    };

    __device__ __forceinline__ void loadR(PreR& p, int n, int rmode, int oz, int opi, int oll, int olu, int otl,
                                          int otu) const
    {
        const double* d = Dp(n);
        const double* ir = Ip(n);
        const double* w = Wp(n);
        fetch<NZ, NZ, EHr>(p.H, d + Lo.D_H, p.sH);
        if (n < N) fetch<NX, NZ, EFr>(p.F, d + Lo.D_F, p.sF);
        if constexpr (NG > 0) fetch<NG, NZ, EGr>(p.G, d + Lo.D_G, p.sG);
        p.dz = lane < NZ ? w[oz + lane] : 0.0;
        p.rg = lane < NZ ? w[Lo.W_rg + lane] : 0.0;
        p.dpi = (lane < NX && n > 0) ? w[opi + lane] : 0.0;
        p.rb = (lane < NX && n < N) ? w[Lo.W_rb + lane] : 0.0;
        load_slots_rm(rmode, d, ir, w, Lo.W_rdl, Lo.W_rdu, p.m, p.rdl, p.rdu, p.ll, p.lu, p.tl, p.tu, p.a1, p.a2,
                      p.a3, p.a4);
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
            const int c = slot(t);
            p.sll[t] = p.slu[t] = p.stl[t] = p.stu[t] = 0.0;
            if (c < NC) {
                p.sll[t] = w[oll + c];
                p.slu[t] = w[olu + c];
                p.stl[t] = w[otl + c];
                p.stu[t] = w[otu + c];
            }
        }
    }

    struct OutR {
        double rg, rb, rdl[NCT], rdu[NCT], rml[NCT], rmu[NCT];
    };

    __device__ __forceinline__ void flushR(int n, const OutR& o) const
    {
        double* w = Wp(n);
        if (lane < NZ) w[Lo.W_irg + lane] = o.rg;
        if (n < N && lane < NX) w[Lo.W_irb + lane] = o.rb;
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
            const int c = slot(t);
            if (c < NC) {
                w[Lo.W_irdl + c] = o.rdl[t];
                w[Lo.W_irdu + c] = o.rdu[t];
                w[Lo.W_irml + c] = o.rml[t];
                w[Lo.W_irmu + c] = o.rmu[t];
            }
        }
    }

    __device__ __forceinline__ double passR(int rmode, double shift, int oz, int opi, int oll, int olu, int otl,
                                            int otu) const
    {
        Smem& s = S();
        double nr = 0.0;
        PreR p;
        OutR o;
        loadR(p, N, rmode, oz, opi, oll, olu, otl, otu);
        for (int n = N; n >= 0; --n) {
            const int cur = n & 1, nxt = cur ^ 1;
            commit<NZ, NZ, EHr>(s.M, LDZ, p.H, p.sH);
            if (n < N) commit<NX, NZ, EFr>(s.F, LDX, p.F, p.sF);
            if constexpr (NG > 0) commit<NG, NZ, EGr>(s.G, LDG, p.G, p.sG);
            const double dz = p.dz, dpi = p.dpi, rg = p.rg, rb = p.rb;
            double m[NCT], rdl[NCT], rdu[NCT], ll[NCT], lu[NCT], tl[NCT], tu[NCT], rml[NCT], rmu[NCT];
            double sll[NCT], slu[NCT], stl[NCT], stu[NCT];
#pragma unroll
            for (int t = 0; t < NCT; ++t) {
                m[t] = p.m[t];
                rdl[t] = p.rdl[t];
                rdu[t] = p.rdu[t];
                ll[t] = p.ll[t];
                lu[t] = p.lu[t];
                tl[t] = p.tl[t];
                tu[t] = p.tu[t];
                sll[t] = p.sll[t];
                slu[t] = p.slu[t];
                stl[t] = p.stl[t];
                stu[t] = p.stu[t];
                rm_value(rmode, shift, ll[t], lu[t], tl[t], tu[t], p.a1[t], p.a2[t], p.a3[t], p.a4[t], rml[t],
                         rmu[t]);
            }
            if (n < N) flushR(n + 1, o);
            if (n > 0) loadR(p, n - 1, rmode, oz, opi, oll, olu, otl, otu);
            if (n == N && lane < NX) {
                s.xn[nxt][lane] = 0.0;
                s.pin[nxt][lane] = 0.0;
            }
            if (lane < NZ) s.z[lane] = dz;
            if (lane < NX) s.t2[lane] = dpi;
            if constexpr (NG > 0) {
#pragma unroll
                for (int t = 0; t < NCT; ++t) {
                    const int c = slot(t);
                    if (c >= NZ && c < NC) s.t1[c - NZ] = m[t] * (sll[t] - slu[t]);
                }
            }
            wsync();
            // g row: H dz + F' dpi_{n+1} - [0; dpi_n] - C' dlam + r_g
            o.rg = 0.0;
            if (lane < NZ) {
                const int j = lane;
                double acc = rg;
#pragma unroll
                for (int k = 0; k < NZ; ++k) acc += s.M[j + k * LDZ] * s.z[k];
                if (n < N) {
#pragma unroll
                    for (int i = 0; i < NX; ++i) acc += s.F[i + j * LDX] * s.pin[nxt][i];
                }
                if (j >= NU) acc -= s.t2[j - NU];
                acc -= m[0] * (sll[0] - slu[0]);
                if constexpr (NG > 0) {
#pragma unroll
                    for (int r = 0; r < NG; ++r) acc -= s.G[r + j * LDG] * s.t1[r];
                }
                o.rg = acc;
                nr = nmax(nr, fabs(acc));
            }
            // b row: F dz - dx_{n+1} + r_b
            o.rb = 0.0;
            if (n < N && lane < NX) {
                double acc = rb;
#pragma unroll
                for (int k = 0; k < NZ; ++k) acc += s.F[lane + k * LDX] * s.z[k];
                o.rb = acc - s.xn[nxt][lane];
                nr = nmax(nr, fabs(o.rb));
            }
            // d rows: -C dz + dt + r_d ; m rows: T dlam + Lam dt + r_m
#pragma unroll
            for (int t = 0; t < NCT; ++t) {
                const int c = slot(t);
                o.rdl[t] = o.rdu[t] = o.rml[t] = o.rmu[t] = 0.0;
                if (c < NC && m[t] != 0.0) {
                    double gz;
                    if (c < NZ) {
                        gz = dz;
                    } else {
                        const int r = c - NZ;
                        gz = 0.0;
#pragma unroll
                        for (int k = 0; k < NZ; ++k) gz += s.G[r + k * LDG] * s.z[k];
                    }
                    o.rdl[t] = -gz + stl[t] + rdl[t];
                    o.rdu[t] = gz + stu[t] + rdu[t];
                    o.rml[t] = tl[t] * sll[t] + ll[t] * stl[t] + rml[t];
                    o.rmu[t] = tu[t] * slu[t] + lu[t] * stu[t] + rmu[t];
                    nr = nmax(nr, nmax(nmax(fabs(o.rdl[t]), fabs(o.rdu[t])), nmax(fabs(o.rml[t]), fabs(o.rmu[t]))));
                }
            }
            if (lane >= NU && lane < NZ) s.xn[cur][lane - NU] = dz;
            if (lane < NX) s.pin[cur][lane] = dpi;
            wsync();
        }
        flushR(0, o);
        return wave_max(nr);
    }

    // ==================================================================
    // Pass X (mixed path): step += correction, then the step length and the
    // duality-measure sums of pass B for the corrected step.
    // ==================================================================
    __device__ __forceinline__ double passX(int oz, int opi, int oll, int olu, int otl, int otu, double sg,
                                            double& o_s1, double& o_s2) const
    {
        double amin = HUGE_VAL, s1 = 0.0, s2 = 0.0;
        for (int n = 0; n <= N; ++n) {
            const double* d = Dp(n);
            const double* ir = Ip(n);
            double* w = Wp(n);
            if (lane < NZ) w[oz + lane] += sg * w[Lo.W_edz + lane];
            if (lane < NX && n > 0) w[opi + lane] += sg * w[Lo.W_edpi + lane];
#pragma unroll
            for (int t = 0; t < NCT; ++t) {
                const int c = slot(t);
                if (c >= NC) continue;
                double m, lo_, hi_;
                slot_bounds(d, c, m, lo_, hi_);
                if (m == 0.0) continue;
                const double dll = w[oll + c] + sg * w[Lo.W_edll + c];
                const double dlu = w[olu + c] + sg * w[Lo.W_edlu + c];
                const double dtl = w[otl + c] + sg * w[Lo.W_edtl + c];
                const double dtu = w[otu + c] + sg * w[Lo.W_edtu + c];
                w[oll + c] = dll;
                w[olu + c] = dlu;
                w[otl + c] = dtl;
                w[otu + c] = dtu;
                const double ll = ir[Lo.I_ll + c], lu = ir[Lo.I_lu + c], tl = ir[Lo.I_tl + c], tu = ir[Lo.I_tu + c];
                if (dll < 0.0) amin = fmin(amin, -ll * __builtin_amdgcn_rcp(dll));
                if (dlu < 0.0) amin = fmin(amin, -lu * __builtin_amdgcn_rcp(dlu));
                if (dtl < 0.0) amin = fmin(amin, -tl * __builtin_amdgcn_rcp(dtl));
                if (dtu < 0.0) amin = fmin(amin, -tu * __builtin_amdgcn_rcp(dtu));
                s1 += ll * dtl + dll * tl + lu * dtu + dlu * tu;
                s2 += dll * dtl + dlu * dtu;
            }
        }
        o_s1 = wave_sum(s1);
        o_s2 = wave_sum(s2);
        return wave_min(amin);
    }

    // Iterative refinement of the step at the given offsets (Section 3.4).
    // Stops when ||r_ir|| <= ir_tol * max(1, ||r||), after max_steps
    // corrections, or when a correction did not lower ||r_ir|| (that
    // correction is then subtracted again, so the step kept is the best one
    // seen).  Updates amax, s1, s2 for the step kept; nir0 returns the
    // residual norm of the unrefined step (the balance build's accuracy
    // check of the factors); returns the corrections kept.
    __device__ __forceinline__ int refine(int rmode, double shift, double rnorm, int max_steps, int oz, int opi,
                                          int oll, int olu, int otl, int otu, double& amax, double& s1, double& s2,
                                          double& nir0) const
    {
        int steps = 0;
        double prev = HUGE_VAL;
        for (int it = 0;; ++it) {
            const double nir = passR(rmode, shift, oz, opi, oll, olu, otl, otu);
            __syncthreads();
            if (it == 0) nir0 = nir;
            const bool back = it > 0 && !(nir < prev);
            if (!back && (!(nir > P.ir_tol * rnorm) || it == max_steps)) break;
            if (!back) {
                prev = nir;
                passC(RM_IR, 0.0, Lo.W_irg, Lo.W_irb, Lo.W_irdl, Lo.W_irdu);
                __syncthreads();
                double t1, t2;
                passB(RM_IR, 0.0, Lo.W_irb, Lo.W_irdl, Lo.W_irdu, Lo.W_edz, Lo.W_edpi, Lo.W_edll, Lo.W_edlu,
                      Lo.W_edtl, Lo.W_edtu, t1, t2);
                __syncthreads();
            }
            amax = passX(oz, opi, oll, olu, otl, otu, back ? -1.0 : 1.0, s1, s2);
            __syncthreads();
            if (back) {
                --steps;
                break;
            }
            ++steps;
        }
        return steps;
    }

    // cold start: y = 0, pi = 0, t = max(C y - d, 1), lam = 1 (masked slots 0)
    // Initial point (P.warm): cold start y = 0, pi = 0, t = max(C y - d, 1),
    // lam = 1; with a primal guess in the iterate records (warm start of
    // Section 4.2) y is kept and the rest set as in the cold start at that y;
    // with a primal and dual guess everything is kept, multipliers and
    // slacks clamped below as in the iterate update.
    __device__ __forceinline__ void init(int warm) const
    {
        for (int n = 0; n <= N; ++n) {
            const double* d = Dp(n);
            double* ir = Ip(n);
            if (warm == 0 && lane < NZ) ir[Lo.I_z + lane] = 0.0;
            if (warm != 2 && lane < NX) ir[Lo.I_pi + lane] = 0.0;
#pragma unroll
            for (int t = 0; t < NCT; ++t) {
                const int c = slot(t);
                if (c >= NC) continue;
                double m, lo, hi;
                slot_bounds(d, c, m, lo, hi);
                const bool on = m != 0.0;
                if (warm == 2) {
                    ir[Lo.I_ll + c] = on ? fmax(ir[Lo.I_ll + c], P.lam_min) : 0.0;
                    ir[Lo.I_lu + c] = on ? fmax(ir[Lo.I_lu + c], P.lam_min) : 0.0;
                    ir[Lo.I_tl + c] = on ? fmax(ir[Lo.I_tl + c], P.t_min) : 0.0;
                    ir[Lo.I_tu + c] = on ? fmax(ir[Lo.I_tu + c], P.t_min) : 0.0;
                    if constexpr (SOFT) {
                        const bool sf = d[Lo.D_sm + c] != 0.0;
                        if (!sf) {
                            ir[Lo.I_sl + c] = 0.0;
                            ir[Lo.I_su + c] = 0.0;
                        }
                        ir[Lo.I_lsl + c] = sf ? fmax(ir[Lo.I_lsl + c], P.lam_min) : 0.0;
                        ir[Lo.I_lsu + c] = sf ? fmax(ir[Lo.I_lsu + c], P.lam_min) : 0.0;
                        ir[Lo.I_tsl + c] = sf ? fmax(ir[Lo.I_tsl + c], P.t_min) : 0.0;
                        ir[Lo.I_tsu + c] = sf ? fmax(ir[Lo.I_tsu + c], P.t_min) : 0.0;
                    }
                    continue;
                }
                double gz = 0.0;
                if (warm == 1) {
                    if (c < NZ) {
                        gz = ir[Lo.I_z + c];
                    } else {
                        for (int j = 0; j < NZ; ++j) gz += d[Lo.D_G + (c - NZ) + j * NG] * ir[Lo.I_z + j];
                    }
                }
                ir[Lo.I_ll + c] = on ? 1.0 : 0.0;
                ir[Lo.I_lu + c] = on ? 1.0 : 0.0;
                ir[Lo.I_tl + c] = on ? (warm == 1 ? fmax(gz - lo, 1.0) : fmax(-lo, 1.0)) : 0.0;
                ir[Lo.I_tu + c] = on ? (warm == 1 ? fmax(hi - gz, 1.0) : fmax(hi, 1.0)) : 0.0;
                if constexpr (SOFT) {
                    // slacks s = 0, or (primal guess) the guess: the soft rows' t =
                    // max(G z + s^l - lo, 1) and max(hi - G z + s^u, 1), the bound rows
                    // t_s = max(s - ls, 1), lam_s = 1; slots without slacks hold zeros
                    const bool sf = d[Lo.D_sm + c] != 0.0;
                    const double sl0 = (sf && warm == 1) ? ir[Lo.I_sl + c] : 0.0;
                    const double su0 = (sf && warm == 1) ? ir[Lo.I_su + c] : 0.0;
                    if (sf && warm == 1) {
                        ir[Lo.I_tl + c] = fmax(gz + sl0 - lo, 1.0);
                        ir[Lo.I_tu + c] = fmax(hi - gz + su0, 1.0);
                    }
                    ir[Lo.I_sl + c] = sl0;
                    ir[Lo.I_su + c] = su0;
                    ir[Lo.I_lsl + c] = sf ? 1.0 : 0.0;
                    ir[Lo.I_lsu + c] = sf ? 1.0 : 0.0;
                    ir[Lo.I_tsl + c] = sf ? fmax(sl0 - d[Lo.D_lls + c], 1.0) : 0.0;
                    ir[Lo.I_tsu + c] = sf ? fmax(su0 - d[Lo.D_lus + c], 1.0) : 0.0;
                }
            }
        }
        __syncthreads();
    }

    __device__ __forceinline__ void copy_step_out(double* out) const
    {
        for (int n = 0; n <= N; ++n) {
            double* o = out + (size_t)n * Lo.IREC;
            const double* w = Wp(n);
            if (lane < NZ) o[Lo.I_z + lane] = w[Lo.W_dz + lane];
            if (lane < NX) o[Lo.I_pi + lane] = w[Lo.W_dpi + lane];
#pragma unroll
            for (int t = 0; t < NCT; ++t) {
                const int c = slot(t);
                if (c >= NC) continue;
                o[Lo.I_ll + c] = w[Lo.W_dll + c];
                o[Lo.I_lu + c] = w[Lo.W_dlu + c];
                o[Lo.I_tl + c] = w[Lo.W_dtl + c];
                o[Lo.I_tu + c] = w[Lo.W_dtu + c];
                if constexpr (SOFT) {
                    if (Dp(n)[Lo.D_sm + c] != 0.0) {
                        o[Lo.I_sl + c] = w[Lo.W_dsl + c];
                        o[Lo.I_su + c] = w[Lo.W_dsu + c];
                        o[Lo.I_lsl + c] = w[Lo.W_dlsl + c];
                        o[Lo.I_lsu + c] = w[Lo.W_dlsu + c];
                        o[Lo.I_tsl + c] = w[Lo.W_dtsl + c];
                        o[Lo.I_tsu + c] = w[Lo.W_dtsu + c];
                    }
                }
            }
        }
    }

    // ------------------------------------------------------------------
    // Driver.  Solve mode: the IPM from a cold start.  Newton mode: one
    // Newton step at the stored iterate with r_m = lam.*t - tau.  Every pass
    // has a single call site so that its code is emitted once.
    // ------------------------------------------------------------------
    // resume: continue from the iterate records (a primal-dual warm start:
    // the launch that stopped there left them as the next iteration would
    // find them); itcap > 0: at most itcap iterations in this launch
    // (iteration blocks of the server)
    // it0, ir0: iterations and refinement steps done before this launch on
    // the same instance (a mixed solve continued by the FP64 kernel)
    __device__ __forceinline__ void run(DevStat* st, double* step_out, int fell_back, int resume, int itcap, int it0,
                                        int ir0) const
    {
        const bool newton_mode = P.mode == KMODE_NEWTON;
        const bool absf = ABS;
        if (!newton_mode) init(resume ? 2 : P.warm);
        const int cap = itcap > 0 ? min(P.iter_max, itcap) : P.iter_max;
        int status = ST_MAX_ITER, k = 0;
        double ng = 0, nb = 0, nd = 0, nm = 0, mu = 0.0, slt = 0.0;
        const double inv2nc = nc > 0 ? 1.0 / (2.0 * nc) : 0.0;
        const double shift0 = newton_mode ? P.tau : 0.0;
        bool upd = false, rejected = false;
        double alpha = 0.0;
        int ir_steps = 0;
        // absolute formulation: once the loop ends, one more pass A (delta
        // form, no update, no factorization) evaluates the residuals at the
        // returned iterate; it reuses the single call site of pass A
        bool final_pass = false;
        int k_exit = 0;
        // balance build: the iteration is factored with the array algorithm
        // (after its Cholesky factors failed the accuracy check)
        bool qr = false, refactor = false;
        int qr_refactors = 0;
        for (k = 0;; ++k) {
            // residuals at the (updated) iterate; factorization unless the
            // last step was rejected as too short
            const bool fact_ok =
                passA(upd, alpha, shift0, !rejected && !final_pass && (newton_mode || k < cap), absf && !final_pass, qr,
                      ng, nb, nd, nm, slt);
            __syncthreads();
            mu = slt * inv2nc;
            if (final_pass) {
                k = k_exit;
                if (ng != ng || nb != nb || nd != nd || nm != nm) status = ST_NAN;
                break;
            }
            if (rejected) {
                status = ST_MIN_STEP;
                if (absf) {
                    final_pass = true;
                    k_exit = k;
                    upd = false;
                    continue;
                }
                break;
            }
            if (MIXED && !newton_mode && !fact_ok) {
                status = ST_FALLBACK;  // FP32 factorization broke down
                break;
            }
            if (!newton_mode && absf) {
                // absolute formulation (mode speed_abs): exit on the duality
                // measure alone
                if (mu != mu) {
                    status = ST_NAN;
                    break;
                }
                if (mu <= P.tol_comp || k >= cap) {
                    status = mu <= P.tol_comp ? ST_SUCCESS : ST_MAX_ITER;
                    final_pass = true;
                    k_exit = k;
                    upd = false;
                    continue;
                }
            } else if (!newton_mode) {
                if (ng != ng || nb != nb || nd != nd || nm != nm || mu != mu) {
                    status = ST_NAN;
                    break;
                }
                if (ng <= P.tol_stat && nb <= P.tol_eq && nd <= P.tol_ineq && nm <= P.tol_comp) {
                    status = ST_SUCCESS;
                    break;
                }
                if (k >= cap) {
                    status = ST_MAX_ITER;
                    break;
                }
            }
            if constexpr (BALANCE) {
                // a breakdown of the Cholesky factorization fails the check too
                if (!fact_ok && !qr && !newton_mode) refactor = true;
            }
            // round 0: predictor (affine step; in Newton mode the step itself)
            // round 1: Mehrotra corrector; round 2: predictor-centering step
            // when the conditional corrector is rejected (Section 4.2)
            double amax = HUGE_VAL, mu_aff = 0.0, smu = 0.0;
            for (int round = 0; round < 3 && !refactor; ++round) {
                const int rmode = round == 1 ? RM_CORRECTOR : RM_SHIFT;
                const double shift = round == 0 ? shift0 : smu;
                const bool aff = round == 0 && !newton_mode;
                if (round > 0) {
                    passC(rmode, shift, Lo.W_rg, Lo.W_rb, Lo.W_rdl, Lo.W_rdu);
                    __syncthreads();
                }
                double s1, s2;
                const int oll = aff ? Lo.W_all : Lo.W_dll, olu = aff ? Lo.W_alu : Lo.W_dlu;
                const int otl = aff ? Lo.W_atl : Lo.W_dtl, otu = aff ? Lo.W_atu : Lo.W_dtu;
                amax = passB(rmode, shift, Lo.W_rb, Lo.W_rdl, Lo.W_rdu, Lo.W_dz, Lo.W_dpi, oll, olu, otl, otu, s1, s2);
                __syncthreads();
                if constexpr (REFINE) {
                    // refinement of the prediction-centering-correction
                    // direction (Section 4.2); the affine predictor only
                    // feeds the centering parameter and the corrector
                    // right-hand side and is used unrefined.  Balance build:
                    // the predictor's residual checks the accuracy of this
                    // iteration's Cholesky factors
                    const bool dir = (round > 0 || newton_mode || nc == 0) && (KM != KM_F64 || P.ir_max > 0);
                    const bool check = BALANCE && !qr && !newton_mode && round == 0;
                    if (dir || check) {
                        const double rnorm = fmax(1.0, fmax(fmax(ng, nb), fmax(nd, nm)));
                        double nir0 = 0.0;
                        ir_steps += refine(rmode, shift, rnorm, dir ? P.ir_max : 0, Lo.W_dz, Lo.W_dpi, oll, olu, otl,
                                           otu, amax, s1, s2, nir0);
                        if (check && !(nir0 <= P.ir_tol * rnorm)) {
                            refactor = true;
                            break;
                        }
                    }
                }
                if (newton_mode || nc == 0) break;
                const double a = fmin(amax, 1.0);
                const double mu_a = (slt + a * s1 + a * a * s2) * inv2nc;
                if (round == 0) {
                    mu_aff = fmax(0.0, mu_a);
                    const double ratio = mu > 0.0 ? mu_aff / mu : 0.0;
                    smu = ratio * ratio * ratio * mu;
                } else if (round == 1) {
                    if (!(mu_a > P.corr_ratio * mu_aff)) break;
                } else {
                    break;
                }
            }
            if constexpr (BALANCE) {
                if (refactor) {
                    // start the iteration over (no step taken) with the array
                    // algorithm; the next iteration starts with Cholesky again
                    refactor = false;
                    qr = true;
                    upd = false;
                    ++qr_refactors;
                    --k;
                    continue;
                }
                qr = false;
            }
            if (newton_mode) break;
            alpha = fmin(1.0, P.gamma * amax);
            upd = true;
            rejected = alpha < P.alpha_min;
        }
        if (newton_mode) {
            copy_step_out(step_out);
            status = ST_SUCCESS;
            k = 0;
        }
        // the mixed path hands instances it could not finish to the FP64 kernel
        if (MIXED && !newton_mode && (status == ST_NAN || status == ST_MIN_STEP)) status = ST_FALLBACK;
        // a finite iterate is handed over as it is: the FP64 kernel continues
        // the solve from it instead of starting over
        if (MIXED && status == ST_FALLBACK)
            fell_back = (__builtin_isfinite(ng) && __builtin_isfinite(nb) && __builtin_isfinite(nd) &&
                         __builtin_isfinite(nm) && __builtin_isfinite(mu))
                            ? FB_RESUME
                            : FB_COLD;
        if (lane == 0) {
            st->status = status;
            st->iters = it0 + k;
            st->ir_steps = ir0 + ir_steps;
            st->fell_back = fell_back;
            st->qr_refactors = qr_refactors;
            st->mu = mu;
            st->res[0] = ng;
            st->res[1] = nb;
            st->res[2] = nd;
            st->res[3] = nm;
        }
    }
};

// Occupancy: small stage blocks fit two waves per SIMD; larger ones get the
// whole register file (256 VGPRs + 256 AGPRs) of one wave instead of spilling.
__host__ __device__ constexpr int ipm_max_waves(int nz, bool mixed) { return (nz > 24 || (mixed && nz > 16)) ? 1 : 2; }

template <int NX, int NU, int NG, int KM>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(1, ipm_max_waves(NX + NU, KM == KM_MIXED || KM == KM_BALANCE)))) void ipm_kernel(const InstDesc* __restrict__ desc, int count,
                                                    const double* __restrict__ data, double* __restrict__ iter,
                                                    double* __restrict__ work, double* __restrict__ step_out,
                                                    DevStat* __restrict__ stat, KParams P)
{
    using S = Ipm<NX, NU, NG, KM>;
    const int b = blockIdx.x;
    if (b >= count) return;
    const InstDesc ds = desc[b];
    int fell_back = FB_NONE, resume = ds.resume, itcap = ds.itcap, it0 = 0, ir0 = 0;
    if (P.mode == KMODE_FALLBACK) {
        // second launch after the mixed kernel: only instances it handed over,
        // continued from their iterate within the remaining iteration budget
        const DevStat s0 = stat[ds.index];
        if (s0.status != ST_FALLBACK) return;
        fell_back = FB_DONE;
        if (s0.fell_back == FB_RESUME) {
            resume = 1;
            it0 = s0.iters;
            ir0 = s0.ir_steps;
            itcap = max(1, P.iter_max - it0);
        }
    }
    const S ipm(data + ds.data, iter + ds.iter, work + ds.work, ds.N, ds.nc, P);
    ipm.run(stat + ds.index, step_out + ds.iter, fell_back, resume, itcap, it0, ir0);
}

template <int NX, int NU, int NG, int KM>
void launch_ipm(const InstDesc* desc, int count, const double* data, double* iter, double* work, double* step,
                DevStat* stat, KParams P, hipStream_t stream)
{
    hipLaunchKernelGGL((ipm_kernel<NX, NU, NG, KM>), dim3(count), dim3(WAVE), 0, stream, desc, count, data, iter,
                       work, step, stat, P);
}

}  // namespace oqp
