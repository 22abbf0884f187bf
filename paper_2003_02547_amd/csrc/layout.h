// Device memory layout of the batched OCP-QP IPM.
//
// Every instance is padded to the stage sizes (NX, NU, NG) of the kernel
// variant ("bucket") that solves it.  Padded inputs carry unit Hessian
// diagonal and zero coupling, padded general rows are masked, so the padded
// problem has the same minimiser (padded components are exactly zero).
//
// One instance = N+1 stage records, each a fixed number of doubles, stored
// contiguously so that one workgroup streams its own instance stage by stage
// with coalesced loads.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define OQP_HD __host__ __device__
#else
#define OQP_HD
#endif

namespace oqp {

OQP_HD constexpr int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct Layout {
    int NX, NU, NG, NZ, NC;
    int SOFT;  // 1: soft layout (slack blocks present)
    // problem data record (doubles), one per stage
    int D_F, D_H, D_g, D_b, D_bm, D_blo, D_bhi, D_G, D_gm, D_glo, D_ghi, SREC;
    // iterate record (doubles), one per stage: z, pi_n, lam_l, lam_u, t_l, t_u
    int I_z, I_pi, I_ll, I_lu, I_tl, I_tu, IREC;
    // workspace record (doubles), one per stage
    int W_rg, W_rb, W_rdl, W_rdu, W_yu, W_pv, W_dz, W_dpi, W_dll, W_dlu, W_dtl, W_dtu;
    int W_all, W_alu, W_atl, W_atu, W_irg, W_irb, W_irdl, W_irdu, W_irml, W_irmu;
    int W_edz, W_edpi, W_edll, W_edlu, W_edtl, W_edtu, W_L, W_dinv, W_V, WREC;
    // soft constraints (Section 2.2), present only in a soft layout, one
    // entry per constraint slot: data (slot mask, slack Hessians Zl, Zu,
    // gradients zl, zu, lower bounds lls, lus), iterate (slacks s^l, s^u,
    // multipliers and slacks of their bounds), workspace (slack
    // stationarity and bound residuals, step, affine step)
    int D_sm, D_Zl, D_Zu, D_zl, D_zu, D_lls, D_lus;
    int I_sl, I_su, I_lsl, I_lsu, I_tsl, I_tsu;
    int W_rsl, W_rsu, W_rdsl, W_rdsu, W_dsl, W_dsu, W_dlsl, W_dlsu, W_dtsl, W_dtsu, W_alsl, W_alsu, W_atsl, W_atsu;
};

// F = [B A] is NX x NZ column-major, H is NZ x NZ column-major (full
// symmetric), G is NG x NZ column-major.  Constraint slots per stage: NC =
// NZ box slots (one per component of z = [u; x], masked by bm) followed by
// NG general rows (masked by gm).
// A soft layout (soft = true) appends the slack blocks to each record.
OQP_HD constexpr Layout make_layout(int NX, int NU, int NG, bool soft = false)
{
    Layout L{};
    L.NX = NX; L.NU = NU; L.NG = NG; L.NZ = NX + NU; L.NC = NX + NU + NG;
    L.SOFT = soft ? 1 : 0;
    const int NZ = L.NZ, NC = L.NC;
    int o = 0;
    L.D_F = o; o += NX * NZ;
    L.D_H = o; o += NZ * NZ;
    L.D_g = o; o += NZ;
    L.D_b = o; o += NX;
    L.D_bm = o; o += NZ;
    L.D_blo = o; o += NZ;
    L.D_bhi = o; o += NZ;
    L.D_G = o; o += NG * NZ;
    L.D_gm = o; o += NG;
    L.D_glo = o; o += NG;
    L.D_ghi = o; o += NG;
    {
        const int ns = soft ? NC : 0;
        L.D_sm = o; o += ns;
        L.D_Zl = o; o += ns;
        L.D_Zu = o; o += ns;
        L.D_zl = o; o += ns;
        L.D_zu = o; o += ns;
        L.D_lls = o; o += ns;
        L.D_lus = o; o += ns;
    }
    L.SREC = round_up(o, 8);
    o = 0;
    L.I_z = o; o += NZ;
    L.I_pi = o; o += NX;
    L.I_ll = o; o += NC;
    L.I_lu = o; o += NC;
    L.I_tl = o; o += NC;
    L.I_tu = o; o += NC;
    {
        const int ns = soft ? NC : 0;
        L.I_sl = o; o += ns;
        L.I_su = o; o += ns;
        L.I_lsl = o; o += ns;
        L.I_lsu = o; o += ns;
        L.I_tsl = o; o += ns;
        L.I_tsu = o; o += ns;
    }
    L.IREC = round_up(o, 8);
    o = 0;
    L.W_rg = o; o += NZ;
    L.W_rb = o; o += NX;
    L.W_rdl = o; o += NC;
    L.W_rdu = o; o += NC;
    L.W_yu = o; o += round_up(NU, 1);
    L.W_pv = o; o += NX;
    L.W_dz = o; o += NZ;
    L.W_dpi = o; o += NX;
    L.W_dll = o; o += NC;
    L.W_dlu = o; o += NC;
    L.W_dtl = o; o += NC;
    L.W_dtu = o; o += NC;
    L.W_all = o; o += NC;
    L.W_alu = o; o += NC;
    L.W_atl = o; o += NC;
    L.W_atu = o; o += NC;
    L.W_irg = o; o += NZ;
    L.W_irb = o; o += NX;
    L.W_irdl = o; o += NC;
    L.W_irdu = o; o += NC;
    L.W_irml = o; o += NC;
    L.W_irmu = o; o += NC;
    L.W_edz = o; o += NZ;
    L.W_edpi = o; o += NX;
    L.W_edll = o; o += NC;
    L.W_edlu = o; o += NC;
    L.W_edtl = o; o += NC;
    L.W_edtu = o; o += NC;
    o = round_up(o, 8);
    L.W_L = o; o += NZ * NZ;
    L.W_dinv = o; o += NZ;
    // [L_{n+1}' F; sqrt(w) G] of the stage, used only by the global-memory
    // mode of the block kernel (stage blocks above 64) and by the wide-stage
    // kernel (also for more than 64 general rows)
    L.W_V = o; o += (NX + NU > 64 || NG > 64) ? (NX + NG) * NZ : 0;
    {
        const int ns = soft ? NC : 0;
        L.W_rsl = o; o += ns;
        L.W_rsu = o; o += ns;
        L.W_rdsl = o; o += ns;
        L.W_rdsu = o; o += ns;
        L.W_dsl = o; o += ns;
        L.W_dsu = o; o += ns;
        L.W_dlsl = o; o += ns;
        L.W_dlsu = o; o += ns;
        L.W_dtsl = o; o += ns;
        L.W_dtsu = o; o += ns;
        L.W_alsl = o; o += ns;
        L.W_alsu = o; o += ns;
        L.W_atsl = o; o += ns;
        L.W_atsu = o; o += ns;
    }
    L.WREC = round_up(o, 8);
    return L;
}

// Per-instance descriptor (device).  Offsets are in doubles from the base of
// the respective region.
struct InstDesc {
    int64_t data;   // stage records of the problem data
    int64_t iter;   // iterate records (the solution region)
    int64_t work;   // workspace records
    int32_t N;      // horizon
    int32_t nc;     // number of two-sided constraints (box + general)
    int32_t index;  // position of the instance in the caller's batch
    int32_t resume; // 1: continue from the iterate records (iteration blocks of the server)
    int32_t nx, nu, ng;  // padded stage sizes (read by the runtime-sized block kernel)
    int32_t itcap;  // > 0: at most this many iterations in this launch
    int32_t nuN;    // inputs of the terminal stage (0: the wide-stage kernel skips its padded input block)
    int32_t pad;
};

// Partial condensing (Section 3.5), one descriptor per instance.  Offsets
// are in doubles; the original QP keeps its own record layout (stage sizes
// onx, onu, ong), the condensed QP uses the layout of the kernel that solves
// it (cnx, cnu, cng).
struct CondDesc {
    int64_t odata;   // original data records (N + 1)
    int64_t oiter;   // expanded iterate records (N + 1), original layout
    int64_t cdata;   // condensed data records (N2 + 1)
    int64_t citer;   // condensed iterate records (N2 + 1)
    int32_t N, N2;   // original and condensed horizon
    int32_t tab;     // int offset of the stage table: (nx, nu, nbx, ng) per
                     // original stage, then the N2 + 1 block starts
    int32_t onx, onu, ong;
    int32_t cnx, cnu, cng;
    int32_t pad;
};

// One workgroup of the condensing and expansion kernels: block b of
// instance inst (b = N2 is the terminal stage).
struct CondItem {
    int32_t inst;
    int32_t block;
};

// Per-instance result written by the kernel.
struct DevStat {
    int32_t status;
    int32_t iters;
    int32_t ir_steps;
    int32_t fell_back;  // the mixed path handed the instance to the FP64 kernel (FB_*)
    double mu;
    double res[4];  // inf-norms of r_g, r_b, r_d, lam.*t at the returned iterate
    int32_t qr_refactors;  // balance build: iterations factored again with the array algorithm
    int32_t pad;
};

// Solver arguments passed by value to every launch.
struct KParams {
    double tol_stat, tol_eq, tol_ineq, tol_comp;
    double alpha_min, gamma, lam_min, t_min, reg_prim, corr_ratio, ir_tol;
    double tau;         // Newton-step entry: r_m = lam.*t - tau
    int32_t iter_max;
    int32_t ir_max;
    int32_t mode;       // KMODE_SOLVE or KMODE_NEWTON
    int32_t warm;       // initial point of a solve: 0 cold, 1 primal guess, 2 primal and dual guess
};

enum { KMODE_SOLVE = 0, KMODE_NEWTON = 1, KMODE_FALLBACK = 2 };
// Compiled kernel builds: FP64 delta formulation, mixed (FP32 factorization
// and sweeps, FP64 refinement), FP64 absolute formulation, FP64 with the
// QR-based (array algorithm) factorization, FP64 delta formulation with
// soft constraints (soft layout), FP64 Cholesky checked by its refinement
// residual with the array algorithm as fallback (one-wave kernel).
enum { KM_F64 = 0, KM_MIXED = 1, KM_ABS = 2, KM_ROBUST = 3, KM_SOFT = 4, KM_BALANCE = 5 };
enum { ST_SUCCESS = 0, ST_MAX_ITER = 1, ST_MIN_STEP = 2, ST_NAN = 3, ST_FALLBACK = 4 };
// DevStat.fell_back: 0 solved by the launch's own kernel, 1 finished by the
// FP64 kernel; between the mixed launch and the FP64 one, a handed-over
// instance holds FB_RESUME (its iterate is finite: the FP64 kernel continues
// from it) or FB_COLD (it starts the FP64 solve over)
enum { FB_NONE = 0, FB_DONE = 1, FB_COLD = 2, FB_RESUME = 3 };

}  // namespace oqp
