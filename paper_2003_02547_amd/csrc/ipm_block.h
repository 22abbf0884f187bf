// Block kernel of the batched OCP-QP interior-point method: one 256-thread
// workgroup (four waves) per instance, for stage blocks too large for the
// one-wave kernel to hold in registers.
//
// The method, passes and Riccati equations are those of the one-wave kernel
// (square-root Riccati recursion of Section 3.3 on the reduced system
// eq:alg:kkt, Mehrotra predictor-corrector of Section 4.2, FP64 iterative
// refinement of Section 3.4 in the mixed path), with the same device record
// layout, so the two kernels are interchangeable per instance.  What differs
// is the mapping onto the hardware:
//   * stage sizes are runtime values read from the instance descriptor, so
//     one launch solves instances of different sizes (the host orders them
//     by estimated cost, largest first);
//   * the stage matrices of the sweep go through registers spread over all
//     256 threads, prefetched one stage ahead, and are staged in LDS;
//   * the products U = L_{n+1}' [B A] and M += V'V run on all four waves with
//     4 x 4 register tiles; row-wise work (residual rows, constraint slots)
//     takes one thread per row or slot;
//   * the Cholesky factorization and the triangular solves run on wave 0
//     with one row per lane (rows of the factor held in registers up to the
//     compile-time bound ZM on the stage block).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "dev_common.h"
#include "layout.h"

namespace oqp {

constexpr int BT = 256;    // threads per instance
constexpr int BGMAX = 64;  // general rows per stage supported by the block kernel

// LDS plan (offsets in doubles) for padded stage sizes NX, NU, NG.
struct BLds {
    int ldm, ldf, ldg, ldx, ldv;  // odd leading dimensions: column-strided access spreads over the banks
    int oM, oF, oG, oLx, oV, oz, orb, ot1, ot2, oe, ows, oxn, opin, opn, odv, odd, ol11, ocol, ored, oflag;
    // global-memory mode, stage matrix held in registers (stage blocks up to
    // 160): a panel of 16 rows of V, the column panel of the factor below the
    // diagonal tile, the diagonal tile, and one chunk (16 rows) of L_{n+1} and
    // F that the V panel is built from
    int ldu, oUp, oPn, oDg, oCA, oCB;
    int total;
};

OQP_HD constexpr int bmaxi(int a, int b) { return a > b ? a : b; }

// Global-memory mode (stage blocks above 64): the stage matrix and its
// factor live in the instance's factor record, F and G are read in place,
// U' = [L_{n+1}' F; sqrt(w) G] goes to a workspace block, and LDS holds only
// vectors.
OQP_HD constexpr bool block_global(int NX, int NU) { return NX + NU > 64; }

OQP_HD constexpr BLds make_blds(int NX, int NU, int NG)
{
    const int NZ = NX + NU, NC = NZ + NG, NV = NX + NG;
    const bool gl = block_global(NX, NU);
    BLds s{};
    s.ldm = NZ | 1;
    s.ldf = NX | 1;
    s.ldg = NG | 1;
    s.ldx = NX | 1;
    s.ldv = NV | 1;
    int o = 0;
    s.oM = o; o += gl ? 0 : s.ldm * NZ;              // H / stage matrix / factor; factor columns in the forward sweeps
    s.oF = o; o += gl ? 0 : s.ldf * NZ;              // [B A]
    s.oG = o; o += (gl || NG == 0) ? 0 : s.ldg * NZ; // G
    s.oLx = o; o += gl ? 0 : s.ldx * NX;             // L_{n+1} (lower, zero strict upper)
    s.oV = o; o += gl ? 0 : s.ldv * NZ;              // [U; sqrt(w) G]
    s.oz = o; o += NZ;
    s.orb = o; o += bmaxi(NX, 1);
    s.ot1 = o; o += bmaxi(bmaxi(NX, NG), 1);
    s.ot2 = o; o += bmaxi(NX, 1);
    s.oe = o; o += NC;
    s.ows = o; o += NC;
    s.oxn = o; o += 2 * bmaxi(NX, 1);
    s.opin = o; o += 2 * bmaxi(NX, 1);
    s.opn = o; o += 2 * bmaxi(NX, 1);
    s.odv = o; o += NZ;
    s.odd = o; o += NZ;                              // FP64 running diagonal (mixed Cholesky)
    // diagonal block of the current Cholesky panel; with the next region, the
    // two reflector buffers of the array algorithm (2 (NV + 2) doubles)
    s.ol11 = o; o += bmaxi(16 * 16, 2 * (NV + 2) - 64);
    s.ocol = o; o += 64;
    s.ored = o; o += 32;
    s.oflag = o; o += 2;
    s.ldu = NZ | 1;
    const bool tiles = gl && NZ <= 160;
    s.oUp = o; o += tiles ? 16 * s.ldu : 0;
    s.oPn = o; o += tiles ? NZ * 17 : 0;
    s.oDg = o; o += tiles ? 16 * 17 : 0;
    s.oCA = o; o += tiles ? 16 * 17 : 0;
    // the chunk of F shares the panel of V: each panel's chunks are consumed
    // before its rows of V are stored, and the syrk reads of the previous
    // panel end before the first chunk of the next (barriers in between);
    // 64 KB at nz = 160, so two workgroups fit a CU
    s.oCB = s.oUp;
    s.total = o;
    return s;
}

// Position (row r, column c) of element e = start + BT t of a column-major
// block with R rows, advanced without a division per element.
struct Walk {
    int r, c, sr, sc, R;
    __device__ __forceinline__ Walk(int R_, int start) : R(R_)
    {
        const int q = R_ > 0 ? R_ : 1;
        r = start % q;
        c = start / q;
        sr = BT % q;
        sc = BT / q;
    }
    __device__ __forceinline__ void next()
    {
        r += sr;
        c += sc;
        if (r >= R) {
            r -= R;
            ++c;
        }
    }
};

__device__ __forceinline__ double* blds()
{
    extern __shared__ double oqp_blds_dyn[];
    return oqp_blds_dyn;
}

template <int KM, int ZM, int GM, bool GL>
struct Blk {
    static constexpr bool MIXED = KM == KM_MIXED;
    static constexpr bool ABS = KM == KM_ABS;  // absolute formulation (Section 3.2)
    static constexpr bool SOFT = KM == KM_SOFT;  // soft constraints (Section 2.2), soft layout
    // factorization by the array algorithm (Section 4.2, mode robust), or
    // Cholesky factors checked by the predictor's refinement residual with the
    // array algorithm when they fail the check (mode balance)
    static constexpr bool ROBUST = KM == KM_ROBUST;
    static constexpr bool BALANCE = KM == KM_BALANCE;
    // refinement of the prediction-centering-correction direction
    static constexpr bool REFINE = MIXED || ROBUST || BALANCE || KM == KM_F64;
    using TS = typename std::conditional<MIXED, float, double>::type;
    Layout Lo;
    BLds S;
    int NX, NU, NG, NZ, NC, NV;
    const double* __restrict__ dat;
    double* __restrict__ itr;
    double* __restrict__ wk;
    int N, nc, tid, lane, wid;
    const KParams& P;
    // leading dimensions of the stage blocks (LDS copies, or the records in
    // global-memory mode)
    int ldm, ldf, ldg, ldx, ldv;
    // global-memory mode: stage blocks of the current stage
    mutable double* cM;
    mutable const double* cF;
    mutable const double* cG;
    mutable const double* cLx;
    mutable const double* cXC;
    mutable double* cV;
    mutable const double* cH;  // global-memory mode: H of the current stage (data record)

    __device__ __forceinline__ Blk(const InstDesc& ds, const double* d, double* i, double* w, const KParams& P_)
        : Lo(make_layout(ds.nx, ds.nu, ds.ng, SOFT)), S(make_blds(ds.nx, ds.nu, ds.ng)), NX(ds.nx), NU(ds.nu), NG(ds.ng),
          NZ(ds.nx + ds.nu), NC(ds.nx + ds.nu + ds.ng), NV(ds.nx + ds.ng), dat(d + ds.data), itr(i + ds.iter),
          wk(w + ds.work), N(ds.N), nc(ds.nc), tid((int)threadIdx.x), lane((int)threadIdx.x & 63),
          wid((int)threadIdx.x >> 6), P(P_)
    {
        if constexpr (GL) {
            ldm = NZ;
            ldf = NX;
            ldg = NG;
            ldx = NZ;
            ldv = NV;
        } else {
            ldm = S.ldm;
            ldf = S.ldf;
            ldg = S.ldg;
            ldx = S.ldx;
            ldv = S.ldv;
        }
        cM = cV = nullptr;
        cF = cG = cLx = cXC = cH = nullptr;
    }

    __device__ __forceinline__ const double* Dp(int n) const { return dat + (size_t)n * Lo.SREC; }
    __device__ __forceinline__ double* Ip(int n) const { return itr + (size_t)n * Lo.IREC; }
    __device__ __forceinline__ double* Wp(int n) const { return wk + (size_t)n * Lo.WREC; }

    // stage blocks: LDS copies, or the records themselves in global-memory mode
    __device__ __forceinline__ double* M() const { return GL ? cM : blds() + S.oM; }
    __device__ __forceinline__ double* F() const { return GL ? const_cast<double*>(cF) : blds() + S.oF; }
    __device__ __forceinline__ double* G() const { return GL ? const_cast<double*>(cG) : blds() + S.oG; }
    __device__ __forceinline__ double* Lx() const { return GL ? const_cast<double*>(cLx) : blds() + S.oLx; }
    __device__ __forceinline__ double* V() const { return GL ? cV : blds() + S.oV; }
    // first x-column of the next stage's factor (passes B and C)
    __device__ __forceinline__ const double* XC() const { return GL ? cXC : blds() + S.oM + NU * ldm; }
    __device__ __forceinline__ double* ddv() const { return blds() + S.odd; }
    __device__ __forceinline__ double* l11() const { return blds() + S.ol11; }
    __device__ __forceinline__ double* z() const { return blds() + S.oz; }
    __device__ __forceinline__ double* rbv() const { return blds() + S.orb; }
    __device__ __forceinline__ double* t1() const { return blds() + S.ot1; }
    __device__ __forceinline__ double* t2() const { return blds() + S.ot2; }
    __device__ __forceinline__ double* ev() const { return blds() + S.oe; }
    __device__ __forceinline__ double* wsv() const { return blds() + S.ows; }
    __device__ __forceinline__ double* xn(int p) const { return blds() + S.oxn + p * (NX > 0 ? NX : 1); }
    __device__ __forceinline__ double* pin(int p) const { return blds() + S.opin + p * (NX > 0 ? NX : 1); }
    __device__ __forceinline__ double* pn(int p) const { return blds() + S.opn + p * (NX > 0 ? NX : 1); }
    __device__ __forceinline__ double* dv() const { return blds() + S.odv; }
    __device__ __forceinline__ double* col() const { return blds() + S.ocol; }
    __device__ __forceinline__ double* red() const { return blds() + S.ored; }
    __device__ __forceinline__ double* flag() const { return blds() + S.oflag; }

    __device__ __forceinline__ static double rnd(double x) { return (double)(TS)x; }

    // Thread index re-materialised inside a loop body: the empty volatile asm
    // keeps the compiler from hoisting per-thread address arithmetic of every
    // pass to the top of the kernel, where it would stay live (and occupy
    // registers) for the whole solve.
    __device__ __forceinline__ static int opq(int v)
    {
        asm volatile("" : "+v"(v));
        return v;
    }

    // sum_{k < n} a[k sa] b[k sb] in type T with four independent partial
    // sums, so that several LDS reads are in flight at once
    template <typename T>
    __device__ __forceinline__ static T dot(const double* a, int sa, const double* b, int sb, int n)
    {
        T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        int k = 0;
        if constexpr (GL) {
            // global-memory mode (operands in HBM/L2): 16 loads issued
            // together, the sums taken in the same order as below
            for (; k + 16 <= n; k += 16) {
                double av[16], bv[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    av[q] = a[(k + q) * sa];
                    bv[q] = b[(k + q) * sb];
                }
#pragma unroll
                for (int q = 0; q < 16; q += 4) {
                    s0 += (T)av[q] * (T)bv[q];
                    s1 += (T)av[q + 1] * (T)bv[q + 1];
                    s2 += (T)av[q + 2] * (T)bv[q + 2];
                    s3 += (T)av[q + 3] * (T)bv[q + 3];
                }
            }
        }
#pragma unroll 2
        for (; k + 4 <= n; k += 4) {
            const double a0 = a[k * sa], a1 = a[(k + 1) * sa], a2 = a[(k + 2) * sa], a3 = a[(k + 3) * sa];
            const double b0 = b[k * sb], b1 = b[(k + 1) * sb], b2 = b[(k + 2) * sb], b3 = b[(k + 3) * sb];
            s0 += (T)a0 * (T)b0;
            s1 += (T)a1 * (T)b1;
            s2 += (T)a2 * (T)b2;
            s3 += (T)a3 * (T)b3;
        }
        for (; k < n; ++k) s0 += (T)a[k * sa] * (T)b[k * sb];
        return (s0 + s1) + (s2 + s3);
    }

    // ------------------------------------------------------------------
    // block reductions (fixed combination order: identical in every thread)
    // ------------------------------------------------------------------
    __device__ __forceinline__ void reduce4(double& a, double& b, double& c, double& d, double& e) const
    {
        a = wave_max(a);
        b = wave_max(b);
        c = wave_max(c);
        d = wave_max(d);
        e = wave_sum(e);
        double* r = red();
        __syncthreads();
        if (lane == 0) {
            r[wid * 5 + 0] = a;
            r[wid * 5 + 1] = b;
            r[wid * 5 + 2] = c;
            r[wid * 5 + 3] = d;
            r[wid * 5 + 4] = e;
        }
        __syncthreads();
        a = nmax(nmax(r[0], r[5]), nmax(r[10], r[15]));
        b = nmax(nmax(r[1], r[6]), nmax(r[11], r[16]));
        c = nmax(nmax(r[2], r[7]), nmax(r[12], r[17]));
        d = nmax(nmax(r[3], r[8]), nmax(r[13], r[18]));
        e = (r[4] + r[9]) + (r[14] + r[19]);
        __syncthreads();
    }

    __device__ __forceinline__ double bmin_sum2(double amin, double& s1, double& s2) const
    {
        amin = wave_min(amin);
        s1 = wave_sum(s1);
        s2 = wave_sum(s2);
        double* r = red();
        __syncthreads();
        if (lane == 0) {
            r[wid * 3 + 0] = amin;
            r[wid * 3 + 1] = s1;
            r[wid * 3 + 2] = s2;
        }
        __syncthreads();
        amin = fmin(fmin(r[0], r[3]), fmin(r[6], r[9]));
        s1 = (r[1] + r[4]) + (r[7] + r[10]);
        s2 = (r[2] + r[5]) + (r[8] + r[11]);
        __syncthreads();
        return amin;
    }

    __device__ __forceinline__ double bmax1(double v) const
    {
        v = wave_max(v);
        double* r = red();
        __syncthreads();
        if (lane == 0) r[wid] = v;
        __syncthreads();
        v = nmax(nmax(r[0], r[1]), nmax(r[2], r[3]));
        __syncthreads();
        return v;
    }

    // ------------------------------------------------------------------
    // stage prefetch: three flat blocks of global memory (element e = tid +
    // BT t of each) into registers, committed to LDS at the next stage
    // ------------------------------------------------------------------
    static constexpr int EA = GL ? 1 : (ZM * ZM + BT - 1) / BT;           // H, or the factor columns
    static constexpr int EF = GL ? 1 : (ZM * ZM + BT - 1) / BT;           // F
    static constexpr int EG = (GL || GM == 0) ? 1 : (GM * ZM + BT - 1) / BT;

    struct Pre {
        double a[EA], f[EF], g[EG];
        const double* sa;   // block a (or, for the factor columns, its first part)
        const double* sa2;  // second part of block a from element na1 on
        const double* sf;
        const double* sg;
        int na1, na, nf, ng;
    };

    __device__ __forceinline__ void fetch(Pre& p) const
    {
        if constexpr (GL) return;
        // element offsets recomputed per stage, not held across the loop
        const int tdo = opaque(tid);
#pragma unroll
        for (int t = 0; t < EA; ++t) {
            const int e = tdo + BT * t;
            const double* src = e < p.na1 ? p.sa : p.sa2;
            p.a[t] = e < p.na ? src[e] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < EF; ++t) {
            const int e = tdo + BT * t;
            p.f[t] = e < p.nf ? p.sf[e] : 0.0;
        }
        if constexpr (GM > 0) {
#pragma unroll
            for (int t = 0; t < EG; ++t) {
                const int e = tdo + BT * t;
                p.g[t] = e < p.ng ? p.sg[e] : 0.0;
            }
        }
    }

    __device__ __forceinline__ void commit(const Pre& p, double* da, double* df, double* dg) const
    {
        if constexpr (GL) return;
        const int tdo = opaque(tid);
        {
            Walk q(NZ, tdo);
#pragma unroll
            for (int t = 0; t < EA; ++t) {
                const int e = tdo + BT * t;
                if (e < p.na) da[q.r + q.c * ldm] = p.a[t];
                q.next();
            }
        }
        {
            Walk q(NX, tdo);
#pragma unroll
            for (int t = 0; t < EF; ++t) {
                const int e = tdo + BT * t;
                if (e < p.nf) df[q.r + q.c * ldf] = p.f[t];
                q.next();
            }
        }
        if constexpr (GM > 0) {
            Walk q(NG, tdo);
#pragma unroll
            for (int t = 0; t < EG; ++t) {
                const int e = tdo + BT * t;
                if (e < p.ng) dg[q.r + q.c * ldg] = p.g[t];
                q.next();
            }
        }
    }

    // H, F, G of stage n (passes A and R)
    __device__ __forceinline__ void seg_hfg(Pre& p, int n) const
    {
        const double* d = Dp(n);
        p.sa = p.sa2 = d + Lo.D_H;
        p.na1 = p.na = NZ * NZ;
        p.sf = d + Lo.D_F;
        p.nf = n < N ? NX * NZ : 0;
        p.sg = d + Lo.D_G;
        p.ng = NG * NZ;
    }

    // factor columns (u-columns of stage n, x-columns of stage n + 1, both
    // in the NZ x NZ column-major factor layout), F and G of stage n
    // (passes B and C)
    __device__ __forceinline__ void seg_lfg(Pre& p, int n) const
    {
        const double* d = Dp(n);
        p.sa = Wp(n) + Lo.W_L;
        p.sa2 = n < N ? Wp(n + 1) + Lo.W_L : p.sa;
        p.na1 = NZ * NU;
        p.na = n < N ? NZ * NZ : NZ * NU;
        p.sf = d + Lo.D_F;
        p.nf = n < N ? NX * NZ : 0;
        p.sg = d + Lo.D_G;
        p.ng = NG * NZ;
    }

    // global-memory mode: point the stage blocks at the records of stage n.
    // Pass A builds the stage matrix in the stage's factor record (H copied
    // in first; the factor then stays there) with L_{n+1} read from the next
    // stage's record; pass R reads H in place; passes B and C read the u
    // columns of this stage's factor and the x columns of the next one's.
    __device__ __forceinline__ void stage_A(int n, bool qr) const
    {
        if constexpr (GL) {
            const double* d = Dp(n);
            cM = Wp(n) + Lo.W_L;
            cF = d + Lo.D_F;
            cG = d + Lo.D_G;
            cLx = n < N ? Wp(n + 1) + Lo.W_L + NU + NU * NZ : cM;
            cV = Wp(n) + Lo.W_V;
            cH = d + Lo.D_H;
            // the stage matrix is built in the factor record, from a copy of H,
            // unless it is held in registers
            if (!use_tiles(qr))
                for (int e = opq(tid); e < NZ * NZ; e += BT) cM[e] = cH[e];
        }
    }
    __device__ __forceinline__ void stage_R(int n) const
    {
        if constexpr (GL) {
            const double* d = Dp(n);
            cM = const_cast<double*>(d + Lo.D_H);
            cF = d + Lo.D_F;
            cG = d + Lo.D_G;
        }
    }
    __device__ __forceinline__ void stage_BC(int n) const
    {
        if constexpr (GL) {
            const double* d = Dp(n);
            cM = Wp(n) + Lo.W_L;
            cXC = n < N ? Wp(n + 1) + Lo.W_L + NU * NZ : cM;
            cF = d + Lo.D_F;
            cG = d + Lo.D_G;
        }
    }

    // constraint slot data: mask, lower, upper (slot c: box on z_c for c <
    // NZ, general row c - NZ otherwise)
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
            m = lo = hi = 0.0;
        }
    }

    // Slack elimination of a soft slot c (Section 2.2).  The slot's slack
    // pair (s^l, s^u) enters the lower row as G z + s^l and the upper row as
    // -G z + s^u, each with its own bound row s >= ls (multiplier lam_s,
    // slack t_s).  Given the row terms el = (lam_l rd_l - rm_l) / t_l and eu
    // (same for the upper row) and the barrier weights wl, wu, the slack rows
    // of the Newton system read
    //   D_l ds^l + wl G dz = -g_l,   D_u ds^u - wu G dz = -g_u,
    //   D = Z + w + w_s,  g = r_s - e - e_s,  e_s = (lam_s rd_s - rm_s) / t_s,
    // so that eliminating ds turns the row terms into e + w g / D (and the
    // weights into w (Z + w_s) / D, applied in pass A).  r_s, rd_s are read
    // from the workspace pass A wrote, rm_s per rmode as in slot_rm.
    struct SoftE {
        double Dl, Du, gl, gu, lsl, lsu, tsl, tsu, rmsl, rmsu, rdsl, rdsu;
    };
    __device__ __forceinline__ SoftE soft_terms(const double* d, const double* ir, const double* w, int c, int rmode,
                                                double shift, double wl, double wu, double& el, double& eu) const
    {
        SoftE q;
        q.lsl = ir[Lo.I_lsl + c];
        q.lsu = ir[Lo.I_lsu + c];
        q.tsl = ir[Lo.I_tsl + c];
        q.tsu = ir[Lo.I_tsu + c];
        q.rdsl = w[Lo.W_rdsl + c];
        q.rdsu = w[Lo.W_rdsu + c];
        q.rmsl = q.lsl * q.tsl - shift;
        q.rmsu = q.lsu * q.tsu - shift;
        if (rmode == RM_CORRECTOR) {
            q.rmsl += w[Lo.W_alsl + c] * w[Lo.W_atsl + c];
            q.rmsu += w[Lo.W_alsu + c] * w[Lo.W_atsu + c];
        }
        const double itsl = rcp_nr(q.tsl), itsu = rcp_nr(q.tsu);
        const double esl = (q.lsl * q.rdsl - q.rmsl) * itsl;
        const double esu = (q.lsu * q.rdsu - q.rmsu) * itsu;
        q.Dl = d[Lo.D_Zl + c] + wl + q.lsl * itsl;
        q.Du = d[Lo.D_Zu + c] + wu + q.lsu * itsu;
        q.gl = w[Lo.W_rsl + c] - el - esl;
        q.gu = w[Lo.W_rsu + c] - eu - esu;
        el += wl * q.gl * rcp_nr(q.Dl);
        eu += wu * q.gu * rcp_nr(q.Du);
        return q;
    }

    // ------------------------------------------------------------------
    // dense kernels on LDS blocks
    // ------------------------------------------------------------------

    // C(i, j) op= sum_{k < K} A(k, i) B(k, j) for i < m, j < n (only j <= i
    // when `lower`), with A(k, i) = A[k sak + i sai] and B(k, j) = B[k sbk +
    // j sbj], on the matrix cores: 16 x 16 output tiles spread over the four
    // waves, K in steps of 4 (v_mfma_f64_16x16x4f64; in the mixed path FP32
    // operands and accumulation, v_mfma_f32_16x16x4f32).  Operand lanes:
    // A(k0 + lane / 16, i0 + lane % 16), B(k0 + lane / 16, j0 + lane % 16);
    // result register r of a lane: row i0 + 4 r + lane / 16 (FP64) or
    // i0 + 4 (lane / 16) + r (FP32), column j0 + lane % 16.  Loads use
    // clamped in-range indices and zero out-of-range operands, so every lane
    // stays active.  op: 0 store, 1 add, -1 subtract.
    __device__ __forceinline__ void mma_tn(const double* A, int sak, int sai, const double* B, int sbk, int sbj, int m,
                                           int n, int K, double* C, int ldc, int op, bool lower) const
    {
        using V4 = TS __attribute__((ext_vector_type(4)));
        if (m <= 0 || n <= 0 || K <= 0) return;
        const int TM = (m + 15) >> 4, TN = (n + 15) >> 4;
        const int l16 = lane & 15, lk = lane >> 4;
        for (int t = opq(wid); t < TM * TN; t += BT / 64) {
            const int ti = t % TM, tj = t / TM;
            if (lower && ti < tj) continue;
            const int i = 16 * ti + l16, j = 16 * tj + l16;
            const bool iv = i < m, jv = j < n;
            const double* pa = A + min(i, m - 1) * sai;
            const double* pb = B + min(j, n - 1) * sbj;
            V4 acc = {0, 0, 0, 0};
#pragma unroll 4
            for (int k0 = 0; k0 < K; k0 += 4) {
                const int k = k0 + lk;
                const int kc = min(k, K - 1);
                const double av = pa[kc * sak], bv = pb[kc * sbk];
                const bool kv = k < K;
                const TS a = (iv && kv) ? (TS)av : (TS)0;
                const TS b = (jv && kv) ? (TS)bv : (TS)0;
                if constexpr (MIXED)
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
                else
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * ti + (MIXED ? 4 * lk + r : 4 * r + lk);
                const int col = 16 * tj + l16;
                if (row < m && col < n && (!lower || col <= row)) {
                    double* c = C + row + col * ldc;
                    if (op == 0) *c = (double)acc[r];
                    else if (op > 0) *c += (double)acc[r];
                    else *c = MIXED ? (double)((TS)*c - acc[r]) : *c - (double)acc[r];
                }
            }
        }
    }

    // V[i][k] = sum_l Lx[l][i] F[l][k] (i < NX, k < NZ); Lx lower with zero
    // strict upper part
    __device__ __forceinline__ void trmm_LtF() const
    {
        mma_tn(Lx(), 1, ldx, F(), 1, ldf, NX, NZ, NX, V(), ldv, 0, false);
    }

    // M[i][k] += sum_{r0 <= r < NV} V[r][i] V[r][k] on the lower triangle
    __device__ __forceinline__ void syrk_VtV(int r0) const
    {
        mma_tn(V() + r0, 1, ldv, V() + r0, 1, ldv, NZ, NZ, NV - r0, M(), ldm, 1, true);
    }

    // Blocked right-looking Cholesky of M (NZ x NZ, lower triangle read) with
    // panels of PW columns.  Writes L (zero strict upper part) back into M and
    // 1/L_ii into dv.  Every thread calls it; returns false (in every thread)
    // when a pivot is not positive.  Mixed path: FP32 entries and updates,
    // each row's diagonal accumulated in FP64 (FP64 pivots).
    //
    // Stage blocks above 64 (global-memory mode): wave 0 factors the PW x PW
    // diagonal block (one row per lane, rows in registers, column entries by
    // readlane) and copies it to LDS; every thread then solves one row of the
    // block below it against that factor (L21 = M21 L11^{-T}), and all
    // threads apply the panel to the trailing lower triangle with 4 x 4
    // register tiles.
    static constexpr int PW = 16;

    // Stage blocks up to 64 (LDS mode): wave 0 holds every row of a panel
    // (one row per lane, rows in registers) and applies each column to the
    // rows below it in lock-step; all waves then apply the panel to the
    // trailing lower triangle.
    __device__ __forceinline__ bool cholesky_wave() const
    {
        double* m = M();
        double dd = 0.0;  // wave 0: FP64 running diagonal of row `lane` (mixed path)
        bool ok = true;
        if (wid == 0 && MIXED) dd = lane < NZ ? m[lane + lane * ldm] : 1.0;
        for (int p0 = 0; p0 < NZ; p0 += PW) {
            const int pw = min(PW, NZ - p0);
            if (wid == 0) {
                double r[PW];
#pragma unroll
                for (int q = 0; q < PW; ++q) {
                    r[q] = (lane >= p0 && lane < NZ && q < pw) ? m[lane + (p0 + q) * ldm] : 0.0;
                    if constexpr (MIXED) r[q] = rnd(r[q]);
                }
#pragma unroll
                for (int q = 0; q < PW; ++q) {
                    if (q >= pw) continue;
                    const int j = p0 + q;
                    const double piv = MIXED ? bcast(dd, j) : bcast(r[q], j);
                    ok = ok && (piv > 0.0);
                    const double inv = rsqrt_nr(piv);
                    const double lij = MIXED ? rnd(r[q] * inv) : r[q] * inv;
                    if (lane == j) {
                        dv()[j] = inv;
                        r[q] = piv * inv;
                    } else if (lane > j) {
                        r[q] = lij;
                        if constexpr (MIXED) dd -= lij * lij;
                    } else {
                        r[q] = 0.0;
                    }
                    // rank-1 update of the rest of the panel; column entries
                    // come from the lanes that hold them (readlane)
#pragma unroll
                    for (int q2 = q + 1; q2 < PW; ++q2)
                        if (q2 < pw) r[q2] = (double)((TS)r[q2] - (TS)lij * (TS)bcast(lij, p0 + q2));
                }
                if (lane < NZ) {
#pragma unroll
                    for (int q = 0; q < PW; ++q)
                        if (q < pw) m[lane + (p0 + q) * ldm] = r[q];
                }
            }
            __syncthreads();
            // trailing update of rows/columns p1.. with the panel
            const int p1 = p0 + pw;
            const int nt = NZ - p1;
            if (nt > 0) {
                mma_tn(m + p1 + p0 * ldm, ldm, 1, m + p1 + p0 * ldm, ldm, 1, nt, nt, pw, m + p1 + p1 * ldm, ldm, -1,
                       true);
                __syncthreads();
            }
        }
        if (wid == 0 && lane == 0) flag()[0] = 1.0;
        __syncthreads();
        if (wid == 0 && !ok && lane == 0) flag()[0] = 0.0;
        __syncthreads();
        return flag()[0] != 0.0;
    }

    __device__ __forceinline__ bool cholesky() const
    {
        if constexpr (!GL) return cholesky_wave();
        double* m = M();
        double* dd = ddv();
        double* lb = l11();
        bool ok = true;
        if constexpr (MIXED) {
            for (int i = opq(tid); i < NZ; i += BT) dd[i] = m[i + i * ldm];
            __syncthreads();
        }
        for (int p0 = 0; p0 < NZ; p0 += PW) {
            const int pw = min(PW, NZ - p0);
            const int p1 = p0 + pw;
            // diagonal block on wave 0: lane q holds row p0 + q
            if (wid == 0) {
                const bool act = lane < pw;
                const int i = p0 + min(lane, pw - 1);
                double r[PW];
#pragma unroll
                for (int q = 0; q < PW; ++q) {
                    const double v = m[i + (p0 + min(q, pw - 1)) * ldm];
                    r[q] = (act && q < pw) ? (MIXED ? rnd(v) : v) : 0.0;
                }
                double d = (MIXED && act) ? dd[i] : 1.0;
#pragma unroll
                for (int q = 0; q < PW; ++q) {
                    if (q >= pw) continue;
                    const double piv = MIXED ? bcast(d, q) : bcast(r[q], q);
                    ok = ok && (piv > 0.0);
                    const double inv = rsqrt_nr(piv);
                    const double lij = MIXED ? rnd(r[q] * inv) : r[q] * inv;
                    if (lane == q) {
                        dv()[p0 + q] = inv;
                        r[q] = piv * inv;
                    } else if (lane > q) {
                        r[q] = lij;
                        if constexpr (MIXED) d -= lij * lij;
                    } else {
                        r[q] = 0.0;
                    }
#pragma unroll
                    for (int q2 = q + 1; q2 < PW; ++q2)
                        if (q2 < pw) r[q2] = (double)((TS)r[q2] - (TS)lij * (TS)bcast(lij, q2));
                }
                if (act) {
#pragma unroll
                    for (int q = 0; q < PW; ++q)
                        if (q < pw) {
                            m[i + (p0 + q) * ldm] = r[q];
                            lb[lane + q * PW] = r[q];
                        }
                    if constexpr (MIXED) dd[i] = d;
                }
            }
            __syncthreads();
            // rows below the block: L21 = M21 L11^{-T}, one row per thread;
            // rows above it get zeros in the panel columns
            for (int i = opq(tid); i < NZ; i += BT) {
                if (i < p0) {
                    for (int q = 0; q < pw; ++q) m[i + (p0 + q) * ldm] = 0.0;
                    continue;
                }
                if (i < p1) continue;
                double r[PW];
#pragma unroll
                for (int q = 0; q < PW; ++q) {
                    const double v = m[i + (p0 + min(q, pw - 1)) * ldm];
                    r[q] = MIXED ? rnd(v) : v;
                }
                double d = MIXED ? dd[i] : 0.0;
#pragma unroll
                for (int q = 0; q < PW; ++q) {
                    if (q >= pw) continue;
                    TS acc = (TS)r[q];
#pragma unroll
                    for (int c = 0; c < q; ++c) acc -= (TS)r[c] * (TS)lb[q + c * PW];
                    r[q] = MIXED ? rnd((double)acc * dv()[p0 + q]) : (double)acc * dv()[p0 + q];
                    if constexpr (MIXED) d -= r[q] * r[q];
                }
#pragma unroll
                for (int q = 0; q < PW; ++q)
                    if (q < pw) m[i + (p0 + q) * ldm] = r[q];
                if constexpr (MIXED) dd[i] = d;
            }
            __syncthreads();
            // trailing update of rows/columns p1.. with the panel
            const int nt = NZ - p1;
            if (nt > 0) {
                mma_tn(m + p1 + p0 * ldm, ldm, 1, m + p1 + p0 * ldm, ldm, 1, nt, nt, pw, m + p1 + p1 * ldm, ldm, -1,
                       true);
                __syncthreads();
            }
        }
        if (wid == 0 && lane == 0) flag()[0] = ok ? 1.0 : 0.0;
        __syncthreads();
        const bool res = flag()[0] != 0.0;
        __syncthreads();
        return res;
    }

    // Array algorithm (Section 4.2, modes robust and balance): with M holding
    // L, the Cholesky factor of Phi (zero strict upper part), and V the rows
    // [U; sqrt(w) G] (rows r0.. of V), Householder reflections of the array
    // [L'; V] leave an upper-triangular R with R'R = Phi + V'V, i.e. the factor
    // of the normal matrix, without forming V'V.  Reflection j takes the
    // column j of V into R(j, j) (beta = +norm, so the diagonal stays
    // positive; v0 computed without cancellation when R(j, j) > 0) and is
    // applied to the columns k > j.  L = R' is written back into M (lower
    // part) and 1/L_jj into dv.  Threads: column k = t / RG with RG threads
    // (a power of two, lanes of one wave) summing interleaved rows; each
    // reflection takes one barrier, its vector in one of two LDS buffers.
    // Every thread calls it.
    __device__ __forceinline__ void qr_update(int r0) const
    {
        double* m = M();
        double* v = V();
        double* rb = l11();  // two buffers of NV + 2 doubles: v / v0 per row, then tau
        const int nvr = NV - r0;
        int rg = 1;
        while (rg * 2 * NZ <= BT && rg < 64) rg *= 2;
        const int k = tid / rg, q = tid % rg;
        const bool act = k < NZ;
        // column 0's reflection: its threads hold the squared norm of V(:, 0)
        auto colnorm = [&](int c) {
            double sq = 0.0;
            if (act && k == c)
                for (int r = q; r < nvr; r += rg) {
                    const double x = v[(r0 + r) + c * ldv];
                    sq += x * x;
                }
            for (int o = 1; o < rg; o <<= 1) sq += __shfl_xor(sq, o);
            return sq;
        };
        double sg = colnorm(0);
        for (int j = 0; j < NZ; ++j) {
            double* buf = rb + (j & 1) * (NV + 2);
            if (act && k == j) {
                // reflection j from R(j, j) = L(j, j) and V(:, j)
                const double a = m[j + j * ldm];
                const double beta = sqrt(a * a + sg);
                const double v0 = a <= 0.0 ? a - beta : -sg / (a + beta);
                const double tau = sg == 0.0 ? 0.0 : 2.0 * v0 * v0 / (sg + v0 * v0);
                const double iv0 = sg == 0.0 ? 0.0 : 1.0 / v0;
                for (int r = q; r < nvr; r += rg) buf[r] = v[(r0 + r) + j * ldv] * iv0;
                if (q == 0) {
                    buf[NV] = tau;
                    m[j + j * ldm] = beta;
                }
            }
            __syncthreads();
            if (act && k > j) {
                const double tau = buf[NV];
                double sd = 0.0;
                for (int r = q; r < nvr; r += rg) sd += buf[r] * v[(r0 + r) + k * ldv];
                for (int o = 1; o < rg; o <<= 1) sd += __shfl_xor(sd, o);
                double* rjk = m + k + j * ldm;  // R(j, k) = L(k, j)
                sd += *rjk;
                const double ts = tau * sd;
                for (int r = q; r < nvr; r += rg) v[(r0 + r) + k * ldv] -= ts * buf[r];
                if (q == 0) *rjk -= ts;  // the column's threads are lanes of one wave: all read it above
            }
            if (j + 1 < NZ) sg = colnorm(j + 1);
        }
        __syncthreads();
        for (int i = opq(tid); i < NZ; i += BT) dv()[i] = 1.0 / m[i + i * ldm];
        __syncthreads();
    }

    // ------------------------------------------------------------------
    // Global-memory mode with the stage matrix in registers (stage blocks up
    // to 160, FP64 and mixed builds): the lower 16 x 16 tiles of
    // M = Phi + V'V are matrix-core accumulators spread over the four waves
    // (tile t in row-major lower order belongs to wave t mod 4), so the
    // products and the Cholesky factorization never go through global memory
    // until the factor itself is written out.
    //   * M starts as H (read from the data record) plus the box weights;
    //   * V is formed 16 rows at a time in LDS: rows of U = L_{n+1}' F from
    //     chunks of 16 rows of L_{n+1} and F staged in LDS (the next chunk's
    //     loads in flight while the current one is multiplied), then the rows
    //     sqrt(w) G; each panel updates every tile of M (M += Vp' Vp);
    //   * right-looking Cholesky by 16-column panels: the diagonal tile is
    //     factored on wave 0 (one row per lane), the tiles below it are
    //     solved against it one row per thread in LDS, the panel column is
    //     written to the stage's factor record, and the trailing tiles are
    //     updated on the matrix cores from that LDS panel.
    // Mixed path: FP32 operands and accumulators, the running diagonal of
    // every row in FP64 (the pivots) as in the other factorizations.
    // ------------------------------------------------------------------
    static constexpr int RT = 14;  // tiles per wave: 4 x 14 >= 55, the lower tiles of a 160-wide block
    // sequential triangular sweeps of wave 0 (forward and backward
    // substitution with a diagonal block): factor entries loaded PCH columns
    // at a time, ahead of the dependent steps.  The global-memory mode reads
    // the factor from HBM/L2 (16 at a time: 3 % on the large-stage batch);
    // the LDS-resident builds load one per step (16 at a time cost them
    // registers and 6 % on the uneven batch).
    static constexpr int PCH = GL ? 16 : 1;
    static constexpr bool TILES = GL && !ROBUST;
    using V4 = TS __attribute__((ext_vector_type(4)));

    __device__ __forceinline__ static V4 mfma4(TS a, TS b, V4 c)
    {
        if constexpr (MIXED)
            return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
        else
            return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // v, opaque to the optimizer: lane offsets derived from it inside a loop
    // are recomputed there instead of being held in registers across it
    __device__ __forceinline__ static int opaque(int v)
    {
        asm volatile("" : "+v"(v));
        return v;
    }
    // tile row of accumulator register r of this lane (column: lane % 16)
    __device__ __forceinline__ int arow(int r) const { return MIXED ? 4 * (lane >> 4) + r : 4 * r + (lane >> 4); }
    // (balance build: not in an iteration factored with the array
    // algorithm, which needs V in the stage's workspace block)
    __device__ __forceinline__ bool use_tiles(bool qr) const { return TILES && NZ <= 160 && !(BALANCE && qr); }

    // Factor the stage matrix of stage n (n < N: with the rows of U; NG > 0:
    // with the rows sqrt(w) G) into the factor record cM; 1/L_ii to dv.
    // Returns false (in every thread) when a pivot is not positive.
    __device__ __forceinline__ bool factor_tiles(int n, const double* hd) const
    {
        const int TMt = (NZ + 15) >> 4, NTt = TMt * (TMt + 1) / 2;
        const int l16 = lane & 15, lk = lane >> 4;
        const int ldu = S.ldu;
        double* up = blds() + S.oUp;  // Vp[k][j], k < 16, ld ldu
        double* lp = blds() + S.oPn;  // panel column below the diagonal tile: [row][q], ld 17
        double* dg = blds() + S.oDg;  // diagonal tile [row][q], ld 17
        double* ca = blds() + S.oCA;  // chunk of L_{n+1}: [k][i], k < 16, ld 17
        double* cb = blds() + S.oCB;  // chunk of F: [k][j], k < 16, ld ldu
        double* dd = ddv();           // running FP64 diagonal (mixed path)
        const double* wv = wsv();
        V4 acc[RT];
        // tiles of this wave (wave-uniform: scalar registers)
        const int w0 = __builtin_amdgcn_readfirstlane(wid);
        int tI[RT], tJ[RT];
#pragma unroll
        for (int s = 0; s < RT; ++s) {
            const int t = w0 + 4 * s;
            int ti = 0;
            while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
            tI[s] = t < NTt ? ti : -1;
            tJ[s] = t < NTt ? t - ti * (ti + 1) / 2 : -1;
        }
        // ---- U = L_{n+1}' F, 16 rows at a time, to the stage's V block
        // (row-major, rows 0 .. NX-1, ld NZ), before the stage matrix takes
        // the accumulators: the two are never live together ----
        const int npu = n < N ? (NX + 15) >> 4 : 0, npg = (NG + 15) >> 4;
        constexpr int KC = 16;                         // rows of L_{n+1} and F per chunk
        constexpr int CA = 16 * KC / BT;               // L_{n+1} chunk elements per thread
        constexpr int CB = (KC * 160 + BT - 1) / BT;  // F chunk elements per thread
        double* const vw = cV;
        for (int pnl = 0; pnl < npu; ++pnl) {
            // U rows 16 pnl ..: U(r, j) = sum_{l >= r} L(l, r) F(l, j); output
            // tile columns jt = wid, wid + 4, wid + 8 of the panel
            V4 ua[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) ua[q] = V4{0, 0, 0, 0};
            const int l_first = 16 * pnl;
            const int nch = (NX - l_first + KC - 1) / KC;
            double pa[CA], pb[CB];
            // element idx of a chunk: row kk = idx mod KC (contiguous in
            // the column-major records), column idx / KC
            auto fetch_chunk = [&](int l0) {
#pragma unroll
                for (int e = 0; e < CA; ++e) {
                    const int idx = tid + BT * e;
                    const int kk = idx % KC, i = idx / KC;
                    const int l = l0 + kk;
                    pa[e] = (l < NX && l_first + i < NX) ? cLx[l + (l_first + i) * ldx] : 0.0;
                }
#pragma unroll
                for (int e = 0; e < CB; ++e) {
                    const int idx = tid + BT * e;
                    const int kk = idx % KC, j = idx / KC;
                    const int l = l0 + kk;
                    pb[e] = (j < NZ && l < NX) ? cF[l + j * ldf] : 0.0;
                }
            };
            fetch_chunk(l_first);
            for (int c = 0; c < nch; ++c) {
                __syncthreads();  // the previous chunk has been read
#pragma unroll
                for (int e = 0; e < CA; ++e) {
                    const int idx = tid + BT * e;
                    ca[(idx % KC) * 17 + idx / KC] = pa[e];
                }
#pragma unroll
                for (int e = 0; e < CB; ++e) {
                    const int idx = tid + BT * e;
                    const int kk = idx % KC, j = idx / KC;
                    if (j < NZ) cb[kk * ldu + j] = pb[e];
                }
                __syncthreads();
                if (c + 1 < nch) fetch_chunk(l_first + KC * (c + 1));
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const int jt = w0 + 4 * q;
                    if (jt < TMt) {
                        const int j = min(16 * jt + l16, NZ - 1);
#pragma unroll
                        for (int k4 = 0; k4 < KC / 4; ++k4) {
                            const int kk = 4 * k4 + lk;
                            const TS a = (TS)ca[kk * 17 + l16];
                            const TS b = (16 * jt + l16 < NZ) ? (TS)cb[kk * ldu + j] : (TS)0;
                            ua[q] = mfma4(a, b, ua[q]);
                        }
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int jt = w0 + 4 * q;
                if (jt < TMt) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * pnl + arow(r), j = 16 * jt + l16;
                        if (j < NZ && row < NX) vw[row * NZ + j] = (double)ua[q][r];
                    }
                }
            }
        }
        // ---- M = H + diag(box weights) + reg I ----
#pragma unroll
        for (int s = 0; s < RT; ++s) {
            const int t = w0 + 4 * s;
            const int ti = tI[s], tj = tJ[s];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * ti + arow(r), c = 16 * tj + l16;
                double v = 0.0;
                if (t < NTt) {
                    if (row < NZ && c < NZ) v = hd[row + c * NZ];
                    if (row == c) v += row < NZ ? wv[row] + P.reg_prim : 1.0;
                }
                acc[s][r] = (TS)v;
            }
        }
        if constexpr (MIXED) {
            // FP64 running diagonal (the pivots): M_ii in FP64, the squares of
            // V's columns added panel by panel below
            for (int i = opq(tid); i < NZ; i += BT) dd[i] = hd[i + i * NZ] + wv[i] + P.reg_prim;
        }
        // ---- M += V'V, 16 rows of V at a time through LDS ----
        for (int pnl = 0; pnl < npu + npg; ++pnl) {
            // the previous panel's products are done with up (and U is stored)
            __syncthreads();
            // all of a thread's loads issued before its LDS stores (element
            // offsets recomputed per panel, not held across the loop)
            constexpr int EV = (16 * 160 + BT - 1) / BT;
            const int tdo = opaque(tid);
            double vv[EV];
            if (pnl < npu) {
                const int r0 = 16 * pnl;
#pragma unroll
                for (int t = 0; t < EV; ++t) {
                    const int e = tdo + BT * t, kk = e / NZ, j = e % NZ, row = r0 + kk;
                    vv[t] = (e < 16 * NZ && row < NX) ? vw[row * NZ + j] : 0.0;
                }
            } else {
                // rows sqrt(w) G of general rows 16 (pnl - npu) ..
                const int g0 = 16 * (pnl - npu);
#pragma unroll
                for (int t = 0; t < EV; ++t) {
                    const int e = tdo + BT * t, kk = e / NZ, j = e % NZ, g = g0 + kk;
                    vv[t] = (e < 16 * NZ && g < NG) ? sqrt(wv[NZ + g]) * cG[g + j * ldg] : 0.0;
                }
            }
#pragma unroll
            for (int t = 0; t < EV; ++t) {
                const int e = tdo + BT * t;
                if (e < 16 * NZ) up[(e / NZ) * ldu + e % NZ] = vv[t];
            }
            __syncthreads();
            if constexpr (MIXED) {
                for (int i = opq(tid); i < NZ; i += BT) {
                    double sq = 0.0;
#pragma unroll
                    for (int kk = 0; kk < 16; ++kk) sq += up[kk * ldu + i] * up[kk * ldu + i];
                    dd[i] += sq;
                }
            }
            // one k-step over all tiles at a time (the same order of products
            // in every tile), so that the operands held in registers stay
            // those of one k-step
            const int l16o = opaque(l16), lko = opaque(lk);
#pragma unroll
            for (int s = 0; s < RT; ++s) {
                if (tI[s] >= 0) {
                    const int ti = tI[s], tj = tJ[s];
                    const int i = min(16 * ti + l16o, NZ - 1), j = min(16 * tj + l16o, NZ - 1);
                    const bool iv = 16 * ti + l16o < NZ, jv = 16 * tj + l16o < NZ;
#pragma unroll
                    for (int k4 = 0; k4 < 4; ++k4) {
                        const int kk = 4 * k4 + lko;
                        const TS a = iv ? (TS)up[kk * ldu + i] : (TS)0;
                        const TS b = jv ? (TS)up[kk * ldu + j] : (TS)0;
                        acc[s] = mfma4(a, b, acc[s]);
                    }
                }
            }
        }
        // ---- Cholesky by 16-column panels ----
        bool ok = true;
        double* fm = cM;
        for (int p = 0; p < TMt; ++p) {
            const int l16o = opaque(l16), lko = opaque(lk);
            __syncthreads();  // the previous panel's trailing products are done with dg / pn
            // the tiles of column p to LDS
#pragma unroll
            for (int s = 0; s < RT; ++s) {
                if (tI[s] >= 0) {
                    const int ti = tI[s], tj = tJ[s];
                    if (tj == p) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int rr = MIXED ? 4 * lko + r : 4 * r + lko;
                            if (ti == p) dg[rr * 17 + l16o] = (double)acc[s][r];
                            else if (16 * ti + rr < NZ) lp[(16 * ti + rr) * 17 + l16o] = (double)acc[s][r];
                        }
                    }
                }
            }
            __syncthreads();
            const int p0 = 16 * p, pw = min(16, NZ - p0);
            // diagonal tile on wave 0: lane q holds row p0 + q
            if (wid == 0) {
                double r[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) r[q] = (lane < 16) ? dg[lane * 17 + q] : 0.0;
                double d = (MIXED && lane < pw) ? dd[p0 + lane] : 1.0;
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    if (q >= pw) continue;
                    const double piv = MIXED ? bcast(d, q) : bcast(r[q], q);
                    ok = ok && (piv > 0.0);
                    const double inv = rsqrt_nr(piv);
                    const double lij = MIXED ? rnd(r[q] * inv) : r[q] * inv;
                    if (lane == q) {
                        dv()[p0 + q] = inv;
                        r[q] = piv * inv;
                    } else if (lane > q) {
                        r[q] = lij;
                        if constexpr (MIXED) d -= lij * lij;
                    } else {
                        r[q] = 0.0;
                    }
#pragma unroll
                    for (int q2 = q + 1; q2 < 16; ++q2)
                        if (q2 < pw) r[q2] = (double)((TS)r[q2] - (TS)lij * (TS)bcast(lij, q2));
                }
                if (lane < 16) {
#pragma unroll
                    for (int q = 0; q < 16; ++q) dg[lane * 17 + q] = r[q];
                }
            }
            __syncthreads();
            // rows below: L21 = M21 L11^{-T}, one row per thread
            for (int i = p0 + 16 + opq(tid); i < NZ; i += BT) {
                double r[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) r[q] = MIXED ? rnd(lp[i * 17 + q]) : lp[i * 17 + q];
                double d = MIXED ? dd[i] : 0.0;
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    if (q >= pw) continue;
                    TS a = (TS)r[q];
#pragma unroll
                    for (int c = 0; c < q; ++c) a -= (TS)r[c] * (TS)dg[q * 17 + c];
                    r[q] = MIXED ? rnd((double)a * dv()[p0 + q]) : (double)a * dv()[p0 + q];
                    if constexpr (MIXED) d -= r[q] * r[q];
                }
#pragma unroll
                for (int q = 0; q < 16; ++q) lp[i * 17 + q] = r[q];
                if constexpr (MIXED) dd[i] = d;
            }
            __syncthreads();
            // panel column to the factor record (zeros above the diagonal tile)
            for (int i = opq(tid); i < NZ; i += BT) {
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    if (q >= pw) continue;
                    double v = 0.0;
                    if (i >= p0 + 16) v = lp[i * 17 + q];
                    else if (i >= p0 && i - p0 >= q) v = dg[(i - p0) * 17 + q];
                    fm[i + (p0 + q) * NZ] = v;
                }
            }
            // trailing tiles (i, j), p < j <= i: M_ij -= L_ip L_jp'
#pragma unroll
            for (int s = 0; s < RT; ++s) {
                if (tI[s] >= 0) {
                    const int ti = tI[s], tj = tJ[s];
                    if (tj > p) {
                        const int i = 16 * ti + l16o, j = 16 * tj + l16o;
                        const bool iv = i < NZ, jv = j < NZ;
#pragma unroll
                        for (int k4 = 0; k4 < 4; ++k4) {
                            const int kk = 4 * k4 + lko;
                            const TS a = iv ? -(TS)lp[i * 17 + kk] : (TS)0;
                            const TS b = jv ? (TS)lp[j * 17 + kk] : (TS)0;
                            acc[s] = mfma4(a, b, acc[s]);
                        }
                    }
                }
            }
        }
        if (wid == 0 && lane == 0) flag()[0] = 1.0;
        __syncthreads();
        if (wid == 0 && !ok && lane == 0) flag()[0] = 0.0;
        __syncthreads();
        const bool res = flag()[0] != 0.0;
        __syncthreads();
        return res;
    }

    // Forward substitution with the (u, u) block of the factor in M (u
    // columns): wave 0 solves y = L_uu^{-1} m_u (rows j < NU, one per lane,
    // di = 1/L_jj), then every thread of rows NU <= i < NZ forms
    // p_i = m_i - L_xu(i, :) y.  mv is this thread's row value (row tid);
    // returns y_tid or p_tid.  Every thread calls it; uses ev() as scratch.
    __device__ __forceinline__ double fwd_subst_u(double mv, double di) const
    {
        const double* m = M();
        double* yv = ev();
        mv = rnd(mv);
        if (wid == 0) {
            double v = mv;
            // PCH columns of the factor at a time, their loads issued
            // together ahead of the dependent steps
            for (int j0 = 0; j0 < NU; j0 += PCH) {
                double lc[PCH];
#pragma unroll
                for (int q = 0; q < PCH; ++q) {
                    const int j = j0 + q;
                    lc[q] = (j < NU && lane > j && lane < NU) ? m[lane + j * ldm] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < PCH; ++q) {
                    const int j = j0 + q;
                    if (j >= NU) break;
                    const double y = rnd(bcast(v, j) * bcast(di, j));
                    if (lane == j) v = y;
                    else if (lane > j && lane < NU) v = (double)((TS)v - (TS)lc[q] * (TS)y);
                }
            }
            if (lane < NU) yv[lane] = v;
        }
        __syncthreads();
        const int i = opq(tid);
        if (i < NU) return yv[i];
        if (i < NZ) return (double)((TS)mv - dot<TS>(m + i, ldm, yv, 1, NU));
        return 0.0;
    }

    // Blocked triangular solves with a lower-triangular n x n block L (leading
    // dimension ld) and 1/L_ii in di (LDS), on a vector x in LDS: wave 0
    // solves each 64-row diagonal block (one row per lane), all threads
    // update the remaining rows.  Every thread calls them.
    __device__ __forceinline__ void trsv_lower(const double* L, int ld, int n, double* x, const double* di) const
    {
        for (int b0 = 0; b0 < n; b0 += 64) {
            const int bn = min(64, n - b0);
            if (wid == 0) {
                double v = lane < bn ? rnd(x[b0 + lane]) : 0.0;
                // PCH columns at a time, their loads issued together
                for (int c0 = 0; c0 < bn; c0 += PCH) {
                    double lc[PCH], dc[PCH];
#pragma unroll
                    for (int q = 0; q < PCH; ++q) {
                        const int c = c0 + q;
                        lc[q] = (c < bn && lane > c && lane < bn) ? L[(b0 + lane) + (b0 + c) * ld] : 0.0;
                        dc[q] = c < bn ? di[b0 + c] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < PCH; ++q) {
                        const int c = c0 + q;
                        if (c >= bn) break;
                        const double y = rnd(bcast(v, c) * dc[q]);
                        if (lane == c) v = y;
                        else if (lane > c && lane < bn) v = (double)((TS)v - (TS)lc[q] * (TS)y);
                    }
                }
                if (lane < bn) x[b0 + lane] = v;
            }
            __syncthreads();
            for (int i = b0 + bn + opq(tid); i < n; i += BT)
                x[i] = (double)((TS)x[i] - dot<TS>(L + i + b0 * ld, ld, x + b0, 1, bn));
            __syncthreads();
        }
    }

    __device__ __forceinline__ void trsv_lower_t(const double* L, int ld, int n, double* x, const double* di) const
    {
        for (int b1 = n; b1 > 0; b1 -= 64) {
            const int b0 = max(0, b1 - 64), bn = b1 - b0;
            if (wid == 0) {
                double v = lane < bn ? rnd(x[b0 + lane]) : 0.0;
                // PCH rows of L at a time (from the last), their loads
                // issued together
                for (int c1 = bn; c1 > 0; c1 -= PCH) {
                    double lc[PCH], dc[PCH];
#pragma unroll
                    for (int q = 0; q < PCH; ++q) {
                        const int c = c1 - 1 - q;
                        lc[q] = (c >= 0 && lane < c) ? L[(b0 + c) + (b0 + lane) * ld] : 0.0;
                        dc[q] = c >= 0 ? di[b0 + c] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < PCH; ++q) {
                        const int c = c1 - 1 - q;
                        if (c < 0) break;
                        const double xv = rnd(bcast(v, c) * dc[q]);
                        if (lane == c) v = xv;
                        else if (lane < c) v = (double)((TS)v - (TS)lc[q] * (TS)xv);
                    }
                }
                if (lane < bn) x[b0 + lane] = v;
            }
            __syncthreads();
            for (int i = opq(tid); i < b0; i += BT)
                x[i] = (double)((TS)x[i] - dot<TS>(L + b0 + i * ld, 1, x + b0, 1, bn));
            __syncthreads();
        }
    }

    // ==================================================================
    // Pass A: apply the previous step (optional), residuals at the iterate,
    // barrier terms, factorization and the right-hand-side sweep for r_m =
    // lam.*t - shift.  Returns whether every pivot was positive.
    // ==================================================================
    // With absf (absolute formulation, Section 3.2) the right-hand side is
    // built from the data alone, -[g; b; d; r_m - 2 Lam T e]; the residual
    // products are skipped and their norms not formed.
    __device__ __forceinline__ bool passA(bool upd, double alpha, double shift, bool factor, bool absf, bool qr,
                                          double& o_g, double& o_b, double& o_d, double& o_m, double& o_lt) const
    {
        double mg = 0.0, mb = 0.0, md = 0.0, mm = 0.0, slt = 0.0;
        bool fact_ok = true;
        Pre pre;
        seg_hfg(pre, N);
        fetch(pre);
        for (int n = N; n >= 0; --n) {
            const int cur = n & 1, nxt = cur ^ 1;
            commit(pre, M(), F(), G());
            stage_A(n, qr);
            const double* d = Dp(n);
            double* ir = Ip(n);
            double* w = Wp(n);
            // row j = tid (< NZ), state row i = tid (< NX), slot c = tid (< NC)
            const int j = opq(tid);
            double g = 0.0, zz = 0.0, dz = 0.0, b = 0.0, pi = 0.0, dpi = 0.0;
            if (j < NZ) {
                g = d[Lo.D_g + j];
                zz = ir[Lo.I_z + j];
                if (upd) dz = w[Lo.W_dz + j];
            }
            if (j < NX) {
                if (n < N) b = d[Lo.D_b + j];
                pi = ir[Lo.I_pi + j];
                if (upd && n > 0) dpi = w[Lo.W_dpi + j];
            }
            double m = 0.0, lo = 0.0, hi = 0.0, ll = 0.0, lu = 0.0, tl = 0.0, tu = 0.0;
            if (j < NC) {
                slot_bounds(d, j, m, lo, hi);
                ll = ir[Lo.I_ll + j];
                lu = ir[Lo.I_lu + j];
                tl = ir[Lo.I_tl + j];
                tu = ir[Lo.I_tu + j];
                if (upd && m != 0.0) {
                    ll = fmax(ll + alpha * w[Lo.W_dll + j], P.lam_min);
                    lu = fmax(lu + alpha * w[Lo.W_dlu + j], P.lam_min);
                    tl = fmax(tl + alpha * w[Lo.W_dtl + j], P.t_min);
                    tu = fmax(tu + alpha * w[Lo.W_dtu + j], P.t_min);
                }
            }
            // slack pair of a soft slot and the multipliers and slacks of its
            // bounds, after the step (clamped like the rows)
            double sm = 0.0, sl = 0.0, su = 0.0, lsl = 0.0, lsu = 0.0, tsl = 0.0, tsu = 0.0;
            if constexpr (SOFT) {
                if (j < NC) sm = d[Lo.D_sm + j];
                if (sm != 0.0) {
                    sl = ir[Lo.I_sl + j];
                    su = ir[Lo.I_su + j];
                    lsl = ir[Lo.I_lsl + j];
                    lsu = ir[Lo.I_lsu + j];
                    tsl = ir[Lo.I_tsl + j];
                    tsu = ir[Lo.I_tsu + j];
                    if (upd) {
                        sl += alpha * w[Lo.W_dsl + j];
                        su += alpha * w[Lo.W_dsu + j];
                        lsl = fmax(lsl + alpha * w[Lo.W_dlsl + j], P.lam_min);
                        lsu = fmax(lsu + alpha * w[Lo.W_dlsu + j], P.lam_min);
                        tsl = fmax(tsl + alpha * w[Lo.W_dtsl + j], P.t_min);
                        tsu = fmax(tsu + alpha * w[Lo.W_dtsu + j], P.t_min);
                    }
                }
            }
            if (n > 0) {
                seg_hfg(pre, n - 1);
                fetch(pre);  // next stage of the sweep
            }
            if (upd) {
                zz += alpha * dz;
                if (n > 0) pi += alpha * dpi;
            }
            if (n == N && j < NX) {
                xn(nxt)[j] = 0.0;
                pin(nxt)[j] = 0.0;
                pn(nxt)[j] = 0.0;
            }
            if (j < NZ) z()[j] = zz;
            if (j < NX) t2()[j] = pi;
            if (j >= NZ && j < NC) t1()[j - NZ] = m * (ll - lu);
            __syncthreads();

            // r_g = H z + g + F' pi_{n+1} - [0; pi_n] - C' lam
            double rg = 0.0;
            if (absf) {
                if (j < NZ) rg = g;
            } else if (j < NZ) {
                const double* mh = use_tiles(qr) ? cH : M();
                const double* zv = z();
                double acc = g + dot<double>(mh + j, ldm, zv, 1, NZ);
                if (n < N) acc += dot<double>(F() + j * ldf, 1, pin(nxt), 1, NX);
                if (j >= NU) acc -= t2()[j - NU];
                acc -= m * (ll - lu);
                acc -= dot<double>(G() + j * ldg, 1, t1(), 1, NG);
                rg = acc;
                mg = nmax(mg, fabs(rg));
            }
            // r_b = F z + b - x_{n+1}
            double rb = 0.0;
            if (absf) {
                if (n < N && j < NX) rb = b;
            } else if (n < N && j < NX) {
                const double acc = b + dot<double>(F() + j, ldf, z(), 1, NZ);
                rb = acc - xn(nxt)[j];
                mb = nmax(mb, fabs(rb));
            }
            // r_d, complementarity, barrier weights, reduced-gradient terms
            double rdl = 0.0, rdu = 0.0;
            if (j < NC) {
                double e = 0.0, wsum = 0.0;
                if (m != 0.0) {
                    if (absf) {
                        rdl = lo;
                        rdu = -hi;
                    } else {
                        double gz;
                        if (j < NZ) {
                            gz = zz;
                        } else {
                            gz = dot<double>(G() + (j - NZ), ldg, z(), 1, NZ);
                        }
                        rdl = -gz + tl + lo;
                        rdu = gz + tu - hi;
                        if constexpr (SOFT) {
                            // a soft row holds its slack: G z + s^l, -G z + s^u
                            rdl -= sl;
                            rdu -= su;
                        }
                        md = nmax(md, nmax(fabs(rdl), fabs(rdu)));
                    }
                    const double a1 = ll * tl, a2 = lu * tu;
                    mm = nmax(mm, nmax(a1, a2));
                    slt += a1 + a2;
                    const double itl = rcp_nr(tl), itu = rcp_nr(tu);
                    const double wl = ll * itl, wu = lu * itu;
                    wsum = wl + wu;
                    // r_m / t, with r_m = lam t - shift (delta) or -lam t - shift (absolute)
                    const double ml = absf ? -ll - shift * itl : ll - shift * itl;
                    const double mu_ = absf ? -lu - shift * itu : lu - shift * itu;
                    e = (wl * rdl - ml) - (wu * rdu - mu_);
                    if constexpr (SOFT) {
                        if (sm != 0.0) {
                            // slack rows: stationarity r_s = Z s + z - lam_row -
                            // lam_s, bound rows rd_s = -s + t_s + ls, their
                            // complementarity; then the slack elimination
                            const double Zl = d[Lo.D_Zl + j], Zu = d[Lo.D_Zu + j];
                            const double rsl = Zl * sl + d[Lo.D_zl + j] - ll - lsl;
                            const double rsu = Zu * su + d[Lo.D_zu + j] - lu - lsu;
                            const double rdsl = -sl + tsl + d[Lo.D_lls + j];
                            const double rdsu = -su + tsu + d[Lo.D_lus + j];
                            mg = nmax(mg, nmax(fabs(rsl), fabs(rsu)));
                            md = nmax(md, nmax(fabs(rdsl), fabs(rdsu)));
                            const double a3 = lsl * tsl, a4 = lsu * tsu;
                            mm = nmax(mm, nmax(a3, a4));
                            slt += a3 + a4;
                            const double itsl = rcp_nr(tsl), itsu = rcp_nr(tsu);
                            const double wsl = lsl * itsl, wsu = lsu * itsu;
                            const double esl = wsl * rdsl - (lsl - shift * itsl);
                            const double esu = wsu * rdsu - (lsu - shift * itsu);
                            const double iDl = rcp_nr(Zl + wl + wsl), iDu = rcp_nr(Zu + wu + wsu);
                            const double el = wl * rdl - ml, eu = wu * rdu - mu_;
                            const double gl = rsl - el - esl, gu = rsu - eu - esu;
                            e = (el + wl * gl * iDl) - (eu + wu * gu * iDu);
                            wsum = wl * (Zl + wsl) * iDl + wu * (Zu + wsu) * iDu;
                            w[Lo.W_rsl + j] = rsl;
                            w[Lo.W_rsu + j] = rsu;
                            w[Lo.W_rdsl + j] = rdsl;
                            w[Lo.W_rdsu + j] = rdsu;
                            if (upd) {
                                ir[Lo.I_sl + j] = sl;
                                ir[Lo.I_su + j] = su;
                                ir[Lo.I_lsl + j] = lsl;
                                ir[Lo.I_lsu + j] = lsu;
                                ir[Lo.I_tsl + j] = tsl;
                                ir[Lo.I_tsu + j] = tsu;
                            }
                        }
                    }
                }
                ev()[j] = e;
                wsv()[j] = wsum;
                if (upd && m != 0.0) {
                    ir[Lo.I_ll + j] = ll;
                    ir[Lo.I_lu + j] = lu;
                    ir[Lo.I_tl + j] = tl;
                    ir[Lo.I_tu + j] = tu;
                }
                w[Lo.W_rdl + j] = rdl;
                w[Lo.W_rdu + j] = rdu;
            }
            if (j < NX) rbv()[j] = rb;
            if (upd) {
                if (j < NZ) ir[Lo.I_z + j] = zz;
                if (j < NX && n > 0) ir[Lo.I_pi + j] = pi;
            }
            if (j < NZ) w[Lo.W_rg + j] = rg;
            if (n < N && j < NX) w[Lo.W_rb + j] = rb;
            __syncthreads();

            if (factor && use_tiles(qr)) {
                fact_ok = factor_tiles(n, cH) && fact_ok;
            } else if (factor) {
                // Phi = H + diag(box weights) + reg I ; V = [L_{n+1}' F ; sqrt(w_g) G]
                if (j < NZ) M()[j + j * ldm] += wsv()[j] + P.reg_prim;
                {
                    const double* gg = G();
                    const double* wv = wsv();
                    double* v = V();
                    for (int e = tid; e < NG * NZ; e += BT) {
                        const int r = e % NG, k = e / NG;
                        v[NX + r + k * ldv] = sqrt(wv[NZ + r]) * gg[r + k * ldg];
                    }
                }
                if (n < N) trmm_LtF();
                __syncthreads();
                // the array algorithm (robust build; balance build when this
                // iteration's Cholesky factors failed the accuracy check)
                // factors Phi + V'V without forming V'V
                const bool arr = ROBUST || (BALANCE && qr);
                if (!arr) {
                    if (n < N || NG > 0) syrk_VtV(n < N ? 0 : NX);
                    __syncthreads();
                }
                fact_ok = cholesky() && fact_ok;
                if (arr && (n < N || NG > 0)) qr_update(n < N ? 0 : NX);
            }
            if (factor) {

                // reduced gradient and cost-to-go terms
                double mv = 0.0;
                if (j < NZ) {
                    mv = rg - ev()[j] - dot<double>(G() + j * ldg, 1, ev() + NZ, 1, NG);
                }
                if (n < N) {
                    const double* L = Lx();
                    if (j < NX) t1()[j] = (double)dot<TS>(L + j + j * ldx, 1, rbv() + j, 1, NX - j);
                    __syncthreads();
                    if (j < NX) t2()[j] = (double)((TS)pn(nxt)[j] + dot<TS>(L + j, ldx, t1(), 1, j + 1));
                    __syncthreads();
                    if (j < NZ) mv = (double)((TS)mv + dot<TS>(F() + j * ldf, 1, t2(), 1, NX));
                }
                {
                    const double di = j < NZ ? dv()[j] : 0.0;
                    mv = fwd_subst_u(mv, di);
                    if (j < NZ) w[Lo.W_dinv + j] = di;
                    if (j < NU) w[Lo.W_yu + j] = mv;
                    else if (j < NZ) {
                        w[Lo.W_pv + j - NU] = mv;
                        pn(cur)[j - NU] = mv;
                    }
                }
                // factor to global memory; its (x, x) block becomes L_{n+1} of
                // the next stage of the sweep (in global-memory mode the
                // factor is already in its record and is read from there)
                if constexpr (!GL) {
                    const double* mf = M();
                    double* wl = w + Lo.W_L;
                    Walk q(NZ, tid);
                    for (int e = tid; e < NZ * NZ; e += BT) {
                        wl[e] = mf[q.r + q.c * ldm];
                        q.next();
                    }
                    double* L = Lx();
                    Walk qx(NX, tid);
                    for (int e = tid; e < NX * NX; e += BT) {
                        L[qx.r + qx.c * ldx] = mf[(NU + qx.r) + (NU + qx.c) * ldm];
                        qx.next();
                    }
                }
            }
            if (j >= NU && j < NZ) xn(cur)[j - NU] = zz;
            if (j < NX) pin(cur)[j] = pi;
            __syncthreads();
        }
        reduce4(mg, mb, md, mm, slt);
        o_g = mg;
        o_b = mb;
        o_d = md;
        o_m = mm;
        o_lt = slt;
        return fact_ok;
    }

    // slot values used by the right-hand-side sweeps: r_m (lower, upper) of
    // slot c per rmode
    __device__ __forceinline__ void slot_rm(int rmode, double shift, const double* w, int c, double ll, double lu,
                                            double tl, double tu, double& rml, double& rmu) const
    {
        if (rmode == RM_IR) {
            rml = w[Lo.W_irml + c];
            rmu = w[Lo.W_irmu + c];
            return;
        }
        rml = ll * tl - shift;
        rmu = lu * tu - shift;
        if (rmode == RM_CORRECTOR) {
            rml += w[Lo.W_all + c] * w[Lo.W_atl + c];
            rmu += w[Lo.W_alu + c] * w[Lo.W_atu + c];
        }
        if (ABS) {
            // absolute formulation: r_m - 2 lam t
            rml -= 2.0 * ll * tl;
            rmu -= 2.0 * lu * tu;
        }
    }

    // cost-to-go of the right-hand side: returns mv + F'(Lxx (Lxx' rb) + pn)
    // for row j, with Lxx(i, k) = xc[(NU + i) + k ldm] (xc: first x-column of
    // the next stage's factor) and rb, pn in LDS; every thread must call it
    __device__ __forceinline__ double cost_to_go_x(double mv, const double* xc, const double* pnv) const
    {
        const int j = opq(tid);
        if (j < NX) t1()[j] = (double)dot<TS>(xc + (NU + j) + j * ldm, 1, rbv() + j, 1, NX - j);
        __syncthreads();
        if (j < NX) t2()[j] = (double)((TS)pnv[j] + dot<TS>(xc + (NU + j), ldm, t1(), 1, j + 1));
        __syncthreads();
        if (j < NZ) mv = (double)((TS)mv + dot<TS>(F() + j * ldf, 1, t2(), 1, NX));
        return mv;
    }

    // ==================================================================
    // Pass C: backward right-hand-side sweep with the stored factors for the
    // RHS (r_g, r_b, r_d) at offsets og, ob, odl, odu and r_m per rmode.
    // ==================================================================
    __device__ __forceinline__ void passC(int rmode, double shift, int og, int ob, int odl, int odu) const
    {
        Pre pre;
        seg_lfg(pre, N);
        fetch(pre);
        for (int n = N; n >= 0; --n) {
            const int cur = n & 1, nxt = cur ^ 1;
            commit(pre, M(), F(), G());
            stage_BC(n);
            const double* d = Dp(n);
            const double* ir = Ip(n);
            const double* w = Wp(n);
            const int j = opq(tid);
            const double di = j < NU ? w[Lo.W_dinv + j] : 0.0;
            const double rg = j < NZ ? w[og + j] : 0.0;
            const double rb = (j < NX && n < N) ? w[ob + j] : 0.0;
            if (j < NC) {
                double m, lo, hi;
                slot_bounds(d, j, m, lo, hi);
                double e = 0.0;
                if (m != 0.0) {
                    const double ll = ir[Lo.I_ll + j], lu = ir[Lo.I_lu + j];
                    const double tl = ir[Lo.I_tl + j], tu = ir[Lo.I_tu + j];
                    double rml, rmu;
                    slot_rm(rmode, shift, w, j, ll, lu, tl, tu, rml, rmu);
                    const double itl = rcp_nr(tl), itu = rcp_nr(tu);
                    e = (ll * w[odl + j] - rml) * itl - (lu * w[odu + j] - rmu) * itu;
                    if constexpr (SOFT) {
                        if (d[Lo.D_sm + j] != 0.0) {
                            double el = (ll * w[odl + j] - rml) * itl, eu = (lu * w[odu + j] - rmu) * itu;
                            soft_terms(d, ir, w, j, rmode, shift, ll * itl, lu * itu, el, eu);
                            e = el - eu;
                        }
                    }
                }
                ev()[j] = e;
            }
            if (n == N && j < NX) pn(nxt)[j] = 0.0;
            if (j < NX) rbv()[j] = rb;
            if (n > 0) {
                seg_lfg(pre, n - 1);
                fetch(pre);
            }
            __syncthreads();
            double mv = 0.0;
            if (j < NZ) {
                mv = rg - ev()[j] - dot<double>(G() + j * ldg, 1, ev() + NZ, 1, NG);
            }
            if (n < N) mv = cost_to_go_x(mv, XC(), pn(nxt));
            mv = fwd_subst_u(mv, di);
            {
                double* wo = Wp(n);
                if (j < NU) wo[Lo.W_yu + j] = mv;
                else if (j < NZ) {
                    wo[Lo.W_pv + j - NU] = mv;
                    pn(cur)[j - NU] = mv;
                }
            }
            __syncthreads();
        }
    }

    // ==================================================================
    // Pass B: forward substitution and recovery of dt, dlam.  Writes dz, dpi
    // to (oz, opi) and dlam, dt to (oll, olu, otl, otu).  Returns the largest
    // alpha keeping lam, t >= 0 (uncapped; HUGE_VAL if unblocked) and s1 =
    // sum(lam dt + dlam t), s2 = sum(dlam dt).
    // ==================================================================
    __device__ __forceinline__ double passB(int rmode, double shift, int ob, int odl, int odu, int oz, int opi, int oll, int olu,
                            int otl, int otu, double& o_s1, double& o_s2) const
    {
        double amin = HUGE_VAL, s1 = 0.0, s2 = 0.0;
        // dx_0 = -(L0 L0')^{-1} p_0 with L0 the (x, x) block of stage 0
        {
            const int j = tid;
            double* w0 = Wp(0);
            const double* L;
            int ld;
            if constexpr (GL) {
                L = w0 + Lo.W_L + NU + NU * NZ;
                ld = NZ;
            } else {
                double* Ls = Lx();
                Walk qx(NX, tid);
                for (int e = tid; e < NX * NX; e += BT) {
                    Ls[qx.r + qx.c * ldx] = w0[Lo.W_L + (NU + qx.r) + (NU + qx.c) * NZ];
                    qx.next();
                }
                L = Ls;
                ld = ldx;
            }
            if (j < NX) {
                xn(0)[j] = -w0[Lo.W_pv + j];
                dv()[j] = w0[Lo.W_dinv + NU + j];
                w0[opi + j] = 0.0;
            }
            __syncthreads();
            trsv_lower(L, ld, NX, xn(0), dv());
            trsv_lower_t(L, ld, NX, xn(0), dv());
        }
        Pre pre;
        seg_lfg(pre, 0);
        fetch(pre);
        for (int n = 0; n <= N; ++n) {
            const int cur = n & 1, nxt = cur ^ 1;
            commit(pre, M(), F(), G());
            stage_BC(n);
            const double* d = Dp(n);
            const double* ir = Ip(n);
            double* w = Wp(n);
            const int j = opq(tid);
            const double di = j < NU ? w[Lo.W_dinv + j] : 0.0;
            const double yu = j < NU ? w[Lo.W_yu + j] : 0.0;
            const double rb = (j < NX && n < N) ? w[ob + j] : 0.0;
            const double pnx = (j < NX && n < N) ? Wp(n + 1)[Lo.W_pv + j] : 0.0;
            double m = 0.0, rdl = 0.0, rdu = 0.0, ll = 0.0, lu = 0.0, tl = 0.0, tu = 0.0, rml = 0.0, rmu = 0.0;
            if (j < NC) {
                double lo, hi;
                slot_bounds(d, j, m, lo, hi);
                if (m != 0.0) {
                    rdl = w[odl + j];
                    rdu = w[odu + j];
                    ll = ir[Lo.I_ll + j];
                    lu = ir[Lo.I_lu + j];
                    tl = ir[Lo.I_tl + j];
                    tu = ir[Lo.I_tu + j];
                    slot_rm(rmode, shift, w, j, ll, lu, tl, tu, rml, rmu);
                }
            }
            if (n < N) {
                seg_lfg(pre, n + 1);
                fetch(pre);
            }
            __syncthreads();
            // v = y_u + L_xu' dx ; back-substitution with L_uu'
            if (wid == 0) {
                const double* mu = M();
                const double* x = xn(cur);
                double v = 0.0;
                if (lane < NU) v = (double)((TS)yu + dot<TS>(mu + NU + lane * ldm, 1, x, 1, NX));
                // PCH rows of L_uu at a time (from the last), their loads
                // issued together
                for (int c1 = NU; c1 > 0; c1 -= PCH) {
                    double lc[PCH];
#pragma unroll
                    for (int q = 0; q < PCH; ++q) {
                        const int c = c1 - 1 - q;
                        lc[q] = (c >= 0 && lane < c) ? mu[c + lane * ldm] : 0.0;
                    }
#pragma unroll
                    for (int q = 0; q < PCH; ++q) {
                        const int c = c1 - 1 - q;
                        if (c < 0) break;
                        const double xv = rnd(bcast(v, c) * bcast(di, c));
                        if (lane == c) v = xv;
                        else if (lane < c) v = (double)((TS)v - (TS)lc[q] * (TS)xv);
                    }
                }
                if (lane < NU) {
                    z()[lane] = -v;
                    w[oz + lane] = ABS ? -v - ir[Lo.I_z + lane] : -v;
                }
            }
            if (j >= NU && j < NZ) {
                const double dz = xn(cur)[j - NU];
                z()[j] = dz;
                w[oz + j] = ABS ? dz - ir[Lo.I_z + j] : dz;
            }
            __syncthreads();
            if (n < N) {
                const double* xc = XC();
                if (j < NX) xn(nxt)[j] = (double)((TS)rb + dot<TS>(F() + j, ldf, z(), 1, NZ));
                __syncthreads();
                if (j < NX) t1()[j] = (double)dot<TS>(xc + (NU + j) + j * ldm, 1, xn(nxt) + j, 1, NX - j);
                __syncthreads();
                if (j < NX) {
                    const double pv = (double)((TS)pnx + dot<TS>(xc + (NU + j), ldm, t1(), 1, j + 1));
                    Wp(n + 1)[opi + j] = ABS ? pv - Ip(n + 1)[Lo.I_pi + j] : pv;
                }
            }
            // constraint steps, step length, duality-measure sums
            if (j < NC) {
                double dll = 0.0, dlu = 0.0, dtl = 0.0, dtu = 0.0;
                if (m != 0.0) {
                    double gdz;
                    if (j < NZ) {
                        gdz = z()[j];
                    } else {
                        gdz = dot<double>(G() + (j - NZ), ldg, z(), 1, NZ);
                    }
                    double dsl = 0.0, dsu = 0.0;
                    if constexpr (SOFT) {
                        if (d[Lo.D_sm + j] != 0.0) {
                            // slack steps and the steps of their bound rows
                            const double itl = rcp_nr(tl), itu = rcp_nr(tu);
                            const double wl = ll * itl, wu = lu * itu;
                            double el = (ll * rdl - rml) * itl, eu = (lu * rdu - rmu) * itu;
                            const SoftE q = soft_terms(d, ir, w, j, rmode, shift, wl, wu, el, eu);
                            dsl = -(q.gl + wl * gdz) * rcp_nr(q.Dl);
                            dsu = -(q.gu - wu * gdz) * rcp_nr(q.Du);
                            const double dtsl = dsl - q.rdsl, dtsu = dsu - q.rdsu;
                            const double dlsl = -(q.rmsl + q.lsl * dtsl) * rcp_nr(q.tsl);
                            const double dlsu = -(q.rmsu + q.lsu * dtsu) * rcp_nr(q.tsu);
                            if (dlsl < 0.0) amin = fmin(amin, -q.lsl * __builtin_amdgcn_rcp(dlsl));
                            if (dlsu < 0.0) amin = fmin(amin, -q.lsu * __builtin_amdgcn_rcp(dlsu));
                            if (dtsl < 0.0) amin = fmin(amin, -q.tsl * __builtin_amdgcn_rcp(dtsl));
                            if (dtsu < 0.0) amin = fmin(amin, -q.tsu * __builtin_amdgcn_rcp(dtsu));
                            s1 += q.lsl * dtsl + dlsl * q.tsl + q.lsu * dtsu + dlsu * q.tsu;
                            s2 += dlsl * dtsl + dlsu * dtsu;
                            // the affine step keeps only what the corrector reads
                            const bool aff = oll == Lo.W_all;
                            if (!aff) {
                                w[Lo.W_dsl + j] = dsl;
                                w[Lo.W_dsu + j] = dsu;
                            }
                            w[(aff ? Lo.W_alsl : Lo.W_dlsl) + j] = dlsl;
                            w[(aff ? Lo.W_alsu : Lo.W_dlsu) + j] = dlsu;
                            w[(aff ? Lo.W_atsl : Lo.W_dtsl) + j] = dtsl;
                            w[(aff ? Lo.W_atsu : Lo.W_dtsu) + j] = dtsu;
                        }
                    }
                    if constexpr (SOFT) {
                        dtl = gdz + dsl - rdl;
                        dtu = -gdz + dsu - rdu;
                    } else {
                        dtl = gdz - rdl;
                        dtu = -gdz - rdu;
                    }
                    dll = -(rml + ll * dtl) * rcp_nr(tl);
                    dlu = -(rmu + lu * dtu) * rcp_nr(tu);
                    if (ABS) {
                        // absolute formulation: full-step iterate minus the
                        // current one (eq:alg:pdipm:step)
                        dtl -= tl;
                        dtu -= tu;
                        dll -= ll;
                        dlu -= lu;
                    }
                    if (dll < 0.0) amin = fmin(amin, -ll * __builtin_amdgcn_rcp(dll));
                    if (dlu < 0.0) amin = fmin(amin, -lu * __builtin_amdgcn_rcp(dlu));
                    if (dtl < 0.0) amin = fmin(amin, -tl * __builtin_amdgcn_rcp(dtl));
                    if (dtu < 0.0) amin = fmin(amin, -tu * __builtin_amdgcn_rcp(dtu));
                    s1 += ll * dtl + dll * tl + lu * dtu + dlu * tu;
                    s2 += dll * dtl + dlu * dtu;
                }
                w[oll + j] = dll;
                w[olu + j] = dlu;
                w[otl + j] = dtl;
                w[otu + j] = dtu;
            }
            __syncthreads();
        }
        amin = bmin_sum2(amin, s1, s2);
        o_s1 = s1;
        o_s2 = s2;
        return amin;
    }

    // ==================================================================
    // Pass R (mixed path): FP64 residual r_ir = K step + r of the Newton
    // system for the step at (oz, opi, oll, olu, otl, otu); written to the
    // refinement arrays.  Returns its inf-norm.
    // ==================================================================
    __device__ __forceinline__ double passR(int rmode, double shift, int oz, int opi, int oll, int olu, int otl, int otu) const
    {
        double nr = 0.0;
        Pre pre;
        seg_hfg(pre, N);
        fetch(pre);
        for (int n = N; n >= 0; --n) {
            const int cur = n & 1, nxt = cur ^ 1;
            commit(pre, M(), F(), G());
            stage_R(n);
            const double* d = Dp(n);
            const double* ir = Ip(n);
            double* w = Wp(n);
            const int j = opq(tid);
            const double dz = j < NZ ? w[oz + j] : 0.0;
            const double rg = j < NZ ? w[Lo.W_rg + j] : 0.0;
            const double dpi = (j < NX && n > 0) ? w[opi + j] : 0.0;
            const double rb = (j < NX && n < N) ? w[Lo.W_rb + j] : 0.0;
            double m = 0.0, rdl = 0.0, rdu = 0.0, ll = 0.0, lu = 0.0, tl = 0.0, tu = 0.0, rml = 0.0, rmu = 0.0;
            double sll = 0.0, slu = 0.0, stl = 0.0, stu = 0.0;
            if (j < NC) {
                double lo, hi;
                slot_bounds(d, j, m, lo, hi);
                if (m != 0.0) {
                    rdl = w[Lo.W_rdl + j];
                    rdu = w[Lo.W_rdu + j];
                    ll = ir[Lo.I_ll + j];
                    lu = ir[Lo.I_lu + j];
                    tl = ir[Lo.I_tl + j];
                    tu = ir[Lo.I_tu + j];
                    slot_rm(rmode, shift, w, j, ll, lu, tl, tu, rml, rmu);
                    sll = w[oll + j];
                    slu = w[olu + j];
                    stl = w[otl + j];
                    stu = w[otu + j];
                }
            }
            if (n > 0) {
                seg_hfg(pre, n - 1);
                fetch(pre);
            }
            if (n == N && j < NX) {
                xn(nxt)[j] = 0.0;
                pin(nxt)[j] = 0.0;
            }
            if (j < NZ) z()[j] = dz;
            if (j < NX) t2()[j] = dpi;
            if (j >= NZ && j < NC) t1()[j - NZ] = m * (sll - slu);
            __syncthreads();
            // g row: H dz + F' dpi_{n+1} - [0; dpi_n] - C' dlam + r_g
            double org = 0.0, orb = 0.0;
            if (j < NZ) {
                const double* mh = M();
                const double* zv = z();
                double acc = rg + dot<double>(mh + j, ldm, zv, 1, NZ);
                if (n < N) acc += dot<double>(F() + j * ldf, 1, pin(nxt), 1, NX);
                if (j >= NU) acc -= t2()[j - NU];
                acc -= m * (sll - slu);
                acc -= dot<double>(G() + j * ldg, 1, t1(), 1, NG);
                org = acc;
                nr = nmax(nr, fabs(acc));
                w[Lo.W_irg + j] = org;
            }
            // b row: F dz - dx_{n+1} + r_b
            if (n < N && j < NX) {
                const double acc = rb + dot<double>(F() + j, ldf, z(), 1, NZ);
                orb = acc - xn(nxt)[j];
                nr = nmax(nr, fabs(orb));
                w[Lo.W_irb + j] = orb;
            }
            // d rows: -C dz + dt + r_d ; m rows: T dlam + Lam dt + r_m
            if (j < NC) {
                double ordl = 0.0, ordu = 0.0, orml = 0.0, ormu = 0.0;
                if (m != 0.0) {
                    double gz;
                    if (j < NZ) {
                        gz = dz;
                    } else {
                        gz = dot<double>(G() + (j - NZ), ldg, z(), 1, NZ);
                    }
                    ordl = -gz + stl + rdl;
                    ordu = gz + stu + rdu;
                    orml = tl * sll + ll * stl + rml;
                    ormu = tu * slu + lu * stu + rmu;
                    nr = nmax(nr, nmax(nmax(fabs(ordl), fabs(ordu)), nmax(fabs(orml), fabs(ormu))));
                }
                w[Lo.W_irdl + j] = ordl;
                w[Lo.W_irdu + j] = ordu;
                w[Lo.W_irml + j] = orml;
                w[Lo.W_irmu + j] = ormu;
            }
            if (j >= NU && j < NZ) xn(cur)[j - NU] = dz;
            if (j < NX) pin(cur)[j] = dpi;
            __syncthreads();
        }
        return bmax1(nr);
    }

    // ==================================================================
    // Pass X (mixed path): step += correction, then the step length and the
    // duality-measure sums of pass B for the corrected step.  Stages are
    // independent here, so the loop runs over all (stage, row) pairs.
    // ==================================================================
    __device__ __forceinline__ double passX(int oz, int opi, int oll, int olu, int otl, int otu, double sg, double& o_s1,
                                            double& o_s2) const
    {
        double amin = HUGE_VAL, s1 = 0.0, s2 = 0.0;
        for (int e = tid; e < (N + 1) * NZ; e += BT) {
            double* w = Wp(e / NZ);
            const int j = e % NZ;
            w[oz + j] += sg * w[Lo.W_edz + j];
        }
        for (int e = tid; e < N * NX; e += BT) {
            double* w = Wp(1 + e / NX);
            const int i = e % NX;
            w[opi + i] += sg * w[Lo.W_edpi + i];
        }
        for (int e = tid; e < (N + 1) * NC; e += BT) {
            const int n = e / NC, c = e % NC;
            const double* d = Dp(n);
            const double* ir = Ip(n);
            double* w = Wp(n);
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
        amin = bmin_sum2(amin, s1, s2);
        o_s1 = s1;
        o_s2 = s2;
        return amin;
    }

    // Iterative refinement of the step at the given offsets (Section 3.4):
    // each correction solves the Newton system with the refinement residual
    // as right-hand side.  Stops when ||r_ir|| <= ir_tol * rnorm, after
    // max_steps corrections, or when a correction did not lower ||r_ir||
    // (that correction is then subtracted again, so the step kept is the best
    // one seen).  Updates amax, s1, s2 for the step kept; nir0 returns the
    // residual norm of the unrefined step (the balance build's accuracy check
    // of the factors); returns the corrections kept.
    __device__ __forceinline__ int refine(int rmode, double shift, double rnorm, int max_steps, int oz, int opi, int oll,
                                          int olu, int otl, int otu, double& amax, double& s1, double& s2,
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
                double t1v, t2v;
                passB(RM_IR, 0.0, Lo.W_irb, Lo.W_irdl, Lo.W_irdu, Lo.W_edz, Lo.W_edpi, Lo.W_edll, Lo.W_edlu, Lo.W_edtl,
                      Lo.W_edtu, t1v, t2v);
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
    // Initial point (P.warm), as in the one-wave kernel: cold start, primal
    // guess (y kept, the rest as in the cold start at that y), or primal and
    // dual guess (kept, multipliers and slacks clamped below).
    __device__ __forceinline__ void init(int warm) const
    {
        if (warm == 0)
            for (int e = tid; e < (N + 1) * NZ; e += BT) Ip(e / NZ)[Lo.I_z + e % NZ] = 0.0;
        if (warm != 2)
            for (int e = tid; e < (N + 1) * NX; e += BT) Ip(e / NX)[Lo.I_pi + e % NX] = 0.0;
        for (int e = tid; e < (N + 1) * NC; e += BT) {
            const int n = e / NC, c = e % NC;
            double m, lo, hi;
            const double* d = Dp(n);
            slot_bounds(d, c, m, lo, hi);
            const bool on = m != 0.0;
            double* ir = Ip(n);
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
        __threadfence_block();
        __syncthreads();
    }

    __device__ __forceinline__ void copy_step_out(double* out) const
    {
        for (int e = tid; e < (N + 1) * NZ; e += BT) {
            const int n = e / NZ, j = e % NZ;
            out[(size_t)n * Lo.IREC + Lo.I_z + j] = Wp(n)[Lo.W_dz + j];
        }
        for (int e = tid; e < (N + 1) * NX; e += BT) {
            const int n = e / NX, i = e % NX;
            out[(size_t)n * Lo.IREC + Lo.I_pi + i] = Wp(n)[Lo.W_dpi + i];
        }
        for (int e = tid; e < (N + 1) * NC; e += BT) {
            const int n = e / NC, c = e % NC;
            double* o = out + (size_t)n * Lo.IREC;
            const double* w = Wp(n);
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

    // ------------------------------------------------------------------
    // Driver (same iteration logic as the one-wave kernel).
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
        // returned iterate, through the single call site of pass A
        bool final_pass = false;
        int k_exit = 0;
        // balance build: the iteration is factored with the array algorithm
        // (after its Cholesky factors failed the accuracy check)
        bool qr = false, refactor = false;
        int qr_refactors = 0;
        for (k = 0;; ++k) {
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
                status = ST_FALLBACK;
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
                    // direction (Section 4.2; the FP64 build when asked for
                    // by a positive ir_max, Section 3.4); the affine
                    // predictor only feeds the centering parameter and the
                    // corrector right-hand side and is used unrefined.
                    // Balance build: the predictor's residual checks the
                    // accuracy of this iteration's Cholesky factors
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
        if (MIXED && !newton_mode && (status == ST_NAN || status == ST_MIN_STEP)) status = ST_FALLBACK;
        // a finite iterate is handed over as it is: the FP64 kernel continues
        // the solve from it instead of starting over
        if (MIXED && status == ST_FALLBACK)
            fell_back = (__builtin_isfinite(ng) && __builtin_isfinite(nb) && __builtin_isfinite(nd) &&
                         __builtin_isfinite(nm) && __builtin_isfinite(mu))
                            ? FB_RESUME
                            : FB_COLD;
        if (tid == 0) {
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

// Waves per SIMD the register budget is sized for: two in every build, so
// that two instances share a CU and hide each other's latency wherever LDS
// allows it.  The uneven batch of 4096 runs 13 % faster (mixed path 7 %)
// than at one wave per SIMD.  The stage prefetch recomputes its element
// offsets per stage, so the 32- and 64-wide builds fit 256 registers with no
// spill (with general rows at 64: 4-26; they had spilled up to 410); the
// 32-wide build with general rows, one wave per SIMD before, runs the
// 8-mass batch condensed to 15 stages 33 % faster at two.  The
// global-memory mode takes two as well: its stage matrix sits in matrix-core
// accumulators (112 registers per lane in FP64), L_{n+1}' F is formed before
// they are live, and the lane offsets of the tile loops are recomputed per
// panel, so the build fits 256 registers with a few spills outside the
// factorization; LDS is 64 KB at nz = 160.  One batch of 256 large stages
// (one workgroup per CU) runs 6 % slower than the one-wave build with the
// whole register file; two such batches in flight, which share every CU,
// 44 % faster.
__host__ __device__ constexpr int block_waves(int zm, int gm)
{
    return 2;
}

// ZM > 64 selects the global-memory mode; WV overrides the register budget
// (64-wide blocks with general rows at one wave per SIMD, for launches whose
// LDS keeps a CU to one workgroup anyway: that build spills nothing).
template <int KM, int ZM, int GM, int WV = block_waves(ZM, GM)>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(WV, WV))) void ipm_block_kernel(
    const InstDesc* __restrict__ desc, int count, const double* __restrict__ data, double* __restrict__ iter,
    double* __restrict__ work, double* __restrict__ step_out, DevStat* __restrict__ stat, KParams P)
{
    const int b = blockIdx.x;
    if (b >= count) return;
    const InstDesc ds = desc[b];
    int fell_back = FB_NONE, resume = ds.resume, itcap = ds.itcap, it0 = 0, ir0 = 0;
    if (P.mode == KMODE_FALLBACK) {
        // only instances the mixed kernel handed over, continued from their
        // iterate within the remaining iteration budget
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
    const Blk<KM, ZM, GM, (ZM > 64)> ipm(ds, data, iter, work, P);
    ipm.run(stat + ds.index, step_out + ds.iter, fell_back, resume, itcap, it0, ir0);
}

}  // namespace oqp
