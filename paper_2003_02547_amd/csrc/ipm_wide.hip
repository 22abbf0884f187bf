// Wide-stage kernel of the batched IPM (FP64, delta formulation, Mehrotra
// predictor-corrector of Section 4.2) for stage blocks beyond the block
// kernel's limits: more than 64 inputs, more than 64 general rows or more
// than 256 constraint slots in a stage.  These are the QPs of full
// condensing (Section 3.5 with one block: a single stage holding every input
// and, as general rows, the state boxes of every later stage) and other wide
// stages.  For such a QP the factorization of stage 0 is the dense Cholesky
// factorization of the condensed Hessian plus barrier terms, the KKT solver
// Section 3.3 names for condensed QPs (they have no equality constraints
// left but the one that carries the terminal state).
//
// One 256-thread workgroup solves one instance.  Rows, columns and
// constraint slots are distributed over the threads in strided loops, so no
// stage size is bounded by the workgroup size.  The stage matrices live in
// the workspace records (HBM):
//   M = H + diag(box weights) + reg I + V'V,  V = [Lxx_{n+1}' F; sqrt(w) G]
// is formed on the matrix cores (v_mfma_f64_16x16x4f64: the trmm and the
// syrk) and factored in place by a right-looking Cholesky in 16-column
// panels: wave 0 factors the diagonal block (one row per lane), every thread
// solves rows of the panel below it, and the trailing lower triangle takes
// the panel's rank-16 update on the matrix cores.  Triangular solves of the
// sweeps are blocked the same way (wave 0 on the 16 x 16 diagonal block,
// then all threads on the rows below or above it).
//
// A terminal stage N without inputs (the usual case, and the case of every
// condensed QP of an OCP QP without terminal inputs) has only padded input
// components, with a unit Hessian and nothing else, so their step is zero:
// only its state block is factored and swept.
#include <hip/hip_runtime.h>
#include <math.h>

#include "dev_common.h"
#include "ipm_launch.h"
#include "layout.h"

namespace oqp {

namespace {

constexpr int WT = 256;  // threads per workgroup
constexpr int PW = 16;   // panel width of the factorization and the solves

// LDS plan (offsets in doubles) for padded stage sizes NX, NU, NG
struct WLds {
    int oz, oe, ows, omv, ot1, ot2, orb, oxn, opin, opn, ol11, odi, ored, oflag, total;
};

__host__ __device__ inline WLds make_wlds(int NX, int NU, int NG)
{
    const int NZ = NX + NU, NC = NZ + NG, X = NX > 0 ? NX : 1;
    WLds s{};
    int o = 0;
    s.oz = o; o += NZ;          // z (residual pass) or the step of z (forward pass)
    s.oe = o; o += NC;          // per slot: lam_l - lam_u (residual pass), then e
    s.ows = o; o += NC;         // per slot: w_l + w_u
    s.omv = o; o += NZ;         // reduced gradient / sweep vector of the stage
    s.ot1 = o; o += X;
    s.ot2 = o; o += X;
    s.orb = o; o += X;
    s.oxn = o; o += 2 * X;      // x_{n+1} (or its step), two buffers
    s.opin = o; o += 2 * X;     // pi_{n+1}, two buffers
    s.opn = o; o += 2 * X;      // p_{n+1} of the sweep, two buffers
    s.ol11 = o; o += PW * PW;   // diagonal block of the current panel
    s.odi = o; o += PW;         // its inverse diagonal
    s.ored = o; o += 32;
    s.oflag = o; o += 2;
    s.total = o;
    return s;
}

__device__ __forceinline__ double* wlds()
{
    extern __shared__ double oqp_wlds_dyn[];
    return oqp_wlds_dyn;
}

// thread index re-materialised inside loop bodies (keeps per-thread address
// arithmetic from being hoisted and held live across the whole solve)
__device__ __forceinline__ int opq(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// sum_{k < n} a[k sa] b[k sb]: eight loads of each operand issued before
// their products, so that eight memory round trips overlap (the stage
// records mostly come from HBM: a dependent chain would pay one trip each)
__device__ __forceinline__ double dot(const double* a, int sa, const double* b, int sb, int n)
{
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int k = 0;
    // 16 loads issued together, the sums taken in the order of the loop below
    for (; k + 16 <= n; k += 16) {
        double av[16], bv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            av[u] = a[(k + u) * sa];
            bv[u] = b[(k + u) * sb];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) s[u & 7] += av[u] * bv[u];
    }
    for (; k + 8 <= n; k += 8) {
        double av[8], bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            av[u] = a[(k + u) * sa];
            bv[u] = b[(k + u) * sb];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += av[u] * bv[u];
    }
    for (; k < n; ++k) s[0] += a[k * sa] * b[k * sb];
    return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

struct Wide {
    Layout Lo;
    WLds S;
    int NX, NU, NG, NZ, NC, NV;
    const double* __restrict__ dat;
    double* __restrict__ itr;
    double* __restrict__ wk;
    int N, nc, nuN, tid, lane, wid;
    const KParams& P;

    __device__ __forceinline__ Wide(const InstDesc& ds, const double* d, double* i, double* w, const KParams& P_)
        : Lo(make_layout(ds.nx, ds.nu, ds.ng)), S(make_wlds(ds.nx, ds.nu, ds.ng)), NX(ds.nx), NU(ds.nu), NG(ds.ng),
          NZ(ds.nx + ds.nu), NC(ds.nx + ds.nu + ds.ng), NV(ds.nx + ds.ng), dat(d + ds.data), itr(i + ds.iter),
          wk(w + ds.work), N(ds.N), nc(ds.nc), nuN(ds.nuN), tid((int)threadIdx.x), lane((int)threadIdx.x & 63),
          wid((int)threadIdx.x >> 6), P(P_)
    {
    }

    __device__ __forceinline__ const double* Dp(int n) const { return dat + (size_t)n * Lo.SREC; }
    __device__ __forceinline__ double* Ip(int n) const { return itr + (size_t)n * Lo.IREC; }
    __device__ __forceinline__ double* Wp(int n) const { return wk + (size_t)n * Lo.WREC; }

    __device__ __forceinline__ double* z() const { return wlds() + S.oz; }
    __device__ __forceinline__ double* ev() const { return wlds() + S.oe; }
    __device__ __forceinline__ double* wsv() const { return wlds() + S.ows; }
    __device__ __forceinline__ double* mv() const { return wlds() + S.omv; }
    __device__ __forceinline__ double* t1() const { return wlds() + S.ot1; }
    __device__ __forceinline__ double* t2() const { return wlds() + S.ot2; }
    __device__ __forceinline__ double* rbv() const { return wlds() + S.orb; }
    __device__ __forceinline__ double* xn(int p) const { return wlds() + S.oxn + p * (NX > 0 ? NX : 1); }
    __device__ __forceinline__ double* pin(int p) const { return wlds() + S.opin + p * (NX > 0 ? NX : 1); }
    __device__ __forceinline__ double* pn(int p) const { return wlds() + S.opn + p * (NX > 0 ? NX : 1); }
    __device__ __forceinline__ double* l11() const { return wlds() + S.ol11; }
    __device__ __forceinline__ double* di11() const { return wlds() + S.odi; }
    __device__ __forceinline__ double* red() const { return wlds() + S.ored; }
    __device__ __forceinline__ double* flag() const { return wlds() + S.oflag; }

    // first component of z_n taking part in the factorization and the
    // sweeps: the state block only at a terminal stage without inputs
    __device__ __forceinline__ int zb(int n) const { return (n == N && nuN == 0) ? NU : 0; }
    // factor of stage n (NZ x NZ, column-major, zero strict upper part) and
    // its (x, x) block
    __device__ __forceinline__ double* Lf(int n) const { return Wp(n) + Lo.W_L; }
    __device__ __forceinline__ const double* Lxx(int n) const { return Wp(n) + Lo.W_L + NU + NU * NZ; }

    __device__ __forceinline__ void slot_bounds(const double* d, int c, double& m, double& lo, double& hi) const
    {
        if (c < NZ) {
            m = d[Lo.D_bm + c];
            lo = d[Lo.D_blo + c];
            hi = d[Lo.D_bhi + c];
        } else {
            m = d[Lo.D_gm + (c - NZ)];
            lo = d[Lo.D_glo + (c - NZ)];
            hi = d[Lo.D_ghi + (c - NZ)];
        }
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

    // ------------------------------------------------------------------
    // dense kernels on HBM blocks
    // ------------------------------------------------------------------

    // C(i, j) op= sum_{k < K} A(k, i) B(k, j) for i < m, j < n (only j <= i
    // when `lower`), A(k, i) = A[k sak + i sai], B(k, j) = B[k sbk + j sbj]:
    // 16 x 16 output tiles over the four waves, K in steps of 4 on
    // v_mfma_f64_16x16x4f64.  Operand lanes: A(k0 + lane / 16, i0 + lane %
    // 16), B(k0 + lane / 16, j0 + lane % 16); accumulator register r of a
    // lane holds row i0 + 4 r + lane / 16, column j0 + lane % 16.  Loads use
    // clamped in-range indices and zero out-of-range operands, so every lane
    // stays active.  op: 0 store, 1 add, -1 subtract.
    __device__ __forceinline__ void mma_tn(const double* A, int sak, int sai, const double* B, int sbk, int sbj, int m,
                                           int n, int K, double* C, int ldc, int op, bool lower) const
    {
        using V4 = double __attribute__((ext_vector_type(4)));
        if (m <= 0 || n <= 0) return;
        const int TM = (m + 15) >> 4, TN = (n + 15) >> 4;
        const int l16 = lane & 15, lk = lane >> 4;
        for (int t = opq(wid); t < TM * TN; t += WT / 64) {
            const int ti = t % TM, tj = t / TM;
            if (lower && ti < tj) continue;
            const int i = 16 * ti + l16, j = 16 * tj + l16;
            const bool iv = i < m, jv = j < n;
            const double* pa = A + min(i, m - 1) * sai;
            const double* pb = B + min(j, n - 1) * sbj;
            V4 acc = {0.0, 0.0, 0.0, 0.0};
            // K in chunks of 16: the chunk's eight operand loads are issued
            // before its four matrix-core steps
            for (int k0 = 0; k0 < K; k0 += 16) {
                double av[4], bv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int kc = min(k0 + 4 * q + lk, K - 1);
                    av[q] = pa[kc * sak];
                    bv[q] = pb[kc * sbk];
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool kv = k0 + 4 * q + lk < K;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64((iv && kv) ? av[q] : 0.0, (jv && kv) ? bv[q] : 0.0, acc,
                                                               0, 0, 0);
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * ti + 4 * r + lk;
                const int col = 16 * tj + l16;
                if (row < m && col < n && (!lower || col <= row)) {
                    double* c = C + row + col * ldc;
                    if (op == 0) *c = acc[r];
                    else if (op > 0) *c += acc[r];
                    else *c -= acc[r];
                }
            }
        }
    }

    // In-place Cholesky factorization of the n x n matrix at m (column-major,
    // leading dimension ld, lower triangle read, strict upper part zero):
    // L with L L' = M in the lower triangle, 1/L_ii into dinv.  Every thread
    // calls it; returns false in every thread when a pivot is not positive.
    __device__ __forceinline__ bool cholesky(double* m, int ld, int n, double* dinv) const
    {
        bool ok = true;
        for (int p0 = 0; p0 < n; p0 += PW) {
            const int pw = min(PW, n - p0);
            const int p1 = p0 + pw;
            if (wid == 0) {
                // diagonal block: lane q holds row p0 + q
                const bool act = lane < pw;
                const int i = p0 + min(lane, pw - 1);
                double r[PW];
#pragma unroll
                for (int q = 0; q < PW; ++q) {
                    const double v = m[i + (p0 + min(q, pw - 1)) * ld];
                    r[q] = (act && q < pw && q <= lane) ? v : 0.0;
                }
#pragma unroll
                for (int q = 0; q < PW; ++q) {
                    if (q >= pw) continue;
                    const double piv = bcast(r[q], q);
                    ok = ok && (piv > 0.0);
                    const double inv = 1.0 / sqrt(piv);
                    const double lij = r[q] * inv;
                    if (lane == q) {
                        r[q] = piv * inv;
                        if (act) {
                            dinv[p0 + q] = inv;
                            di11()[q] = inv;
                        }
                    } else if (lane > q) {
                        r[q] = lij;
                    } else {
                        r[q] = 0.0;
                    }
                    // rank-1 update of the rows below; the upper part stays zero
#pragma unroll
                    for (int q2 = q + 1; q2 < PW; ++q2) {
                        if (q2 >= pw) continue;
                        const double l2 = bcast(lij, q2);
                        if (lane > q) r[q2] -= lij * l2;
                    }
                }
                if (act) {
#pragma unroll
                    for (int q = 0; q < PW; ++q) {
                        if (q < pw) {
                            m[i + (p0 + q) * ld] = r[q];
                            l11()[lane + PW * q] = r[q];
                        }
                    }
                }
            }
            __syncthreads();
            // panel below the diagonal block: L21 = M21 L11^{-T}, one row per
            // thread (forward substitution with the LDS copy of L11)
            const double* lb = l11();
            const double* dd = di11();
            for (int i = p1 + opq(tid); i < n; i += WT) {
                double x[PW];
#pragma unroll
                for (int q = 0; q < PW; ++q) x[q] = q < pw ? m[i + (p0 + q) * ld] : 0.0;
#pragma unroll
                for (int q = 0; q < PW; ++q) {
                    if (q >= pw) continue;
                    double s = x[q];
#pragma unroll
                    for (int k = 0; k < q; ++k) s -= x[k] * lb[q + PW * k];
                    x[q] = s * dd[q];
                }
#pragma unroll
                for (int q = 0; q < PW; ++q)
                    if (q < pw) m[i + (p0 + q) * ld] = x[q];
            }
            __syncthreads();
            // trailing lower triangle: M22 -= L21 L21'
            const int nt = n - p1;
            if (nt > 0) {
                mma_tn(m + p1 + p0 * ld, ld, 1, m + p1 + p0 * ld, ld, 1, nt, nt, pw, m + p1 + p1 * ld, ld, -1, true);
                __syncthreads();
            }
        }
        if (tid == 0) flag()[0] = 1.0;
        __syncthreads();
        if (wid == 0 && !ok && lane == 0) flag()[0] = 0.0;
        __syncthreads();
        const bool res = flag()[0] != 0.0;
        __syncthreads();
        return res;
    }

    // x <- L^{-1} x for the n x n lower factor at L (leading dimension ld,
    // inverse diagonal dinv); x in LDS.  Every thread calls it.
    __device__ __forceinline__ void trsv_lower(const double* L, int ld, int n, double* x, const double* dinv) const
    {
        for (int p0 = 0; p0 < n; p0 += PW) {
            const int pw = min(PW, n - p0);
            const int p1 = p0 + pw;
            if (wid == 0) {
                // the block's row of this lane and its pivot inverse are
                // loaded first, then the substitution runs from registers
                const bool act = lane < pw;
                const int i = p0 + min(lane, pw - 1);
                double lr[PW];
#pragma unroll
                for (int q = 0; q < PW; ++q) lr[q] = (act && q < pw) ? L[i + (p0 + q) * ld] : 0.0;
                const double dl = act ? dinv[i] : 1.0;
                double v = act ? x[i] : 0.0;
#pragma unroll
                for (int q = 0; q < PW; ++q) {
                    if (q >= pw) break;
                    const double xq = bcast(v, q) * bcast(dl, q);
                    if (lane == q) v = xq;
                    else if (lane > q && act) v -= lr[q] * xq;
                }
                if (act) x[i] = v;
            }
            __syncthreads();
            for (int i = p1 + opq(tid); i < n; i += WT) x[i] -= dot(L + i + p0 * ld, ld, x + p0, 1, pw);
            __syncthreads();
        }
    }

    // x <- L^{-T} x (same arguments as trsv_lower)
    __device__ __forceinline__ void trsv_lower_t(const double* L, int ld, int n, double* x, const double* dinv) const
    {
        if (n <= 0) return;
        for (int p0 = ((n - 1) / PW) * PW; p0 >= 0; p0 -= PW) {
            const int pw = min(PW, n - p0);
            if (wid == 0) {
                const bool act = lane < pw;
                const int i = p0 + min(lane, pw - 1);
                double lc[PW];
#pragma unroll
                for (int q = 0; q < PW; ++q) lc[q] = (act && q < pw) ? L[(p0 + q) + i * ld] : 0.0;
                const double dl = act ? dinv[i] : 1.0;
                double v = act ? x[i] : 0.0;
#pragma unroll
                for (int q = PW - 1; q >= 0; --q) {
                    if (q >= pw) continue;
                    const double xq = bcast(v, q) * bcast(dl, q);
                    if (lane == q) v = xq;
                    else if (lane < q) v -= lc[q] * xq;
                }
                if (act) x[i] = v;
            }
            __syncthreads();
            for (int i = opq(tid); i < p0; i += WT) x[i] -= dot(L + p0 + i * ld, 1, x + p0, 1, pw);
            __syncthreads();
        }
    }

    // y = Lxx' v (upper-triangular product) then r = p + Lxx y, for the
    // NX x NX factor Lxx (leading dimension NZ): the cost-to-go P v + p with
    // P = Lxx Lxx'.  v, p, r in LDS (r may alias p); t1 is scratch.
    __device__ __forceinline__ void ctg(const double* L, const double* v, const double* p, double* r) const
    {
        for (int i = opq(tid); i < NX; i += WT) t1()[i] = dot(L + i + i * NZ, 1, v + i, 1, NX - i);
        __syncthreads();
        for (int i = opq(tid); i < NX; i += WT) t2()[i] = p[i] + dot(L + i, NZ, t1(), 1, i + 1);
        __syncthreads();
        for (int i = opq(tid); i < NX; i += WT) r[i] = t2()[i];
        __syncthreads();
    }

    // ------------------------------------------------------------------
    // Initial point (cold start, primal guess, or primal-dual guess)
    // ------------------------------------------------------------------
    __device__ __forceinline__ void init(int warm) const
    {
        if (warm == 0)
            for (int e = tid; e < (N + 1) * NZ; e += WT) Ip(e / NZ)[Lo.I_z + e % NZ] = 0.0;
        if (warm != 2 && NX > 0)
            for (int e = tid; e < (N + 1) * NX; e += WT) Ip(e / NX)[Lo.I_pi + e % NX] = 0.0;
        __syncthreads();
        for (int e = tid; e < (N + 1) * NC; e += WT) {
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
                continue;
            }
            double gz = 0.0;
            if (warm == 1) gz = c < NZ ? ir[Lo.I_z + c] : dot(d + Lo.D_G + (c - NZ), NG, ir + Lo.I_z, 1, NZ);
            ir[Lo.I_ll + c] = on ? 1.0 : 0.0;
            ir[Lo.I_lu + c] = on ? 1.0 : 0.0;
            ir[Lo.I_tl + c] = on ? (warm == 1 ? fmax(gz - lo, 1.0) : fmax(-lo, 1.0)) : 0.0;
            ir[Lo.I_tu + c] = on ? (warm == 1 ? fmax(hi - gz, 1.0) : fmax(hi, 1.0)) : 0.0;
        }
        __syncthreads();
    }

    // ==================================================================
    // Pass A: update of the iterate by alpha times the stored step (when
    // upd), residuals of eq:alg:pdipm:delta and their norms, barrier weights
    // w = lam / t, and (when factor) the backward factorization of every
    // stage.  The right-hand sides are formed by pass C.
    // ==================================================================
    __device__ __forceinline__ bool passA(bool upd, double alpha, bool factor, double& o_g, double& o_b, double& o_d,
                                          double& o_m, double& o_lt) const
    {
        double mg = 0.0, mb = 0.0, md = 0.0, mm = 0.0, slt = 0.0;
        bool fact_ok = true;
        for (int n = N; n >= 0; --n) {
            const int cur = n & 1, nxt = cur ^ 1;
            const int z0 = zb(n);
            const double* d = Dp(n);
            double* ir = Ip(n);
            double* w = Wp(n);
            // slots: step and clamps; lam_l - lam_u of each slot
            for (int c = opq(tid); c < NC; c += WT) {
                double m, lo, hi;
                slot_bounds(d, c, m, lo, hi);
                double dl = 0.0;
                if (m != 0.0) {
                    double ll = ir[Lo.I_ll + c], lu = ir[Lo.I_lu + c];
                    if (upd) {
                        ll = fmax(ll + alpha * w[Lo.W_dll + c], P.lam_min);
                        lu = fmax(lu + alpha * w[Lo.W_dlu + c], P.lam_min);
                        const double tl = fmax(ir[Lo.I_tl + c] + alpha * w[Lo.W_dtl + c], P.t_min);
                        const double tu = fmax(ir[Lo.I_tu + c] + alpha * w[Lo.W_dtu + c], P.t_min);
                        ir[Lo.I_ll + c] = ll;
                        ir[Lo.I_lu + c] = lu;
                        ir[Lo.I_tl + c] = tl;
                        ir[Lo.I_tu + c] = tu;
                    }
                    dl = m * (ll - lu);
                }
                ev()[c] = dl;
            }
            // primal rows and dynamics multipliers
            for (int j = opq(tid); j < NZ; j += WT) {
                double zz = ir[Lo.I_z + j];
                if (upd && j >= z0) zz += alpha * w[Lo.W_dz + j];
                if (j < z0) zz = 0.0;
                z()[j] = zz;
                if (upd) ir[Lo.I_z + j] = zz;
            }
            for (int i = opq(tid); i < NX; i += WT) {
                double pi = 0.0;
                if (n > 0) {
                    pi = ir[Lo.I_pi + i];
                    if (upd) {
                        pi += alpha * w[Lo.W_dpi + i];
                        ir[Lo.I_pi + i] = pi;
                    }
                }
                t2()[i] = pi;
                if (n == N) {
                    xn(nxt)[i] = 0.0;
                    pin(nxt)[i] = 0.0;
                }
            }
            __syncthreads();
            // r_g = H z + g + F' pi_{n+1} - [0; pi_n] - G' (lam_l - lam_u)
            for (int j = z0 + opq(tid); j < NZ; j += WT) {
                double acc = d[Lo.D_g + j] + dot(d + Lo.D_H + j, NZ, z(), 1, NZ);
                if (n < N) acc += dot(d + Lo.D_F + j * NX, 1, pin(nxt), 1, NX);
                if (j >= NU) acc -= t2()[j - NU];
                acc -= ev()[j];
                acc -= dot(d + Lo.D_G + j * NG, 1, ev() + NZ, 1, NG);
                mg = nmax(mg, fabs(acc));
                w[Lo.W_rg + j] = acc;
            }
            // r_b = F z + b - x_{n+1}
            for (int i = opq(tid); i < NX; i += WT) {
                double rb = 0.0;
                if (n < N) {
                    rb = d[Lo.D_b + i] + dot(d + Lo.D_F + i, NX, z(), 1, NZ) - xn(nxt)[i];
                    mb = nmax(mb, fabs(rb));
                    w[Lo.W_rb + i] = rb;
                }
                rbv()[i] = rb;
            }
            __syncthreads();
            // r_d, complementarity, barrier weights, right-hand-side terms
            for (int c = opq(tid); c < NC; c += WT) {
                double m, lo, hi;
                slot_bounds(d, c, m, lo, hi);
                double wsum = 0.0, rdl = 0.0, rdu = 0.0;
                if (m != 0.0) {
                    const double ll = ir[Lo.I_ll + c], lu = ir[Lo.I_lu + c];
                    const double tl = ir[Lo.I_tl + c], tu = ir[Lo.I_tu + c];
                    const double gz = c < NZ ? z()[c] : dot(d + Lo.D_G + (c - NZ), NG, z(), 1, NZ);
                    rdl = -gz + tl + lo;
                    rdu = gz + tu - hi;
                    md = nmax(md, nmax(fabs(rdl), fabs(rdu)));
                    const double a1 = ll * tl, a2 = lu * tu;
                    mm = nmax(mm, nmax(a1, a2));
                    slt += a1 + a2;
                    wsum = ll / tl + lu / tu;
                }
                w[Lo.W_rdl + c] = rdl;
                w[Lo.W_rdu + c] = rdu;
                wsv()[c] = wsum;
            }
            __syncthreads();
            if (factor) fact_ok = factor_stage(n) && fact_ok;
            // x_n and pi_n for the stage before
            for (int i = opq(tid); i < NX; i += WT) {
                xn(cur)[i] = z()[NU + i];
                pin(cur)[i] = t2()[i];
            }
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

    // M = H + diag(w) + reg I + V'V with V = [Lxx_{n+1}' F; sqrt(w_g) G],
    // factored in place (stage N: its state block only).  Barrier weights of
    // the stage in wsv.
    __device__ __forceinline__ bool factor_stage(int n) const
    {
        const int z0 = zb(n), nz = NZ - z0;
        const double* d = Dp(n);
        double* w = Wp(n);
        double* m = w + Lo.W_L;
        double* V = w + Lo.W_V;
        for (int e = opq(tid); e < nz * nz; e += WT) {
            const int r = z0 + e % nz, c = z0 + e / nz;
            double v = 0.0;
            if (r >= c) v = d[Lo.D_H + r + c * NZ] + (r == c ? wsv()[r] + P.reg_prim : 0.0);
            m[r + c * NZ] = v;
        }
        for (int e = opq(tid); e < NG * nz; e += WT) {
            const int r = e % NG, k = z0 + e / NG;
            V[NX + r + k * NV] = sqrt(wsv()[NZ + r]) * d[Lo.D_G + r + k * NG];
        }
        if (n < N) mma_tn(Lxx(n + 1), 1, NZ, d + Lo.D_F, 1, NX, NX, NZ, NX, V, NV, 0, false);
        __syncthreads();
        const int r0 = n < N ? 0 : NX;
        mma_tn(V + r0 + z0 * NV, 1, NV, V + r0 + z0 * NV, 1, NV, nz, nz, NV - r0, m + z0 + z0 * NZ, NZ, 1, true);
        __syncthreads();
        return cholesky(m + z0 + z0 * NZ, NZ, nz, w + Lo.W_dinv + z0);
    }

    // r_m (lower, upper) of slot c per rmode
    __device__ __forceinline__ void slot_rm(int rmode, double shift, const double* w, int c, double ll, double lu,
                                            double tl, double tu, double& rml, double& rmu) const
    {
        rml = ll * tl - shift;
        rmu = lu * tu - shift;
        if (rmode == RM_CORRECTOR) {
            rml += w[Lo.W_all + c] * w[Lo.W_atl + c];
            rmu += w[Lo.W_alu + c] * w[Lo.W_atu + c];
        }
    }

    // ==================================================================
    // Pass C: backward right-hand-side sweep with the stored factors, for the
    // residuals of pass A and r_m per rmode: y_u = Luu^{-1} m_u and
    // p_n = m_x - Lxu y_u of every stage (workspace W_yu, W_pv).
    // ==================================================================
    __device__ __forceinline__ void passC(int rmode, double shift) const
    {
        for (int n = N; n >= 0; --n) {
            const int cur = n & 1, nxt = cur ^ 1;
            const int z0 = zb(n);
            const double* d = Dp(n);
            const double* ir = Ip(n);
            double* w = Wp(n);
            for (int c = opq(tid); c < NC; c += WT) {
                double m, lo, hi;
                slot_bounds(d, c, m, lo, hi);
                double e = 0.0;
                if (m != 0.0) {
                    const double ll = ir[Lo.I_ll + c], lu = ir[Lo.I_lu + c];
                    const double tl = ir[Lo.I_tl + c], tu = ir[Lo.I_tu + c];
                    double rml, rmu;
                    slot_rm(rmode, shift, w, c, ll, lu, tl, tu, rml, rmu);
                    e = (ll * w[Lo.W_rdl + c] - rml) / tl - (lu * w[Lo.W_rdu + c] - rmu) / tu;
                }
                ev()[c] = e;
            }
            for (int i = opq(tid); i < NX; i += WT) {
                rbv()[i] = n < N ? w[Lo.W_rb + i] : 0.0;
                if (n == N) pn(nxt)[i] = 0.0;
            }
            __syncthreads();
            // reduced gradient: r_g - e_box - G' e_gen
            for (int j = z0 + opq(tid); j < NZ; j += WT)
                mv()[j] = w[Lo.W_rg + j] - ev()[j] - dot(d + Lo.D_G + j * NG, 1, ev() + NZ, 1, NG);
            // cost-to-go of the next stage: + F' (P_{n+1} r_b + p_{n+1})
            if (n < N) {
                ctg(Lxx(n + 1), rbv(), pn(nxt), t2());
                for (int j = opq(tid); j < NZ; j += WT) mv()[j] += dot(d + Lo.D_F + j * NX, 1, t2(), 1, NX);
            }
            __syncthreads();
            const double* L = w + Lo.W_L;
            if (z0 < NU) trsv_lower(L, NZ, NU, mv(), w + Lo.W_dinv);
            for (int k = opq(tid); k < NU; k += WT) w[Lo.W_yu + k] = z0 < NU ? mv()[k] : 0.0;
            for (int i = opq(tid); i < NX; i += WT) {
                const double p = mv()[NU + i] - (z0 < NU ? dot(L + NU + i, NZ, mv(), 1, NU) : 0.0);
                w[Lo.W_pv + i] = p;
                pn(cur)[i] = p;
            }
            __syncthreads();
        }
    }

    // ==================================================================
    // Pass B: forward substitution and recovery of dt, dlam.  Writes dz, dpi
    // (W_dz, W_dpi) and dlam, dt to (oll, olu, otl, otu).  Returns the
    // largest alpha keeping lam, t >= 0 (uncapped; HUGE_VAL if unblocked) and
    // s1 = sum(lam dt + dlam t), s2 = sum(dlam dt).
    // ==================================================================
    __device__ __forceinline__ double passB(int rmode, double shift, int oll, int olu, int otl, int otu, double& o_s1,
                                            double& o_s2) const
    {
        double amin = HUGE_VAL, s1 = 0.0, s2 = 0.0;
        // dx_0 = -(Lxx Lxx')^{-1} p_0 with Lxx the state block of stage 0
        {
            double* w0 = Wp(0);
            for (int i = opq(tid); i < NX; i += WT) {
                xn(0)[i] = -w0[Lo.W_pv + i];
                w0[Lo.W_dpi + i] = 0.0;
            }
            __syncthreads();
            trsv_lower(Lxx(0), NZ, NX, xn(0), w0 + Lo.W_dinv + NU);
            trsv_lower_t(Lxx(0), NZ, NX, xn(0), w0 + Lo.W_dinv + NU);
        }
        for (int n = 0; n <= N; ++n) {
            const int cur = n & 1, nxt = cur ^ 1;
            const int z0 = zb(n);
            const double* d = Dp(n);
            const double* ir = Ip(n);
            double* w = Wp(n);
            const double* L = w + Lo.W_L;
            // du = -Luu^{-T} (y_u + Lxu' dx)
            if (z0 < NU) {
                for (int k = opq(tid); k < NU; k += WT)
                    mv()[k] = w[Lo.W_yu + k] + dot(L + NU + k * NZ, 1, xn(cur), 1, NX);
                __syncthreads();
                trsv_lower_t(L, NZ, NU, mv(), w + Lo.W_dinv);
            }
            for (int j = opq(tid); j < NZ; j += WT) {
                const double dz = j < z0 ? 0.0 : (j < NU ? -mv()[j] : xn(cur)[j - NU]);
                z()[j] = dz;
                w[Lo.W_dz + j] = dz;
            }
            __syncthreads();
            if (n < N) {
                // dx_{n+1} = F dz + r_b, dpi_{n+1} = P_{n+1} dx_{n+1} + p_{n+1}
                for (int i = opq(tid); i < NX; i += WT)
                    xn(nxt)[i] = w[Lo.W_rb + i] + dot(d + Lo.D_F + i, NX, z(), 1, NZ);
                double* w1 = Wp(n + 1);
                for (int i = opq(tid); i < NX; i += WT) pn(nxt)[i] = w1[Lo.W_pv + i];
                __syncthreads();
                ctg(Lxx(n + 1), xn(nxt), pn(nxt), t2());
                for (int i = opq(tid); i < NX; i += WT) w1[Lo.W_dpi + i] = t2()[i];
            }
            // constraint steps, step length, duality-measure sums
            for (int c = opq(tid); c < NC; c += WT) {
                double m, lo, hi;
                slot_bounds(d, c, m, lo, hi);
                double dll = 0.0, dlu = 0.0, dtl = 0.0, dtu = 0.0;
                if (m != 0.0) {
                    const double ll = ir[Lo.I_ll + c], lu = ir[Lo.I_lu + c];
                    const double tl = ir[Lo.I_tl + c], tu = ir[Lo.I_tu + c];
                    double rml, rmu;
                    slot_rm(rmode, shift, w, c, ll, lu, tl, tu, rml, rmu);
                    const double gdz = c < NZ ? z()[c] : dot(d + Lo.D_G + (c - NZ), NG, z(), 1, NZ);
                    dtl = gdz - w[Lo.W_rdl + c];
                    dtu = -gdz - w[Lo.W_rdu + c];
                    dll = -(rml + ll * dtl) / tl;
                    dlu = -(rmu + lu * dtu) / tu;
                    if (dll < 0.0) amin = fmin(amin, -ll / dll);
                    if (dlu < 0.0) amin = fmin(amin, -lu / dlu);
                    if (dtl < 0.0) amin = fmin(amin, -tl / dtl);
                    if (dtu < 0.0) amin = fmin(amin, -tu / dtu);
                    s1 += ll * dtl + dll * tl + lu * dtu + dlu * tu;
                    s2 += dll * dtl + dlu * dtu;
                }
                w[oll + c] = dll;
                w[olu + c] = dlu;
                w[otl + c] = dtl;
                w[otu + c] = dtu;
            }
            __syncthreads();
        }
        amin = bmin_sum2(amin, s1, s2);
        o_s1 = s1;
        o_s2 = s2;
        return amin;
    }

    __device__ __forceinline__ void copy_step_out(double* out) const
    {
        for (int n = 0; n <= N; ++n) {
            double* o = out + (size_t)n * Lo.IREC;
            const double* w = Wp(n);
            for (int j = opq(tid); j < NZ; j += WT) o[Lo.I_z + j] = w[Lo.W_dz + j];
            for (int i = opq(tid); i < NX; i += WT) o[Lo.I_pi + i] = w[Lo.W_dpi + i];
            for (int c = opq(tid); c < NC; c += WT) {
                o[Lo.I_ll + c] = w[Lo.W_dll + c];
                o[Lo.I_lu + c] = w[Lo.W_dlu + c];
                o[Lo.I_tl + c] = w[Lo.W_dtl + c];
                o[Lo.I_tu + c] = w[Lo.W_dtu + c];
            }
        }
        __syncthreads();
    }

    // ------------------------------------------------------------------
    // Driver.  Solve mode: the IPM from the initial point.  Newton mode: one
    // Newton step at the stored iterate with r_m = lam.*t - tau.
    // ------------------------------------------------------------------
    __device__ __forceinline__ void run(DevStat* st, double* step_out, int resume, int itcap) const
    {
        const bool newton_mode = P.mode == KMODE_NEWTON;
        if (!newton_mode) init(resume ? 2 : P.warm);
        const int cap = itcap > 0 ? min(P.iter_max, itcap) : P.iter_max;
        int status = ST_MAX_ITER, k = 0;
        double ng = 0, nb = 0, nd = 0, nm = 0, mu = 0.0, slt = 0.0;
        const double inv2nc = nc > 0 ? 1.0 / (2.0 * nc) : 0.0;
        const double shift0 = newton_mode ? P.tau : 0.0;
        bool upd = false, rejected = false;
        double alpha = 0.0;
        for (k = 0;; ++k) {
            const bool fact_ok = passA(upd, alpha, !rejected && (newton_mode || k < cap), ng, nb, nd, nm, slt);
            mu = slt * inv2nc;
            if (rejected) {
                status = ST_MIN_STEP;
                break;
            }
            if (!newton_mode) {
                if (!fact_ok || ng != ng || nb != nb || nd != nd || nm != nm || mu != mu) {
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
            // round 0: predictor (in Newton mode the step itself); round 1:
            // Mehrotra corrector; round 2: predictor-centering step when the
            // conditional corrector is rejected (Section 4.2)
            double amax = HUGE_VAL, mu_aff = 0.0, smu = 0.0;
            for (int round = 0; round < 3; ++round) {
                const int rmode = round == 1 ? RM_CORRECTOR : RM_SHIFT;
                const double shift = round == 0 ? shift0 : smu;
                const bool aff = round == 0 && !newton_mode;
                passC(rmode, shift);
                double s1, s2;
                amax = aff ? passB(rmode, shift, Lo.W_all, Lo.W_alu, Lo.W_atl, Lo.W_atu, s1, s2)
                           : passB(rmode, shift, Lo.W_dll, Lo.W_dlu, Lo.W_dtl, Lo.W_dtu, s1, s2);
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
        if (tid == 0) {
            st->status = status;
            st->iters = k;
            st->ir_steps = 0;
            st->fell_back = FB_NONE;
            st->qr_refactors = 0;
            st->mu = mu;
            st->res[0] = ng;
            st->res[1] = nb;
            st->res[2] = nd;
            st->res[3] = nm;
        }
    }
};

}  // namespace

// Three workgroups per CU (130 VGPRs).  Forcing four (114 VGPRs, no spills)
// keeps a whole batch of 1024 fully condensed 8-mass instances resident but
// makes the solve slower (104 -> 123 ms): more instances' stage matrices
// compete for the same L2.
__global__ __launch_bounds__(WT) void ipm_wide_kernel(const InstDesc* __restrict__ desc, int count,
                                                      const double* __restrict__ data, double* __restrict__ iter,
                                                      double* __restrict__ work, double* __restrict__ step_out,
                                                      DevStat* __restrict__ stat, KParams P)
{
    const int b = blockIdx.x;
    // no mixed build: nothing is ever handed over to this kernel
    if (b >= count || P.mode == KMODE_FALLBACK) return;
    const InstDesc ds = desc[b];
    const Wide ipm(ds, data, iter, work, P);
    ipm.run(stat + ds.index, step_out + ds.iter, ds.resume, ds.itcap);
}

int wide_lds_bytes(int nx, int nu, int ng) { return (int)sizeof(double) * make_wlds(nx, nu, ng).total; }

int wide_launch(const InstDesc* desc, int count, const double* data, double* iter, double* work, double* step,
                DevStat* stat, const KParams& P, size_t lds_bytes, void* stream)
{
    if (count <= 0) return 0;
    hipLaunchKernelGGL(ipm_wide_kernel, dim3(count), dim3(WT), lds_bytes, (hipStream_t)stream, desc, count, data, iter,
                       work, step, stat, P);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace oqp
