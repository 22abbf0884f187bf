// Partial condensing of batched OCP QPs and expansion of their solutions
// (Section 3.5), on gfx950.
//
// A block of stages [s0, s1) becomes one stage of the condensed QP with
// input u_bar = [u_s0; ...; u_{s1-1}] and state x_bar = x_s0 (the state at the
// block start stays a variable).  One 256-thread workgroup condenses one
// block of one instance: it steps the affine maps x_n = Gam_n [u_bar; x_bar] +
// gam_n through the block (Gam_{n+1} = A_n Gam_n + B_n S_n, S_n selecting u_n
// from u_bar), in LDS, and accumulates along the way
//   H_bar += E_n' H_n E_n,  g_bar += E_n' (H_n e_n + g_n),
// with E_n = [S_n; Gam_n] and e_n = [0; gam_n], into the condensed record in
// HBM; the block's end map is the condensed dynamics [B_bar A_bar], b_bar.
// Input boxes keep their mask at their offset in u_bar, the box on x_s0 stays
// a box, state boxes of later stages become general rows Gam_n[i, :] with
// bounds shifted by gam_n[i], and general rows become D_n S_n + C_n Gam_n with
// bounds shifted by C_n gam_n.  Rows of a condensed stage are ordered stage by
// stage: state-box rows (increasing component), then general rows.
//
// Expansion maps the condensed solution back: inputs and block-start states
// are copied, interior states follow from the dynamics, every constraint
// takes the multipliers and slacks of its condensed row, the dynamics
// multiplier at a block end is the condensed one, and interior dynamics
// multipliers solve the state rows of the stationarity residual r_g of
// eq:alg:pdipm:delta, backwards through the block:
//   pi_n = (H_n z_n + g_n)_x + A_n' pi_{n+1} - G_{n,x}' (lam_l - lam_u).
//
// Both kernels run once per solve (not per IPM iteration).  Instances and
// blocks are independent: the grid is one workgroup per (instance, block),
// the terminal stage N being a block of its own.
#include <hip/hip_runtime.h>

#include "layout.h"

namespace oqp {

static constexpr int CT = 256;  // threads per workgroup

// dynamic LDS of the condensing kernel (doubles): the maps Gam (two buffers,
// onx x cnz), W = H_n E_n ((onx + onu) x cnz), gam (two buffers), w
struct CondLds {
    int G0, G1, W, g0, g1, w, total;
};

__host__ __device__ inline CondLds cond_lds(int onx, int onu, int cnz)
{
    CondLds L{};
    int o = 0;
    L.G0 = o; o += onx * cnz;
    L.G1 = o; o += onx * cnz;
    L.W = o; o += (onx + onu) * cnz;
    L.g0 = o; o += onx;
    L.g1 = o; o += onx;
    L.w = o; o += onx + onu;
    L.total = o;
    return L;
}

struct BlockRange {
    int s0, s1;
};

__device__ inline BlockRange block_range(const CondDesc& D, const int* bs, int b)
{
    return b < D.N2 ? BlockRange{bs[b], bs[b + 1]} : BlockRange{D.N, D.N + 1};
}

__global__ void __launch_bounds__(CT) pcond_condense_kernel(const CondDesc* __restrict__ cds,
                                                            const CondItem* __restrict__ items,
                                                            const int* __restrict__ tab,
                                                            const double* __restrict__ odata,
                                                            double* __restrict__ cdata)
{
    extern __shared__ double lds[];
    const CondItem it = items[blockIdx.x];
    const CondDesc D = cds[it.inst];
    const int tid = (int)threadIdx.x;
    const Layout Lo = make_layout(D.onx, D.onu, D.ong);
    const Layout Lc = make_layout(D.cnx, D.cnu, D.cng);
    const int* st = tab + D.tab;  // nx, nu, nbx, ng per original stage
    const int* bs = st + 4 * (D.N + 1);
    const int b = it.block;
    const BlockRange br = block_range(D, bs, b);
    const int ONX = Lo.NX, ONU = Lo.NU, ONZ = Lo.NZ, ONG = Lo.NG > 0 ? Lo.NG : 1;
    const int CNX = Lc.NX, CNU = Lc.NU, CNZ = Lc.NZ, CNG = Lc.NG > 0 ? Lc.NG : 1;
    const CondLds C = cond_lds(ONX, ONU, CNZ);
    double* out = cdata + D.cdata + (int64_t)b * Lc.SREC;
    const int nxs = st[4 * br.s0];
    int nU = 0;
    for (int n = br.s0; n < br.s1; ++n) nU += st[4 * n + 1];

    double* G = lds + C.G0;
    double* Gn = lds + C.G1;
    double* g = lds + C.g0;
    double* gn = lds + C.g1;
    double* W = lds + C.W;
    double* w = lds + C.w;
    for (int e = tid; e < Lc.SREC; e += CT) out[e] = 0.0;
    // Gam at the block start: x_s0 = x_bar
    for (int e = tid; e < ONX * CNZ; e += CT) {
        const int i = e % ONX, c = e / ONX;
        G[e] = (i < nxs && c == CNU + i) ? 1.0 : 0.0;
    }
    for (int i = tid; i < ONX; i += CT) g[i] = 0.0;
    __syncthreads();
    // padded components: unit Hessian diagonal
    for (int c = tid; c < CNZ; c += CT)
        if ((c >= nU && c < CNU) || c >= CNU + nxs) out[Lc.D_H + c + c * CNZ] = 1.0;

    int off = 0, row = 0;
    for (int n = br.s0; n < br.s1; ++n) {
        const int nx = st[4 * n], nu = st[4 * n + 1], nbx = st[4 * n + 2], ng = st[4 * n + 3];
        const int nz = nu + nx;
        const double* rec = odata + D.odata + (int64_t)n * Lo.SREC;
        const double* H = rec + Lo.D_H;
        const double* Gr = rec + Lo.D_G;
        // E_n = [S_n; Gam_n] is zero in the columns of the inputs of later
        // stages: only the na active columns (inputs up to this stage, then
        // the block-start state) take part in W and in the update of H_bar
        const int nin = off + nu, na = nin + nxs;
        // W = H_n E_n, w = H_n e_n + g_n (rows: u_n then x_n)
        for (int e = tid; e < nz * na; e += CT) {
            const int r = e % nz, a = e / nz;
            const int c = a < nin ? a : CNU + (a - nin);
            const int hr = r < nu ? r : ONU + (r - nu);
            double acc = (c >= off && c < off + nu) ? H[hr + (c - off) * ONZ] : 0.0;
            for (int i = 0; i < nx; ++i) acc += H[hr + (ONU + i) * ONZ] * G[i + c * ONX];
            W[r + c * nz] = acc;
        }
        for (int r = tid; r < nz; r += CT) {
            const int hr = r < nu ? r : ONU + (r - nu);
            double acc = rec[Lo.D_g + hr];
            for (int i = 0; i < nx; ++i) acc += H[hr + (ONU + i) * ONZ] * g[i];
            w[r] = acc;
        }
        __syncthreads();
        // H_bar += E_n' W on the lower triangle (mirrored once at the end of
        // the block, so H_bar is exactly symmetric), g_bar += E_n' w.  Each
        // thread updates four entries per round: their four loads of H_bar
        // are in flight together
        for (int e0 = tid; e0 < na * na; e0 += 4 * CT) {
            int ix[4];
            double cur[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = e0 + q * CT;
                const int a1 = e % na, a2 = e / na;
                ix[q] = -1;
                if (e < na * na && a1 >= a2) {
                    const int c1 = a1 < nin ? a1 : CNU + (a1 - nin), c2 = a2 < nin ? a2 : CNU + (a2 - nin);
                    ix[q] = c1 + c2 * CNZ;
                }
                cur[q] = ix[q] >= 0 ? out[Lc.D_H + ix[q]] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (ix[q] < 0) continue;
                const int c1 = ix[q] % CNZ, c2 = ix[q] / CNZ;
                double acc = (c1 >= off && c1 < off + nu) ? W[(c1 - off) + c2 * nz] : 0.0;
                for (int i = 0; i < nx; ++i) acc += G[i + c1 * ONX] * W[(nu + i) + c2 * nz];
                out[Lc.D_H + ix[q]] = cur[q] + acc;
            }
        }
        for (int c1 = tid; c1 < CNZ; c1 += CT) {
            double acc = (c1 >= off && c1 < off + nu) ? w[c1 - off] : 0.0;
            for (int i = 0; i < nx; ++i) acc += G[i + c1 * ONX] * w[nu + i];
            out[Lc.D_g + c1] += acc;
        }
        // input boxes
        for (int j = tid; j < nu; j += CT)
            if (rec[Lo.D_bm + j] != 0.0) {
                out[Lc.D_bm + off + j] = 1.0;
                out[Lc.D_blo + off + j] = rec[Lo.D_blo + j];
                out[Lc.D_bhi + off + j] = rec[Lo.D_bhi + j];
            }
        if (n == br.s0) {
            // box on the block-start state
            for (int i = tid; i < nx; i += CT)
                if (rec[Lo.D_bm + ONU + i] != 0.0) {
                    out[Lc.D_bm + CNU + i] = 1.0;
                    out[Lc.D_blo + CNU + i] = rec[Lo.D_blo + ONU + i];
                    out[Lc.D_bhi + CNU + i] = rec[Lo.D_bhi + ONU + i];
                }
        } else {
            // interior state boxes become general rows
            for (int e = tid; e < nx * CNZ; e += CT) {
                const int i = e % nx, c = e / nx;
                if (rec[Lo.D_bm + ONU + i] == 0.0) continue;
                int rk = 0;
                for (int l = 0; l < i; ++l) rk += rec[Lo.D_bm + ONU + l] != 0.0 ? 1 : 0;
                const int rho = row + rk;
                out[Lc.D_G + rho + c * CNG] = G[i + c * ONX];
                if (c == 0) {
                    out[Lc.D_gm + rho] = 1.0;
                    out[Lc.D_glo + rho] = rec[Lo.D_blo + ONU + i] - g[i];
                    out[Lc.D_ghi + rho] = rec[Lo.D_bhi + ONU + i] - g[i];
                }
            }
            row += nbx;
        }
        // general rows
        for (int e = tid; e < ng * CNZ; e += CT) {
            const int r = e % ng, c = e / ng;
            double acc = (c >= off && c < off + nu) ? Gr[r + (c - off) * ONG] : 0.0;
            for (int i = 0; i < nx; ++i) acc += Gr[r + (ONU + i) * ONG] * G[i + c * ONX];
            out[Lc.D_G + (row + r) + c * CNG] = acc;
        }
        for (int r = tid; r < ng; r += CT) {
            double sh = 0.0;
            for (int i = 0; i < nx; ++i) sh += Gr[r + (ONU + i) * ONG] * g[i];
            out[Lc.D_gm + row + r] = 1.0;
            out[Lc.D_glo + row + r] = rec[Lo.D_glo + r] - sh;
            out[Lc.D_ghi + row + r] = rec[Lo.D_ghi + r] - sh;
        }
        row += ng;
        // step the maps through the dynamics of stage n
        if (n < D.N) {
            const int nxn = st[4 * (n + 1)];
            const double* F = rec + Lo.D_F;
            for (int e = tid; e < nxn * CNZ; e += CT) {
                const int i = e % nxn, c = e / nxn;
                double acc = (c >= off && c < off + nu) ? F[i + (c - off) * ONX] : 0.0;
                for (int l = 0; l < nx; ++l) acc += F[i + (ONU + l) * ONX] * G[l + c * ONX];
                Gn[i + c * ONX] = acc;
            }
            for (int i = tid; i < nxn; i += CT) {
                double acc = rec[Lo.D_b + i];
                for (int l = 0; l < nx; ++l) acc += F[i + (ONU + l) * ONX] * g[l];
                gn[i] = acc;
            }
        }
        __syncthreads();
        double* t = G; G = Gn; Gn = t;
        t = g; g = gn; gn = t;
        off += nu;
    }
    // upper triangle of H_bar from the lower one (the padded unit diagonal
    // has no off-diagonal entries)
    __syncthreads();
    for (int e = tid; e < CNZ * CNZ; e += CT) {
        const int r = e % CNZ, c = e / CNZ;
        if (r < c) out[Lc.D_H + e] = out[Lc.D_H + c + r * CNZ];
    }
    // condensed dynamics: the map at the block end
    if (b < D.N2) {
        const int nxn = st[4 * br.s1];
        for (int e = tid; e < nxn * CNZ; e += CT) {
            const int i = e % nxn, c = e / nxn;
            out[Lc.D_F + i + c * CNX] = G[i + c * ONX];
        }
        for (int i = tid; i < nxn; i += CT) out[Lc.D_b + i] = g[i];
    }
}

__device__ inline void copy_slot(double* o, const Layout& Lo, int so, const double* c, const Layout& Lc, int sc)
{
    o[Lo.I_ll + so] = c[Lc.I_ll + sc];
    o[Lo.I_lu + so] = c[Lc.I_lu + sc];
    o[Lo.I_tl + so] = c[Lc.I_tl + sc];
    o[Lo.I_tu + so] = c[Lc.I_tu + sc];
}

__global__ void __launch_bounds__(CT) pcond_expand_kernel(const CondDesc* __restrict__ cds,
                                                          const CondItem* __restrict__ items,
                                                          const int* __restrict__ tab,
                                                          const double* __restrict__ odata,
                                                          const double* __restrict__ citer, double* oiter)
{
    const CondItem it = items[blockIdx.x];
    const CondDesc D = cds[it.inst];
    const int tid = (int)threadIdx.x;
    const Layout Lo = make_layout(D.onx, D.onu, D.ong);
    const Layout Lc = make_layout(D.cnx, D.cnu, D.cng);
    const int* st = tab + D.tab;
    const int* bs = st + 4 * (D.N + 1);
    const int b = it.block;
    const BlockRange br = block_range(D, bs, b);
    const int ONX = Lo.NX, ONU = Lo.NU, ONZ = Lo.NZ, ONG = Lo.NG > 0 ? Lo.NG : 1;
    const int CNU = Lc.NU, CNZ = Lc.NZ;
    const double* crec = citer + D.citer + (int64_t)b * Lc.IREC;
    double* obase = oiter + D.oiter;
    const int nxs = st[4 * br.s0];

    for (int n = br.s0; n < br.s1; ++n) {
        double* orc = obase + (int64_t)n * Lo.IREC;
        for (int e = tid; e < Lo.IREC; e += CT) orc[e] = 0.0;
    }
    __syncthreads();
    // inputs, block-start state and the dynamics multiplier at the block start
    {
        int off = 0;
        for (int n = br.s0; n < br.s1; ++n) {
            const int nu = st[4 * n + 1];
            double* orc = obase + (int64_t)n * Lo.IREC;
            for (int j = tid; j < nu; j += CT) orc[Lo.I_z + j] = crec[Lc.I_z + off + j];
            off += nu;
        }
        double* o0 = obase + (int64_t)br.s0 * Lo.IREC;
        for (int i = tid; i < nxs; i += CT) {
            o0[Lo.I_z + ONU + i] = crec[Lc.I_z + CNU + i];
            if (br.s0 > 0) o0[Lo.I_pi + i] = crec[Lc.I_pi + i];
        }
    }
    __syncthreads();
    // interior states from the dynamics
    for (int n = br.s0; n + 1 < br.s1; ++n) {
        const int nx = st[4 * n], nu = st[4 * n + 1], nxn = st[4 * (n + 1)];
        const double* rec = odata + D.odata + (int64_t)n * Lo.SREC;
        const double* F = rec + Lo.D_F;
        const double* z = obase + (int64_t)n * Lo.IREC + Lo.I_z;
        double* xo = obase + (int64_t)(n + 1) * Lo.IREC + Lo.I_z + ONU;
        for (int i = tid; i < nxn; i += CT) {
            double acc = rec[Lo.D_b + i];
            for (int j = 0; j < nu; ++j) acc += F[i + j * ONX] * z[j];
            for (int l = 0; l < nx; ++l) acc += F[i + (ONU + l) * ONX] * z[ONU + l];
            xo[i] = acc;
        }
        __syncthreads();
    }
    // multipliers and slacks of every constraint
    {
        int off = 0, row = 0;
        for (int n = br.s0; n < br.s1; ++n) {
            const int nx = st[4 * n], nu = st[4 * n + 1], nbx = st[4 * n + 2], ng = st[4 * n + 3];
            const double* rec = odata + D.odata + (int64_t)n * Lo.SREC;
            double* orc = obase + (int64_t)n * Lo.IREC;
            for (int j = tid; j < nu; j += CT) copy_slot(orc, Lo, j, crec, Lc, off + j);
            if (n == br.s0) {
                for (int i = tid; i < nx; i += CT) copy_slot(orc, Lo, ONU + i, crec, Lc, CNU + i);
            } else {
                for (int i = tid; i < nx; i += CT) {
                    if (rec[Lo.D_bm + ONU + i] == 0.0) continue;
                    int rk = 0;
                    for (int l = 0; l < i; ++l) rk += rec[Lo.D_bm + ONU + l] != 0.0 ? 1 : 0;
                    copy_slot(orc, Lo, ONU + i, crec, Lc, CNZ + row + rk);
                }
                row += nbx;
            }
            for (int r = tid; r < ng; r += CT) copy_slot(orc, Lo, ONZ + r, crec, Lc, CNZ + row + r);
            row += ng;
            off += nu;
        }
    }
    __syncthreads();
    // interior dynamics multipliers, backwards from the condensed one at the
    // block end
    if (b < D.N2) {
        const double* pend = citer + D.citer + (int64_t)(b + 1) * Lc.IREC + Lc.I_pi;
        for (int n = br.s1 - 1; n > br.s0; --n) {
            const int nx = st[4 * n], nu = st[4 * n + 1], ng = st[4 * n + 3], nxn = st[4 * (n + 1)];
            const double* rec = odata + D.odata + (int64_t)n * Lo.SREC;
            const double* H = rec + Lo.D_H;
            const double* F = rec + Lo.D_F;
            const double* Gr = rec + Lo.D_G;
            double* orc = obase + (int64_t)n * Lo.IREC;
            const double* pn = n + 1 == br.s1 ? pend : obase + (int64_t)(n + 1) * Lo.IREC + Lo.I_pi;
            for (int i = tid; i < nx; i += CT) {
                const int hr = ONU + i;
                double acc = rec[Lo.D_g + hr];
                for (int j = 0; j < nu; ++j) acc += H[hr + j * ONZ] * orc[Lo.I_z + j];
                for (int l = 0; l < nx; ++l) acc += H[hr + (ONU + l) * ONZ] * orc[Lo.I_z + ONU + l];
                for (int r = 0; r < nxn; ++r) acc += F[r + hr * ONX] * pn[r];
                if (rec[Lo.D_bm + hr] != 0.0) acc -= orc[Lo.I_ll + hr] - orc[Lo.I_lu + hr];
                for (int r = 0; r < ng; ++r) acc -= Gr[r + hr * ONG] * (orc[Lo.I_ll + ONZ + r] - orc[Lo.I_lu + ONZ + r]);
                orc[Lo.I_pi + i] = acc;
            }
            __syncthreads();
        }
    }
}

int cond_lds_bytes(int onx, int onu, int cnz) { return (int)(sizeof(double) * cond_lds(onx, onu, cnz).total); }

int cond_launch(int expand, const CondDesc* cds, const CondItem* items, int nitems, const int* tab,
                const double* odata, double* cdata, const double* citer, double* oiter, size_t lds_bytes,
                void* stream)
{
    if (nitems <= 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    if (expand)
        hipLaunchKernelGGL(pcond_expand_kernel, dim3(nitems), dim3(CT), 0, s, cds, items, tab, odata, citer, oiter);
    else
        hipLaunchKernelGGL(pcond_condense_kernel, dim3(nitems), dim3(CT), lds_bytes, s, cds, items, tab, odata,
                           cdata);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace oqp
