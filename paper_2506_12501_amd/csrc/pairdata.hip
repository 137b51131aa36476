// pairdata.hip -- primitive-pair data for one side of a class of shellsets.
//
// For every shell pair and every primitive pair (zeta_a, zeta_b) it writes
//   zeta_p, P (Sec. 2.1, after Eq. (8)) and the Hermite-to-AO matrix
//   H_ab^p = sum_{a,b} C^a C^b E_ab^p   (Eq. (19); C = identity for Cartesian)
// with E from the recursion of Eqs. (10)-(11) bootstrapped by Eq. (14), and
// all primitive prefactors folded in:
//   bra: 2 pi^{5/2} K_AB c_a c_b / zeta_p        (from [0]^(m), Eq. (27))
//   ket: (-1)^{l_q} K_CD c_c c_d / zeta_q         (sign of Eq. (25))
// A single-function solid side (3-/2-centre, Sec. 2.2.3) keeps only the
// terminal Hermites p = a, whose coefficient is (2 zeta_a)^{-l_a} (Eq. (16));
// its H is the bare C and the primitive weight goes to [0]^(m) instead.
// A single-function Cartesian side uses the 2-centre recursion with a unit
// partner (zeta_b = 0, b = 0).
#include "kernels.h"

namespace mdx {


__device__ __forceinline__ void cart_of(int l, int idx, int &ax, int &ay, int &az)
{
    // inverse of the Cartesian order (l,0,0),(l-1,1,0),(l-1,0,1),...
    int s = 0;
    while ((s + 1) * (s + 2) / 2 <= idx) ++s;
    az = idx - s * (s + 1) / 2;
    ay = s - az;
    ax = l - s;
}

// LDS of one item (one primitive pair, or one pair of a grouped side)
struct PdLayout {
    int EA, EB, ET;   // E[3][EA][EB][ET]
    int na, nb;       // output functions per centre
};

__host__ __device__ inline PdLayout pd_layout(const SideGeom &g)
{
    PdLayout L;
    const int d = g.role == 2 ? 1 : 0;
    const int lb = g.lb < 0 ? 0 : g.lb;
    L.EA = g.la + d + 1;
    L.EB = lb + d + 1;
    L.ET = g.la + lb + 2 * d + 1;
    L.na = nfunc(g.la, g.cart);
    L.nb = g.lb >= 0 ? nfunc(lb, g.cart) : 1;
    return L;
}

constexpr int PD_NTM = 10;      // nonzero Cartesian terms per real solid harmonic, l <= 7
constexpr int PD_THREADS = 256;

// doubles of one item's E table plus its prefactor slot (kept even for 16-byte alignment)
__host__ __device__ inline int pd_item_doubles(const SideGeom &g)
{
    const PdLayout L = pd_layout(g);
    return (3 * L.EA * L.EB * L.ET + 2) & ~1;
}

__host__ __device__ inline size_t pairdata_lds_bytes(const SideGeom &g, int per_block)
{
    const PdLayout L = pd_layout(g);
    const size_t nf = L.na + L.nb;
    return ((size_t)per_block * pd_item_doubles(g) + nf * PD_NTM) * 8 + (nf + nf * PD_NTM * 3) * 4;
}

// H elements a typical item writes (rows x padded columns; the derivative
// role six blocks).  The last primitive of a pair also zeroes the rows up to
// the next 16-row tile, in more passes of the same threads; sizing groups by
// that rare case gave an s item 128 threads for its 16 elements.
static int pd_item_elements(const SideGeom &g)
{
    if (g.grouped) return (g.role == 0 ? g.rows_per_block : g.nterm) * g.ncolp;
    if (g.role == 1) return g.rows_per_block * g.ncolp;
    return (g.role == 2 ? 6 : 1) * g.nh * g.ncolp;
}

// Items per 256-thread workgroup: each item gets a power-of-two group of
// threads, about one thread per four H elements (at least 4, for the three
// E recursions; at most the whole workgroup).  Small s/p items share a
// workgroup: a workgroup's fixed latency (record loads, recursion, barrier)
// is paid once for up to 64 items.
static int pd_per_block(const SideGeom &g)
{
    const int e = pd_item_elements(g);
    int t = 4;
    while (t < PD_THREADS && 4 * t < e) t *= 2;
    return PD_THREADS / t;
}

// workgroup blk of the launch of one side record
__device__ __forceinline__ void pairdata_block(const PairDataArgs &a, int blk)
{
    const SideGeom &g = a.g;
    const int G = a.per_block;                      // items of this workgroup
    const int T = PD_THREADS / G;                   // threads of one item
    const int slot = (int)threadIdx.x / T, lt = (int)threadIdx.x % T;
    const int item = blk * G + slot;
    const int nitem = g.grouped ? g.npair : a.nitems;
    const bool live = item < nitem;                 // dead slots still reach every barrier
    // one item = one primitive pair of a pair (items), or one pair (grouped side)
    int pair = 0, k = 0;
    if (live) {
        if (g.grouped) {
            pair = item;
        } else {
            const int2 it = a.items[item];
            pair = it.x;
            k = it.y;
        }
    }
    const PairRec pr = a.pairs[pair];
    const int np = pr.ka * pr.kb;
    const int la = g.la;
    const int lb = g.lb < 0 ? 0 : g.lb;
    const PdLayout PL = pd_layout(g);
    const int EA = PL.EA, EB = PL.EB, ET = PL.ET;
    extern __shared__ double pd_smem[];
    double *Eb = pd_smem + slot * pd_item_doubles(g);         // [3][EA][EB][ET] of this item
#define E(ax, i, j, t) Eb[(((ax) * EA + (i)) * EB + (j)) * ET + (t)]
    double &sh_pref = Eb[3 * EA * EB * ET];
    double *ta_w = pd_smem + G * pd_item_doubles(g);       // [na][NTM], shared by the items
    double *tb_w = ta_w + PL.na * PD_NTM;                   // [nb][NTM]
    int *ta_n = (int *)(tb_w + PL.nb * PD_NTM);             // [na]
    int *tb_n = ta_n + PL.na;                               // [nb]
    int *ta_c = tb_n + PL.nb;                               // [na][NTM][3]
    int *tb_c = ta_c + PL.na * PD_NTM * 3;                  // [nb][NTM][3]

    if (live && lt == 0 && k == 0) a.nprim[pair] = np;

    const double A0 = a.center[3 * pr.sa], A1 = a.center[3 * pr.sa + 1], A2 = a.center[3 * pr.sa + 2];
    double B[3] = {A0, A1, A2};
    if (g.lb >= 0) {
        B[0] = a.center[3 * pr.sb]; B[1] = a.center[3 * pr.sb + 1]; B[2] = a.center[3 * pr.sb + 2];
    }
    const double Av[3] = {A0, A1, A2};

    if (g.grouped) {
        // single-function solid side: primitive records carry the weights
        if (!live) return;                          // no barrier on this path
        for (int kk = lt; kk < g.kmax; kk += T) {
            PrimRec r{};
            if (kk < np) {
                const double z = a.expo[pr.offa + kk], c = a.coef[pr.offa + kk];
                const double w = c * pow(2.0 * z, -(double)la) / z;
                r.p = z; r.Px = A0; r.Py = A1; r.Pz = A2;
                r.ws = (g.role == 0 ? 2.0 * 17.493418327624862 : 1.0) * w;   // 2 pi^{5/2}
                r.wt = (g.role == 1 && (la & 1)) ? -1.0 : 1.0;
            } else {
                r.p = 1.0; r.Px = A0; r.Py = A1; r.Pz = A2; r.ws = 0.0; r.wt = 0.0;
            }
            a.prim[pair * g.kmax + kk] = r;
        }
        const double sgn = (g.role == 1 && (la & 1)) ? -1.0 : 1.0;
        double *Hp = a.H + (int64_t)pair * g.pair_stride;
        const int nrows = g.rows_per_block;
        for (int e = lt; e < nrows * g.ncolp; e += T) {
            const int row = e / g.ncolp, col = e % g.ncolp;
            double v = 0.0;
            if (row < g.nterm && col < g.ncol) v = sgn * (g.cart ? (row == col ? 1.0 : 0.0) : a.Ca[col * ncart(la) + row]);
            Hp[e] = v;
        }
        // bra role pads rows to 16
        if (g.role == 0)
            for (int e = nrows * g.ncolp + lt; e < g.pair_stride; e += T) Hp[e] = 0.0;
        return;
    }

    // nonzero Cartesian->solid terms of every output function, both centres
    // (at most PD_NTM nonzero terms per real solid harmonic; one per Cartesian);
    // class constants, built once per workgroup
    constexpr int NTM = PD_NTM;
    const int nb_out = g.lb >= 0 ? nfunc(lb, g.cart) : 1;
    const int na_out = nfunc(la, g.cart);
    for (int side = 0; side < 2; ++side) {
        const int l = side == 0 ? la : lb, nout = side == 0 ? na_out : nb_out;
        const double *C = side == 0 ? a.Ca : a.Cb;
        const bool unit = side == 1 && g.lb < 0;
        for (int mo = (int)threadIdx.x; mo < nout; mo += PD_THREADS) {
            int n = 0;
            for (int ic = 0; ic < ncart(l); ++ic) {
                const double w = unit ? 1.0 : (g.cart ? (ic == mo ? 1.0 : 0.0) : C[mo * ncart(l) + ic]);
                if (w == 0.0 || n == NTM) continue;
                int x, y, z;
                cart_of(l, ic, x, y, z);
                (side == 0 ? ta_c : tb_c)[(mo * NTM + n) * 3 + 0] = x;
                (side == 0 ? ta_c : tb_c)[(mo * NTM + n) * 3 + 1] = y;
                (side == 0 ? ta_c : tb_c)[(mo * NTM + n) * 3 + 2] = z;
                (side == 0 ? ta_w : tb_w)[mo * NTM + n] = w;
                ++n;
            }
            (side == 0 ? ta_n : tb_n)[mo] = n;
        }
    }

    const bool valid = live && k < np;
    double za = 1.0, zb = 0.0, ca = 0.0, cb = 1.0;
    if (valid) {
        const int ka = k / pr.kb, kb = k % pr.kb;
        za = a.expo[pr.offa + ka];
        ca = a.coef[pr.offa + ka];
        if (g.lb >= 0) {
            zb = a.expo[pr.offb + kb];
            cb = a.coef[pr.offb + kb];
        }
    }
    const double p = za + zb;
    const double i2p = 0.5 / p;
    if (lt < 3) {
        const int ax = lt;
        // X_PA = (zeta_b/p)(B - A) and X_PB = (zeta_a/p)(A - B): both exactly 0
        // when the two centres coincide (P - A formed from a rounded P is not)
        const double XPA = zb / p * (B[ax] - Av[ax]), XPB = za / p * (Av[ax] - B[ax]);
        // Eqs. (10), (11) with E^0_00 = 1 (the exponential is applied below)
        E(ax, 0, 0, 0) = 1.0;
        // the derivative-bra role also needs a+1 and b+1 (d/dA of Eq. (1))
        const int la_e = la + (g.role == 2), lb_e = lb + (g.role == 2);
        for (int i = 0; i <= la_e; ++i) {
            if (i > 0)
                for (int t = 0; t <= i; ++t) {
                    double v = XPA * (t <= i - 1 ? E(ax, i - 1, 0, t) : 0.0);
                    if (t > 0) v += i2p * E(ax, i - 1, 0, t - 1);
                    if (t + 1 <= i - 1) v += (t + 1) * E(ax, i - 1, 0, t + 1);
                    E(ax, i, 0, t) = v;
                }
            for (int j = 1; j <= lb_e; ++j)
                for (int t = 0; t <= i + j; ++t) {
                    double v = XPB * (t <= i + j - 1 ? E(ax, i, j - 1, t) : 0.0);
                    if (t > 0) v += i2p * E(ax, i, j - 1, t - 1);
                    if (t + 1 <= i + j - 1) v += (t + 1) * E(ax, i, j - 1, t + 1);
                    E(ax, i, j, t) = v;
                }
        }
    }
    if (lt == 0) {
        const double dx = Av[0] - B[0], dy = Av[1] - B[1], dz = Av[2] - B[2];
        const double K = valid ? exp(-za * zb / p * (dx * dx + dy * dy + dz * dz)) * ca * cb : 0.0;
        const double pref = K / p;   // + 2 pi^{5/2} on the bra
        sh_pref = g.role != 1 ? 2.0 * 17.493418327624862 * pref : pref;
        if (live) {
            PrimRec r{};
            r.p = valid ? p : 1.0;
            // P = A + (zeta_b/p)(B - A): exactly A on one centre, so P - Q of two
            // one-centre pairs on the same atom is exactly 0
            r.Px = Av[0] + zb / p * (B[0] - Av[0]);
            r.Py = Av[1] + zb / p * (B[1] - Av[1]);
            r.Pz = Av[2] + zb / p * (B[2] - Av[2]);
            r.ws = valid ? 1.0 : 0.0;
            // terminal weight (-1)^L K c c / (zeta_q (2 zeta_q)^L), Eqs. (17), (40)
            r.wt = valid ? ((g.L & 1) ? -1.0 : 1.0) * pref * pow(2.0 * p, -(double)g.L) : 0.0;
            a.prim[pair * g.kmax + k] = r;
        }
    }
    __syncthreads();
    if (!live) return;
    const double pref = sh_pref;

    // rows of this primitive block
    int row0, nrows;
    double *Hp;
    if (g.role != 1) {
        row0 = k * g.nh;
        nrows = g.nh;
        // the pair's last primitive also zeroes the rows up to the next 16-row tile
        if (k == np - 1) nrows = round_up(np * g.nh, 16) - row0;
        Hp = a.H + (int64_t)pair * g.pair_stride;
    } else {
        row0 = 0;
        nrows = g.rows_per_block;
        Hp = a.H + (int64_t)pair * g.pair_stride + (int64_t)k * g.rows_per_block * g.ncolp;
    }
    if (g.role == 2) {
        // derivative bra: d/dA_i of x_A^a exp(-zeta_a r_A^2) is 2 zeta_a (a+1_i) - a_i (a-1_i)
        // (likewise for B), so along axis i the Hermite coefficient of the derivative is
        // 2 zeta_a E^{a+1,b}_t - a_i E^{a-1,b}_t, expanded about the same P up to order L+1.
        auto e1 = [&](int ax, int i, int j, int t) -> double {
            return (i >= 0 && j >= 0 && t <= i + j) ? E(ax, i, j, t) : 0.0;
        };
        // stored transposed, Hd[d][col][row] (rows contiguous): the backward
        // kernel reads 16 consecutive rows of one function per lane group
        const int64_t dstride = (int64_t)g.rows_per_block * g.ncolp;
        for (int e = lt; e < 6 * nrows * g.ncolp; e += T) {
            const int d = e / (nrows * g.ncolp), rem = e - d * nrows * g.ncolp;
            const int row = row0 + rem % nrows, col = rem / nrows;
            const int rk = row - k * g.nh;
            double v = 0.0;
            if (valid && rk < g.nh && col < g.ncol) {
                const Tuv r = herm_tuv(rk);
                const int tv[3] = {r.t, r.u, r.v};
                const int dax = d % 3;
                const bool onA = d < 3;
                const int ma = col / nb_out, mb = col % nb_out;
                double s = 0.0;
                for (int i = 0; i < ta_n[ma]; ++i)
                    for (int j = 0; j < tb_n[mb]; ++j) {
                        double f = ta_w[ma * NTM + i] * tb_w[mb * NTM + j];
                        for (int ax = 0; ax < 3 && f != 0.0; ++ax) {
                            const int ai = ta_c[(ma * NTM + i) * 3 + ax], bi = tb_c[(mb * NTM + j) * 3 + ax], t = tv[ax];
                            double c;
                            if (ax != dax) c = e1(ax, ai, bi, t);
                            else if (onA) c = 2.0 * za * e1(ax, ai + 1, bi, t) - ai * e1(ax, ai - 1, bi, t);
                            else c = 2.0 * zb * e1(ax, ai, bi + 1, t) - bi * e1(ax, ai, bi - 1, t);
                            f *= c;
                        }
                        s += f;
                    }
                v = pref * s;
            }
            Hp[d * dstride + (int64_t)col * g.rows_per_block + row] = v;
        }
        return;
    }
    for (int e = lt; e < nrows * g.ncolp; e += T) {
        const int row = row0 + e / g.ncolp, col = e % g.ncolp;
        // Hermite triple of this row
        int h = -1;
        if (g.role == 0) {
            const int rk = row - k * g.nh;
            if (rk < g.nh && valid) h = rk;
        } else if (valid) {
            const int nnt = nherm(g.L - 1);
            if (row < nnt) h = row;
            else if (row >= g.ntpad && row < g.ntpad + g.nterm) h = nnt + (row - g.ntpad);
        }
        double v = 0.0;
        if (h >= 0 && col < g.ncol) {
            const Tuv r = herm_tuv(h);
            const int ma = col / nb_out, mb = col % nb_out;
            double s = 0.0;
            for (int i = 0; i < ta_n[ma]; ++i) {
                const int *ca = ta_c + (ma * NTM + i) * 3;
                const int ax = ca[0], ay = ca[1], az = ca[2];
                for (int j = 0; j < tb_n[mb]; ++j) {
                    const int *cb = tb_c + (mb * NTM + j) * 3;
                    const int bx = cb[0], by = cb[1], bz = cb[2];
                    if (r.t > ax + bx || r.u > ay + by || r.v > az + bz) continue;
                    s += ta_w[ma * NTM + i] * tb_w[mb * NTM + j] * E(0, ax, bx, r.t) * E(1, ay, by, r.u) * E(2, az, bz, r.v);
                }
            }
            v = pref * s;
            if (g.role == 1 && ((r.t + r.u + r.v) & 1)) v = -v;
        }
        Hp[(int64_t)row * g.ncolp + col] = v;
    }
}

#undef E

__global__ void __launch_bounds__(PD_THREADS) pairdata_kernel(PairDataArgs a) { pairdata_block(a, blockIdx.x); }

// Several side records in one launch: workgroups base[r] .. base[r+1]-1 are
// record r's (records without items own none).  A launch of every record of
// a plan lets the hardware spread them over the chip instead of running the
// records one after another on a few streams.
__global__ void __launch_bounds__(PD_THREADS) pairdata_multi_kernel(PairDataMulti m)
{
    const int b = blockIdx.x;
    int lo = 0, hi = m.nrec;   // base[lo] <= b < base[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (m.base[mid] <= b) lo = mid;
        else hi = mid;
    }
    const PairDataArgs a = m.recs[lo];
    pairdata_block(a, b - m.base[lo]);
}

int pairdata_prepare(PairDataArgs &a, size_t &lds)
{
    a.per_block = pd_per_block(a.g);
    const int nitem = a.g.grouped ? a.g.npair : a.nitems;
    lds = pairdata_lds_bytes(a.g, a.per_block);
    return (nitem + a.per_block - 1) / a.per_block;
}

void launch_pairdata(const PairDataArgs &a0, hipStream_t s)
{
    PairDataArgs a = a0;
    size_t lds = 0;
    const int nblk = pairdata_prepare(a, lds);
    if (nblk > 0) hipLaunchKernelGGL(pairdata_kernel, dim3(nblk), dim3(PD_THREADS), lds, s, a);
}

void launch_pairdata_multi(const PairDataMulti &m, int nblk, size_t lds, hipStream_t s)
{
    if (nblk > 0) hipLaunchKernelGGL(pairdata_multi_kernel, dim3(nblk), dim3(PD_THREADS), lds, s, m);
}

}  // namespace mdx
