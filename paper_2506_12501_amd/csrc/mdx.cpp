// mdx.cpp -- host runtime behind include/mdx.h: validation, planning, pair-data
// and integral launches.  No device allocation happens inside a call; all
// scratch lives in the caller's workspace, or, for mdx_eri_batch_noalloc, in a
// static device buffer defined here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mdx.h"
#include "kernels.h"
#include "mdx_internal.h"
#include "runtime.h"

#include "boys_table.inc"

using namespace mdx;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

mdx_status mdx::fail(mdx_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

extern "C" const char *mdx_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *mdx_status_string(mdx_status s)
{
    switch (s) {
    case MDX_OK: return "MDX_OK";
    case MDX_EINVAL: return "MDX_EINVAL";
    case MDX_EUNSUPPORTED: return "MDX_EUNSUPPORTED";
    case MDX_EWORKSPACE: return "MDX_EWORKSPACE";
    case MDX_ENOMEM: return "MDX_ENOMEM";
    case MDX_EDEVICE: return "MDX_EDEVICE";
    }
    return "unknown mdx_status";
}

#define HIP_TRY HIP_TRY2

// ---------------------------------------------------------------------------
// real solid harmonics by recursion in l (Helgaker, Jorgensen & Olsen,
// Molecular Electronic-Structure Theory, Sec. 6.4.2), Racah normalised:
//   S_{l+1,l+1}  = sqrt(2^{d(l,0)} (2l+1)/(2l+2)) (x S_{ll} - (1-d(l,0)) y S_{l,-l})
//   S_{l+1,-l-1} = sqrt(2^{d(l,0)} (2l+1)/(2l+2)) (y S_{ll} + (1-d(l,0)) x S_{l,-l})
//   S_{l+1,m}    = ((2l+1) z S_{lm} - sqrt((l+m)(l-m)) r^2 S_{l-1,m}) / sqrt((l+m+1)(l-m+1))
// Polynomials are dense cubes of coefficients c[ax][ay][az].
// ---------------------------------------------------------------------------
namespace {
constexpr int SH_L = 8;
constexpr int SH_D = SH_L + 1;
struct Poly {
    double c[SH_D][SH_D][SH_D];
};

void solid_tables(std::vector<std::vector<double>> &out)   // out[l] = [nsph][ncart]
{
    std::vector<std::vector<Poly>> S(SH_L + 1);
    for (int l = 0; l <= SH_L; ++l) S[l].assign(2 * l + 1, Poly{});
    S[0][0].c[0][0][0] = 1.0;
    auto at = [&](int l, int m) -> Poly & { return S[l][m + l]; };
    for (int l = 0; l < SH_L; ++l) {
        const double f = std::sqrt((l == 0 ? 2.0 : 1.0) * (2 * l + 1) / (2.0 * l + 2));
        Poly &top = at(l + 1, l + 1), &bot = at(l + 1, -l - 1);
        const Poly &Sll = at(l, l), &Slm = at(l, -l);
        for (int i = 0; i <= l; ++i)
            for (int j = 0; j <= l - i; ++j)
                for (int k = 0; k <= l - i - j; ++k) {
                    top.c[i + 1][j][k] += f * Sll.c[i][j][k];
                    bot.c[i][j + 1][k] += f * Sll.c[i][j][k];
                    if (l > 0) {
                        top.c[i][j + 1][k] -= f * Slm.c[i][j][k];
                        bot.c[i + 1][j][k] += f * Slm.c[i][j][k];
                    }
                }
        for (int m = -l; m <= l; ++m) {
            Poly &d = at(l + 1, m);
            const double den = std::sqrt((double)(l + m + 1) * (l - m + 1));
            const Poly &s1 = at(l, m);
            for (int i = 0; i <= l; ++i)
                for (int j = 0; j <= l - i; ++j)
                    for (int k = 0; k <= l - i - j; ++k) d.c[i][j][k + 1] += (2 * l + 1) * s1.c[i][j][k] / den;
            if (l >= 1 && std::abs(m) <= l - 1) {
                const double g = std::sqrt((double)(l + m) * (l - m)) / den;
                const Poly &s2 = at(l - 1, m);
                for (int i = 0; i <= l - 1; ++i)
                    for (int j = 0; j <= l - 1 - i; ++j)
                        for (int k = 0; k <= l - 1 - i - j; ++k) {
                            const double v = g * s2.c[i][j][k];
                            d.c[i + 2][j][k] -= v;
                            d.c[i][j + 2][k] -= v;
                            d.c[i][j][k + 2] -= v;
                        }
            }
        }
    }
    out.assign(SH_L + 1, {});
    for (int l = 0; l <= SH_L; ++l) {
        const int nc = ncart(l);
        out[l].assign((size_t)(2 * l + 1) * nc, 0.0);
        for (int m = 0; m < 2 * l + 1; ++m) {
            int idx = 0;
            for (int ax = l; ax >= 0; --ax)
                for (int ay = l - ax; ay >= 0; --ay) {
                    out[l][(size_t)m * nc + idx] = S[l][m].c[ax][ay][l - ax - ay];
                    ++idx;
                }
        }
    }
}
}  // namespace

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
// Scratch of mdx_eri_batch_noalloc: one copy per device, alive until the
// process ends.  Host code must never use this name as a device address (on
// the host it is only a stand-in); its device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[MDX_NOALLOC_SCRATCH_BYTES];

static std::mutex scratch_mu;
static std::map<int, char *> scratch_addr;   // device -> device address of `scratch`

static hipError_t scratch_of_device(int device, char **ptr)
{
    std::lock_guard<std::mutex> lk(scratch_mu);
    auto it = scratch_addr.find(device);
    if (it != scratch_addr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // the current device's copy
    if (e != hipSuccess) return e;
    scratch_addr[device] = (char *)p;
    *ptr = (char *)p;
    return hipSuccess;
}

extern "C" mdx_status mdx_create(int device, mdx_ctx **out)
{
    if (!out) return fail(MDX_EINVAL, "mdx_create: null output pointer");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(MDX_EINVAL, "mdx_create: device %d of %d", device, ndev);
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(MDX_EDEVICE, "mdx_create: device %d is %s, libmdx is built for gfx950", device, prop.gcnArchName);
    mdx_ctx *c = new (std::nothrow) mdx_ctx();
    if (!c) return fail(MDX_ENOMEM, "mdx_create: out of host memory");
    c->device = device;
    c->ncu = prop.multiProcessorCount;
    {
        const hipError_t es = scratch_of_device(device, &c->scratch);   // device is current (hipSetDevice above)
        if (es != hipSuccess) {
            delete c;
            return fail(MDX_EDEVICE, "mdx_create: static scratch of device %d: %s", device, hipGetErrorString(es));
        }
    }
    // Boys table
    static_assert(sizeof(mdx_boys_table_host) == sizeof(double) * BOYS_EXP_OFF, "Boys table shape");
    std::vector<double> btab(BOYS_EXP_OFF + BOYS_NROW);
    std::memcpy(btab.data(), mdx_boys_table_host, sizeof(mdx_boys_table_host));
    for (int k = 0; k < BOYS_NROW; ++k) btab[BOYS_EXP_OFF + k] = std::exp(-(double)k / BOYS_STEP_INV);
    hipError_t e = hipMalloc((void **)&c->boys, btab.size() * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(c->boys, btab.data(), btab.size() * sizeof(double), hipMemcpyHostToDevice);
    // solid harmonics, l <= 8
    std::vector<std::vector<double>> sol;
    solid_tables(sol);
    c->solid_host = sol;
    size_t tot = 0;
    for (auto &v : sol) tot += v.size();
    if (e == hipSuccess) e = hipMalloc((void **)&c->solid, tot * sizeof(double));
    size_t off = 0;
    for (int l = 0; l <= 8 && e == hipSuccess; ++l) {
        c->solid_off[l] = off;
        e = hipMemcpy(c->solid + off, sol[l].data(), sol[l].size() * sizeof(double), hipMemcpyHostToDevice);
        off += sol[l].size();
    }
    // terminal ket matrices: 2-centre kets (lc, ld <= MDX_LMAX_4C) and single functions (l <= MDX_LMAX_3C)
    std::vector<double> T;
    for (int cart = 0; cart < 2 && e == hipSuccess; ++cart) {
        for (int lc = 0; lc <= MDX_LMAX_4C; ++lc)
            for (int ld = 0; ld <= MDX_LMAX_4C; ++ld) {
                c->tket_off[cart][lc][ld] = T.size();
                build_tket(c, lc, ld, cart != 0, T);
            }
        for (int l = 0; l <= MDX_LMAX_3C; ++l) {
            c->tket1_off[cart][l] = T.size();
            build_tket(c, l, -1, cart != 0, T);
        }
    }
    if (e == hipSuccess) e = hipMalloc((void **)&c->tket, T.size() * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(c->tket, T.data(), T.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        mdx_destroy(c);
        return fail(MDX_EDEVICE, "mdx_create: %s", hipGetErrorString(e));
    }
    *out = c;
    return MDX_OK;
}

extern "C" void mdx_destroy(mdx_ctx *c)
{
    if (!c) return;
    hipSetDevice(c->device);
    if (c->boys) hipFree(c->boys);
    if (c->solid) hipFree(c->solid);
    if (c->tket) hipFree(c->tket);
    delete c;
}

// T[q][cd] for the terminal Hermites q (level L = lc+ld) of a ket:
//   2-centre: sum over Cartesian c, d with c + d = q of C^c C^d (Eqs. (17), (39))
//   single function (ld < 0): C^q
// rows padded to a multiple of 4, columns to 16.
void mdx::build_tket(mdx_ctx *c, int lc, int ld, bool cart, std::vector<double> &T)
{
    const int L = lc + std::max(ld, 0);
    const int nt = ncart(L), ntp = round_up(nt, 4);
    const int nc = nfunc(lc, cart), nd = ld >= 0 ? nfunc(ld, cart) : 1;
    const int ncol = nc * nd, ncolp = round_up(ncol, 16);
    const size_t base = T.size();
    T.resize(base + (size_t)ntp * ncolp, 0.0);
    auto cart_list = [](int l) {
        std::vector<std::array<int, 3>> v;
        for (int ax = l; ax >= 0; --ax)
            for (int ay = l - ax; ay >= 0; --ay) v.push_back({ax, ay, l - ax - ay});
        return v;
    };
    const auto cl = cart_list(lc);
    const auto dl = cart_list(std::max(ld, 0));
    const auto &Cc = c->solid_host[lc];
    const auto &Cd = c->solid_host[std::max(ld, 0)];
    for (int mc = 0; mc < nc; ++mc)
        for (int md = 0; md < nd; ++md) {
            const int col = mc * nd + md;
            for (size_t ic = 0; ic < cl.size(); ++ic) {
                const double fc = cart ? (ic == (size_t)mc ? 1.0 : 0.0) : Cc[(size_t)mc * cl.size() + ic];
                if (fc == 0.0) continue;
                for (size_t id = 0; id < dl.size(); ++id) {
                    const double fd = (cart || ld < 0) ? ((ld < 0 || id == (size_t)md) ? 1.0 : 0.0)
                                                       : Cd[(size_t)md * dl.size() + id];
                    if (fd == 0.0) continue;
                    const int t = cl[ic][0] + dl[id][0], u = cl[ic][1] + dl[id][1], v = cl[ic][2] + dl[id][2];
                    const int q = herm_index(t, u, v) - nherm(L - 1);
                    T[base + (size_t)q * ncolp + col] += fc * fd;
                }
            }
        }
}

// ---------------------------------------------------------------------------
// mdx_boys
// ---------------------------------------------------------------------------
extern "C" mdx_status mdx_boys(mdx_ctx *c, int32_t n, const double *x, int mmax, double *F, mdx_stream_t s)
{
    if (!c) return fail(MDX_EINVAL, "mdx_boys: null context");
    if (n < 0) return fail(MDX_EINVAL, "mdx_boys: n = %d < 0", n);
    if (mmax < 0 || mmax > MDX_BOYS_MAX_M) return fail(MDX_EUNSUPPORTED, "mdx_boys: mmax = %d outside [0, %d]", mmax, MDX_BOYS_MAX_M);
    if (n > 0 && (!x || !F)) return fail(MDX_EINVAL, "mdx_boys: null x or F");
    if (n == 0) return MDX_OK;
    HIP_TRY(hipSetDevice(c->device));
    launch_boys(x, n, mmax, F, c->boys, (hipStream_t)s);
    HIP_TRY(hipGetLastError());
    return MDX_OK;
}
