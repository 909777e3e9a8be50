// Host-side checks of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer: md_create's validation, the table construction
// (knots on a bin grid, knots inside bins, knots too close for any table),
// workspace planning, the option switches and the calls that need md_bind, all
// through the C ABI and without any device work.  Built with the host half of
// md_runtime.hip instrumented (tests/test_host_sanitizers.py); prints one line
// per failed expectation and exits nonzero if there was any.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "include/md.h"

namespace {

int failures = 0;

void expect(int got, int want, const char* what)
{
    if (got != want) {
        std::printf("FAIL %s: got %d, want %d\n", what, got, want);
        ++failures;
    }
}

// A potential of ns species with npk pair and ndk density knots spaced `step`
// below `rc` (amplitudes of no physical meaning), plus knot offsets `jitter`.
struct Pot {
    std::vector<double> pa, pr, da, dr, c, m;
    md_potential p{};
    Pot(int ns, int npk, int ndk, double rc, double step, double jitter = 0.0)
    {
        for (int a = 0; a < ns * ns; ++a) {
            for (int k = 0; k < npk; ++k) {
                pa.push_back(0.5 - 0.6 * k / std::max(npk - 1, 1));
                pr.push_back(rc - step * (npk - 1 - k) - (k + 1 < npk ? jitter * (k + 1) : 0.0));
            }
            for (int k = 0; k < ndk; ++k) {
                da.push_back(1.0 + k);
                dr.push_back(rc - 0.5 - step * (ndk - 1 - k) - (k + 1 < ndk ? jitter * (k + 2) : 0.0));
            }
        }
        for (int a = 0; a < ns; ++a) {
            c.push_back(1.0 - 0.3 * a);
            m.push_back(55.845 - 40.0 * a);
        }
        p.n_species = ns;
        p.n_pair_knots = npk;
        p.n_dens_knots = ndk;
        p.reserved = 0;
        p.pair_a = pa.data();
        p.pair_r = pr.data();
        p.dens_A = da.data();
        p.dens_R = dr.data();
        p.emb_c = c.data();
        p.mass_amu = m.data();
    }
};

struct Cfg {
    std::vector<int64_t> off;
    std::vector<double> box, origin, vp, nh_t, nh_q, pr_p, pr_w, hmat;
    std::vector<uint8_t> per;
    md_config c{};
    explicit Cfg(std::vector<int64_t> sizes, double L = 28.7)
    {
        off.push_back(0);
        for (int64_t n : sizes) off.push_back(off.back() + n);
        const int R = (int)sizes.size();
        for (int r = 0; r < R; ++r)
            for (int a = 0; a < 3; ++a) {
                box.push_back(L + r);
                per.push_back(1);
            }
        c.n_replicas = R;
        c.max_neighbours = 48;
        c.rebuild_every = 10;
        c.precision = MD_FP64;
        c.nbr_mode = MD_NBR_FULL;
        c.lanes_per_atom = 0;
        c.atom_offset = off.data();
        c.box = box.data();
        c.periodic = per.data();
        c.skin = 0.3;
        c.dt_fs = 1.0;
        c.integrator = MD_VERLET;
    }
};

// Creates, sizes, toggles every option and destroys one context; returns the
// md_create code.
int exercise(const md_config& cfg, const md_potential& pot, const char* what)
{
    md_ctx* ctx = nullptr;
    const int rc = md_create(&cfg, &pot, &ctx);
    if (rc != MD_OK) {
        if (ctx) {
            if (std::strlen(md_last_error(ctx)) == 0) {
                std::printf("FAIL %s: rejection without a message\n", what);
                ++failures;
            }
            md_destroy(ctx);
        }
        return rc;
    }
    size_t bytes = 0;
    expect(md_workspace_bytes(ctx, &bytes), MD_OK, "md_workspace_bytes");
    if (bytes == 0) {
        std::printf("FAIL %s: empty workspace\n", what);
        ++failures;
    }
    // every option with a few values, legal or not; the return code only has
    // to be one of the documented ones and the state must stay consistent
    for (int32_t opt = 0; opt <= 20; ++opt)
        for (int64_t v : {-1LL, 0LL, 1LL, 2LL, 4LL, 8LL, 64LL, 222LL, 444LL, 1024LL, (1LL << 40)}) {
            const int r = md_set_option(ctx, opt, v);
            if (r != MD_OK && r != MD_ERR_ARG && r != MD_ERR_STATE && r != MD_ERR_DEVICE) {
                std::printf("FAIL %s: option %d value %lld gave %d\n", what, opt, (long long)v, r);
                ++failures;
            }
            int64_t back = 0;
            (void)md_get_option(ctx, opt, &back);
        }
    expect(md_set_option(ctx, MD_OPT_TIMING, 0), MD_OK, "timing off");
    expect(md_workspace_bytes(ctx, &bytes), MD_OK, "md_workspace_bytes after options");
    // calls that need md_bind
    expect(md_step(ctx, 1, nullptr), MD_ERR_STATE, "md_step before md_bind");
    expect(md_build_neighbours(ctx, nullptr), MD_ERR_STATE, "md_build_neighbours before md_bind");
    md_energies e;
    expect(md_energy(ctx, &e, nullptr), MD_ERR_STATE, "md_energy before md_bind");
    expect(md_bind(ctx, nullptr, nullptr, 0), MD_ERR_ARG, "md_bind without state");
    md_destroy(ctx);
    return rc;
}

}  // namespace

int main()
{
    int cases = 0;
    // one species on the 0.02 A grid, two species, knots inside bins (split
    // tables), 16 + 4 knots, knots closer than r_c / 4096 (no table)
    Pot fe(1, 6, 2, 4.1, 0.38);
    Pot fec(2, 6, 2, 4.1, 0.38);
    Pot split(1, 6, 2, 4.1, 0.38, 0.00731);
    Pot many(1, 16, 4, 4.1, 0.12, 0.0013);
    Pot close(1, 6, 2, 4.1, 0.38, 0.0);
    close.pr[2] += 3e-4;               // off every bin grid,
    close.pr[1] = close.pr[2] - 1e-5;  // and a second knot 1e-5 A below it
    Pot bad_dens(1, 6, 2, 4.1, 0.38);
    bad_dens.da[0] = -1.0;
    Pot bad_sym(2, 6, 2, 4.1, 0.38);
    bad_sym.pa[1 * 6 + 0] += 1.0;  // pair (0, 1) differs from (1, 0)
    Pot bad_mass(1, 6, 2, 4.1, 0.38);
    bad_mass.m[0] = 0.0;

    for (int prec : {MD_FP64, MD_MIXED})
        for (int mode : {MD_NBR_FULL, MD_NBR_HALF_ATOMIC}) {
            Cfg one({2000});
            one.c.precision = prec;
            one.c.nbr_mode = mode;
            expect(exercise(one.c, fe.p, "one species"), MD_OK, "one species"), ++cases;
            expect(exercise(one.c, fec.p, "two species"), MD_OK, "two species"), ++cases;
            expect(exercise(one.c, split.p, "split tables"), MD_OK, "split tables"), ++cases;
            expect(exercise(one.c, many.p, "16 + 4 knots"), MD_OK, "16 + 4 knots"), ++cases;
            expect(exercise(one.c, close.p, "close knots"), prec == MD_MIXED ? MD_ERR_POTENTIAL : MD_OK,
                   "close knots"), ++cases;
            Cfg batch({500, 1200, 64, 3000});
            batch.c.precision = prec;
            batch.c.nbr_mode = mode;
            expect(exercise(batch.c, fec.p, "batch"), MD_OK, "batch"), ++cases;
        }
    {
        Cfg nvt({800, 900});
        nvt.nh_t = {300.0, 600.0};
        nvt.nh_q = {1e5, 1e5};
        nvt.c.nh_temperature = nvt.nh_t.data();
        nvt.c.nh_mass = nvt.nh_q.data();
        expect(exercise(nvt.c, fe.p, "thermostat"), MD_OK, "thermostat"), ++cases;
        Cfg pr({2000});
        pr.pr_p = {1.0};
        pr.pr_w = {1e4};
        pr.c.pr_pressure_gpa = pr.pr_p.data();
        pr.c.pr_mass = pr.pr_w.data();
        expect(exercise(pr.c, fe.p, "barostat"), MD_OK, "barostat"), ++cases;
        Cfg tri({2000});
        tri.hmat = {28.7, 0.0, 0.0, 0.0, 28.7, 0.0, 28.7, 0.0, 28.7};  // edges (L, 0, L), (0, L, 0), (0, 0, L)
        tri.c.box_matrix = tri.hmat.data();
        expect(exercise(tri.c, fe.p, "box matrix"), MD_OK, "box matrix"), ++cases;
        Cfg gear({2000});
        gear.c.integrator = MD_GEAR3;
        expect(exercise(gear.c, fe.p, "gear"), MD_OK, "gear"), ++cases;
        Cfg slab({1500});
        slab.per[2] = 0;
        slab.box[2] = 8.0;
        expect(exercise(slab.c, fe.p, "thin free axis"), MD_OK, "thin free axis"), ++cases;
    }
    // rejected configurations
    {
        Cfg c({2000});
        expect(exercise(c.c, bad_dens.p, "negative density"), MD_ERR_POTENTIAL, "negative density"), ++cases;
        expect(exercise(c.c, bad_sym.p, "asymmetric pair"), MD_ERR_POTENTIAL, "asymmetric pair"), ++cases;
        expect(exercise(c.c, bad_mass.p, "zero mass"), MD_ERR_POTENTIAL, "zero mass"), ++cases;
        Cfg small({2000}, 8.7);
        expect(exercise(small.c, fe.p, "box too small"), MD_ERR_BOX, "box too small"), ++cases;
        struct Bad {
            const char* what;
            void (*edit)(md_config&);
        } bad[] = {
            {"cap 0", [](md_config& k) { k.max_neighbours = 0; }},
            {"rebuild 0", [](md_config& k) { k.rebuild_every = 0; }},
            {"precision 7", [](md_config& k) { k.precision = 7; }},
            {"nbr_mode 3", [](md_config& k) { k.nbr_mode = 3; }},
            {"lanes 3", [](md_config& k) { k.lanes_per_atom = 3; }},
            {"skin < 0", [](md_config& k) { k.skin = -0.1; }},
            {"dt nan", [](md_config& k) { k.dt_fs = std::nan(""); }},
            {"no replicas", [](md_config& k) { k.n_replicas = 0; }},
        };
        for (const Bad& b : bad) {
            Cfg k({2000});
            b.edit(k.c);
            expect(exercise(k.c, fe.p, b.what), MD_ERR_ARG, b.what), ++cases;
        }
        Cfg neg({2000, 100});
        neg.off[2] = 1000;  // offsets decrease
        expect(exercise(neg.c, fe.p, "decreasing offsets"), MD_ERR_ARG, "decreasing offsets"), ++cases;
    }
    expect(md_create(nullptr, &fe.p, nullptr), MD_ERR_ARG, "null config"), ++cases;
    std::printf("%d cases, %d failures\n", cases, failures);
    return failures == 0 ? 0 : 1;
}
