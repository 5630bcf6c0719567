// Host-only code of the runtime, run under AddressSanitizer and
// UndefinedBehaviorSanitizer with no GPU: configuration checks, the list and
// workspace plans behind md_workspace_size and md_admit, the log-spaced MSD
// schedule, the RSA and lattice initial states, and md_init's error path
// when no device is present.  The runtime source is included whole so that
// its file-local helpers (the initial-state generators) can be called.
// Exit status 0 and no sanitizer report: every check passed.
#include "runtime.cpp"

#include <cstdio>

static int g_failures = 0;
#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond); \
            ++g_failures;                                                            \
        }                                                                            \
    } while (0)

static kamd_config config(int precision, int dim)
{
    kamd_config c;
    std::memset(&c, 0, sizeof c);
    const double eps[3] = {1.0, 1.5, 0.5}, sig[3] = {1.0, 0.8, 0.88};
    for (int p = 0; p < 3; ++p) {
        c.model.eps[p] = eps[p];
        c.model.sigma[p] = sig[p];
    }
    c.model.rc_factor = 2.5;
    c.precision = precision;
    c.dt = 0.005;
    c.skin = 0.3;
    c.init_mode = KAMD_INIT_RSA;
    c.min_dist = 0.8;
    c.dim = dim;
    return c;
}

static kamd_replica replica(int n, int n_a, double rho, int dim, uint64_t seed, int64_t offset = 0)
{
    kamd_replica r;
    r.offset = offset;
    r.n = n;
    r.n_a = n_a;
    r.box = dim == 2 ? std::sqrt(n / rho) : std::cbrt(n / rho);
    r.temperature = 1.0;
    r.seed = seed;
    return r;
}

static void check_workspace_sizes()
{
    for (int prec = 0; prec < 3; ++prec)
        for (int dim : {3, 2}) {
            kamd_config c = config(prec, dim);
            for (int n : {1, 2, 64, 65, 1000, 32000}) {
                kamd_replica r = replica(n, (4 * n) / 5, dim == 2 ? 1.204 : 1.2, dim, 7);
                if (r.box <= 2.0 * (2.5 + c.skin)) r.box = 2.0 * (2.5 + c.skin) + 0.5;
                size_t b = 0;
                CHECK(md_workspace_size(&c, &r, 1, &b) == KAMD_OK);
                CHECK(b > 0 && b % 256 == 0);
                for (int div : {1, 2}) {
                    c.cell_div = div;
                    size_t b2 = 0;
                    CHECK(md_workspace_size(&c, &r, 1, &b2) == KAMD_OK);
                }
                c.cell_div = 0;
            }
        }
    // one-species replicas and a batch of uneven sizes
    kamd_config c = config(KAMD_PREC_MIXED, 3);
    std::vector<kamd_replica> reps;
    int64_t off = 0;
    for (int k = 0; k < 40; ++k) {
        const int n = 250 + 197 * k;
        const int na = k % 5 == 0 ? 0 : (k % 5 == 1 ? n : (4 * n) / 5);
        reps.push_back(replica(n, na, 1.2, 3, 100 + k, off));
        off += n;
    }
    size_t b = 0;
    CHECK(md_workspace_size(&c, reps.data(), (int)reps.size(), &b) == KAMD_OK);
    // refusals
    kamd_replica small = replica(1000, 800, 1.2, 3, 1);
    small.box = 5.0;  // cutoff + skin beyond L/2
    CHECK(md_workspace_size(&c, &small, 1, &b) == KAMD_EBOX);
    kamd_replica bad = replica(1000, 1200, 1.2, 3, 1);
    CHECK(md_workspace_size(&c, &bad, 1, &b) == KAMD_EINVAL);
    CHECK(md_workspace_size(&c, nullptr, 1, &b) == KAMD_EINVAL);
    CHECK(md_workspace_size(nullptr, &small, 1, &b) == KAMD_EINVAL);
    kamd_replica r = replica(1000, 800, 1.2, 3, 1);
    CHECK(md_workspace_size(&c, &r, 1, nullptr) == KAMD_EINVAL);
    CHECK(md_workspace_size(&c, &r, 0, &b) == KAMD_EINVAL);
    kamd_config cb = c;
    cb.cell_div = 3;
    CHECK(md_workspace_size(&cb, &r, 1, &b) == KAMD_EINVAL);
    cb = c;
    cb.precision = 7;
    CHECK(md_workspace_size(&cb, &r, 1, &b) == KAMD_EINVAL);
    CHECK(std::strlen(md_last_error(nullptr)) > 0);
}

static void check_admission()
{
    kamd_config c = config(KAMD_PREC_MIXED, 3);
    std::vector<kamd_replica> reps;
    for (int k = 0; k < 16; ++k) reps.push_back(replica(20000 + 5000 * k, 16000 + 4000 * k, 1.2, 3, 200 + k));
    size_t one = 0;
    CHECK(md_workspace_size(&c, reps.data(), 1, &one) == KAMD_OK);
    std::vector<int32_t> adm(reps.size(), -1);
    int32_t cnt = -1;
    CHECK(md_admit(&c, reps.data(), (int)reps.size(), (size_t)1 << 40, adm.data(), &cnt) == KAMD_OK);
    CHECK(cnt == (int)reps.size());
    CHECK(md_admit(&c, reps.data(), (int)reps.size(), one, adm.data(), &cnt) == KAMD_OK);
    CHECK(cnt == 1 && adm[0] == 1);
    CHECK(md_admit(&c, reps.data(), (int)reps.size(), 0, adm.data(), &cnt) == KAMD_OK);
    CHECK(cnt == 0);
    CHECK(md_admit(&c, reps.data(), 0, 0, adm.data(), &cnt) == KAMD_EINVAL);
}

static void check_log_schedule()
{
    int32_t cnt = 0;
    CHECK(md_log_schedule(1000, 1.0, 60, nullptr, 0, &cnt) == KAMD_OK);
    CHECK(cnt == 50);
    std::vector<int32_t> out(cnt);
    CHECK(md_log_schedule(1000, 1.0, 60, out.data(), cnt, &cnt) == KAMD_OK);
    for (int i = 1; i < cnt; ++i) CHECK(out[i] > out[i - 1]);
    CHECK(out.front() >= 1 && out.back() == 1000);
    // a short output buffer is filled, not overrun
    std::vector<int32_t> few(5, -1);
    CHECK(md_log_schedule(100000, 1.0, 200, few.data(), 5, &cnt) == KAMD_OK);
    CHECK(cnt > 5 && few[4] > few[3]);
    CHECK(md_log_schedule(0, 1.0, 60, nullptr, 0, &cnt) == KAMD_EINVAL);
    CHECK(md_log_schedule(10, 0.1, 60, nullptr, 0, &cnt) == KAMD_EINVAL);
    CHECK(md_log_schedule(10, 1.0, 0, nullptr, 0, &cnt) == KAMD_EINVAL);
}

static void check_initial_states()
{
    for (int dim : {3, 2}) {
        // the planar density 1.204 lies above the jamming coverage of random
        // sequential addition of discs of diameter 0.8, so planar boxes here
        // are at half that density
        for (int n : {1, 2, 500, 4000}) {
            kamd_replica r = replica(n, (4 * n) / 5, dim == 2 ? 0.6 : 1.2, dim, 11);
            std::vector<double> x, y, z;
            const bool ok = rsa_positions(r, dim, 0.8, x, y, z);
            if (!ok) std::fprintf(stderr, "RSA failed: dim %d n %d\n", dim, n);
            CHECK(ok);
            CHECK((int)x.size() == n && (int)y.size() == n && (int)z.size() == n);
            for (int i = 0; i < n; ++i) {
                CHECK(x[i] >= 0.0 && x[i] < r.box && y[i] >= 0.0 && y[i] < r.box);
                CHECK(dim == 2 ? z[i] == 0.0 : (z[i] >= 0.0 && z[i] < r.box));
            }
            lattice_positions(r, dim, x, y, z);
            CHECK((int)x.size() == n);
            for (int i = 0; i < n; ++i) CHECK(x[i] > 0.0 && x[i] < r.box);
        }
        // a density RSA cannot reach: the budget ends the attempt (then the
        // lattice is used)
        kamd_replica dense = replica(300, 240, 3.0, dim, 12);
        std::vector<double> x, y, z;
        CHECK(!rsa_positions(dense, dim, 0.8, x, y, z));
    }
}

static void check_init_without_device()
{
    kamd_config c = config(KAMD_PREC_MIXED_FIXED, 3);
    kamd_replica r = replica(1000, 800, 1.2, 3, 5);
    kamd_state st;
    std::memset(&st, 0, sizeof st);
    kamd_ctx *ctx = reinterpret_cast<kamd_ctx *>(&c);  // overwritten with NULL on error
    const int rc = md_init(&ctx, &c, &r, 1, &st, nullptr, 0, nullptr);
    CHECK(rc == KAMD_EHIP || rc == KAMD_ENOMEM);
    CHECK(ctx == nullptr);
    CHECK(std::strlen(md_last_error(nullptr)) > 0);
    CHECK(md_init(nullptr, &c, &r, 1, &st, nullptr, 0, nullptr) == KAMD_EINVAL);
    CHECK(md_destroy(nullptr) == KAMD_EINVAL || md_destroy(nullptr) == KAMD_OK);
}

int main()
{
    check_workspace_sizes();
    check_admission();
    check_log_schedule();
    check_initial_states();
    check_init_without_device();
    std::printf("runtime host driver: %d failed checks\n", g_failures);
    return g_failures ? 1 : 0;
}
