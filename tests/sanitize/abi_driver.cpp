// abi_driver.cpp -- drives the host side of the C ABI in a process built for
// AddressSanitizer and UBSan (the library's host code instrumented, device
// code untouched). Test infrastructure only.
//
//   abi_driver host    argument and canonical-form checks that end before any
//                      device work: status strings, spx_validate_csr_host on
//                      every class of malformed CSR, and the descriptor /
//                      argument rejections of the entry points (no GPU needed)
//   abi_driver serve   the solve server end to end on the GPU: HBM pool
//                      carving and reuse, queueing under a small budget, the
//                      worker thread, cancellation, budget rejection and
//                      destroy with requests still queued; every finished
//                      solution's residual checked on the host
//
// Prints one line per check and "abi_driver ok" at the end; exits non-zero on
// the first failed check (the sanitizers abort on their own findings).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include <hip/hip_runtime.h>

#include "spx.h"

namespace {

int g_checks = 0;

void expect(bool ok, const char *what)
{
    ++g_checks;
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (last error: %s)\n", what, spx_last_error());
        std::exit(1);
    }
}

void expect_status(spx_status got, spx_status want, const char *what)
{
    ++g_checks;
    if (got != want) {
        std::fprintf(stderr, "FAILED: %s: got %s, want %s (last error: %s)\n", what, spx_status_string(got),
                     spx_status_string(want), spx_last_error());
        std::exit(1);
    }
    std::printf("ok   %-58s %s\n", what, spx_status_string(got));
}

struct Csr {
    int32_t n = 0;
    std::vector<int32_t> rowptr, col;
    std::vector<double> val;
};

// 2D 5-point Laplacian on an m x m grid (Dirichlet boundary eliminated).
Csr poisson2d(int m)
{
    Csr A;
    A.n = m * m;
    A.rowptr.push_back(0);
    for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
            const int r = i + m * j;
            auto put = [&](int c, double v) {
                A.col.push_back(c);
                A.val.push_back(v);
            };
            if (j > 0) put(r - m, -1.0);
            if (i > 0) put(r - 1, -1.0);
            put(r, 4.0);
            if (i + 1 < m) put(r + 1, -1.0);
            if (j + 1 < m) put(r + m, -1.0);
            A.rowptr.push_back((int32_t)A.col.size());
        }
    return A;
}

spx_status validate(const Csr &A)
{
    return spx_validate_csr_host(A.n, A.n, (int64_t)A.col.size(), A.rowptr.data(), A.col.data());
}

void host_checks()
{
    for (int s = 0; s <= (int)SPX_CANCELLED; ++s) expect(spx_status_string((spx_status)s) != nullptr, "status string");
    expect(std::strlen(spx_status_string((spx_status)999)) > 0, "status string of an unknown code");

    const Csr good = poisson2d(12);
    expect_status(validate(good), SPX_OK, "validate_csr_host: canonical 5-point 12x12");
    {
        Csr A = good;
        A.rowptr[0] = 1;
        expect_status(validate(A), SPX_ERR_FORMAT, "validate_csr_host: rowptr[0] != 0");
    }
    {
        Csr A = good;
        std::swap(A.rowptr[5], A.rowptr[6]);
        expect_status(validate(A), SPX_ERR_FORMAT, "validate_csr_host: decreasing rowptr");
    }
    {
        Csr A = good;
        A.rowptr[A.n] -= 1;
        expect_status(validate(A), SPX_ERR_FORMAT, "validate_csr_host: rowptr[n] != nnz");
    }
    {
        Csr A = good;
        A.col[40] = A.n;  // one past the last column
        expect_status(validate(A), SPX_ERR_RANGE, "validate_csr_host: column >= n");
        A.col[40] = -3;
        expect_status(validate(A), SPX_ERR_RANGE, "validate_csr_host: negative column");
    }
    {
        Csr A = good;
        const int32_t p = A.rowptr[20];
        std::swap(A.col[p], A.col[p + 1]);
        expect_status(validate(A), SPX_ERR_UNSORTED, "validate_csr_host: swapped columns");
    }
    {
        Csr A = good;
        const int32_t p = A.rowptr[30];
        A.col[p + 1] = A.col[p];
        expect_status(validate(A), SPX_ERR_DUPLICATE, "validate_csr_host: repeated column");
    }
    expect_status(spx_validate_csr_host(4, 4, 0, nullptr, nullptr), SPX_ERR_ARG, "validate_csr_host: null rowptr");
    expect(std::strlen(spx_last_error()) > 0, "last error text after a rejection");

    // descriptor and argument rejections: all decided on the host
    spx_matrix bad{};
    bad.fmt = SPX_CSR;
    bad.val_type = SPX_F64;
    bad.nrows = -1;
    double dummy[4] = {0, 0, 0, 0};
    expect_status(spx_spmv(nullptr, dummy, dummy, 1.0, 0.0, nullptr), SPX_ERR_ARG, "spmv: null descriptor");
    expect_status(spx_spmv(&bad, dummy, dummy, 1.0, 0.0, nullptr), SPX_ERR_ARG, "spmv: negative size");
    bad.nrows = 4;
    bad.ncols = 4;
    bad.fmt = (spx_format)17;
    expect_status(spx_spmv(&bad, dummy, dummy, 1.0, 0.0, nullptr), SPX_ERR_ARG, "spmv: unknown format");
    bad.fmt = SPX_CSR;
    expect_status(spx_csr_spmv(&bad, dummy, dummy, 1.0, 0.0, nullptr), SPX_ERR_ARG, "csr_spmv: CSR without rowptr");
    bad.fmt = SPX_SELLP;
    bad.slice_size = 48;
    expect_status(spx_validate(&bad, nullptr), SPX_ERR_ARG, "validate: SELL-P slice size not a power of two");
    spx_solve_opts o{};
    o.tol = 1e-10;
    o.maxit = 10;
    size_t bytes = 0;
    expect_status(spx_solve_workspace(99, &bad, &o, &bytes), SPX_ERR_ARG, "solve_workspace: bad descriptor");
    expect_status(spx_cg_solve(nullptr, dummy, dummy, &o, nullptr, 0, nullptr, nullptr), SPX_ERR_ARG,
                  "cg_solve: null descriptor");
    expect_status(spx_cg_batch(nullptr, 1, nullptr, 0, nullptr), SPX_ERR_ARG, "cg_batch: null systems");
    expect_status(spx_cg_batch_noalloc(nullptr, 1, nullptr), SPX_ERR_ARG, "cg_batch_noalloc: null systems");
    expect_status(spx_server_create(nullptr, nullptr), SPX_ERR_ARG, "server_create: null config");
    uint64_t t = 0;
    expect_status(spx_serve_submit(nullptr, nullptr, &t), SPX_ERR_ARG, "serve_submit: null server");
}

double relres(const Csr &A, const std::vector<double> &b, const std::vector<double> &x)
{
    double rr = 0, bb = 0;
    for (int32_t i = 0; i < A.n; ++i) {
        double s = b[(size_t)i];
        for (int32_t p = A.rowptr[(size_t)i]; p < A.rowptr[(size_t)i + 1]; ++p) s -= A.val[(size_t)p] * x[(size_t)A.col[(size_t)p]];
        rr += s * s;
        bb += b[(size_t)i] * b[(size_t)i];
    }
    return std::sqrt(rr / bb);
}

void serve_checks()
{
    int ndev = 0;
    expect(hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0, "a GPU is visible");
    // a budget that holds only a few of the systems at once: admission waits
    // for memory to be freed, and the pool is carved and reused many times
    spx_server_config cfg{};
    cfg.device = 0;
    cfg.max_slots = 16;
    cfg.hbm_budget_bytes = size_t(4) << 20;
    spx_server *srv = nullptr;
    expect_status(spx_server_create(&cfg, &srv), SPX_OK, "server_create (4 MiB budget)");
    const int kReq = 48;
    std::vector<Csr> mats;
    std::vector<std::vector<double>> bs, xs;
    std::vector<uint64_t> tickets;
    for (int k = 0; k < kReq; ++k) {
        mats.push_back(poisson2d(8 + (k * 7) % 57));
        const Csr &A = mats.back();
        std::vector<double> b((size_t)A.n);
        for (int32_t i = 0; i < A.n; ++i) b[(size_t)i] = std::sin(0.37 * i + k);
        bs.push_back(b);
        xs.emplace_back((size_t)A.n, 0.0);
    }
    for (int k = 0; k < kReq; ++k) {
        const Csr &A = mats[(size_t)k];
        spx_request r{};
        r.n = A.n;
        r.solver = (k % 5 == 3) ? SPX_SOLVER_BICGSTAB : SPX_SOLVER_CG;
        r.nnz = (int64_t)A.col.size();
        r.rowptr = A.rowptr.data();
        r.colidx = A.col.data();
        r.vals = A.val.data();
        r.b = bs[(size_t)k].data();
        r.x_out = xs[(size_t)k].data();
        r.tol = 1e-8;
        uint64_t t = 0;
        expect(spx_serve_submit(srv, &r, &t) == SPX_OK, "serve_submit");
        tickets.push_back(t);
    }
    std::printf("ok   %-58s %d requests\n", "serve_submit under a small budget", kReq);
    // cancel a few (each either ends CANCELLED or had already finished)
    for (int k = 5; k < kReq; k += 9) expect(spx_serve_cancel(srv, tickets[(size_t)k]) == SPX_OK, "serve_cancel");
    int done = 0, nc = 0;
    for (int k = 0; k < kReq; ++k) {
        spx_solve_info info{};
        const spx_status st = spx_serve_wait(srv, tickets[(size_t)k], 120.0, &info);
        if (st == SPX_CANCELLED) {
            expect(k % 9 == 5, "only cancelled tickets end CANCELLED");
            ++nc;
            continue;
        }
        expect(st == SPX_OK, "serve_wait: converged");
        expect(relres(mats[(size_t)k], bs[(size_t)k], xs[(size_t)k]) <= 1e-8, "served solution: relative residual");
        ++done;
    }
    std::printf("ok   %-58s %d solved, %d cancelled\n", "served results checked on the host", done, nc);
    // a request that can never fit is refused at once
    {
        const Csr big = poisson2d(600);
        std::vector<double> b((size_t)big.n, 1.0);
        spx_request r{};
        r.n = big.n;
        r.solver = SPX_SOLVER_CG;
        r.nnz = (int64_t)big.col.size();
        r.rowptr = big.rowptr.data();
        r.colidx = big.col.data();
        r.vals = big.val.data();
        r.b = b.data();
        r.tol = 1e-8;
        uint64_t t = 0;
        expect_status(spx_serve_submit(srv, &r, &t), SPX_ERR_BUDGET, "serve_submit: larger than the budget");
    }
    spx_server_stats stats{};
    expect_status(spx_server_get_stats(srv, &stats), SPX_OK, "server_get_stats");
    expect(stats.pool_bytes_in_use == 0 && stats.pool_bytes_peak <= cfg.hbm_budget_bytes, "pool drained, peak in budget");
    // destroy with work still queued: every ticket must end (no leak, no hang)
    for (int k = 0; k < 12; ++k) {
        const Csr &A = mats[(size_t)(k + 30)];
        spx_request r{};
        r.n = A.n;
        r.solver = SPX_SOLVER_CG;
        r.nnz = (int64_t)A.col.size();
        r.rowptr = A.rowptr.data();
        r.colidx = A.col.data();
        r.vals = A.val.data();
        r.b = bs[(size_t)k + 30].data();
        r.tol = 1e-8;
        uint64_t t = 0;
        expect(spx_serve_submit(srv, &r, &t) == SPX_OK, "serve_submit before destroy");
    }
    expect_status(spx_server_destroy(srv), SPX_OK, "server_destroy with requests queued");
}

}  // namespace

int main(int argc, char **argv)
{
    const char *mode = argc > 1 ? argv[1] : "host";
    if (std::strcmp(mode, "host") == 0) {
        host_checks();
    } else if (std::strcmp(mode, "serve") == 0) {
        host_checks();
        serve_checks();
    } else {
        std::fprintf(stderr, "usage: abi_driver host|serve\n");
        return 2;
    }
    std::printf("abi_driver ok (%d checks)\n", g_checks);
    return 0;
}
