// C-ABI of the full-order side: a FOM handle (sparse operators and source
// on the device), rank-2 FOM stepping, the Galerkin projection onto given
// bases, and POD of a snapshot matrix.  Validation is synchronous and comes
// before any enqueue, as for the ROM entry points.
//
// POD (Sec. 4.4: left singular vectors of the snapshot matrix, kept by a
// cumulative-energy criterion) of a tall-skinny snapshot matrix X (n x ns)
// that may be numerically rank deficient (snapshots of one wave field
// often are):
//   1. G = X^T X on the device; its eigen-decomposition G = V L V^T on the
//      host (one-sided Jacobi, Hestenes); the numerical rank r counts the
//      eigenvalues above 100 ns u l_1.
//   2. Y = X V_r (device), orthonormalised by two Cholesky QR passes
//      (Gram products and Y R^{-1} on the device): Q spans the dominant
//      r-dimensional subspace; cond(Y) <= sqrt(l_1 / l_r) keeps the passes
//      well inside their range.
//   3. Rayleigh-Ritz: B = Q^T X (device), its SVD B = U_B S W^T on the host
//      (one-sided Jacobi on the columns of B), modes Phi = Q U_B (device).
// The singular values from step 3 carry the relative error of an SVD of X
// (u sigma_1 / sigma_i), not the squared one of the Gram matrix.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "rom_internal.h"

struct rom_fom {
    int device = 0;
    int nv = 0, ns = 0;
    double dt = 0.0;
    int source = 0;
    rom::FomCsr av, as;
    double *f = nullptr;
    void *mem = nullptr;          // one device block holding everything above
};

namespace {

using rom::api_fail;
using rom::api_hip_fail;

void dfree(void *p) {
    if (p) (void)hipFree(p);
}

bool finite_all(const double *x, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) return false;
    return true;
}

rom_status check_csr(int nrows, int ncols, const int32_t *ptr, const int32_t *col, const double *val,
                     const std::string &what) {
    if (!ptr || (ptr[nrows] > 0 && (!col || !val))) return api_fail(ROM_E_ARG, what + ": NULL array");
    if (ptr[0] != 0) return api_fail(ROM_E_ARG, what + ": row pointer must start at 0");
    for (int r = 0; r < nrows; ++r)
        if (ptr[r + 1] < ptr[r]) return api_fail(ROM_E_ARG, what + ": row pointers must not decrease");
    const int64_t nnz = ptr[nrows];
    for (int64_t k = 0; k < nnz; ++k)
        if (col[k] < 0 || col[k] >= ncols) return api_fail(ROM_E_ARG, what + ": column index out of range");
    if (!finite_all(val, (size_t)nnz)) return api_fail(ROM_E_NONFINITE, what + ": non-finite value");
    return ROM_OK;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Padded (ELL) copy of a CSR operator when its longest row has at most 8
// entries: width W in {2, 4, 8}, entries in stored order, unused slots
// column -1 and value 0.  W = 0: no copy (the kernels use the CSR form).
struct Ell {
    int W = 0;
    std::vector<int> col;
    std::vector<double> val;
};

Ell make_ell(int nrows, const int32_t *ptr, const int32_t *col, const double *val) {
    Ell E;
    int wmax = 0;
    for (int r = 0; r < nrows; ++r) wmax = std::max(wmax, (int)(ptr[r + 1] - ptr[r]));
    if (wmax > 8) return E;
    E.W = wmax <= 2 ? 2 : (wmax <= 4 ? 4 : 8);
    E.col.assign((size_t)nrows * E.W, -1);
    E.val.assign((size_t)nrows * E.W, 0.0);
    for (int r = 0; r < nrows; ++r)
        for (int k = ptr[r]; k < ptr[r + 1]; ++k) {
            E.col[(size_t)r * E.W + (k - ptr[r])] = col[k];
            E.val[(size_t)r * E.W + (k - ptr[r])] = val[k];
        }
    return E;
}

// ---- small dense linear algebra on the host (column-major n x n) ---------

// Upper Cholesky factor R of the symmetric positive definite A (A = R^T R);
// false if a pivot is not positive.
bool cholesky_upper(const std::vector<double> &A, int n, std::vector<double> &R) {
    R.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i <= j; ++i) {
            double s = A[(size_t)j * n + i];
            for (int k = 0; k < i; ++k) s -= R[(size_t)i * n + k] * R[(size_t)j * n + k];
            if (i == j) {
                if (!(s > 0.0)) return false;
                R[(size_t)j * n + j] = sqrt(s);
            } else {
                R[(size_t)j * n + i] = s / R[(size_t)i * n + i];
            }
        }
    }
    return true;
}

// Inverse of an upper triangular R (back substitution per column).
void inverse_upper(const std::vector<double> &R, int n, std::vector<double> &Ri) {
    Ri.assign((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
        Ri[(size_t)j * n + j] = 1.0 / R[(size_t)j * n + j];
        for (int i = j - 1; i >= 0; --i) {
            double s = 0.0;
            for (int k = i + 1; k <= j; ++k) s += R[(size_t)k * n + i] * Ri[(size_t)j * n + k];
            Ri[(size_t)j * n + i] = -s / R[(size_t)i * n + i];
        }
    }
}

// One Hestenes rotation of columns p, q of the m x c column-major A:
// makes them orthogonal; returns whether it rotated.  A column whose squared
// norm is at most `tiny` (eps^2 times the squared Frobenius norm of A) is
// numerically zero: rounding noise keeps such columns from ever testing
// orthogonal, and their rotations cannot change any column above the floor,
// so pairs with one are skipped.
bool rotate_pair(double *A, int m, int p, int q, double tiny) {
    const double eps = 2.220446049250313e-16;
    double *ap = A + (size_t)p * m, *aq = A + (size_t)q * m;
    double alpha = 0.0, beta = 0.0, gamma = 0.0;
    for (int i = 0; i < m; ++i) {
        alpha += ap[i] * ap[i];
        beta += aq[i] * aq[i];
        gamma += ap[i] * aq[i];
    }
    if (alpha <= tiny || beta <= tiny) return false;
    if (gamma == 0.0 || fabs(gamma) <= eps * sqrt(alpha * beta)) return false;
    const double zeta = (beta - alpha) / (2.0 * gamma);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
    for (int i = 0; i < m; ++i) {
        const double x = ap[i], y = aq[i];
        ap[i] = cs * x - sn * y;
        aq[i] = sn * x + cs * y;
    }
    return true;
}

// Singular values (descending, c of them) and left singular vectors of the
// m x c column-major A by one-sided Jacobi (Hestenes): rotate column pairs
// until all are orthogonal to working precision; then sigma_j = |a_j| and
// u_j = a_j / sigma_j (U is m x c; columns of zero norm stay zero).  Pairs
// are visited in round-robin order (each round pairs every column with one
// other, so its rotations touch disjoint columns), and the rounds of larger
// problems are shared out over host threads; the order of a round does not
// change its result, so the output does not depend on the thread count.
void jacobi_svd_left(std::vector<double> A, int m, int c, std::vector<double> &sigma, std::vector<double> &U) {
    double fro2 = 0.0;
    for (size_t i = 0; i < A.size(); ++i) fro2 += A[i] * A[i];
    const double tiny = 4.930380657631324e-32 * fro2;      // eps^2 |A|_F^2
    const int cc = c + (c & 1);                  // even count; index c (if any) is a dummy
    const int npair = cc / 2;
    int nthr = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
    if ((double)npair * m < 32768.0) nthr = 1;   // too little work per round to share
    nthr = std::min(nthr, std::max(1, npair / 4));
    // circle method: position 0 fixed, the others rotate one place per round
    std::vector<int> ring(cc);
    for (int i = 0; i < cc; ++i) ring[i] = i;
    std::atomic<int> arrive{0}, gen{0};
    std::atomic<bool> rotated{false}, done{false};
    auto barrier = [&](int nth) {
        const int g = gen.load(std::memory_order_acquire);
        if (arrive.fetch_add(1, std::memory_order_acq_rel) == nth - 1) {
            arrive.store(0, std::memory_order_relaxed);
            gen.fetch_add(1, std::memory_order_acq_rel);
        } else {
            while (gen.load(std::memory_order_acquire) == g) std::this_thread::yield();
        }
    };
    auto worker = [&](int tid) {
        for (int sweep = 0; sweep < 80; ++sweep) {
            for (int r = 0; r < cc - 1; ++r) {
                for (int k = tid; k < npair; k += nthr) {
                    int p = ring[k], q = ring[cc - 1 - k];
                    if (p > q) std::swap(p, q);
                    if (q < c && rotate_pair(A.data(), m, p, q, tiny)) rotated.store(true, std::memory_order_relaxed);
                }
                barrier(nthr);
                if (tid == 0) {                  // next round's pairing
                    const int last = ring[cc - 1];
                    for (int i = cc - 1; i > 1; --i) ring[i] = ring[i - 1];
                    if (cc > 1) ring[1] = last;
                }
                barrier(nthr);
            }
            if (tid == 0) {
                done.store(!rotated.load(std::memory_order_relaxed), std::memory_order_relaxed);
                rotated.store(false, std::memory_order_relaxed);
            }
            barrier(nthr);
            if (done.load(std::memory_order_relaxed)) break;
        }
    };
    if (nthr == 1) {
        worker(0);
    } else {
        std::vector<std::thread> pool;
        for (int t = 1; t < nthr; ++t) pool.emplace_back(worker, t);
        worker(0);
        for (std::thread &th : pool) th.join();
    }
    std::vector<double> nrm(c);
    for (int j = 0; j < c; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += A[(size_t)j * m + i] * A[(size_t)j * m + i];
        nrm[j] = sqrt(s);
    }
    std::vector<int> order(c);
    for (int j = 0; j < c; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nrm[a] > nrm[b]; });
    sigma.assign(c, 0.0);
    U.assign((size_t)m * c, 0.0);
    for (int jj = 0; jj < c; ++jj) {
        const int j = order[jj];
        sigma[jj] = nrm[j];
        if (nrm[j] > 0.0)
            for (int i = 0; i < m; ++i) U[(size_t)jj * m + i] = A[(size_t)j * m + i] / nrm[j];
    }
}

// Gram matrix G = X^T X (n x n) of the row-major X (N x n), on the device,
// copied to the host.
rom_status gram(const double *X, int64_t N, int n, double *part, double *Gd, std::vector<double> &G,
                hipStream_t st) {
    hipError_t e = rom::launch_gemm_tn(X, X, N, n, n, part, Gd, st);
    G.assign((size_t)n * n, 0.0);
    if (e == hipSuccess) e = hipMemcpyAsync(G.data(), Gd, sizeof(double) * G.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return api_hip_fail(e, "rom_pod: Gram product");
    for (int j = 0; j < n; ++j)           // exact symmetry (the two triangles round alike anyway)
        for (int i = 0; i < j; ++i) G[(size_t)i * n + j] = G[(size_t)j * n + i];
    return ROM_OK;
}

}  // namespace

extern "C" {

rom_status rom_fom_create(int32_t nv, int32_t ns, const int32_t *av_ptr, const int32_t *av_col, const double *av_val,
                          const int32_t *as_ptr, const int32_t *as_col, const double *as_val, const double *f,
                          double dt, uint32_t flags, void *stream, rom_fom **out) {
    if (out) *out = nullptr;
    if (!out || !f) return api_fail(ROM_E_ARG, "rom_fom_create: NULL argument");
    if (nv < 1 || ns < 1) return api_fail(ROM_E_ARG, "rom_fom_create: Nv and Ns must be >= 1");
    if (!(dt > 0.0) || !isfinite(dt)) return api_fail(ROM_E_ARG, "rom_fom_create: dt must be finite and > 0");
    if (flags & ~(uint32_t)ROM_SOURCE_GAUSS1) return api_fail(ROM_E_ARG, "rom_fom_create: unknown flag bits");
    rom_status rs = check_csr(nv, ns, av_ptr, av_col, av_val, "rom_fom_create: Av");
    if (rs == ROM_OK) rs = check_csr(ns, nv, as_ptr, as_col, as_val, "rom_fom_create: As");
    if (rs != ROM_OK) return rs;
    if (!finite_all(f, nv)) return api_fail(ROM_E_NONFINITE, "rom_fom_create: non-finite source");
    const int64_t nzv = av_ptr[nv], nzs = as_ptr[ns];
    const size_t b_avp = align256(sizeof(int) * (size_t)(nv + 1)), b_avc = align256(sizeof(int) * (size_t)nzv);
    const size_t b_avv = align256(sizeof(double) * (size_t)nzv), b_asp = align256(sizeof(int) * (size_t)(ns + 1));
    const size_t b_asc = align256(sizeof(int) * (size_t)nzs), b_asv = align256(sizeof(double) * (size_t)nzs);
    const size_t b_f = align256(sizeof(double) * (size_t)nv);
    const Ell ev = make_ell(nv, av_ptr, av_col, av_val), es = make_ell(ns, as_ptr, as_col, as_val);
    const size_t b_evc = align256(sizeof(int) * ev.col.size()), b_evv = align256(sizeof(double) * ev.val.size());
    const size_t b_esc = align256(sizeof(int) * es.col.size()), b_esv = align256(sizeof(double) * es.val.size());
    const size_t total = b_avp + b_avc + b_avv + b_asp + b_asc + b_asv + b_f + b_evc + b_evv + b_esc + b_esv;
    rom_fom *F = new (std::nothrow) rom_fom();
    if (!F) return api_fail(ROM_E_NOMEM, "rom_fom_create: host allocation failed");
    hipError_t e = hipGetDevice(&F->device);
    if (e != hipSuccess) { delete F; return api_hip_fail(e, "rom_fom_create: hipGetDevice"); }
    e = hipMalloc(&F->mem, total);
    if (e != hipSuccess) { delete F; return api_fail(ROM_E_NOMEM, "rom_fom_create: device allocation failed"); }
    char *m = static_cast<char *>(F->mem);
    int *avp = reinterpret_cast<int *>(m); m += b_avp;
    int *avc = reinterpret_cast<int *>(m); m += b_avc;
    double *avv = reinterpret_cast<double *>(m); m += b_avv;
    int *asp = reinterpret_cast<int *>(m); m += b_asp;
    int *asc = reinterpret_cast<int *>(m); m += b_asc;
    double *asv = reinterpret_cast<double *>(m); m += b_asv;
    F->f = reinterpret_cast<double *>(m); m += b_f;
    int *evc = reinterpret_cast<int *>(m); m += b_evc;
    double *evv = reinterpret_cast<double *>(m); m += b_evv;
    int *esc = reinterpret_cast<int *>(m); m += b_esc;
    double *esv = reinterpret_cast<double *>(m);
    hipStream_t st = static_cast<hipStream_t>(stream);
    e = hipMemcpyAsync(avp, av_ptr, sizeof(int) * (size_t)(nv + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nzv) e = hipMemcpyAsync(avc, av_col, sizeof(int) * (size_t)nzv, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nzv) e = hipMemcpyAsync(avv, av_val, sizeof(double) * (size_t)nzv, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(asp, as_ptr, sizeof(int) * (size_t)(ns + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nzs) e = hipMemcpyAsync(asc, as_col, sizeof(int) * (size_t)nzs, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nzs) e = hipMemcpyAsync(asv, as_val, sizeof(double) * (size_t)nzs, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(F->f, f, sizeof(double) * (size_t)nv, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && ev.W)
        e = hipMemcpyAsync(evc, ev.col.data(), sizeof(int) * ev.col.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && ev.W)
        e = hipMemcpyAsync(evv, ev.val.data(), sizeof(double) * ev.val.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && es.W)
        e = hipMemcpyAsync(esc, es.col.data(), sizeof(int) * es.col.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && es.W)
        e = hipMemcpyAsync(esv, es.val.data(), sizeof(double) * es.val.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { dfree(F->mem); delete F; return api_hip_fail(e, "rom_fom_create: upload"); }
    F->nv = nv; F->ns = ns; F->dt = dt; F->source = (flags & ROM_SOURCE_GAUSS1) ? 1 : 0;
    F->av.ptr = avp; F->av.col = avc; F->av.val = avv; F->av.nrows = nv;
    F->as.ptr = asp; F->as.col = asc; F->as.val = asv; F->as.nrows = ns;
    if (ev.W) { F->av.ecol = evc; F->av.eval = evv; F->av.W = ev.W; }
    if (es.W) { F->as.ecol = esc; F->as.eval = esv; F->as.W = es.W; }
    *out = F;
    return ROM_OK;
}

rom_status rom_fom_run(rom_fom *F, int32_t M, const double *mu, int64_t n0, int64_t nsteps, double *V, double *S,
                       void *stream) {
    if (!F || !mu || !V || !S) return api_fail(ROM_E_ARG, "rom_fom_run: NULL argument");
    if (M < 1) return api_fail(ROM_E_ARG, "rom_fom_run: M must be >= 1");
    if (n0 < 0 || nsteps < 0) return api_fail(ROM_E_ARG, "rom_fom_run: n0 and nsteps must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int64_t k = 0; k < nsteps; ++k) {
        hipError_t e = rom::launch_fom_step(F->av, F->as, F->f, mu, M, n0 + k, F->dt, F->source, V, S, st);
        if (e != hipSuccess) return api_hip_fail(e, "rom_fom_run: launch");
    }
    return ROM_OK;
}

rom_status rom_fom_project(rom_fom *F, int32_t kv, int32_t ks, const double *phi_v, const double *phi_s,
                           double *Avs, double *Asv, double *b, void *stream) {
    if (!F || !phi_v || !phi_s || !Avs || !Asv || !b) return api_fail(ROM_E_ARG, "rom_fom_project: NULL argument");
    if (kv < 1 || ks < 1 || kv > F->nv || ks > F->ns)
        return api_fail(ROM_E_ARG, "rom_fom_project: need 1 <= Kv <= Nv and 1 <= Ks <= Ns");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int zmax = std::max({rom::gemm_tn_splits(F->nv, kv, ks), rom::gemm_tn_splits(F->ns, ks, kv),
                               rom::gemm_tn_splits(F->nv, kv, 1)});
    const size_t by = align256(sizeof(double) * (size_t)F->nv * ks), bs = align256(sizeof(double) * (size_t)F->ns * kv);
    const size_t bp = sizeof(double) * (size_t)zmax * kv * ks;
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, by + bs + bp, st);
    if (e != hipSuccess) return api_fail(ROM_E_NOMEM, "rom_fom_project: device allocation failed");
    double *Yv = static_cast<double *>(ws);
    double *Ys = reinterpret_cast<double *>(static_cast<char *>(ws) + by);
    double *part = reinterpret_cast<double *>(static_cast<char *>(ws) + by + bs);
    e = rom::launch_fom_spmm(F->av, phi_s, ks, Yv, st);                       // Av Phi_s  (Nv x Ks)
    if (e == hipSuccess) e = rom::launch_fom_spmm(F->as, phi_v, kv, Ys, st);  // As Phi_v  (Ns x Kv)
    if (e == hipSuccess) e = rom::launch_gemm_tn(phi_v, Yv, F->nv, kv, ks, part, Avs, st);
    if (e == hipSuccess) e = rom::launch_gemm_tn(phi_s, Ys, F->ns, ks, kv, part, Asv, st);
    if (e == hipSuccess) e = rom::launch_gemm_tn(phi_v, F->f, F->nv, kv, 1, part, b, st);
    hipError_t e2 = hipFreeAsync(ws, st);
    if (e != hipSuccess) return api_hip_fail(e, "rom_fom_project: launch");
    if (e2 != hipSuccess) return api_hip_fail(e2, "rom_fom_project: free");
    return ROM_OK;
}

rom_status rom_fom_destroy(rom_fom *F) {
    if (!F) return ROM_OK;
    dfree(F->mem);
    delete F;
    return ROM_OK;
}

rom_status rom_pod(int64_t n, int32_t ns, const double *X, double tol, int32_t kmax, double *phi, double *sigma,
                   int32_t *k_out, void *stream) {
    if (k_out) *k_out = 0;
    if (!X || !phi || !sigma || !k_out) return api_fail(ROM_E_ARG, "rom_pod: NULL argument");
    if (ns < 1 || ns > 2048 || n < ns) return api_fail(ROM_E_ARG, "rom_pod: need 1 <= ns <= 2048 and n >= ns");
    if (kmax < 1 || kmax > ns) return api_fail(ROM_E_ARG, "rom_pod: need 1 <= kmax <= ns");
    if (!(tol < 1.0) || isnan(tol)) return api_fail(ROM_E_ARG, "rom_pod: tol must be < 1 (negative: keep kmax)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // split partials of the largest product that can occur: X^T X, Y^T Y
    // and Q^T X for any rank r <= ns
    size_t np = (size_t)rom::gemm_tn_splits(n, ns, ns) * ns * ns;
    for (int r = 1; r <= ns; ++r) {
        np = std::max(np, (size_t)rom::gemm_tn_splits(n, r, r) * r * r);
        np = std::max(np, (size_t)rom::gemm_tn_splits(n, r, ns) * r * ns);
    }
    const size_t bx = align256(sizeof(double) * (size_t)n * ns), bg = align256(sizeof(double) * (size_t)ns * ns);
    const size_t bp = sizeof(double) * np;
    void *ws = nullptr;
    hipError_t e = hipMalloc(&ws, 2 * bx + 2 * bg + bp);
    if (e != hipSuccess) return api_fail(ROM_E_NOMEM, "rom_pod: device allocation failed");
    char *w = static_cast<char *>(ws);
    double *Ya = reinterpret_cast<double *>(w);
    double *Yb = reinterpret_cast<double *>(w + bx);
    double *Gd = reinterpret_cast<double *>(w + 2 * bx);
    double *Bd = reinterpret_cast<double *>(w + 2 * bx + bg);
    double *part = reinterpret_cast<double *>(w + 2 * bx + 2 * bg);
    const double u = 1.1102230246251565e-16;
    std::vector<double> G, lam, Vg, R, Ri, B, sb, Ub;
    int r = 0, k = 0;
    rom_status rs = gram(X, n, ns, part, Gd, G, st);
    if (rs == ROM_OK) {
        // 1. eigen-decomposition of the Gram matrix (PSD: its SVD) and the rank
        jacobi_svd_left(G, ns, ns, lam, Vg);
        if (!(lam[0] > 0.0) || !isfinite(lam[0])) rs = api_fail(ROM_E_NONFINITE, "rom_pod: zero or non-finite snapshots");
        else
            while (r < ns && lam[r] > 100.0 * ns * u * lam[0]) ++r;
    }
    if (rs == ROM_OK) {
        // 2. Y = X V_r, two Cholesky QR passes -> Q (in Ya)
        e = hipMemcpyAsync(Bd, Vg.data(), sizeof(double) * (size_t)ns * r, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = rom::launch_gemm_nn(X, Bd, n, ns, r, Ya, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rs = api_hip_fail(e, "rom_pod: X V");
        for (int pass = 0; pass < 2 && rs == ROM_OK; ++pass) {
            double *src = pass == 0 ? Ya : Yb, *dst = pass == 0 ? Yb : Ya;
            rs = gram(src, n, r, part, Gd, G, st);
            if (rs != ROM_OK) break;
            if (!cholesky_upper(G, r, R)) {
                rs = api_fail(ROM_E_UNSUPPORTED, "rom_pod: Cholesky QR of the dominant subspace failed");
                break;
            }
            inverse_upper(R, r, Ri);
            e = hipMemcpyAsync(Bd, Ri.data(), sizeof(double) * Ri.size(), hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = rom::launch_gemm_nn(src, Bd, n, r, r, dst, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);     // Ri is read before it is replaced
            if (e != hipSuccess) rs = api_hip_fail(e, "rom_pod: Y R^-1");
        }
    }
    if (rs == ROM_OK) {
        // 3. B = Q^T X (r x ns), its left singular vectors and values
        B.assign((size_t)r * ns, 0.0);
        e = rom::launch_gemm_tn(Ya, X, n, r, ns, part, Gd, st);
        if (e == hipSuccess) e = hipMemcpyAsync(B.data(), Gd, sizeof(double) * B.size(), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rs = api_hip_fail(e, "rom_pod: Q^T X");
    }
    if (rs == ROM_OK) {
        jacobi_svd_left(B, r, ns, sb, Ub);          // r x ns: at most r nonzero sigma
        for (int i = 0; i < ns; ++i)
            sigma[i] = i < r ? sb[i] : sqrt(std::max(lam[i], 0.0));
        double tot = 0.0;
        for (int i = 0; i < ns; ++i) tot += sigma[i] * sigma[i];
        k = kmax;
        if (tol >= 0.0) {
            double c = 0.0;
            k = ns;
            for (int i = 0; i < ns; ++i) {
                c += sigma[i] * sigma[i];
                if (c >= (1.0 - tol) * tot) { k = i + 1; break; }
            }
        }
        k = std::min(std::min(k, (int)kmax), r);
        // Phi = Q U_B[:, :k], zero columns up to kmax
        std::vector<double> Bk((size_t)r * kmax, 0.0);
        for (int j = 0; j < k; ++j) memcpy(&Bk[(size_t)j * r], &Ub[(size_t)j * r], sizeof(double) * r);
        e = hipMemcpyAsync(Bd, Bk.data(), sizeof(double) * Bk.size(), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = rom::launch_gemm_nn(Ya, Bd, n, r, kmax, phi, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rs = api_hip_fail(e, "rom_pod: Q U");
        else *k_out = k;
    }
    (void)hipStreamSynchronize(st);
    dfree(ws);
    return rs;
}

}  // extern "C"
