"""Oracle: restarted right-preconditioned GMRES(m) / flexible GMRES(m).

Test infrastructure only (see oracle/__init__.py).

Sec. 5.2 defines GMRES as the minimal-residual iterate over the Krylov space (standard
Euclidean inner product, D = I).  Sec. 6.1 fixes right preconditioning, the stopping rule
(relative residual reduced by 1e-6) and the iteration cap.  The paper does not state the
orthogonalisation or the least-squares update; this oracle uses:

* classical Gram-Schmidt applied twice (h = V^H w; w -= V h; h' = V^H w; w -= V h'; h += h');
* complex Givens rotations, for (a, b) with r = sqrt(|a|^2 + |b|^2):
  a = 0: c = 0, s = 1, rho = b;  else c = |a|/r, s = (a/|a|) conj(b)/r, rho = (a/|a|) r;
  the rotation maps (x, y) -> (c x + s y, -conj(s) x + c y);
* one iteration = one preconditioner application + one product with A;
* a cycle ends when |g_{j+1}| <= rtol * ||b - A x0|| or after m iterations; then
  x += B^-1 (V y) (standard) or x += Z y with z_j = B^-1 v_j kept (flexible);
* the solve ends when the true relative residual ||b - A x|| / ||b - A x0|| <= rtol, or when
  max_iters iterations have been taken;
* fixed_iters > 0 runs exactly that many iterations (restarting every m) ignoring rtol.

Weighted GMRES (Sec. 5.2 with a Hermitian positive definite D): the iterate minimises
||b - A x||_D = sqrt((b - A x)^H D (b - A x)) over the same Krylov space.  The Arnoldi process
orthonormalises in <v, w>_D = w^H D v (weighted Arnoldi): h_i = <w, v_i>_D = v_i^H (D w), again
classical Gram-Schmidt twice (D w recomputed before each pass), h_{j+1,j} = ||w||_D.  The basis
is then D-orthonormal, so ||beta e_1 - H y||_2 = ||r||_D and the Givens least squares is
unchanged.  Every residual norm of the method (beta, the cycle test, the true-residual test) is
the D-norm: rtol bounds ||b - A x||_D / ||b - A x0||_D.  D = None is the standard method above
(the same operations, not D = I).
"""
import numpy as np


def givens(a, b):
    """(c, s, rho) with c real, mapping (a, b) -> (rho, 0)."""
    if a == 0:
        return 0.0, 1.0 + 0.0j, b
    r = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    ph = a / abs(a)
    return abs(a) / r, ph * np.conj(b) / r, ph * r


def apply_givens(c, s, x, y):
    return c * x + s * y, -np.conj(s) * x + c * y


class Result:
    def __init__(self, x, iters, cycles, converged, relres_true, relres_est, history):
        self.x, self.iters, self.cycles, self.converged = x, iters, cycles, converged
        self.relres_true, self.relres_est, self.history = relres_true, relres_est, history


def gmres(A, b, M=None, x0=None, restart=50, rtol=1e-6, max_iters=1000, flexible=False,
          fixed_iters=0, D=None):
    """A: object with @ (matrix), M: callable preconditioner (None = identity), D: Hermitian
    positive definite weight with @ (None = Euclidean inner product)."""
    n = b.shape[0]
    Mf = (lambda v: v) if M is None else M
    if D is None:
        norm = np.linalg.norm

        def dots(Vj, w):  # v_i^H w
            return Vj.conj() @ w
    else:
        def norm(w):  # ||w||_D
            return np.sqrt(np.real(np.vdot(w, D @ w)))

        def dots(Vj, w):  # <w, v_i>_D = v_i^H D w
            return Vj.conj() @ (D @ w)
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - A @ x
    beta0 = norm(r)
    history = [1.0]
    total = 0
    cycles = 0
    limit = fixed_iters if fixed_iters > 0 else max_iters
    if beta0 == 0.0:
        return Result(x, 0, 0, True, 0.0, 0.0, history)
    est = 1.0
    while True:
        beta = norm(r)
        if fixed_iters == 0 and beta <= rtol * beta0:
            return Result(x, total, cycles, True, beta / beta0, est, history)
        if total >= limit:
            return Result(x, total, cycles, fixed_iters > 0, beta / beta0, est, history)
        cycles += 1
        m = restart
        V = np.zeros((m + 1, n), dtype=np.complex128)
        Z = np.zeros((m, n), dtype=np.complex128) if flexible else None
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(m):
            z = Mf(V[j])
            if flexible:
                Z[j] = z
            w = A @ z
            h = dots(V[: j + 1], w)
            w = w - V[: j + 1].T @ h
            h2 = dots(V[: j + 1], w)
            w = w - V[: j + 1].T @ h2
            h = h + h2
            hn = norm(w)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            if hn > 0:
                V[j + 1] = w / hn
            for i in range(j):
                H[i, j], H[i + 1, j] = apply_givens(cs[i], sn[i], H[i, j], H[i + 1, j])
            c, s, rho = givens(H[j, j], H[j + 1, j])
            cs[j], sn[j] = c, s
            H[j, j], H[j + 1, j] = rho, 0.0
            g[j], g[j + 1] = apply_givens(c, s, g[j], g[j + 1])
            total += 1
            j_end = j + 1
            est = abs(g[j + 1]) / beta0
            history.append(est)
            if fixed_iters == 0 and abs(g[j + 1]) <= rtol * beta0:
                break
            if total >= limit or hn == 0:
                break
        k = j_end
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        if flexible:
            x = x + Z[:k].T @ y
        else:
            x = x + Mf(V[:k].T @ y)
        r = b - A @ x
