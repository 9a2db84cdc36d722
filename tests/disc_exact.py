"""Exact constant-field averages of the discretisation levels (Sec. 4.1)
for tests.  The flux through any sub-loop is eB T times its signed area, a
quadratic form x^T K y in the Gaussian loop coordinates, so
<cos(theta x^T K y)> = det(I + theta^2 C K C K^T)^(-1/2) with C the loop
covariance.  C comes from the discrete loop law and K from the sub-loops'
point lists; nothing here calls the oracle or the library."""
import numpy as np

DISC_PAPER, DISC_FULL = 0, 1


def loop_cov(n):
    """Per-component covariance of the CM-fixed discrete loop law
    exp(-(N/4) sum |y_{i+1} - y_i|^2): (2/N) times the pseudo-inverse of the
    cyclic Laplacian."""
    L = 2 * np.eye(n) - np.roll(np.eye(n), 1, 1) - np.roll(np.eye(n), -1, 1)
    return (2.0 / n) * np.linalg.pinv(L)


def area_form(n, idx):
    """K with x^T K y = signed (shoelace) area of the polygon through the
    points idx[0], idx[1], ... (closed)."""
    K = np.zeros((n, n))
    m = len(idx)
    for j in range(m):
        a, b = idx[j], idx[(j + 1) % m]
        K[a, b] += 0.5
        K[b, a] -= 0.5
    return K


def char_fn(C, K, th):
    return np.linalg.det(np.eye(C.shape[0]) + th * th * C @ K @ C @ K.T) ** -0.5


def classes(n):
    return (list(range(0, n, 2)), list(range(1, n, 4)), list(range(3, n, 4)))


def exact_levels(n, th, mode):
    """Exact constant-field scalar <W> at the three levels (N, N/2, N/4)."""
    C = loop_cov(n)
    c, s, t = (area_form(n, i) for i in classes(n))
    w2 = char_fn(C, c, th)
    if mode == DISC_PAPER:
        w1 = char_fn(C, 0.5 * c + 0.25 * s + 0.25 * t, th)
        w4 = char_fn(C, 0.5 * (s + t), th)
    else:
        w1 = char_fn(C, area_form(n, list(range(n))), th)
        w4 = 0.5 * (char_fn(C, s, th) + char_fn(C, t, th))
    return np.array([w1, w2, w4])
