"""FP64 reference of the learned coarse-lattice correction.

TEST INFRASTRUCTURE ONLY: used by the tests and the smoke check, never by
the product library.  Plain numpy, written for reading, not for speed.

What is computed (the correction is not part of the paper's scheme; the
coarse lattice is the paper's scheme at 4x coarser resolution, Sec. VI-VII):

  restrict(f)       full-weighting restriction by an even factor m: coarse
                    node (X, Y) averages fine nodes (mX + i, mY + j),
                    |i|, |j| <= m/2, with weight 1/2 on the outermost row and
                    column of the window, i.e. the tensor product of
                    [1/2, 1, ..., 1, 1/2] / m in x and in y (periodic).
  features(obs)     per coarse node the 3x3 periodic neighbourhood of the six
                    fields rho, Ux, Uy, Cxx, Cxy, Cyy of the observables
                    array: feature 6 s + f for stencil position
                    s = 3 (dy + 1) + (dx + 1) and field f in that order.
  mlp forward       y = W3 gelu(W2 gelu(W1 x + b1) + b2) + b3 with the exact
                    (erf) GELU, gelu(z) = z Phi(z).
  mlp backward      gradients of the loss mean((y - t)^2) over all entries.
  adam              Kingma & Ba (2015), bias-corrected, in the order of
                    their Algorithm 1.
  source(dJ, dtau)  the body force through which the correction acts:
                    F = dJ + div_h(dtau) with central differences,
                    (div tau)_x = d_x tau_xx + d_y tau_xy,
                    (div tau)_y = d_x tau_xy + d_y tau_yy.
  targets           per coarse node: momentum rho U and polymer stress
                    (tau_xx, tau_xy, tau_yy) of the restricted fine state
                    minus those of the coarse state after one coarse step.

Parameter layout shared with the library's flat parameter vector:
  W1 [hidden][in], b1 [hidden], W2 [hidden][hidden], b2 [hidden],
  W3 [out][hidden], b3 [out]   (each W maps column vectors: z = W x + b).
"""
from __future__ import annotations

import math

import numpy as np

FEATURE_FIELDS = (0, 1, 2, 4, 5, 6)  # rho, Ux, Uy, Cxx, Cxy, Cyy in the observables order
N_FEATURES = 9 * len(FEATURE_FIELDS)
N_OUT = 5  # dJx, dJy, dtau_xx, dtau_xy, dtau_yy


# -- activation -----------------------------------------------------------------------

def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    erf = np.vectorize(math.erf)
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    z = np.asarray(z, dtype=np.float64)
    erf = np.vectorize(math.erf)
    Phi = 0.5 * (1.0 + erf(z / math.sqrt(2.0)))
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return Phi + z * phi


# -- parameters -----------------------------------------------------------------------

def shapes(n_in, hidden, n_out):
    return [("W1", (hidden, n_in)), ("b1", (hidden,)), ("W2", (hidden, hidden)),
            ("b2", (hidden,)), ("W3", (n_out, hidden)), ("b3", (n_out,))]


def n_params(n_in, hidden, n_out):
    return sum(int(np.prod(s)) for _, s in shapes(n_in, hidden, n_out))


def unflatten(theta, n_in, hidden, n_out):
    out, o = {}, 0
    for name, s in shapes(n_in, hidden, n_out):
        n = int(np.prod(s))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(s)
        o += n
    return out


def flatten(p):
    return np.concatenate([np.ravel(p[k]) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


# -- network --------------------------------------------------------------------------

def forward(p, X):
    """X [n][in] -> (Y [n][out], cache)."""
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ p["W1"].T + p["b1"]
    H1 = gelu(Z1)
    Z2 = H1 @ p["W2"].T + p["b2"]
    H2 = gelu(Z2)
    Y = H2 @ p["W3"].T + p["b3"]
    return Y, dict(X=X, Z1=Z1, H1=H1, Z2=Z2, H2=H2)


def loss(Y, T):
    return float(np.mean((Y - T) ** 2))


def backward(p, cache, Y, T):
    """Gradients of mean((Y - T)^2) with respect to every parameter."""
    dY = 2.0 * (Y - T) / Y.size
    g = {}
    g["W3"] = dY.T @ cache["H2"]
    g["b3"] = dY.sum(axis=0)
    dH2 = dY @ p["W3"]
    dZ2 = dH2 * gelu_grad(cache["Z2"])
    g["W2"] = dZ2.T @ cache["H1"]
    g["b2"] = dZ2.sum(axis=0)
    dH1 = dZ2 @ p["W2"]
    dZ1 = dH1 * gelu_grad(cache["Z1"])
    g["W1"] = dZ1.T @ cache["X"]
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init_params(n_in, hidden, n_out, seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases (numpy
    generator; the library draws its own initial weights)."""
    r = np.random.default_rng(seed)
    p = {}
    for name, s in shapes(n_in, hidden, n_out):
        p[name] = (r.uniform(-1, 1, size=s) / math.sqrt(s[1])) if name[0] == "W" else np.zeros(s)
    return p


def correction(p, X, in_mean, in_std, out_mean, out_std):
    """Raw features X [n][in] -> correction [n][out]: the network applied to
    standardised inputs, its outputs mapped back to physical units."""
    Z = (np.asarray(X, dtype=np.float64) - in_mean) / in_std
    Y, _ = forward(p, Z)
    return Y * out_std + out_mean


# -- lattice side ---------------------------------------------------------------------

def restrict(f, m):
    """Full-weighting restriction of the last two axes [..., ny, nx] by m."""
    f = np.asarray(f, dtype=np.float64)
    ny, nx = f.shape[-2:]
    assert m % 2 == 0 and ny % m == 0 and nx % m == 0
    w = np.ones(m + 1)
    w[0] = w[-1] = 0.5
    w /= m
    out = np.zeros(f.shape[:-2] + (ny // m, nx // m))
    for Y in range(ny // m):
        for X in range(nx // m):
            acc = 0.0
            for j in range(m + 1):
                for i in range(m + 1):
                    y = (m * Y + j - m // 2) % ny
                    x = (m * X + i - m // 2) % nx
                    acc = acc + w[j] * w[i] * f[..., y, x]
            out[..., Y, X] = acc
    return out


def features(obs):
    """obs [10][ny][nx] observables -> X [ny nx][54]."""
    obs = np.asarray(obs, dtype=np.float64)
    _, ny, nx = obs.shape
    X = np.zeros((ny * nx, N_FEATURES))
    for y in range(ny):
        for x in range(nx):
            n = y * nx + x
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    s = 3 * (dy + 1) + (dx + 1)
                    for fi, f in enumerate(FEATURE_FIELDS):
                        X[n, 6 * s + fi] = obs[f, (y + dy) % ny, (x + dx) % nx]
    return X


def momentum_stress(obs):
    """[5][ny][nx]: rho Ux, rho Uy, tau_xx, tau_xy, tau_yy of an observables array."""
    obs = np.asarray(obs, dtype=np.float64)
    return np.stack([obs[0] * obs[1], obs[0] * obs[2], obs[7], obs[8], obs[9]])


def targets(obs_fine_restricted, obs_coarse):
    """Y [ny nx][5]: correction that takes the coarse state to the restricted
    fine state (momentum and polymer stress)."""
    d = momentum_stress(obs_fine_restricted) - momentum_stress(obs_coarse)
    return d.reshape(5, -1).T.copy()


def source(corr, ny, nx):
    """corr [ny nx][5] (dJx, dJy, dtau_xx, dtau_xy, dtau_yy) -> F [2][ny][nx]:
    F = dJ - <dJ> + div_h(dtau), central differences, <.> the lattice mean.
    Total momentum is conserved on the fine and on the coarse lattice and by
    the restriction, so the exact correction dJ has zero lattice mean; the
    mean of a predicted one is removed (the divergence has zero mean by
    itself on a periodic lattice)."""
    c = np.asarray(corr, dtype=np.float64).T.reshape(5, ny, nx)

    def dx(a):
        return 0.5 * (np.roll(a, -1, axis=1) - np.roll(a, 1, axis=1))

    def dy(a):
        return 0.5 * (np.roll(a, -1, axis=0) - np.roll(a, 1, axis=0))

    Fx = (c[0] - c[0].mean()) + dx(c[2]) + dy(c[3])
    Fy = (c[1] - c[1].mean()) + dx(c[3]) + dy(c[4])
    return np.stack([Fx, Fy])
