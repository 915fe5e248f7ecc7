"""FP64 reference gradient of unrolled compressed NeNMF -- test
infrastructure only (imported by tests/ alone).

The same computation as ``oracle.nenmf`` on ``oracle.rsi`` output (Sec. 3,
Algorithms 1 and 2; Sec. 2 inner loop) written with differentiable torch
float64 CPU operations, so that torch's autograd gives dL/dX independently
of the HIP adjoint:
  * the bases are thin QR factors with positive diagonal (Householder QR
    with the signs fixed; equal to the oracle's Gram-Schmidt bases when no
    column is numerically deficient, which is checked);
  * L = lambda_max(W) from a symmetric eigensolver;
  * every inner loop takes exactly K projected steps (max(0, .) has
    derivative 1[v > 0]), momentum weights of Sec. 2.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .nenmf import momentum_weights

F64 = torch.float64


def _qr_pos(Y: torch.Tensor, tau2: float) -> torch.Tensor:
    Q, R = torch.linalg.qr(Y, mode="reduced")
    d = torch.diagonal(R)
    # the rank rule must not fire: every pivot well above tau2 * max ||y_i||^2
    scale = float(torch.max(torch.sum(Y.detach() ** 2, dim=0)))
    if float(torch.min(d.detach() ** 2)) <= tau2 * scale:
        raise ValueError("a basis column is numerically deficient; no derivative")
    return Q * torch.sign(d)[None, :]


def rsi(X, omega_L, omega_R, q: int, tau2: float = 1e-9):
    """Algorithm 2, two chains, returning (Q_L, Q_R, X_L, X_R)."""
    oL = torch.as_tensor(np.asarray(omega_L, dtype=np.float64))
    oRt = torch.as_tensor(np.asarray(omega_R, dtype=np.float64)).T
    QL = _qr_pos(X @ oL, tau2)
    QRt = _qr_pos(X.T @ oRt, tau2)
    A = B = QtL = QtRt = None
    for k in range(1, q + 1):
        QtL = _qr_pos(X.T @ QL, tau2)
        QtRt = _qr_pos(X @ QRt, tau2)
        A = X @ QtL
        B = X.T @ QtRt
        if k < q:
            QL = _qr_pos(A, tau2)
            QRt = _qr_pos(B, tau2)
    return QtRt, QtL, B.T, A


def nesterov(Z0, W, B, K: int):
    """Exactly K projected Nesterov steps on Z W - B (rows independent)."""
    L = torch.linalg.eigvalsh(0.5 * (W + W.T))[-1]
    beta = momentum_weights(K)
    Y = Z0
    Zp = Z0
    Z = Z0
    for k in range(1, K + 1):
        Z = torch.relu(Y - (Y @ W - B) / L)
        Y = Z + float(beta[k]) * (Z - Zp)
        Zp = Z
    return Z


def unrolled(X, omega_L, omega_R, G0, F0, q: int, T: int, K: int, tau2: float = 1e-9):
    """(G_T, F_T) of compressed NeNMF with T outer iterations of K inner
    steps each, differentiable in X (and G0, F0)."""
    QL, QR, XL, XR = rsi(X, omega_L, omega_R, q, tau2)
    G, F = G0, F0
    for _ in range(T):
        FR = F @ QR
        G = nesterov(G, FR @ FR.T, XR @ FR.T, K)
        GL = QL.T @ G
        F = nesterov(F.T, GL.T @ GL, (GL.T @ XL).T, K).T
    return G, F


def loss_grad(X, omega_L, omega_R, G0, F0, Gt, Ft, q: int, T: int, K: int):
    """L = ||G_T - Gt||^2 + ||F_T - Ft||^2 and dL/dX, dL/dG0, dL/dF0 (FP64)."""
    Xt = torch.tensor(np.asarray(X, dtype=np.float64), requires_grad=True)
    G0t = torch.tensor(np.asarray(G0, dtype=np.float64), requires_grad=True)
    F0t = torch.tensor(np.asarray(F0, dtype=np.float64), requires_grad=True)
    G, F = unrolled(Xt, omega_L, omega_R, G0t, F0t, q, T, K)
    Lv = torch.sum((G - torch.as_tensor(Gt, dtype=F64)) ** 2) + \
        torch.sum((F - torch.as_tensor(Ft, dtype=F64)) ** 2)
    Lv.backward()
    return Lv.item(), Xt.grad.numpy(), G0t.grad.numpy(), F0t.grad.numpy()


def loss(X, omega_L, omega_R, G0, F0, Gt, Ft, q: int, T: int, K: int) -> float:
    with torch.no_grad():
        G, F = unrolled(torch.as_tensor(np.asarray(X, dtype=np.float64)), omega_L, omega_R,
                        torch.as_tensor(np.asarray(G0, dtype=np.float64)),
                        torch.as_tensor(np.asarray(F0, dtype=np.float64)), q, T, K)
        return float(torch.sum((G - torch.as_tensor(Gt, dtype=F64)) ** 2) +
                     torch.sum((F - torch.as_tensor(Ft, dtype=F64)) ** 2))
