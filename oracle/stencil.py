"""In-place diffusion loop and its reverse pass, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Forward (a `State` loop, Sec. 2.3.1): `for t:(Fin T). u := step (get u)` with the
periodic five-point update

    step(u)[y, x] = u[y, x] + c * (u[y+1, x] + u[y-1, x] + u[y, x+1] + u[y, x-1]
                                   - 4 u[y, x]),       c = 0.2,

indices taken modulo the grid. `get` returns an immutable value (Sec. 5.3.2), so
every read in a step is of the previous field (a Jacobi update).
Loss: L = 1/2 * || u_T - target ||^2.

An optional pointwise non-linear term rho * sin(u[y, x]) may be added to each
step (rho = 0 gives the pure diffusion loop). It is the case in which the
reverse pass needs the primal states: the transpose of the linearized sin reads
cos(u_t) (Sec. 5.3.2: only non-linear operations keep their inputs).

Reverse: the transposed loop. ForTranspose runs the time loop backwards; the
cotangent of u_T is u_T - target; GetTranspose / PutTranspose carry the
cotangent of the state reference through each step, and the transpose of one
step turns each of its five reads into an accumulation into the cotangent of
the cell that was read (LetIndexingTranspose). The step is linear, so nothing
of the primal needs to be saved (only non-linear operations keep their inputs,
Sec. 5.3.2).
"""
from __future__ import annotations

import numpy as np

C = 0.2


def step(u: np.ndarray, c: float = C, rho: float = 0.0) -> np.ndarray:
    u = np.asarray(u, dtype=np.float64)
    nb = (np.roll(u, -1, 0) + np.roll(u, 1, 0) + np.roll(u, -1, 1) + np.roll(u, 1, 1))
    out = u + c * (nb - 4.0 * u)
    if rho != 0.0:
        out = out + rho * np.sin(u)
    return out


def step_transpose(ct_next: np.ndarray, c: float = C, u: np.ndarray | None = None,
                   rho: float = 0.0) -> np.ndarray:
    """Cotangent of u_t from the cotangent of u_{t+1}, written as accumulation:
    the forward cell (y, x) read u[y, x] with weight (1 - 4c) and its four
    neighbours with weight c, so it adds those weights times ct_next[y, x]
    into the corresponding cells of the result."""
    g = np.asarray(ct_next, dtype=np.float64)
    acc = np.zeros_like(g)
    acc += (1.0 - 4.0 * c) * g            # read of u[y, x]
    acc += c * np.roll(g, 1, 0)           # read of u[y+1, x] by cell (y, x): lands at y+1
    acc += c * np.roll(g, -1, 0)          # read of u[y-1, x]
    acc += c * np.roll(g, 1, 1)           # read of u[y, x+1]
    acc += c * np.roll(g, -1, 1)          # read of u[y, x-1]
    if rho != 0.0:                        # rho * sin(u[y, x]) linearizes to rho cos(u) du
        acc += rho * np.cos(np.asarray(u, dtype=np.float64)) * g
    return acc


def forward(u0: np.ndarray, steps: int, c: float = C, rho: float = 0.0,
            keep: bool = False):
    """u_T, or (u_T, [u_0 .. u_{T-1}]) when keep is set."""
    u = np.asarray(u0, dtype=np.float64)
    states = []
    for _ in range(steps):
        if keep:
            states.append(u)
        u = step(u, c, rho)
    return (u, states) if keep else u


def loss_and_grad(u0: np.ndarray, target: np.ndarray, steps: int, c: float = C,
                  rho: float = 0.0):
    """Returns (L, u_T, dL/du0). The forward keeps every state when rho != 0."""
    if rho != 0.0:
        uT, states = forward(u0, steps, c, rho, keep=True)
    else:
        uT, states = forward(u0, steps, c), None
    r = uT - np.asarray(target, dtype=np.float64)
    L = 0.5 * float(np.sum(r * r))
    lam = r
    for t in range(steps - 1, -1, -1):     # ForTranspose: t = T-1 ... 0
        lam = step_transpose(lam, c, states[t] if rho != 0.0 else None, rho)
    return L, uT, lam


def step_tangent(du: np.ndarray, u: np.ndarray, c: float = C, rho: float = 0.0) -> np.ndarray:
    """Tangent of `step` at u along du (the linearized step, Sec. 5.1): the
    diffusion part is linear, so it acts on du unchanged; rho sin(u)
    linearizes to rho cos(u) du, which reads the state u of the same step."""
    du = np.asarray(du, dtype=np.float64)
    nb = (np.roll(du, -1, 0) + np.roll(du, 1, 0) + np.roll(du, -1, 1) + np.roll(du, 1, 1))
    out = du + c * (nb - 4.0 * du)
    if rho != 0.0:
        out = out + rho * np.cos(np.asarray(u, dtype=np.float64)) * du
    return out


def loss_jvp(u0: np.ndarray, target: np.ndarray, du0: np.ndarray, dtarget: np.ndarray,
             steps: int, c: float = C, rho: float = 0.0) -> float:
    """Forward mode of L = 1/2 ||u_T - target||^2 along (du0, dtarget): every
    state is stepped together with its tangent, then
    dL = <u_T - target, du_T - dtarget>."""
    u = np.asarray(u0, dtype=np.float64)
    du = np.asarray(du0, dtype=np.float64)
    for _ in range(steps):
        u, du = step(u, c, rho), step_tangent(du, u, c, rho)
    r = u - np.asarray(target, dtype=np.float64)
    return float(np.sum(r * (du - np.asarray(dtarget, dtype=np.float64))))
