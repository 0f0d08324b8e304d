"""FP64 reference belief propagation on a 4-connected H x W grid MRF.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

Model (Sec. 1, Eq. 1): P(x) is proportional to the product of a pairwise
potential over neighbouring pixel pairs and a unary g_p(x_p) per pixel.
Horizontal pairs are oriented left-to-right and vertical pairs top-to-bottom:
the pair (a, b) contributes F[x_a, x_b].  For the truncated-linear potential
of Sec. 1 and Sec. 6, F is symmetric and the orientation is immaterial; it is
kept so that an asymmetric sparse-compatible F (Sec. 4 allows any
neighbourhood structure) is handled correctly.

Message state
-------------
``inbox[k, r, c, :]`` is the message m_{q->p} into pixel p = (r, c) from its
neighbour q = p + OFFSETS[k]; the four directions are LEFT, RIGHT, UP, DOWN
(where the *sender* sits relative to the receiver).  Slots whose neighbour is
off the grid are never read (a missing neighbour contributes a factor 1);
they hold 1/M.

Message forms (all exact, they must agree up to rounding):
  dense  : Eq. 2 (sum) and Eq. 9 (max), O(M^2)
  split  : Eq. 6 (sum) and Eq. 10 (max)
  sparse : Eq. 7 (sum) and Eq. 11 (max), O(mM) -- the paper's trick

Schedules: synchronous (every message from the previous state), the
checkerboard of [2] (Sec. 2), and the directional sweeps of Sec. 6 (one
sweep = passes in the left, right, up and down directions).

Max-product is taken in the product domain: u(y) = max_x F(x, y) h(x), the
exponential of the log-domain max-sum of Eq. 9-11 with f and fbar read as
potentials.  Every message is normalised to sum 1 right after it is computed
(Sec. 3, below Eq. 2), in both modes.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LEFT, RIGHT, UP, DOWN = 0, 1, 2, 3
# Offset of the sender q relative to the receiver p, per inbox direction.
OFFSETS = {LEFT: (0, -1), RIGHT: (0, 1), UP: (-1, 0), DOWN: (1, 0)}
# A message p -> q with q = p + OFFSETS[o] lands in q's inbox OPPOSITE[o].
OPPOSITE = {LEFT: RIGHT, RIGHT: LEFT, UP: DOWN, DOWN: UP}
DIRS = (LEFT, RIGHT, UP, DOWN)

SUM, MAX = "sum", "max"
SYNC, CHECKERBOARD, SWEEP = "sync", "checkerboard", "sweep"
DENSE, SPLIT, SPARSE = "dense", "split", "sparse"


@dataclass
class Potential:
    """A sparse-compatible pairwise potential (Sec. 4).

    F[x_a, x_b] is the potential of the oriented pair (a, b); compat[x_a, x_b]
    is True when x_a is in Nbd(x_b), i.e. the pair is "compatible".  Outside
    compat, F equals the constant fbar (the sparse compatibility property).
    """

    F: np.ndarray
    compat: np.ndarray
    fbar: float

    def __post_init__(self):
        self.F = np.asarray(self.F, dtype=np.float64)
        self.compat = np.asarray(self.compat, dtype=bool)
        M = self.F.shape[0]
        assert self.F.shape == (M, M) and self.compat.shape == (M, M)
        assert np.all(self.F >= 0.0)
        if not np.all(self.F[~self.compat] == self.fbar):
            raise ValueError("F must equal fbar on every incompatible pair")

    @property
    def M(self) -> int:
        return self.F.shape[0]

    def transposed(self) -> "Potential":
        """The same factor seen from the other end of the pair."""
        return Potential(self.F.T.copy(), self.compat.T.copy(), self.fbar)


@dataclass
class EdgePotentials:
    """A potential per edge (Sec. 4: f_ij with its own fbar_ij and its own
    neighbourhood structure; Sec. 7: not necessarily a function of x_i - x_j).

    types[k] is a Potential; th[r, c] is the type of the horizontal pair
    ((r, c), (r, c+1)) and tv[r, c] that of the vertical pair ((r, c),
    (r+1, c)); each pair is oriented left-to-right / top-to-bottom as above.
    """

    types: list
    th: np.ndarray   # [H, W-1]
    tv: np.ndarray   # [H-1, W]

    def __post_init__(self):
        self.th = np.asarray(self.th, dtype=np.int64)
        self.tv = np.asarray(self.tv, dtype=np.int64)
        assert len(self.types) > 0 and all(t.M == self.types[0].M for t in self.types)

    @property
    def M(self) -> int:
        return self.types[0].M


def edge_type_map(pot, H, W, o):
    """[H, W]: type of the edge from each pixel towards direction o (-1 where
    there is no neighbour)."""
    t = np.full((H, W), -1, dtype=np.int64)
    if o == RIGHT:
        t[:, :W - 1] = pot.th
    elif o == LEFT:
        t[:, 1:] = pot.th
    elif o == DOWN:
        t[:H - 1, :] = pot.tv
    else:
        t[1:, :] = pot.tv
    return t


def messages_towards(h, pot, o, form, tmap=None):
    """Normalised messages u for the h rows (any leading shape) sent towards
    direction o.  With per-edge potentials, tmap gives each row's edge type."""
    if not isinstance(pot, EdgePotentials):
        return normalize(form(h, oriented_potential(pot, o)))
    out = np.zeros_like(h)
    for k, pk in enumerate(pot.types):
        sel = tmap == k
        if np.any(sel):
            out[sel] = normalize(form(h[sel], oriented_potential(pk, o)))
    return out


def truncated_linear(M: int, T: int, alpha: float, fbar: float | None = None) -> Potential:
    """f(x_i, x_j) = exp(-alpha * |x_i - x_j|) for |x_i - x_j| <= T, fbar otherwise.

    With fbar = exp(-alpha*T) this is exp(-alpha * min(|d|, T)) (Sec. 1 and
    Sec. 6).  Nbd(x_j) = {x_i : |x_i - x_j| <= T} inside [0, M-1], so m = 2T+1
    away from the label range ends.  A free fbar keeps f's form inside the
    window (the fbar = 0 variant of Sec. 6 does exactly that).
    """
    if fbar is None:
        fbar = float(np.exp(-alpha * T))
    x = np.arange(M)
    d = np.abs(x[:, None] - x[None, :])
    compat = d <= T
    F = np.where(compat, np.exp(-alpha * d.astype(np.float64)), fbar)
    return Potential(F, compat, float(fbar))


# --------------------------------------------------------------------------
# Single-message updates: h has shape [..., M] (x_i last), result [..., M]
# (x_j last).  `pot` is oriented so that pot.F[x_i, x_j] is the factor
# between the sender's state x_i and the receiver's state x_j.
# --------------------------------------------------------------------------

def message_dense_sum(h, pot):
    """Eq. 2 / Eq. 4: u(x_j) = sum over all x_i of f(x_i, x_j) h(x_i)."""
    return h @ pot.F


def message_split_sum(h, pot):
    """Eq. 6: compatible states with f, every other state with fbar."""
    inside = np.where(pot.compat, pot.F, 0.0)
    outside = np.where(pot.compat, 0.0, pot.fbar)
    return h @ inside + h @ outside


def message_sparse_sum(h, pot):
    """Eq. 7: u(x_j) = sum_{x_i in Nbd(x_j)} (f - fbar) h(x_i) + fbar * sum_{x_i} h(x_i).

    The second term is one sum per message; the first visits only the
    compatible states of each x_j, which is the O(mM) part.
    """
    M = pot.M
    total = h.sum(axis=-1)                      # sum_{x_i} h(x_i), once per message
    u = np.empty(h.shape[:-1] + (M,), dtype=np.float64)
    for xj in range(M):
        nbd = np.nonzero(pot.compat[:, xj])[0]  # Nbd(x_j)
        u[..., xj] = h[..., nbd] @ (pot.F[nbd, xj] - pot.fbar) + pot.fbar * total
    return u


def message_dense_max(h, pot):
    """Eq. 9 in the product domain: u(x_j) = max over all x_i of f(x_i, x_j) h(x_i)."""
    out = np.empty(h.shape[:-1] + (pot.M,), dtype=np.float64)
    for xj in range(pot.M):
        out[..., xj] = np.max(h * pot.F[:, xj], axis=-1)
    return out


def message_split_max(h, pot):
    """Eq. 10: max of (max over Nbd of f h) and (max over the rest of fbar h).

    Exact for any fbar >= 0; an empty part contributes nothing.
    """
    out = np.empty(h.shape[:-1] + (pot.M,), dtype=np.float64)
    for xj in range(pot.M):
        nbd = pot.compat[:, xj]
        inside = np.max(h[..., nbd] * pot.F[nbd, xj], axis=-1)
        if np.all(nbd):
            out[..., xj] = inside
        else:
            out[..., xj] = np.maximum(inside, np.max(pot.fbar * h[..., ~nbd], axis=-1))
    return out


def message_sparse_max(h, pot):
    """Eq. 11: max of (max over Nbd of f h) and fbar * (max over all x_i of h).

    Equals Eq. 9 only when f >= fbar everywhere (Sec. 5); the second term is
    one max per message.
    """
    hmax = np.max(h, axis=-1)                   # once per message
    out = np.empty(h.shape[:-1] + (pot.M,), dtype=np.float64)
    for xj in range(pot.M):
        nbd = np.nonzero(pot.compat[:, xj])[0]
        out[..., xj] = np.maximum(np.max(h[..., nbd] * pot.F[nbd, xj], axis=-1),
                                  pot.fbar * hmax)
    return out


MESSAGE_FORMS = {
    (SUM, DENSE): message_dense_sum,
    (SUM, SPLIT): message_split_sum,
    (SUM, SPARSE): message_sparse_sum,
    (MAX, DENSE): message_dense_max,
    (MAX, SPLIT): message_split_max,
    (MAX, SPARSE): message_sparse_max,
}


def normalize(u):
    """Explicit normalisation after each update (Sec. 3): entries sum to 1."""
    return u / u.sum(axis=-1, keepdims=True)


def stored(msg, storage=None):
    """A message as it is kept in the state.

    storage=None keeps FP64.  storage=numpy.float32 models a state held in
    float32: each message is computed in FP64 from the stored (float32)
    values and rounded once to float32 when it is stored.  This is a model of
    a storage format, not of the method: it measures how far the format
    alone moves BP from the FP64 result.
    """
    return msg if storage is None else np.asarray(msg, dtype=storage).astype(np.float64)


# --------------------------------------------------------------------------
# Grid bookkeeping
# --------------------------------------------------------------------------

def _span(delta, n):
    """Slices (senders, receivers) along one axis for a neighbour offset delta."""
    return (slice(max(0, -delta), n - max(0, delta)),
            slice(max(0, delta), n - max(0, -delta)))


def has_neighbor(H, W):
    """has[k, r, c] is True when pixel (r, c) has a neighbour in direction k."""
    has = np.zeros((4, H, W), dtype=bool)
    for k in DIRS:
        dr, dc = OFFSETS[k]
        (rs, _), (cs, _) = _span(dr, H), _span(dc, W)
        has[k, rs, cs] = True
    return has


def init_messages(H, W, M):
    """Uniform messages 1/M on every directed edge (the usual BP start)."""
    return np.full((4, H, W, M), 1.0 / M, dtype=np.float64)


def oriented_potential(pot, o):
    """Potential seen by a message sent towards direction o.

    A message to the right or downwards goes from the first node of the
    oriented pair to the second (F[x_sender, x_receiver]); to the left or
    upwards it goes from the second to the first (F^T).
    """
    return pot if o in (RIGHT, DOWN) else pot.transposed()


def h_vector(g, inbox, has, o):
    """Eq. 5: h(x_i) = g(x_i) * product of messages into i except the one from the target.

    o is the direction of the target neighbour j from i.  Returns [H, W, M]
    (rows of pixels without that neighbour are computed but never used).
    """
    h = g.copy()
    for k in DIRS:
        if k == o:
            continue
        h = h * np.where(has[k][..., None], inbox[k], 1.0)
    return h


def compute_messages(g, inbox, pot, mode, impl, storage=None):
    """All new outgoing messages from the current state: out[o] is [H, W, M],
    the normalised message each pixel sends to its neighbour in direction o."""
    H, W, _ = g.shape
    has = has_neighbor(H, W)
    form = MESSAGE_FORMS[(mode, impl)]
    out = {}
    for o in DIRS:
        h = h_vector(g, inbox, has, o)
        tmap = edge_type_map(pot, H, W, o) if isinstance(pot, EdgePotentials) else None
        out[o] = stored(messages_towards(h, pot, o, form, tmap), storage)
    return out


def deliver(inbox, out, sender_mask=None):
    """Write each sent message into its receiver's inbox; returns a new state.

    sender_mask[r, c] (optional) selects which senders update.
    """
    _, H, W, _ = inbox.shape
    new = inbox.copy()
    for o in DIRS:
        dr, dc = OFFSETS[o]
        (rs, rq), (cs, cq) = _span(dr, H), _span(dc, W)
        k = OPPOSITE[o]
        if sender_mask is None:
            new[k, rq, cq] = out[o][rs, cs]
        else:
            sel = sender_mask[rs, cs]
            dst = new[k, rq, cq]
            dst[sel] = out[o][rs, cs][sel]
            new[k, rq, cq] = dst
    return new


def sync_step(g, inbox, pot, mode, impl=SPARSE, storage=None):
    """One synchronous (Jacobi) iteration: every message from the previous state."""
    return deliver(inbox, compute_messages(g, inbox, pot, mode, impl, storage))


def colour_mask(H, W, t):
    """Pixels of checkerboard colour t mod 2: (r + c) mod 2 == t mod 2."""
    r, c = np.mgrid[0:H, 0:W]
    return (r + c) % 2 == t % 2


def checkerboard_pass(g, inbox, pot, mode, t, impl=SPARSE, storage=None):
    """Pass t of the bipartite schedule (Sec. 2, [2]): only pixels of colour
    t mod 2 send, using the current state; their receivers are all of the
    other colour, so the pass reads and writes disjoint slots."""
    H, W, _ = g.shape
    return deliver(inbox, compute_messages(g, inbox, pot, mode, impl, storage), colour_mask(H, W, t))


# Directions of the four passes of one sweep (Sec. 6): messages travelling
# left, then right, then up, then down.
SWEEP_ORDER = (LEFT, RIGHT, UP, DOWN)


def sweep_pass(g, inbox, pot, mode, o, impl=SPARSE, storage=None):
    """One directional pass of the sweep schedule (Sec. 6): every message sent
    towards direction o, computed in scan order along o, in place.

    Scanlines (rows for left/right, columns for up/down) are independent;
    along a scanline the senders are visited from the far end towards o, so
    each message uses the one its sender has just received from the opposite
    side in the same pass.  Returns a new state.
    """
    g = np.asarray(g, dtype=np.float64)
    H, W, _ = g.shape
    has = has_neighbor(H, W)
    form = MESSAGE_FORMS[(mode, impl)]
    tmap = edge_type_map(pot, H, W, o) if isinstance(pot, EdgePotentials) else None
    k = OPPOSITE[o]
    dr, dc = OFFSETS[o]
    state = np.array(inbox, dtype=np.float64)
    if dc != 0:
        senders = range(0, W - 1) if dc > 0 else range(W - 1, 0, -1)
        line = lambda s: (slice(None), s)            # column s, every row
    else:
        senders = range(0, H - 1) if dr > 0 else range(H - 1, 0, -1)
        line = lambda s: (s, slice(None))            # row s, every column
    for s in senders:
        src = line(s)
        h = g[src].copy()
        for j in DIRS:
            if j != o:
                h = h * np.where(has[j][src][..., None], state[j][src], 1.0)
        msg = stored(messages_towards(h, pot, o, form, None if tmap is None else tmap[src]), storage)
        dst = line(s + (dc if dc != 0 else dr))
        state[k][dst] = msg
    return state


def sweep(g, inbox, pot, mode, impl=SPARSE, storage=None):
    """One sweep: the four directional passes in SWEEP_ORDER."""
    for o in SWEEP_ORDER:
        inbox = sweep_pass(g, inbox, pot, mode, o, impl, storage)
    return inbox


def run(g, pot, mode=SUM, n_iters=10, schedule=SYNC, impl=SPARSE, inbox=None,
        record=False, storage=None):
    """Run BP from uniform messages (or `inbox`); returns the final state
    (and the list of all states when record=True).  For the checkerboard
    schedule n_iters counts passes, for the sweep schedule whole sweeps.
    storage: see `stored` (the uniform start is rounded the same way)."""
    g = np.asarray(g, dtype=np.float64)
    H, W, M = g.shape
    assert pot.M == M
    state = stored(init_messages(H, W, M), storage) if inbox is None else np.array(inbox, dtype=np.float64)
    states = [state]
    for t in range(n_iters):
        if schedule == SYNC:
            state = sync_step(g, state, pot, mode, impl, storage)
        elif schedule == CHECKERBOARD:
            state = checkerboard_pass(g, state, pot, mode, t, impl, storage)
        elif schedule == SWEEP:
            state = sweep(g, state, pot, mode, impl, storage)
        else:
            raise ValueError(schedule)
        if record:
            states.append(state)
    return (state, states) if record else state


def beliefs(g, inbox):
    """Eq. 3: b_i(x) = g(x) * product of all incoming messages, normalised to sum 1."""
    g = np.asarray(g, dtype=np.float64)
    H, W, _ = g.shape
    has = has_neighbor(H, W)
    b = g.copy()
    for k in DIRS:
        b = b * np.where(has[k][..., None], inbox[k], 1.0)
    return b / b.sum(axis=-1, keepdims=True)


def map_labels(b):
    """Disparity estimate: argmax of the beliefs, lowest label on ties."""
    return np.argmax(b, axis=-1).astype(np.int32)


def top2_margin(b):
    """Difference between the largest and second-largest belief per pixel."""
    if b.shape[-1] < 2:
        return np.full(b.shape[:-1], np.inf)
    s = np.sort(b, axis=-1)
    return s[..., -1] - s[..., -2]


def message_sums(inbox, has=None):
    """Sum over labels of every live message (1 after normalisation)."""
    _, H, W, _ = inbox.shape
    has = has_neighbor(H, W) if has is None else has
    return inbox.sum(axis=-1)[has]


def single_update(g, inbox, pot, mode, r, c, o, impl=SPARSE):
    """One message p -> q (p = (r, c), q its neighbour in direction o) from a
    given state, computed pixel by pixel: used to check sampled outputs of a
    full-size run without running the whole grid."""
    g = np.asarray(g, dtype=np.float64)
    H, W, M = g.shape
    dr, dc = OFFSETS[o]
    assert 0 <= r + dr < H and 0 <= c + dc < W, "target off the grid"
    h = g[r, c].copy()
    for k in DIRS:
        if k == o:
            continue
        kr, kc = r + OFFSETS[k][0], c + OFFSETS[k][1]
        if 0 <= kr < H and 0 <= kc < W:
            h = h * inbox[k, r, c]
    if isinstance(pot, EdgePotentials):
        pot = pot.types[int(edge_type_map(pot, H, W, o)[r, c])]
    u = MESSAGE_FORMS[(mode, impl)](h, oriented_potential(pot, o))
    return normalize(u)


def single_belief(g, inbox, r, c):
    """Eq. 3 at one pixel."""
    g = np.asarray(g, dtype=np.float64)
    H, W, _ = g.shape
    b = g[r, c].copy()
    for k in DIRS:
        kr, kc = r + OFFSETS[k][0], c + OFFSETS[k][1]
        if 0 <= kr < H and 0 <= kc < W:
            b = b * inbox[k, r, c]
    return b / b.sum()
