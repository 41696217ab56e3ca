"""Python binding of the GPU library (``include/ludax.h``).

Argument marshalling only: shapes, dtypes, devices and contiguity are
checked here, raw device pointers and the current HIP stream are handed to
the C ABI, and every step of the computation runs in the library's HIP
kernels.  PyTorch provides device memory and streams.  If the library has
not been built this module raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

TICTACTOE, CONNECT_FOUR, HEX, REVERSI, GOMOKU, YAVALATH, PENTE, WOLF_SHEEP, DRAUGHTS, HASAMI_SHOGI = 1, 2, 3, 4, 5, 6, 7, 8, 9, 10
RUNNING, TERMINAL, TRUNCATED, ILLEGAL = 0, 1, 2, 3
OK, E_INVALID, E_UNSUPPORTED, E_DEVICE = 0, -1, -2, -3

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libludax.so")

# every symbol the public header declares
EXPORTS = ("ludax_game_create", "ludax_game_destroy", "ludax_game_info", "ludax_init",
           "ludax_legal_mask", "ludax_step", "ludax_random_step", "ludax_policy_step", "ludax_playout",
           "ludax_playout_batches",
           "ludax_state_stats", "ludax_aux_sync", "ludax_mixed_create", "ludax_mixed_destroy",
           "ludax_mixed_set_slots",
           "ludax_mixed_get_slots", "ludax_mixed_set_one_grid", "ludax_mixed_get_one_grid",
           "ludax_mixed_playout", "ludax_mixed_playout_noalloc",
           "ludax_mixed_autotune", "ludax_net_create", "ludax_net_destroy", "ludax_net_info", "ludax_net_workspace_bytes",
           "ludax_net_max_batch",
           "ludax_net_pack", "ludax_net_forward", "ludax_net_loss_grad", "ludax_net_adam",
           "ludax_net_estimate", "ludax_net_guided_step", "ludax_net_guided_playout", "ludax_strerror",
           "ludax_last_device_error")

_lock = threading.Lock()
_lib = None


class LudaxError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = f"{where}: {_load().ludax_strerror(code).decode()} ({code})"
        if code == E_DEVICE:
            msg += ": " + _load().ludax_last_device_error().decode()
        super().__init__(msg)
        self.code = code


class _Desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("max_plies", ctypes.c_int32)]


class _State(ctypes.Structure):
    _fields_ = [("board", ctypes.c_void_p), ("to_move", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("winner", ctypes.c_void_p),
                ("passes", ctypes.c_void_p), ("ply", ctypes.c_void_p),
                ("last_action", ctypes.c_void_p), ("aux", ctypes.c_void_p)]


class _Batch(ctypes.Structure):
    _fields_ = [("game", ctypes.c_void_p), ("state", ctypes.POINTER(_State)), ("n", ctypes.c_int64),
                ("game_id_base", ctypes.c_int64), ("reward", ctypes.c_void_p), ("terminal", ctypes.c_void_p),
                ("stats", ctypes.c_void_p)]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build the HIP library first "
                    "(python -c 'import __graft_entry__; __graft_entry__.build()')")
            L = ctypes.CDLL(LIB_PATH)
            vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
            P = ctypes.POINTER
            L.ludax_game_create.argtypes = [P(_Desc), P(vp)]
            L.ludax_game_destroy.argtypes = [vp]
            L.ludax_game_info.argtypes = [vp, P(i32), P(i32), P(i32), P(i32)]
            L.ludax_init.argtypes = [vp, P(_State), i64, vp]
            L.ludax_legal_mask.argtypes = [vp, P(_State), vp, i64, vp]
            L.ludax_step.argtypes = [vp, P(_State), vp, vp, vp, vp, i64, vp]
            L.ludax_random_step.argtypes = [vp, P(_State), ctypes.c_uint64, i64, vp, vp, vp, i64, vp]
            L.ludax_policy_step.argtypes = [vp, P(_State), vp, ctypes.c_uint64, i64, vp, vp, vp, i64, vp]
            L.ludax_playout.argtypes = [vp, P(_State), ctypes.c_uint64, i64, vp, vp, vp, vp, i64,
                                        vp]
            L.ludax_playout_batches.argtypes = [P(_Batch), i32, ctypes.c_uint64, i32, vp]
            L.ludax_state_stats.argtypes = [vp, P(_State), ctypes.c_int32, vp, i64, vp]
            L.ludax_aux_sync.argtypes = [vp, P(_State), i64, vp]
            L.ludax_mixed_create.argtypes = [vp, i32, P(vp)]
            L.ludax_mixed_destroy.argtypes = [vp]
            L.ludax_mixed_set_slots.argtypes = [vp, vp]
            L.ludax_mixed_get_slots.argtypes = [vp, vp]
            L.ludax_mixed_set_one_grid.argtypes = [vp, i32]
            L.ludax_mixed_get_one_grid.argtypes = [vp, P(i32)]
            L.ludax_mixed_playout.argtypes = [vp, ctypes.c_uint64, i64, i64, vp, vp, vp, vp, vp, vp]
            L.ludax_mixed_playout_noalloc.argtypes = [vp, ctypes.c_uint64, i64, i64, vp, vp, vp, vp, vp]
            L.ludax_mixed_autotune.argtypes = [vp, ctypes.c_uint64, i64, i64, i32, vp, vp, vp, vp, vp,
                                               P(ctypes.c_float)]
            f32 = ctypes.c_float
            L.ludax_net_create.argtypes = [i32, i32, P(vp)]
            L.ludax_net_destroy.argtypes = [vp]
            L.ludax_net_info.argtypes = [vp, P(i64), P(i64)]
            L.ludax_net_workspace_bytes.argtypes = [vp, i64, i32, P(i64)]
            L.ludax_net_max_batch.argtypes = [vp, i64, i32, P(i64)]
            L.ludax_net_pack.argtypes = [vp, vp, vp, vp]
            L.ludax_net_forward.argtypes = [vp, vp, vp, vp, vp, i64, vp, vp, vp, vp]
            L.ludax_net_loss_grad.argtypes = [vp, vp, vp, vp, vp, vp, vp, i64, f32, vp, vp, vp, vp]
            L.ludax_net_adam.argtypes = [vp, vp, vp, vp, vp, i32, f32, f32, f32, f32, vp, vp]
            L.ludax_net_estimate.argtypes = [vp, vp, vp, P(_State), i64, vp, vp, vp]
            L.ludax_net_guided_step.argtypes = [vp, vp, vp, vp, P(_State), ctypes.c_uint64, i64, vp, vp, vp, i64,
                                                vp, vp]
            L.ludax_net_guided_playout.argtypes = [vp, vp, vp, vp, P(_State), i32, ctypes.c_uint64, i64, vp, vp,
                                                   i64, vp]
            L.ludax_strerror.argtypes = [ctypes.c_int]
            L.ludax_strerror.restype = ctypes.c_char_p
            L.ludax_last_device_error.argtypes = []
            L.ludax_last_device_error.restype = ctypes.c_char_p
            for name in ("ludax_game_create", "ludax_game_destroy", "ludax_game_info",
                         "ludax_init", "ludax_legal_mask", "ludax_step", "ludax_random_step",
                         "ludax_policy_step", "ludax_playout", "ludax_playout_batches",
                         "ludax_state_stats", "ludax_aux_sync", "ludax_mixed_create", "ludax_mixed_destroy",
                         "ludax_mixed_set_slots", "ludax_mixed_get_slots", "ludax_mixed_set_one_grid",
                         "ludax_mixed_get_one_grid", "ludax_mixed_playout",
                         "ludax_mixed_playout_noalloc", "ludax_mixed_autotune", "ludax_net_create",
                         "ludax_net_destroy", "ludax_net_info", "ludax_net_workspace_bytes", "ludax_net_max_batch",
                         "ludax_net_pack",
                         "ludax_net_forward", "ludax_net_loss_grad", "ludax_net_adam",
                         "ludax_net_estimate", "ludax_net_guided_step", "ludax_net_guided_playout"):
                getattr(L, name).restype = ctypes.c_int
            _lib = L
    return _lib


def lib():
    """The loaded ctypes library (raises if it was not built)."""
    return _load()


def _check(code: int, where: str):
    if code != OK:
        raise LudaxError(code, where)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, dtype, shape, name: str):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Game:
    """An immutable game handle (kind, board size, ply bound)."""

    def __init__(self, kind: int, rows: int, cols: int, max_plies: int = 0):
        L = _load()
        h = ctypes.c_void_p()
        _check(L.ludax_game_create(ctypes.byref(_Desc(kind, rows, cols, max_plies)),
                                   ctypes.byref(h)), "ludax_game_create")
        self._h = h
        self.kind, self.rows, self.cols = kind, rows, cols
        c, a, x, m = (ctypes.c_int32() for _ in range(4))
        _check(L.ludax_game_info(h, ctypes.byref(c), ctypes.byref(a), ctypes.byref(x),
                                 ctypes.byref(m)), "ludax_game_info")
        self.cells, self.num_actions, self.aux_bytes, self.max_plies = c.value, a.value, x.value, m.value

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.ludax_game_destroy(h)
            self._h = None


class State:
    """Device structure-of-arrays state of n environments.  aux=True also
    allocates the game's per-env cache (Hex; see ludax_state.aux), which
    every call on this state then passes."""

    FIELDS = ("board", "to_move", "status", "winner", "passes", "ply", "last_action")

    def __init__(self, game: Game, n: int, device="cuda", aux: bool = False):
        self.n, self.cells = n, game.cells
        self.aux = None
        if aux and game.aux_bytes > 0:
            self.aux = torch.empty((n, game.aux_bytes), dtype=torch.uint8, device=device)
        self.board = torch.empty((n, game.cells), dtype=torch.int8, device=device)
        self.to_move = torch.empty(n, dtype=torch.int8, device=device)
        self.status = torch.empty(n, dtype=torch.int8, device=device)
        self.winner = torch.empty(n, dtype=torch.int8, device=device)
        self.passes = torch.empty(n, dtype=torch.int8, device=device)
        self.ply = torch.empty(n, dtype=torch.int16, device=device)
        self.last_action = torch.empty(n, dtype=torch.int16, device=device)

    def _c(self) -> _State:
        # the checked C view is kept while the same field tensors, at the
        # same addresses, are in place (every call passes it)
        ts = [getattr(self, f) for f in self.FIELDS]
        aux = self.__dict__.get("aux")
        key = tuple(t.data_ptr() for t in ts) + (0 if aux is None else aux.data_ptr(),)
        hit = self.__dict__.get("_cview")
        if hit is not None and hit[0] == key and all(a is b for a, b in zip(hit[1], ts)) and hit[3] is aux:
            return hit[2]
        for f, t in zip(self.FIELDS, ts):
            if not t.is_contiguous() or t.device.type != "cuda":
                raise ValueError(f"state.{f} must be a contiguous device tensor")
        if key[0] % 16:
            raise ValueError("state.board must be 16-byte aligned")
        if aux is not None:
            if aux.dtype != torch.uint8 or not aux.is_contiguous() or aux.device.type != "cuda" or key[-1] % 128:
                raise ValueError("state.aux must be a contiguous, 128-byte aligned uint8 device tensor")
        view = _State(*[ctypes.c_void_p(p) for p in key[:-1]], None if aux is None else ctypes.c_void_p(key[-1]))
        self._cview = (key, ts, view, aux)
        return view

    @classmethod
    def from_tensors(cls, game: Game, aux=None, **fields) -> "State":
        s = cls.__new__(cls)
        s.cells = game.cells
        s.aux = aux
        if aux is not None:
            _need(aux, torch.uint8, (fields["board"].shape[0], game.aux_bytes), "aux")
        s.n = fields["board"].shape[0]
        dt = {"board": torch.int8, "to_move": torch.int8, "status": torch.int8,
              "winner": torch.int8, "passes": torch.int8, "ply": torch.int16,
              "last_action": torch.int16}
        for f in cls.FIELDS:
            t = fields[f]
            shape = (s.n, game.cells) if f == "board" else (s.n,)
            _need(t, dt[f], shape, f)
            setattr(s, f, t)
        return s

    def clone(self) -> "State":
        s = State.__new__(State)
        s.n, s.cells = self.n, self.cells
        s.aux = None if self.aux is None else self.aux.clone()
        for f in self.FIELDS:
            setattr(s, f, getattr(self, f).clone())
        return s

    def cpu(self) -> dict:
        return {f: getattr(self, f).cpu().numpy() for f in self.FIELDS}


def init(game: Game, state: State, stream=None):
    _check(_load().ludax_init(game.handle, ctypes.byref(state._c()), state.n, _stream(stream)),
           "ludax_init")


def aux_sync(game: Game, state: State, stream=None):
    """Rebuild state.aux from the boards (see ludax_aux_sync)."""
    _check(_load().ludax_aux_sync(game.handle, ctypes.byref(state._c()), state.n, _stream(stream)),
           "ludax_aux_sync")


def legal_mask(game: Game, state: State, out: torch.Tensor | None = None, stream=None):
    if out is None:
        out = torch.empty((state.n, game.num_actions), dtype=torch.uint8, device=state.board.device)
    _need(out, torch.uint8, (state.n, game.num_actions), "mask")
    _check(_load().ludax_legal_mask(game.handle, ctypes.byref(state._c()), _ptr(out), state.n,
                                    _stream(stream)), "ludax_legal_mask")
    return out


def step(game: Game, state: State, action: torch.Tensor, want_mask: bool = True, reward=None,
         terminal=None, next_mask=None, stream=None):
    dev = state.board.device
    _need(action, torch.int32, (state.n,), "action")
    if reward is None:
        reward = torch.empty((state.n, 2), dtype=torch.int8, device=dev)
    if terminal is None:
        terminal = torch.empty(state.n, dtype=torch.uint8, device=dev)
    if want_mask and next_mask is None:
        next_mask = torch.empty((state.n, game.num_actions), dtype=torch.uint8, device=dev)
    _need(reward, torch.int8, (state.n, 2), "reward")
    _need(terminal, torch.uint8, (state.n,), "terminal")
    if next_mask is not None:
        _need(next_mask, torch.uint8, (state.n, game.num_actions), "next_mask")
    _check(_load().ludax_step(game.handle, ctypes.byref(state._c()), _ptr(action), _ptr(reward),
                              _ptr(terminal), _ptr(next_mask), state.n, _stream(stream)),
           "ludax_step")
    return reward, terminal, next_mask


def random_step(game: Game, state: State, seed: int, game_id_base: int = 0, game_id=None,
                reward=None, terminal=None, stream=None):
    """One uniform-random ply for every env (see ludax_random_step)."""
    dev = state.board.device
    if reward is None:
        reward = torch.empty((state.n, 2), dtype=torch.int8, device=dev)
    if terminal is None:
        terminal = torch.empty(state.n, dtype=torch.uint8, device=dev)
    _need(reward, torch.int8, (state.n, 2), "reward")
    _need(terminal, torch.uint8, (state.n,), "terminal")
    if game_id is not None:
        _need(game_id, torch.int64, (state.n,), "game_id")
    _check(_load().ludax_random_step(game.handle, ctypes.byref(state._c()),
                                     ctypes.c_uint64(seed & (2**64 - 1)), game_id_base, _ptr(game_id),
                                     _ptr(reward), _ptr(terminal), state.n, _stream(stream)),
           "ludax_random_step")
    return reward, terminal


def policy_step(game: Game, state: State, logits: torch.Tensor, seed: int, game_id_base: int = 0,
                game_id=None, reward=None, terminal=None, stream=None):
    """One ply drawn from softmax(logits) over the legal actions (see
    ludax_policy_step)."""
    dev = state.board.device
    _need(logits, torch.float32, (state.n, game.num_actions), "logits")
    if reward is None:
        reward = torch.empty((state.n, 2), dtype=torch.int8, device=dev)
    if terminal is None:
        terminal = torch.empty(state.n, dtype=torch.uint8, device=dev)
    _need(reward, torch.int8, (state.n, 2), "reward")
    _need(terminal, torch.uint8, (state.n,), "terminal")
    if game_id is not None:
        _need(game_id, torch.int64, (state.n,), "game_id")
    _check(_load().ludax_policy_step(game.handle, ctypes.byref(state._c()), _ptr(logits),
                                     ctypes.c_uint64(seed & (2**64 - 1)), game_id_base, _ptr(game_id),
                                     _ptr(reward), _ptr(terminal), state.n, _stream(stream)),
           "ludax_policy_step")
    return reward, terminal


def playout(game: Game, state: State, seed: int, game_id_base: int = 0, game_id=None, reward=None,
            terminal=None, stats=True, stream=None):
    """stats: True (a fresh zeroed int64[4] is returned), a caller tensor
    (added to), or None (no counters)."""
    dev = state.board.device
    if reward is None:
        reward = torch.empty((state.n, 2), dtype=torch.int8, device=dev)
    if terminal is None:
        terminal = torch.empty(state.n, dtype=torch.uint8, device=dev)
    if stats is True:
        stats = torch.zeros(4, dtype=torch.int64, device=dev)
    _need(reward, torch.int8, (state.n, 2), "reward")
    _need(terminal, torch.uint8, (state.n,), "terminal")
    if stats is not None:
        _need(stats, torch.int64, (4,), "stats")
    if game_id is not None:
        _need(game_id, torch.int64, (state.n,), "game_id")
    _check(_load().ludax_playout(game.handle, ctypes.byref(state._c()),
                                 ctypes.c_uint64(seed & (2**64 - 1)), game_id_base, _ptr(game_id),
                                 _ptr(reward), _ptr(terminal), _ptr(stats), state.n,
                                 _stream(stream)), "ludax_playout")
    return reward, terminal, stats


def playout_batches(batches, seed: int, from_start: bool = True, stream=None):
    """ludax_playout_batches: batches = [(game, state, game_id_base, reward,
    terminal, stats), ...] (reward / terminal / stats as in playout: None
    allocates reward and terminal; stats None = no counters).  Returns the
    (reward, terminal, stats) of every batch."""
    arr = (_Batch * len(batches))()
    keep, out = [], []
    for k, (game, state, base, reward, terminal, stats) in enumerate(batches):
        dev = state.board.device
        if reward is None:
            reward = torch.empty((state.n, 2), dtype=torch.int8, device=dev)
        if terminal is None:
            terminal = torch.empty(state.n, dtype=torch.uint8, device=dev)
        _need(reward, torch.int8, (state.n, 2), "reward")
        _need(terminal, torch.uint8, (state.n,), "terminal")
        if stats is not None:
            _need(stats, torch.int64, (4,), "stats")
        c = state._c()
        keep.append(c)
        arr[k] = _Batch(game.handle, ctypes.pointer(c), state.n, base, reward.data_ptr(), terminal.data_ptr(),
                        None if stats is None else stats.data_ptr())
        out.append((reward, terminal, stats))
    _check(_load().ludax_playout_batches(arr, len(batches), ctypes.c_uint64(seed & (2**64 - 1)),
                                         1 if from_start else 0, _stream(stream)), "ludax_playout_batches")
    return out


class BatchGroup:
    """A fixed list of batches for repeated ludax_playout_batches calls:
    the arguments are checked and marshalled once, and each call only sets
    the game-id bases (the tensors must stay in place between calls).
    batches = [(game, state, reward, terminal, stats), ...] with reward,
    terminal and stats as in playout_batches."""

    def __init__(self, batches):
        self._items = []
        self._arr = (_Batch * len(batches))()
        self._keep = []
        for k, (game, state, reward, terminal, stats) in enumerate(batches):
            dev = state.board.device
            if reward is None:
                reward = torch.empty((state.n, 2), dtype=torch.int8, device=dev)
            if terminal is None:
                terminal = torch.empty(state.n, dtype=torch.uint8, device=dev)
            _need(reward, torch.int8, (state.n, 2), "reward")
            _need(terminal, torch.uint8, (state.n,), "terminal")
            if stats is not None:
                _need(stats, torch.int64, (4,), "stats")
            c = state._c()
            self._keep.append((game, state, c))
            self._arr[k] = _Batch(game.handle, ctypes.pointer(c), state.n, 0, reward.data_ptr(),
                                  terminal.data_ptr(), None if stats is None else stats.data_ptr())
            self._items.append((reward, terminal, stats))
        self._n = len(batches)
        self._fn = _load().ludax_playout_batches

    @property
    def outputs(self):
        return self._items

    def run(self, seed: int, game_id_bases, from_start: bool = True, stream=None, stats=None):
        """stats: None keeps the counters given at construction, else one
        int64[4] tensor (or None) per batch for this call."""
        arr = self._arr
        for k, base in enumerate(game_id_bases):
            arr[k].game_id_base = base
        if stats is not None:
            for k, t in enumerate(stats):
                if t is not None:
                    _need(t, torch.int64, (4,), "stats")
                arr[k].stats = None if t is None else t.data_ptr()
        _check(self._fn(arr, self._n, ctypes.c_uint64(seed & (2**64 - 1)), 1 if from_start else 0,
                        _stream(stream)), "ludax_playout_batches")


def state_stats(game: Game, state: State, sign: int, stats: torch.Tensor, stream=None):
    """stats += sign * (sum of ply, TERMINAL wins of player 1, of player 2,
    draws) over the batch (see ludax_state_stats)."""
    _need(stats, torch.int64, (4,), "stats")
    _check(_load().ludax_state_stats(game.handle, ctypes.byref(state._c()), sign, _ptr(stats),
                                     state.n, _stream(stream)), "ludax_state_stats")
    return stats


class MixedResult:
    """Per-game outputs of a mixed batch (device tensors)."""

    def __init__(self, n_games: int, n_kinds: int, device="cuda"):
        self.winner = torch.empty(n_games, dtype=torch.int8, device=device)
        self.plies = torch.empty(n_games, dtype=torch.int16, device=device)
        self.last_action = torch.empty(n_games, dtype=torch.int16, device=device)
        self.workspace = torch.zeros(n_kinds, dtype=torch.int32, device=device)

    def _ptrs(self):
        return _ptr(self.winner), _ptr(self.plies), _ptr(self.last_action), _ptr(self.workspace)


class Mixed:
    """A mixed persistent batch over several game handles: game id g has
    kind games[g % len(games)] (see ludax_mixed_playout)."""

    def __init__(self, games):
        self.games = list(games)  # the handles must outlive this object
        n = len(self.games)
        arr = (ctypes.c_void_p * n)(*[g.handle.value for g in self.games])
        h = ctypes.c_void_p()
        _check(_load().ludax_mixed_create(arr, n, ctypes.byref(h)), "ludax_mixed_create")
        self._h = h
        self.n_kinds = n

    @property
    def slots(self):
        out = (ctypes.c_int32 * self.n_kinds)()
        _check(_load().ludax_mixed_get_slots(self._h, out), "ludax_mixed_get_slots")
        return list(out)

    @property
    def one_grid(self) -> bool:
        v = ctypes.c_int32()
        _check(_load().ludax_mixed_get_one_grid(self._h, ctypes.byref(v)), "ludax_mixed_get_one_grid")
        return bool(v.value)

    @one_grid.setter
    def one_grid(self, value: bool):
        _check(_load().ludax_mixed_set_one_grid(self._h, 1 if value else 0), "ludax_mixed_set_one_grid")

    @slots.setter
    def slots(self, values):
        arr = (ctypes.c_int32 * self.n_kinds)(*values)
        _check(_load().ludax_mixed_set_slots(self._h, arr), "ludax_mixed_set_slots")

    def _check_out(self, n_games, out):
        if out is None:
            out = MixedResult(n_games, self.n_kinds)
        _need(out.winner, torch.int8, (n_games,), "winner")
        _need(out.plies, torch.int16, (n_games,), "plies")
        _need(out.last_action, torch.int16, (n_games,), "last_action")
        _need(out.workspace, torch.int32, (self.n_kinds,), "workspace")
        return out

    def playout(self, seed: int, id_base: int, n_games: int, out: MixedResult | None = None,
                stats=True, stream=None):
        out = self._check_out(n_games, out)
        if stats is True:
            stats = torch.zeros((self.n_kinds, 4), dtype=torch.int64, device=out.winner.device)
        if stats is not None:
            _need(stats, torch.int64, (self.n_kinds, 4), "stats")
        w, p, l, ws = out._ptrs()
        _check(_load().ludax_mixed_playout(self._h, ctypes.c_uint64(seed & (2**64 - 1)), id_base, n_games,
                                           w, p, l, _ptr(stats), ws, _stream(stream)),
               "ludax_mixed_playout")
        return out, stats

    def playout_noalloc(self, seed: int, id_base: int, n_games: int, out: MixedResult | None = None,
                        stats=True, stream=None):
        """ludax_mixed_playout_noalloc: as playout, with the queue counters in
        the library's static device words instead of out.workspace."""
        out = self._check_out(n_games, out)
        if stats is True:
            stats = torch.zeros((self.n_kinds, 4), dtype=torch.int64, device=out.winner.device)
        if stats is not None:
            _need(stats, torch.int64, (self.n_kinds, 4), "stats")
        w, p, l, _ = out._ptrs()
        _check(_load().ludax_mixed_playout_noalloc(self._h, ctypes.c_uint64(seed & (2**64 - 1)), id_base,
                                                   n_games, w, p, l, _ptr(stats), _stream(stream)),
               "ludax_mixed_playout_noalloc")
        return out, stats

    def autotune(self, seed: int, id_base: int, n_games: int, total_slots: int,
                 out: MixedResult | None = None, stream=None) -> float:
        out = self._check_out(n_games, out)
        best = ctypes.c_float()
        w, p, l, ws = out._ptrs()
        _check(_load().ludax_mixed_autotune(self._h, ctypes.c_uint64(seed & (2**64 - 1)), id_base,
                                            n_games, total_slots, w, p, l, ws, _stream(stream),
                                            ctypes.byref(best)), "ludax_mixed_autotune")
        return best.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.ludax_mixed_destroy(h)
            self._h = None


class Net:
    """The policy/value network of an N x N board (N = 11 or 19); see
    ludax_net_* in include/ludax.h.  Holds the parameters (float32), the
    packed bfloat16 copy and the Adam moments as device tensors."""

    def __init__(self, rows: int, cols: int, params=None, device="cuda"):
        L = _load()
        h = ctypes.c_void_p()
        _check(L.ludax_net_create(rows, cols, ctypes.byref(h)), "ludax_net_create")
        self._h = h
        self.rows, self.cols = rows, cols
        npar, pb = ctypes.c_int64(), ctypes.c_int64()
        _check(L.ludax_net_info(h, ctypes.byref(npar), ctypes.byref(pb)), "ludax_net_info")
        self.n_params, self.packed_bytes = npar.value, pb.value
        self.params = torch.zeros(self.n_params, dtype=torch.float32, device=device)
        self.packed = torch.zeros(self.packed_bytes, dtype=torch.uint8, device=device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._ws = {}
        if params is not None:
            self.load(params)

    def load(self, params):
        p = torch.as_tensor(params, dtype=torch.float32).reshape(-1)
        if p.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {p.numel()}")
        self.params.copy_(p)
        self.pack()

    def pack(self, stream=None):
        _check(_load().ludax_net_pack(self._h, _ptr(self.params), _ptr(self.packed), _stream(stream)),
               "ludax_net_pack")

    def workspace_bytes(self, n: int, training: bool = False) -> int:
        """ludax_net_workspace_bytes: the workspace a batch of n needs."""
        b = ctypes.c_int64()
        _check(_load().ludax_net_workspace_bytes(self._h, n, int(training), ctypes.byref(b)),
               "ludax_net_workspace_bytes")
        return b.value

    def workspace(self, n: int, training: bool = False):
        b = ctypes.c_int64()
        _check(_load().ludax_net_workspace_bytes(self._h, n, int(training), ctypes.byref(b)),
               "ludax_net_workspace_bytes")
        key = (training, self.params.device)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < b.value:
            ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=self.params.device)
            self._ws[key] = ws
        return ws

    def max_batch(self, budget_bytes: int, training: bool = False) -> int:
        """The largest batch whose workspace fits the HBM budget."""
        k = ctypes.c_int64()
        _check(_load().ludax_net_max_batch(self._h, budget_bytes, int(training), ctypes.byref(k)),
               "ludax_net_max_batch")
        return k.value

    def forward(self, board, to_move, logits=None, value=None, stream=None):
        n = board.shape[0]
        dev = board.device
        if logits is None:
            logits = torch.empty((n, self.rows * self.cols), dtype=torch.float32, device=dev)
        if value is None:
            value = torch.empty(n, dtype=torch.float32, device=dev)
        _need(board, torch.int8, (n, self.rows * self.cols), "board")
        _need(to_move, torch.int8, (n,), "to_move")
        _need(logits, torch.float32, (n, self.rows * self.cols), "logits")
        _need(value, torch.float32, (n,), "value")
        ws = self.workspace(n)
        _check(_load().ludax_net_forward(self._h, _ptr(self.params), _ptr(self.packed), _ptr(board),
                                         _ptr(to_move), n, _ptr(logits), _ptr(value), _ptr(ws),
                                         _stream(stream)), "ludax_net_forward")
        return logits, value

    def loss_grad(self, board, to_move, action, z, beta: float = 1.0, grads=None, loss=None, stream=None):
        n = board.shape[0]
        dev = board.device
        if grads is None:
            grads = torch.empty(self.n_params, dtype=torch.float32, device=dev)
        if loss is None:
            loss = torch.empty(2, dtype=torch.float32, device=dev)
        _need(board, torch.int8, (n, self.rows * self.cols), "board")
        _need(to_move, torch.int8, (n,), "to_move")
        _need(action, torch.int16, (n,), "action")
        _need(z, torch.float32, (n,), "z")
        _need(grads, torch.float32, (self.n_params,), "grads")
        _need(loss, torch.float32, (2,), "loss")
        ws = self.workspace(n, training=True)
        _check(_load().ludax_net_loss_grad(self._h, _ptr(self.params), _ptr(self.packed), _ptr(board),
                                           _ptr(to_move), _ptr(action), _ptr(z), n, ctypes.c_float(beta),
                                           _ptr(loss), _ptr(grads), _ptr(ws), _stream(stream)),
               "ludax_net_loss_grad")
        return loss, grads

    def adam(self, grads, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step += 1
        _need(grads, torch.float32, (self.n_params,), "grads")
        _check(_load().ludax_net_adam(self._h, _ptr(self.params), _ptr(grads), _ptr(self.m), _ptr(self.v),
                                      self.step, ctypes.c_float(lr), ctypes.c_float(beta1),
                                      ctypes.c_float(beta2), ctypes.c_float(eps), _ptr(self.packed),
                                      _stream(stream)), "ludax_net_adam")

    def estimate(self, state: "State", out=None, stream=None):
        n = state.n
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=state.board.device)
        _need(out, torch.float32, (n,), "estimate")
        ws = self.workspace(n)
        _check(_load().ludax_net_estimate(self._h, _ptr(self.params), _ptr(self.packed),
                                          ctypes.byref(state._c()), n, _ptr(out), _ptr(ws),
                                          _stream(stream)), "ludax_net_estimate")
        return out

    def guided_step(self, game: "Game", state: "State", seed: int, game_id_base: int = 0, game_id=None,
                    reward=None, terminal=None, stream=None):
        """One network-guided ply of every env (ludax_net_guided_step): the
        forward pass and the policy draw and step, the logits kept on chip."""
        n = state.n
        dev = state.board.device
        if reward is None:
            reward = torch.empty((n, 2), dtype=torch.int8, device=dev)
        if terminal is None:
            terminal = torch.empty(n, dtype=torch.uint8, device=dev)
        _need(reward, torch.int8, (n, 2), "reward")
        _need(terminal, torch.uint8, (n,), "terminal")
        if game_id is not None:
            _need(game_id, torch.int64, (n,), "game_id")
        ws = self.workspace(n)
        _check(_load().ludax_net_guided_step(self._h, _ptr(self.params), _ptr(self.packed), game.handle,
                                             ctypes.byref(state._c()), ctypes.c_uint64(seed & (2**64 - 1)),
                                             game_id_base, _ptr(game_id), _ptr(reward), _ptr(terminal), n,
                                             _ptr(ws), _stream(stream)), "ludax_net_guided_step")
        return reward, terminal

    def guided_playout(self, game: "Game", state: "State", plies: int, seed: int, game_id_base: int = 0,
                       game_id=None, out=None, stream=None):
        """`plies` network-guided plies of every env, then the value cutoff,
        in one kernel (ludax_net_guided_playout); returns estimate [n]."""
        n = state.n
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=state.board.device)
        _need(out, torch.float32, (n,), "estimate")
        if game_id is not None:
            _need(game_id, torch.int64, (n,), "game_id")
        _check(_load().ludax_net_guided_playout(self._h, _ptr(self.params), _ptr(self.packed), game.handle,
                                                ctypes.byref(state._c()), plies, ctypes.c_uint64(seed & (2**64 - 1)),
                                                game_id_base, _ptr(game_id), _ptr(out), n, _stream(stream)),
               "ludax_net_guided_playout")
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.ludax_net_destroy(h)
            self._h = None
