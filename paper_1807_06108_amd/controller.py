"""Python front end of the library: one controller = one context + its
device workspace.  PyTorch supplies device memory and the stream; every
computation runs in the library's kernels (through paper_1807_06108_amd.native).
"""

import ctypes

import numpy as np
import torch

from . import native

_STATS_BYTES = ctypes.sizeof(native.Stats)


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Controller:
    """MPPI-on-jump-diffusion controller resident on one GPU.

    cfg: configuration dict (keys of mppi_jump_config; see workloads.py).
    U0: optional initial control sequence [T, m] (default u_init everywhere).
    """

    def __init__(self, cfg, U0=None, device="cuda", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the controller runs only on the HIP device")
        self.cfg = dict(cfg)
        self.device = torch.device(device)
        self.stream = stream
        self.n, self.m, self.q = native.dims(cfg["dynamics"])
        self.K, self.T = int(cfg["K"]), int(cfg["T"])
        self._c = native.make_config(cfg)
        self.ws_bytes = native.workspace_bytes(cfg)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        U0t = None
        if U0 is not None:
            U0t = torch.as_tensor(np.asarray(U0, dtype=np.float32).reshape(self.T, self.m),
                                  device=self.device).contiguous()
        ctx = ctypes.c_void_p()
        native.check(native.lib().mppi_jump_init(
            ctypes.byref(self._c), _ptr(self.ws), self.ws_bytes, _ptr(U0t),
            _stream_handle(self.stream), ctypes.byref(ctx)))
        self._keep = U0t
        self.ctx = ctx

    # ------------------------------------------------------------- lifecycle
    def close(self):
        if getattr(self, "ctx", None):
            native.lib().mppi_jump_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _s(self):
        """The controller's stream, ordered after the work already queued on
        torch's current stream (the inputs of the call)."""
        cur = torch.cuda.current_stream()
        if self.stream is not None and self.stream != cur:
            self.stream.wait_stream(cur)
        return _stream_handle(self.stream)

    def _publish(self):
        """Order torch's current stream after the controller's stream, so
        that results read on the current stream are complete."""
        cur = torch.cuda.current_stream()
        if self.stream is not None and self.stream != cur:
            cur.wait_stream(self.stream)

    def _state(self, x0):
        x = torch.as_tensor(x0, dtype=torch.float32, device=self.device).contiguous()
        if x.numel() != self.n:
            raise ValueError("state needs %d entries" % self.n)
        return x

    # ------------------------------------------------------------- the method
    def step(self, x0, iters=1):
        """Enqueue `iters` iterations from state x0 (tensor or array [n])."""
        x = self._state(x0)
        native.check(native.lib().mppi_jump_step(self.ctx, _ptr(x), int(iters), self._s()))
        return x

    def control_step(self, x0, iters=1, u0_out=None):
        """Enqueue one MPC control step: `iters` iterations then the shift;
        returns u_0 [m] (device tensor)."""
        x = self._state(x0)
        if u0_out is None:
            u0_out = torch.empty(self.m, dtype=torch.float32, device=self.device)
        native.check(native.lib().mppi_jump_control_step(self.ctx, _ptr(x), int(iters),
                                                         _ptr(u0_out), self._s()))
        self._publish()
        return u0_out

    def rollout(self, x0):
        x = self._state(x0)
        native.check(native.lib().mppi_jump_rollout(self.ctx, _ptr(x), self._s()))
        return x

    def update(self):
        native.check(native.lib().mppi_jump_update(self.ctx, self._s()))

    def shift(self, out=None):
        """Enqueue the receding-horizon shift; returns the executed u_0 [m]
        (a device tensor unless `out` is given)."""
        if out is None:
            out = torch.empty(self.m, dtype=torch.float32, device=self.device)
        native.check(native.lib().mppi_jump_shift(self.ctx, _ptr(out), self._s()))
        self._publish()
        return out

    def plant_step(self, x, u, d, force=None):
        """Simulated plant: x <- Euler(x, u + d) on device tensors, with the
        world-frame body force `force` ([3], quadrotor) if given."""
        native.check(native.lib().mppi_jump_plant_step_force(self.ctx, _ptr(x), _ptr(u), _ptr(d),
                                                             _ptr(force), self._s()))
        self._publish()

    # ------------------------------------------------------------- items
    def _get(self, item, nbytes, dtype, shape):
        out = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        native.check(native.lib().mppi_jump_get(self.ctx, native.ITEM[item], _ptr(out), nbytes, self._s()))
        self._publish()
        return out.view(dtype).reshape(shape)

    @property
    def U(self):
        return self._get("U", self.T * self.m * 4, torch.float32, (self.T, self.m))

    @property
    def S(self):
        return self._get("S", self.K * 8, torch.float64, (self.K,))

    @property
    def W(self):
        return self._get("W", self.K * 8, torch.float64, (self.K,))

    @property
    def eps(self):
        """Perturbations, [T, m, K]."""
        return self._get("EPS", self.T * self.m * self.K * 4, torch.float32, (self.T, self.m, self.K))

    def debug_draws(self):
        """(z_D [K,T,m], N [K,T], z_J [K,T,q]) of the last rollout."""
        K, T = self.K, self.T
        return (self._get("DBG_ZD", K * T * self.m * 4, torch.float32, (K, T, self.m)),
                self._get("DBG_N", K * T * 4, torch.int32, (K, T)),
                self._get("DBG_ZJ", K * T * self.q * 4, torch.float32, (K, T, self.q)))

    def stats(self):
        """Statistics of the last iteration (synchronises)."""
        raw = self._get("STATS", _STATS_BYTES, torch.uint8, (_STATS_BYTES,)).cpu().numpy()
        s = native.Stats.from_buffer_copy(raw.tobytes())
        return dict(rho=s.rho, eta=s.eta, status=s.status, n_finite=s.n_finite,
                    iteration=s.iteration)

    def set_U(self, U):
        t = torch.as_tensor(np.asarray(U, dtype=np.float32).reshape(self.T, self.m),
                            device=self.device).contiguous()
        native.check(native.lib().mppi_jump_set(self.ctx, native.ITEM["U"], _ptr(t), t.numel() * 4, self._s()))
        self._keep = t

    def set_S(self, S):
        t = torch.as_tensor(np.asarray(S, dtype=np.float64).reshape(self.K),
                            device=self.device).contiguous()
        native.check(native.lib().mppi_jump_set(self.ctx, native.ITEM["S"], _ptr(t), t.numel() * 8, self._s()))
        self._keep = t

    # ------------------------------------------------------------- timing
    def profile(self, enable=True):
        native.check(native.lib().mppi_jump_profile(self.ctx, int(bool(enable))))

    def profile_read(self):
        """(summed rollout-kernel ms, launches, iterations) since the last read."""
        ms, n, it = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        native.check(native.lib().mppi_jump_profile_read(self.ctx, ctypes.byref(ms), ctypes.byref(n),
                                                         ctypes.byref(it)))
        return ms.value, n.value, it.value


class Batch:
    """Many controllers advanced by one launch per iteration (batched form).

    controllers: Controller objects created with the same schedule; states:
    their state tensors ([n_i] fp32 on the device), read at every step.
    launch: native.C["MPPI_BATCH_GRID"] (one workgroup per tile) or
    native.C["MPPI_BATCH_PERSISTENT"] (resident workgroups take tiles from a
    device work queue)."""

    def __init__(self, controllers, states, stream=None, launch=0):
        self.controllers = list(controllers)
        self.states = [torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous()
                       for x in states]
        n = len(self.controllers)
        self.stream = stream
        ctxs = (ctypes.c_void_p * n)(*[c.ctx.value for c in self.controllers])
        xs = (ctypes.c_void_p * n)(*[x.data_ptr() for x in self.states])
        nbytes = ctypes.c_size_t()
        native.check(native.lib().mppi_jump_batch_scratch_bytes(ctxs, n, ctypes.byref(nbytes)))
        self.scratch = torch.empty(nbytes.value, dtype=torch.uint8, device="cuda")
        bt = ctypes.c_void_p()
        native.check(native.lib().mppi_jump_batch_create(ctxs, xs, n, _ptr(self.scratch),
                                                         nbytes.value, _stream_handle(stream),
                                                         ctypes.byref(bt)))
        self.bt = bt
        u0 = ctypes.c_void_p()
        native.check(native.lib().mppi_jump_batch_u0(bt, ctypes.byref(u0)))
        off = u0.value - self.scratch.data_ptr()
        self.u0 = self.scratch[off:off + 16 * n].view(torch.float32).view(n, 4)
        self.launch = int(launch)
        native.check(native.lib().mppi_jump_batch_set_launch(bt, self.launch))

    def step(self, iters=1, shift=True):
        native.check(native.lib().mppi_jump_batch_step(self.bt, int(iters), int(bool(shift)),
                                                       _stream_handle(self.stream)))

    def close(self):
        if getattr(self, "bt", None):
            native.lib().mppi_jump_batch_destroy(self.bt)
            self.bt = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchGroup:
    """Sub-batches of one controller set (e.g. one per model), each with its
    own stream, stepped together: every sub-batch's stream waits for torch's
    current stream, launches, and the current stream waits for all of them
    (so a step can be captured in one graph from the current stream)."""

    def __init__(self, batches):
        self.batches = list(batches)

    def step(self, iters=1, shift=True):
        cur = torch.cuda.current_stream()
        for b in self.batches:
            if b.stream is not None:
                b.stream.wait_stream(cur)
            b.step(iters, shift)
        for b in self.batches:
            if b.stream is not None:
                cur.wait_stream(b.stream)

    def close(self):
        for b in self.batches:
            b.close()


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


class Pool:
    """Resident controllers served by ticks over any subset (serving form).

    controllers: Controller objects created with the same schedule.
    max_inflight: number of slots, i.e. ticks that may be in flight at once
    (each on the stream given to tick()).  Host staging is page-locked memory
    owned by this object."""

    def __init__(self, controllers, max_inflight=4, stream=None):
        self.controllers = list(controllers)
        n = self.n = len(self.controllers)
        self.max_inflight = int(max_inflight)
        ctxs = (ctypes.c_void_p * n)(*[c.ctx.value for c in self.controllers])
        dbytes, hbytes = ctypes.c_size_t(), ctypes.c_size_t()
        native.check(native.lib().mppi_jump_pool_bytes(ctxs, n, self.max_inflight,
                                                       ctypes.byref(dbytes), ctypes.byref(hbytes)))
        self.device_bytes, self.host_bytes = dbytes.value, hbytes.value
        self.scratch = torch.empty(dbytes.value, dtype=torch.uint8, device="cuda")
        self._pinned = torch.empty(hbytes.value + 256, dtype=torch.uint8, pin_memory=True)
        off = (-self._pinned.data_ptr()) % 256
        pl = ctypes.c_void_p()
        native.check(native.lib().mppi_jump_pool_create(
            ctxs, n, self.max_inflight, _ptr(self.scratch), dbytes.value,
            ctypes.c_void_p(self._pinned.data_ptr() + off), hbytes.value,
            _stream_handle(stream), ctypes.byref(pl)))
        self.pl = pl
        self._count = [0] * self.max_inflight

    def tick(self, ids, states, dist=None, iters=1, slot=0, stream=None):
        """Enqueue one MPC step for controllers ids (int array [c]) from host
        states [c, 12] (fp32); with dist also step each plant: [c, 4]
        control-channel disturbances, or [c, 8] with a world-frame body
        force in columns 4..6 (quadrotor)."""
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        states = np.ascontiguousarray(states, dtype=np.float32).reshape(len(ids), 12)
        if dist is not None:
            dist = np.asarray(dist, dtype=np.float32).reshape(len(ids), -1)
            full = np.zeros((len(ids), 8), dtype=np.float32)
            full[:, :dist.shape[1]] = dist
            dist = full
        native.check(native.lib().mppi_jump_pool_tick(self.pl, _np_ptr(ids), _np_ptr(states),
                                                      _np_ptr(dist), len(ids), int(iters),
                                                      int(slot), _stream_handle(stream)))
        self._count[slot] = len(ids)

    def replace(self, index, controller, stream=None):
        """Put `controller` at pool position `index` (not in a tick in flight)
        in place of the controller there; synchronises `stream`."""
        native.check(native.lib().mppi_jump_pool_replace(self.pl, int(index), controller.ctx,
                                                         _stream_handle(stream)))
        self.controllers[index] = controller

    def finished(self, slot):
        f = ctypes.c_int32()
        native.check(native.lib().mppi_jump_pool_query(self.pl, int(slot), ctypes.byref(f)))
        return bool(f.value)

    def results(self, slot, plant=True):
        """(ids [c], u0 [c, 4], x_next [c, 12] or None) of the slot's finished
        tick, in request order."""
        c = self._count[slot]
        ids = np.empty(c, dtype=np.int32)
        u0 = np.empty((c, 4), dtype=np.float32)
        xn = np.empty((c, 12), dtype=np.float32) if plant else None
        cnt = ctypes.c_int32()
        native.check(native.lib().mppi_jump_pool_results(self.pl, int(slot), _np_ptr(ids),
                                                         _np_ptr(u0), _np_ptr(xn),
                                                         ctypes.byref(cnt)))
        return ids, u0, xn

    def close(self):
        if getattr(self, "pl", None):
            native.lib().mppi_jump_pool_destroy(self.pl)
            self.pl = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def philox(counters, key0, key1):
    """Device Philox4x32-10 blocks for uint32 counters [n, 4] (numpy)."""
    c = torch.as_tensor(np.ascontiguousarray(counters, dtype=np.uint32).view(np.int32),
                        device="cuda")
    out = torch.empty_like(c)
    n = c.shape[0]
    native.check(native.lib().mppi_jump_philox(_ptr(c), key0, key1, _ptr(out), n,
                                               _stream_handle()))
    return out.cpu().numpy().view(np.uint32)
