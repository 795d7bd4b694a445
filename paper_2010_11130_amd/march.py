"""Slab-by-slab time marching (Section 2.4) on the HIP library.

Slab n's inflow data on its initial plane is slab n-1's trace on its final
plane; every slab is assembled (``hdg_assemble``), gets its own lAIR
hierarchy (``air_setup``, Section 3) and is solved by FGMRES (``air_solve``).

Pipelined mode: the matrix of slab n+1 and therefore its hierarchy do not
depend on slab n's solution -- only the Neumann rows of its right-hand side
do.  Builder threads assemble and set up the next slabs, each on its own HIP
stream, while the calling thread solves slab n; the calling thread then
writes the inflow rows (``hdg_inflow_from_trace``) and refreshes the
right-hand side (``hdg_update_neumann``).  The solve of slab n is the
critical path: every kernel a builder runs competes with it for the GPU, so
one builder (one slab of lookahead) is the default; more builders overlap
each other's host waits but slow the solve down more than they gain.  Both
modes run the same kernels on the same data, so their results agree bit for
bit.
"""
import threading
import time

import torch

from .api import System, Hierarchy


class SlabMarch:
    """March over slabs sharing one mesh (a slab mesh reused with time-shifted
    data) or one mesh per slab.

    mesh:    a ``Mesh`` with boundary kinds set, or a sequence of them (one per slab)
    a_vert:  velocity at the vertices (device tensor), or a sequence (one per slab)
    air_kw:  ``Hierarchy`` options; solve_kw: ``Hierarchy.solve`` options
    builders: pipelined mode, number of builder threads (each with its own
              stream); slab k is built by thread k mod builders
    """

    def __init__(self, mesh, p, nu, a_vert, f_q=None, alpha=0.0, air_kw=None, solve_kw=None, keep=True,
                 builders=1):
        self.mesh, self.p, self.nu, self.a, self.f = mesh, p, float(nu), a_vert, f_q
        self.alpha, self.keep = alpha, keep
        self.builders = builders
        self.air_kw = dict(air_kw or {})
        self.solve_kw = dict(solve_kw or {})

    def _pick(self, x, k):
        return x[k] if isinstance(x, (list, tuple)) else x

    def _build(self, k, g):
        s = System(self._pick(self.mesh, k), self.p, self.nu, self._pick(self.a, k), self._pick(self.f, k), g,
                   alpha=self.alpha, keep=self.keep)
        return s, Hierarchy(s, **self.air_kw)

    def _solve(self, k, s, h, g, prev, on_slab):
        if prev is not None:
            prev[0].trace_to_inflow(prev[1], self._pick(self.mesh, k), g)
            s.update_neumann(g)
        x, info = h.solve(**self.solve_kw)
        if not info["converged"]:
            raise RuntimeError("slab %d did not converge: %s" % (k, info))
        if on_slab is not None:
            on_slab(k, s, h, x, info)
        return x, info

    def run(self, g_slabs, pipelined=True, on_slab=None, stages=None):
        """March over ``len(g_slabs)`` slabs.  ``g_slabs[k]``: device boundary
        data of slab k (``hdg_assemble``'s g_q: Dirichlet data, and for k = 0
        the initial data on the initial plane); for k >= 1 the initial-plane
        rows are overwritten in place by the previous slab's trace.
        ``on_slab(k, system, hierarchy, x, info)`` runs after each solve on the
        calling thread's stream.  Returns the last slab's (system, x, info).
        ``stages`` (sequential mode only): a list that receives per slab the
        seconds spent in assembly, setup and solve (the stream is
        synchronized at each boundary)."""
        if pipelined:
            if stages is not None:
                raise ValueError("stage times are only measured by the sequential march")
            return self._run_pipelined(g_slabs, on_slab)
        prev = None
        last = None
        for k, g in enumerate(g_slabs):
            if stages is None:
                s, h = self._build(k, g)
                x, info = self._solve(k, s, h, g, prev, on_slab)
            else:
                sync = torch.cuda.current_stream().synchronize
                t0 = time.perf_counter()
                s = System(self._pick(self.mesh, k), self.p, self.nu, self._pick(self.a, k), self._pick(self.f, k),
                           g, alpha=self.alpha, keep=self.keep)
                sync()
                t1 = time.perf_counter()
                h = Hierarchy(s, **self.air_kw)
                sync()
                t2 = time.perf_counter()
                x, info = self._solve(k, s, h, g, prev, on_slab)
                sync()
                t3 = time.perf_counter()
                stages.append({"assemble": t1 - t0, "setup": t2 - t1, "solve": t3 - t2, "iters": info["iters"],
                               "levels": h.info["levels"], "op_complexity": h.info["op_complexity"]})
            prev = (s, x)
            last = (s, x, info)
        return last

    def _run_pipelined(self, g_slabs, on_slab):
        S = len(g_slabs)
        nb = max(1, int(self.builders))
        main = torch.cuda.current_stream()
        sides = [torch.cuda.Stream() for _ in range(nb)]      # default priority
        cond = threading.Condition()
        ready = {}              # slab -> (system, hierarchy, event) or exception
        state = {"next": 0, "stop": False}

        def builder(j):
            try:
                with torch.cuda.stream(sides[j]):
                    for k in range(j, S, nb):
                        with cond:
                            # bounded lookahead: at most nb slabs built ahead
                            while not state["stop"] and k - state["next"] > nb:
                                cond.wait()
                            if state["stop"]:
                                return
                        s, h = self._build(k, g_slabs[k])
                        ev = torch.cuda.Event()
                        ev.record(sides[j])
                        with cond:
                            ready[k] = (s, h, ev)
                            cond.notify_all()
            except BaseException as e:   # re-raised by the solving thread
                with cond:
                    ready[-1] = e
                    cond.notify_all()

        # the builders read the boundary data written on the calling stream
        for sd in sides:
            sd.wait_stream(main)
        ths = [threading.Thread(target=builder, args=(j,), daemon=True) for j in range(nb)]
        for th in ths:
            th.start()
        prev = None
        held = None
        last = None
        self.wait_s = 0.0       # time the solving thread waited for builds
        try:
            for k in range(S):
                with cond:
                    t_w = time.perf_counter()
                    while k not in ready and -1 not in ready:
                        cond.wait()
                    self.wait_s += time.perf_counter() - t_w
                    if -1 in ready:
                        raise ready[-1]
                    s, h, ev = ready.pop(k)
                    state["next"] = k + 1
                    cond.notify_all()
                main.wait_event(ev)
                x, info = self._solve(k, s, h, g_slabs[k], prev, on_slab)
                # slab k-1's objects were last used before this solve's final
                # synchronization (its trace fed this slab's inflow): release
                held = None
                prev = (s, x)
                held = (s, h)
                last = (s, x, info)
        finally:
            with cond:
                state["stop"] = True
                cond.notify_all()
            for th in ths:
                th.join()
            ready.clear()
        # every build the calling stream consumed was waited for through its
        # event; builds not consumed (after an error) are dropped after join
        return last
