"""Python API over the C ABI: plans, one-structure evaluation, the autograd
adjoint.  PyTorch provides device memory and the current stream only.
"""
import contextlib
import ctypes

import torch

from . import _lib
from . import autotune as _autotune


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A resolved PSWF-LR evaluation plan for one box and channel set.

    box: 3 orthorhombic edges, or a 3x3 cell whose rows are the lattice
    vectors (triclinic); ps: exponent per channel (1..6); r_c: the
    short-range cutoff (k_c = c / r_c); c: mollifier bandwidth (0: from tol);
    grid: (Mx, My, Mz) or None (from tol); support: window points per axis
    P (0: from tol); c_spread: window bandwidth (0: automatic); check_inputs:
    every call first verifies on the device that positions and charges are
    finite and raises otherwise (synchronous); tile: tile edges, or None for
    the autotuner's cached choice for this shape (timed on single calls)
    when `autotune` is set and the cache has one, else the planner's.
    Plans meant for batched calls should pass autotune=False: a batch fills
    the chip with many structures, so the planner's most efficient tiles win
    there (64-structure training batch: 0.53 ms against 0.74 ms with the
    tiles tuned one structure at a time).
    """

    def __init__(self, box, ps, r_c=5.0, c=12.024, tol=1e-5, grid=None, support=0, c_spread=0.0,
                 max_atoms=1, tile=None, check_inputs=False, autotune=True):
        L = _lib.lib()
        flags = _lib.FLAG_CHECK_INPUTS if check_inputs else 0
        self.params = _lib.make_params(box, ps, r_c, c, tol, grid, support, c_spread, tile, flags=flags)
        h = ctypes.c_void_p()
        _lib.check(L.pswflr_plan_create(ctypes.byref(self.params), int(max_atoms), ctypes.byref(h)))
        self.handle = h
        inf = _lib.Info()
        _lib.check(L.pswflr_plan_info(h, ctypes.byref(inf)))
        if tile is None and autotune:
            # the autotuner's cached choice for this shape, if any
            best = _autotune.cached_tile(tuple(inf.grid), inf.support, inf.n_channels, max_atoms)
            if best is not None and best != tuple(inf.tile):
                prm = _lib.make_params(box, ps, r_c, inf.c, tol, tuple(inf.grid), inf.support, inf.c_spread,
                                       best, flags=flags)
                h2 = ctypes.c_void_p()
                if L.pswflr_plan_create(ctypes.byref(prm), int(max_atoms), ctypes.byref(h2)) == _lib.OK:
                    L.pswflr_plan_destroy(h)
                    self.params, self.handle, h = prm, h2, h2
                    _lib.check(L.pswflr_plan_info(h, ctypes.byref(inf)))
        self.info_raw = inf
        C = inf.n_channels
        self.info = {
            "c": inf.c, "r_c": inf.r_c, "k_c": inf.k_c, "c_spread": inf.c_spread, "eta": inf.eta,
            "h": tuple(inf.h), "volume": inf.volume, "grid": tuple(inf.grid), "support": inf.support,
            "n_channels": C, "kz_keep": inf.kz_keep, "ny_keep": inf.ny_keep, "tile": tuple(inf.tile),
            "cg_spread": inf.cg_spread, "cg_gather": inf.cg_gather, "xcols": inf.xcols,
            "max_atoms": inf.max_atoms, "workspace_bytes": inf.workspace_bytes,
            "grid_offset": inf.grid_offset,
            "self_coef": [inf.self_coef[i] for i in range(C)],
            "zero_coef": [inf.zero_coef[i] for i in range(C)],
            "cell": tuple(tuple(inf.cell[3 * a + b] for b in range(3)) for a in range(3)),
        }
        self.ps = list(ps)
        self.box = tuple(tuple(float(v) for v in b) if hasattr(b, "__len__") else float(b) for b in box)
        self.C = C
        self.max_atoms = int(max_atoms)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                _lib.lib().pswflr_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    @property
    def workspace_bytes(self):
        return int(self.info["workspace_bytes"])

    def new_workspace(self, device="cuda"):
        # caching-allocator blocks are at least 512-byte aligned
        ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)
        assert ws.data_ptr() % 256 == 0
        return ws

    def cell_gradient(self, virial, stream=None):
        """dE/dH [3, 3] (rows of H: lattice vectors) at fixed fractional
        coordinates from a device virial [6] of this plan's execute or
        realspace call: the NPT box derivative, formed on the device."""
        st = stream if stream is not None else torch.cuda.current_stream()
        with torch.cuda.stream(st):
            out = torch.empty(9, dtype=torch.float64, device=virial.device)
        _lib.check(_lib.lib().pswflr_cell_gradient(self.handle, _stream(st), _ptr(virial), _ptr(out)))
        return out.view(3, 3)

    def execute(self, pos, q, forces=True, virial=True, potential=False, workspace=None, stream=None,
                out=None):
        """Evaluate energy [3C + 1] (E_k, E_0, E_self per channel, then
        E_lr = sum_c (E_k + E_0)), forces [N,3], virial [6] and potentials
        [C,N] on `stream` (default: the current stream).  Tensors allocated
        here are allocated on that stream, so the caching allocator does not
        hand them to other work before the call has run.

        pos: float32 [N,3] CUDA tensor; q: float32 [C,N] CUDA tensor.
        """
        _check_inputs(pos, q, self.C, self.max_atoms)
        N = pos.shape[0]
        dev = pos.device
        o = out or {}
        with (torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()):
            ws = workspace if workspace is not None else self.new_workspace(dev)
            energy = o.get("energy")
            if energy is None:
                energy = torch.empty(3 * self.C + 1, dtype=torch.float64, device=dev)
            F = (o.get("forces") if o.get("forces") is not None else
                 torch.empty((N, 3), dtype=torch.float32, device=dev)) if forces else None
            W = (o.get("virial") if o.get("virial") is not None else
                 torch.empty(6, dtype=torch.float64, device=dev)) if virial else None
            phi = (o.get("potential") if o.get("potential") is not None else
                   torch.empty((self.C, N), dtype=torch.float32, device=dev)) if potential else None
        if energy.numel() < 3 * self.C + 1:
            raise ValueError("energy output needs 3C + 1 entries")
        st = _lib.lib().pswflr_execute(self.handle, _stream(stream), _ptr(ws), ws.numel(), N, _ptr(pos),
                                       _ptr(q), _ptr(energy), _ptr(F), _ptr(W), _ptr(phi))
        _lib.check(st)
        return {"energy": energy, "forces": F, "virial": W, "potential": phi, "workspace": ws}

    def realspace(self, pos, q, forces=True, virial=True, potential=False, workspace=None, stream=None):
        """Real-space complement of the split: energy [C] (E_real per
        channel), forces [N,3], virial [6] and potentials [C,N] of
        1/2 sum q_i q_j (1 - G_p(r)) / r^p over pairs closer than r_c."""
        _check_inputs(pos, q, self.C, self.max_atoms)
        N = pos.shape[0]
        dev = pos.device
        with (torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()):
            ws = workspace if workspace is not None else self.new_workspace(dev)
            energy = torch.empty(self.C, dtype=torch.float64, device=dev)
            F = torch.empty((N, 3), dtype=torch.float32, device=dev) if forces else None
            W = torch.empty(6, dtype=torch.float64, device=dev) if virial else None
            phi = torch.empty((self.C, N), dtype=torch.float32, device=dev) if potential else None
        st = _lib.lib().pswflr_realspace(self.handle, _stream(stream), _ptr(ws), ws.numel(), N, _ptr(pos), _ptr(q),
                                         _ptr(energy), _ptr(F), _ptr(W), _ptr(phi))
        _lib.check(st)
        return {"energy": energy, "forces": F, "virial": W, "potential": phi, "workspace": ws}

    def force_vjp(self, workspace, pos, q, v, stream=None):
        """Derivatives of sum_i v_i . F_i in charges [C,N] and positions
        [N,3], after an execute with forces on the same workspace (whose
        potential grid it consumes)."""
        N = pos.shape[0]
        dev = pos.device
        with (torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()):
            gq = torch.empty((self.C, N), dtype=torch.float32, device=dev)
            gp = torch.empty((N, 3), dtype=torch.float32, device=dev)
            vv = v.to(device=dev, dtype=torch.float32).contiguous()
        st = _lib.lib().pswflr_force_vjp(self.handle, _stream(stream), _ptr(workspace), workspace.numel(), N,
                                         _ptr(pos), _ptr(q), _ptr(vv), _ptr(gq), _ptr(gp))
        _lib.check(st)
        return gq, gp

    def backward(self, workspace, pos, q, grad_energy, want_q=True, want_pos=True, stream=None):
        """Adjoint of an energy-only execute on the same workspace."""
        N = pos.shape[0]
        dev = pos.device
        with (torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()):
            gq = torch.empty((self.C, N), dtype=torch.float32, device=dev) if want_q else None
            gp = torch.empty((N, 3), dtype=torch.float32, device=dev) if want_pos else None
            g = grad_energy.to(device=dev, dtype=torch.float64).contiguous()
        st = _lib.lib().pswflr_backward(self.handle, _stream(stream), _ptr(workspace), workspace.numel(), N,
                                        _ptr(pos), _ptr(q), _ptr(g), _ptr(gq), _ptr(gp))
        _lib.check(st)
        return gq, gp


def execute_batch(plans, inputs, forces=True, virial=True, potential=False, workspace=None, stream=None):
    """Evaluate many structures in one batched call (one launch per stage
    over all structures).  inputs: list of (pos [N,3], q [C,N]) CUDA tensors,
    one per plan.  Returns a list of output dicts as Plan.execute does."""
    L = _lib.lib()
    n = len(plans)
    if n != len(inputs):
        raise ValueError("one (pos, q) per plan")
    handles = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    natoms = (ctypes.c_int64 * n)(*[int(x[0].shape[0]) for x in inputs])
    need = ctypes.c_size_t()
    _lib.check(L.pswflr_batch_workspace(n, handles, natoms, ctypes.byref(need)))
    dev = inputs[0][0].device if n else torch.device("cuda")
    ws = workspace if workspace is not None else torch.empty(max(1, need.value), dtype=torch.uint8, device=dev)
    if n == 0:
        _lib.check(L.pswflr_execute_batch(0, handles, (_lib.IO * 1)(), _stream(stream), _ptr(ws), ws.numel()))
        return [], ws
    # outputs live in a few flat tensors (one allocation each, not one per
    # structure); the per-structure dicts hold views of them
    Ns = [int(x[0].shape[0]) for x in inputs]
    Cs = [plan.C for plan in plans]
    e_all = torch.empty(sum(3 * c + 1 for c in Cs), dtype=torch.float64, device=dev)
    f_all = torch.empty((sum(Ns), 3), dtype=torch.float32, device=dev) if forces else None
    v_all = torch.empty((n, 6), dtype=torch.float64, device=dev) if virial else None
    p_all = torch.empty(sum(c * m for c, m in zip(Cs, Ns)), dtype=torch.float32, device=dev) if potential else None
    e_views = torch.split(e_all, [3 * c + 1 for c in Cs])
    f_views = torch.split(f_all, Ns) if forces else [None] * n
    v_views = v_all.unbind(0) if virial else [None] * n
    p_views = ([t.view(c, m) for t, c, m in zip(torch.split(p_all, [c * m for c, m in zip(Cs, Ns)]), Cs, Ns)]
               if potential else [None] * n)
    e_ptr = e_all.data_ptr()
    f_ptr = f_all.data_ptr() if forces else 0
    v_ptr = v_all.data_ptr() if virial else 0
    p_ptr = p_all.data_ptr() if potential else 0
    ios = (_lib.IO * n)()
    outs = []
    eo = fo = po = 0
    for i, (plan, (pos, q)) in enumerate(zip(plans, inputs)):
        _check_inputs(pos, q, plan.C, plan.max_atoms)
        N, C = Ns[i], Cs[i]
        io = ios[i]
        io.n_atoms = N
        io.pos = pos.data_ptr()
        io.q = q.data_ptr()
        io.energy = e_ptr + 8 * eo
        io.forces = f_ptr + 12 * fo if forces else None
        io.virial = v_ptr + 48 * i if virial else None
        io.potential = p_ptr + 4 * po if potential else None
        eo += 3 * C + 1
        fo += N
        po += C * N
        outs.append({"energy": e_views[i], "forces": f_views[i], "virial": v_views[i], "potential": p_views[i]})
    _lib.check(L.pswflr_execute_batch(n, handles, ios, _stream(stream), _ptr(ws), ws.numel()))
    return outs, ws


class Batch:
    """Many structures laid out flat for the batched calls: positions
    [sum N_i, 3] and charges (the blocks [C_i, N_i] one after another) in
    one device tensor each, with the per-structure plans.  The ctypes tables
    (plan handles, atom counts) are built once here, so a call marshals four
    pointers."""

    def __init__(self, plans, n_atoms):
        self.plans = list(plans)
        self.n = len(self.plans)
        self.n_atoms = [int(x) for x in n_atoms]
        self.Cs = [p.C for p in self.plans]
        self.handles = (ctypes.c_void_p * max(1, self.n))(*[p.handle.value for p in self.plans])
        self.natoms = (ctypes.c_int64 * max(1, self.n))(*self.n_atoms)
        self.atoms = sum(self.n_atoms)
        self.qlen = sum(c * m for c, m in zip(self.Cs, self.n_atoms))
        self.elen = sum(3 * c + 1 for c in self.Cs)
        # index of each structure's E_lr in the flat energy array
        ends, e0 = [], 0
        for c in self.Cs:
            ends.append(e0 + 3 * c)
            e0 += 3 * c + 1
        self.elr_index = ends
        need = ctypes.c_size_t()
        _lib.check(_lib.lib().pswflr_batch_workspace(self.n, self.handles, self.natoms, ctypes.byref(need)))
        self.workspace_bytes = max(1, need.value)

    @staticmethod
    def concat(inputs):
        """Flat (pos, q) from a list of per-structure (pos [N,3], q [C,N])."""
        pos = torch.cat([p.reshape(-1) for p, _ in inputs]) if inputs else torch.empty(0)
        q = torch.cat([c.reshape(-1) for _, c in inputs]) if inputs else torch.empty(0)
        return pos.contiguous(), q.contiguous()

    def new_workspace(self, device="cuda"):
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def execute(self, pos, q, forces=True, virial=True, potential=False, workspace=None, stream=None, out=None):
        """One batched call on flat inputs: returns flat energy (blocks
        [3C_i + 1]), forces [sum N_i, 3], virial [n, 6], potentials (blocks
        [C_i, N_i]) and E_lr per structure [n]."""
        dev = pos.device
        if pos.dtype != torch.float32 or q.dtype != torch.float32 or not (pos.is_contiguous() and q.is_contiguous()):
            raise ValueError("pos and q must be contiguous float32 tensors")
        if pos.numel() != 3 * self.atoms or q.numel() != self.qlen:
            raise ValueError("flat inputs do not match the batch's atom and channel counts")
        o = out or {}
        with (torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()):
            ws = workspace if workspace is not None else self.new_workspace(dev)
            e = o.get("energy")
            if e is None:
                e = torch.empty(self.elen, dtype=torch.float64, device=dev)
            F = (o.get("forces") if o.get("forces") is not None else
                 torch.empty((self.atoms, 3), dtype=torch.float32, device=dev)) if forces else None
            W = (o.get("virial") if o.get("virial") is not None else
                 torch.empty((self.n, 6), dtype=torch.float64, device=dev)) if virial else None
            phi = (o.get("potential") if o.get("potential") is not None else
                   torch.empty(self.qlen, dtype=torch.float32, device=dev)) if potential else None
        st = _lib.lib().pswflr_execute_batch_flat(self.n, self.handles, self.natoms, _ptr(pos), _ptr(q), _ptr(e),
                                                  _ptr(F), _ptr(W), _ptr(phi), _stream(stream), _ptr(ws),
                                                  ws.numel())
        _lib.check(st)
        return {"energy": e, "forces": F, "virial": W, "potential": phi, "workspace": ws}

    def backward(self, workspace, pos, q, grad_energy, want_q=True, want_pos=True, stream=None):
        """Adjoint of an energy-only batched call on the same workspace:
        grad_energy [sum C_i] (dL/dE per channel) -> dL/dq (flat blocks) and
        dL/dr [sum N_i, 3]."""
        dev = pos.device
        with (torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()):
            gq = torch.empty(self.qlen, dtype=torch.float32, device=dev) if want_q else None
            gp = torch.empty((self.atoms, 3), dtype=torch.float32, device=dev) if want_pos else None
            g = grad_energy.to(device=dev, dtype=torch.float64).contiguous()
        st = _lib.lib().pswflr_backward_batch_flat(self.n, self.handles, self.natoms, _ptr(pos), _ptr(q), _ptr(g),
                                                   _ptr(gq), _ptr(gp), _stream(stream), _ptr(workspace),
                                                   workspace.numel())
        _lib.check(st)
        return gq, gp


class PSWFLRBatchFunction(torch.autograd.Function):
    """E_lr of every structure of a Batch, [n], as a differentiable function
    of the flat positions and charges: one batched energy-only forward, and
    one batched hand-written adjoint for all structures' gradients."""

    @staticmethod
    def forward(ctx, pos, q, batch):
        ws = batch.new_workspace(pos.device)
        out = batch.execute(pos.detach(), q.detach(), forces=False, virial=False, potential=False, workspace=ws)
        ctx.batch = batch
        ctx.ws = ws
        ctx.save_for_backward(pos.detach(), q.detach())
        idx = torch.tensor(batch.elr_index, device=pos.device, dtype=torch.long)
        return out["energy"].index_select(0, idx)

    @staticmethod
    def backward(ctx, grad_out):
        pos, q = ctx.saved_tensors
        batch = ctx.batch
        reps = torch.tensor(batch.Cs, device=grad_out.device, dtype=torch.long)
        g = torch.repeat_interleave(grad_out.detach().to(torch.float64), reps)   # dL/dE per channel
        gq, gp = batch.backward(ctx.ws, pos, q, g, want_q=ctx.needs_input_grad[1], want_pos=ctx.needs_input_grad[0])
        return (gp.view_as(pos) if gp is not None else None), (gq.view_as(q) if gq is not None else None), None


def lr_energy_batch(pos, q, batch):
    return PSWFLRBatchFunction.apply(pos, q, batch)


def _check_inputs(pos, q, C, max_atoms):
    if not (pos.is_cuda and q.is_cuda):
        raise ValueError("pos and q must be CUDA (HIP) tensors")
    if pos.dtype != torch.float32 or q.dtype != torch.float32:
        raise ValueError("pos and q must be float32")
    if pos.dim() != 2 or pos.shape[1] != 3 or not pos.is_contiguous():
        raise ValueError("pos must be a contiguous [N, 3] tensor")
    if q.dim() != 2 or q.shape[0] != C or q.shape[1] != pos.shape[0] or not q.is_contiguous():
        raise ValueError("q must be a contiguous [C, N] tensor")
    if pos.shape[0] > max_atoms:
        raise ValueError("N exceeds the plan's max_atoms")


def energy_forces(pos, q, box, ps, r_c=5.0, c=12.024, tol=1e-5, grid=None, support=0, c_spread=0.0,
                  virial=True, potential=False):
    """One-shot convenience: build a plan for this structure and evaluate it."""
    plan = Plan(box, ps, r_c=r_c, c=c, tol=tol, grid=grid, support=support, c_spread=c_spread,
                max_atoms=max(1, pos.shape[0]))
    out = plan.execute(pos, q, forces=True, virial=virial, potential=potential)
    out["plan"] = plan
    return out


class PSWFLRFunction(torch.autograd.Function):
    """E_lr = sum_c (E_k + E_0) (the library's last energy entry) as a
    differentiable function of (pos, q).

    Forward runs only the forward transforms (the energy needs no inverse
    FFT) and keeps the spectrum in the plan's workspace; backward runs the
    hand-written adjoint (scaled inverse transforms and the gather) and
    returns dE/dq and dE/dpos.
    """

    @staticmethod
    def forward(ctx, pos, q, plan):
        ws = plan.new_workspace(pos.device)
        out = plan.execute(pos.detach(), q.detach(), forces=False, virial=False, potential=False,
                           workspace=ws)
        ctx.plan = plan
        ctx.ws = ws
        ctx.save_for_backward(pos.detach(), q.detach())
        return out["energy"][3 * plan.C]

    @staticmethod
    def backward(ctx, grad_out):
        pos, q = ctx.saved_tensors
        plan = ctx.plan
        g = grad_out.detach().to(torch.float64).reshape(1).expand(plan.C).contiguous()
        gq, gp = plan.backward(ctx.ws, pos, q, g, want_q=ctx.needs_input_grad[1],
                               want_pos=ctx.needs_input_grad[0])
        return gp, gq, None


def lr_energy(pos, q, plan):
    return PSWFLRFunction.apply(pos, q, plan)


class PSWFLRForces(torch.autograd.Function):
    """Forces F = -dE_lr/dr [N,3] as a differentiable function of (pos, q),
    for losses on forces (force matching): forward is the evaluation with
    forces; backward takes dL/dF and runs the library's second-derivative
    call (Hessian gather of the potential grid, dipole spread through the
    same convolution), once per forward."""

    @staticmethod
    def forward(ctx, pos, q, plan):
        ws = plan.new_workspace(pos.device)
        out = plan.execute(pos.detach(), q.detach(), forces=True, virial=False, potential=False, workspace=ws)
        ctx.plan = plan
        ctx.ws = ws
        ctx.save_for_backward(pos.detach(), q.detach())
        return out["forces"]

    @staticmethod
    def backward(ctx, grad_f):
        pos, q = ctx.saved_tensors
        gq, gp = ctx.plan.force_vjp(ctx.ws, pos, q, grad_f.detach())
        return gp, gq, None


def lr_forces(pos, q, plan):
    return PSWFLRForces.apply(pos, q, plan)
