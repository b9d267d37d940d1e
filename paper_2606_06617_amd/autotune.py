"""Autotuner for the tile schedule of the spreading / gather / binning cells.

For a (grid, support P, channels C, atom count) the planner's default tile
maximises the fraction of useful window work prod B / (B + P - 1).  That
ignores parallelism (few large tiles leave CUs idle on small grids) and the
cost balance between spreading and gathering, so the autotuner times a short
list of candidate tiles on the device with the caller's stream and keeps
the fastest.  Results are cached in a JSON file (path from
PSWFLR_AUTOTUNE_CACHE, default ~/.cache/pswflr/autotune.json) keyed by the
device architecture, grid, P, C and the atom count rounded to a power of two.
api.Plan applies a cached tile by default when the caller names none
(PSWFLR_AUTOTUNE=0 turns that off).
"""
import json
import math
import os
import threading
import time

KERNEL_VERSION = 12
_LOCK = threading.Lock()
_MEMO = {}   # path -> (mtime, size, parsed cache): the file is read again only when it changes


def cache_path():
    return os.environ.get("PSWFLR_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pswflr", "autotune.json"))


def _load():
    path = cache_path()
    try:
        st = os.stat(path)
    except OSError:
        return {}
    got = _MEMO.get(path)
    if got is not None and got[0] == st.st_mtime_ns and got[1] == st.st_size:
        return got[2]
    try:
        with open(path) as f:
            db = json.load(f)
    except (OSError, ValueError):
        return {}
    _MEMO[path] = (st.st_mtime_ns, st.st_size, db)
    return db


def _store(db):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _divisors(m):
    return [d for d in range(1, m + 1) if m % d == 0]


def _tile_fits(bx, by, bz, P, lds=160 * 1024):
    """The kernels' own limits.  Spreading: 4x4x4 blocks, the tile's z edge
    one, two or four blocks deep (NBZ), each wave owning NBZ blocks in each
    of 4/NBZ neighbouring y columns (so the y block count is a multiple of
    4/NBZ and there are at most 8 waves' worth of columns), padded edges
    summing to <= 64.  Gather: a one-channel halo tile of at most 8192
    elements (16 per thread), two such buffers in LDS."""
    pad = lambda b: (b + 3) // 4 * 4
    nbz = pad(bz) // 4
    if nbz not in (1, 2, 4):
        return False
    cpw = 4 // nbz
    nby = pad(by) // 4
    S = pad(bx) + pad(by) + pad(bz)
    if nby % cpw or (pad(bx) // 4) * nby > 8 * cpw or S > 64 or bx * by * bz > 129 * (4 + S):
        return False
    ex, ey, ez = bx + P - 1, by + P - 1, bz + P - 1
    return ex * ey * ez <= 512 * 16 and (2 * 512 * 16 + 96) * 4 <= lds


def tile_feasible(grid, tile, P):
    """A tile the library accepts: the kernels' limits and at most 64
    candidate cells for the spread's screening."""
    if any(m % b for m, b in zip(grid, tile)) or not _tile_fits(tile[0], tile[1], tile[2], P):
        return False
    cells = 1
    for m, b in zip(grid, tile):
        cells *= min(min(m // b - 1, (P - 2) // b + 1) + 1, 8)
    return cells <= 64


def candidate_tiles(grid, P, limit=6):
    """Feasible tiles ranked by useful-work fraction, plus the most parallel
    feasible ones (small grids)."""
    feas = []
    for bx in _divisors(grid[0]):
        for by in _divisors(grid[1]):
            for bz in _divisors(grid[2]):
                if not tile_feasible(grid, (bx, by, bz), P):
                    continue
                eff = bx / (bx + P - 1) * by / (by + P - 1) * bz / (bz + P - 1)
                ncell = (grid[0] // bx) * (grid[1] // by) * (grid[2] // bz)
                feas.append((eff, bx * by * bz, ncell, (bx, by, bz)))
    by_eff = sorted(feas, key=lambda t: (-t[0], -t[1]))
    out = [t[3] for t in by_eff[:limit]]
    # for small grids also try shapes that give at least one tile per CU
    par = sorted([t for t in feas if t[2] >= 256], key=lambda t: (-t[0], -t[1]))
    for t in par[:2]:
        if t[3] not in out:
            out.append(t[3])
    return out


def key_for(arch, grid, P, C, n_atoms):
    nb = 1 << max(0, int(math.ceil(math.log2(max(1, n_atoms)))))
    return "%s|%dx%dx%d|P%d|C%d|N%d|v%d" % (arch, grid[0], grid[1], grid[2], P, C, nb, KERNEL_VERSION)


def lookup(arch, grid, P, C, n_atoms):
    with _LOCK:
        return _load().get(key_for(arch, grid, P, C, n_atoms))


_ARCH = {}


def device_arch(device=None):
    """gfx architecture name of a CUDA device (cached)."""
    import torch
    d = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    if d not in _ARCH:
        _ARCH[d] = torch.cuda.get_device_properties(d).gcnArchName.split(":")[0]
    return _ARCH[d]


def cached_tile(grid, P, C, n_atoms):
    """The tuned tile for this shape on the current device, or None (no entry,
    or PSWFLR_AUTOTUNE=0)."""
    if os.environ.get("PSWFLR_AUTOTUNE", "1") == "0":
        return None
    if not os.path.exists(cache_path()):
        return None
    hit = lookup(device_arch(), grid, P, C, n_atoms)
    return tuple(hit["tile"]) if hit else None


def tune(pos, q, box, ps, r_c=5.0, c=12.024, grid=None, support=0, c_spread=0.0, reps=5, verbose=False):
    """Time candidate tiles for this structure shape; cache and return the best
    tile (a 3-tuple).  pos, q: CUDA tensors as for Plan.execute."""
    import torch

    from .api import Plan
    base = Plan(box, ps, r_c=r_c, c=c, grid=grid, support=support, c_spread=c_spread,
                max_atoms=max(1, pos.shape[0]), autotune=False)
    g, P, C = base.info["grid"], base.info["support"], base.info["n_channels"]
    arch = torch.cuda.get_device_properties(pos.device).gcnArchName.split(":")[0]
    key = key_for(arch, g, P, C, pos.shape[0])
    results = {}
    for tile in candidate_tiles(g, P):
        try:
            plan = Plan(box, ps, r_c=r_c, c=c, grid=g, support=P, c_spread=base.info["c_spread"],
                        max_atoms=max(1, pos.shape[0]), tile=tile)
        except RuntimeError:
            continue
        ws = plan.new_workspace(pos.device)
        out = None
        for _ in range(2):
            out = plan.execute(pos, q, forces=True, virial=True, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = plan.execute(pos, q, forces=True, virial=True, workspace=ws)
        torch.cuda.synchronize()
        results[tile] = (time.perf_counter() - t0) / reps
        del out, ws
        if verbose:
            print("tile", tile, "%.3f ms" % (results[tile] * 1e3), flush=True)
    best = min(results, key=results.get)
    with _LOCK:
        db = _load()
        db[key] = {"tile": list(best), "ms": results[best] * 1e3,
                   "default_ms": results.get(tuple(base.info["tile"]), None) and
                   results[tuple(base.info["tile"])] * 1e3,
                   "tried": {"%dx%dx%d" % t: round(v * 1e3, 4) for t, v in results.items()}}
        _store(db)
    return best
