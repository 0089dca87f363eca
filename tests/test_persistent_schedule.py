"""Host-side model of the persistent ensemble launch (no GPU): the work items, the dataflow wait
set and both schedules, simulated with random interleavings of the workgroups.

The model restates the device protocol of k_step_persist:
- dataflow schedule: items k = s * T + t are handed out in increasing order from one counter, in
  chunks of 8 that a workgroup runs in index order; item (s, t) waits until every tile in its
  wait set has finished step s - 1; the wait set of a tile is the 5 x 5 candidate set of tile
  rows holding its first row and rows
  y0 - 2, y0 - 1, y1, y1 + 1, crossed with the bands holding its first column and columns
  x0 - 2, x0 - 1, x1, x1 + 1 (periodic wrap; rows behind a wall skipped);
- barrier schedule: workgroup w runs tiles w, w + nwg, ... of every step, with a grid barrier
  between steps over every workgroup of the launch.

Checked: (1) the wait set holds every tile whose nodes the tile's step reads (the populations it
pulls for its own nodes and for the one-node phi halo) or whose nodes it overwrites in the other
pair; (2) the dataflow schedule finishes for any number of resident workgroups, from one up, and
for random interleavings (no deadlock, every item exactly once, steps of a tile in order, and no
item starts before its wait set is done); (3) the barrier schedule finishes when every workgroup
of the launch is resident (the cooperative launch guarantees it) and stalls when one is not,
which is why it is launched cooperatively.
"""
import random

import pytest


def tile_geometry(nx, ny, wx, rows):
    w, h = 64 * wx, rows
    return w, h, (nx + w - 1) // w, (ny + h - 1) // h


def wait_set(nx, ny, walls, wx, rows, band, rg):
    w, h, nb, nr = tile_geometry(nx, ny, wx, rows)
    y0, x0 = rg * h, band * w
    y1, x1 = min(y0 + h, ny), min(x0 + w, nx)
    out = set()
    for yy in (y0, y0 - 2, y0 - 1, y1, y1 + 1):
        if not 0 <= yy < ny:
            if walls:
                continue
            yy %= ny
        for xx in (x0, x0 - 2, x0 - 1, x1, x1 + 1):
            out.add((yy // h) * nb + (xx % nx) // w)
    return out


def footprint(nx, ny, walls, wx, rows, band, rg):
    """Tiles owning a node the step of tile (band, rg) reads or writes: the pulls of its own nodes
    (x +- 1, y +- 1), the pulls of the phi halo ring (one node further), and its own nodes (the
    other pair is written there, and read there by every tile whose reach covers it)."""
    w, h, nb, nr = tile_geometry(nx, ny, wx, rows)
    y0, x0 = rg * h, band * w
    y1, x1 = min(y0 + h, ny), min(x0 + w, nx)
    out = set()
    for y in range(y0 - 2, y1 + 2):
        if not 0 <= y < ny:
            if walls:
                continue
            y %= ny
        for x in range(x0 - 2, x1 + 2):
            out.add((y // h) * nb + (x % nx) // w)
    return out


BOXES = [(70, 45, 0, 1, 16), (70, 45, 1, 1, 1), (300, 7, 0, 2, 1), (130, 9, 1, 1, 2), (64, 64, 0, 1, 3),
         (200, 3, 0, 4, 1), (65, 5, 0, 1, 1), (1, 1, 0, 1, 1), (129, 2, 1, 2, 1), (257, 130, 0, 4, 3)]


@pytest.mark.parametrize("nx,ny,walls,wx,rows", BOXES)
def test_wait_set_covers_the_footprint(nx, ny, walls, wx, rows):
    w, h, nb, nr = tile_geometry(nx, ny, wx, rows)
    for rg in range(nr):
        for band in range(nb):
            assert footprint(nx, ny, walls, wx, rows, band, rg) <= wait_set(nx, ny, walls, wx, rows, band, rg)


def _tiles(boxes):
    """Global tile list (box, tile) in box order, as the launch's tile table."""
    out = []
    for b, (nx, ny, walls, wx, rows) in enumerate(boxes):
        w, h, nb, nr = tile_geometry(nx, ny, wx, rows)
        out += [(b, t) for t in range(nb * nr)]
    return out


def simulate(boxes, nsteps, nwg, resident, schedule, rng, chunk=8):
    """Event simulation: `resident` of the nwg workgroups run (the others never start, as
    workgroups that have not been dispatched); each running workgroup, picked at random, makes one
    move.  Dataflow: grab the next `chunk` items from the counter, then for each item in order
    wait for its wait set and run it.  Barrier: workgroup w runs tiles w, w + nwg, ... of every
    step and arrives at a grid barrier between steps.  Returns True when every item completed,
    False on a stall (no running workgroup can move)."""
    tiles = _tiles(boxes)
    T = len(tiles)
    total = nsteps * T
    done = {bt: 0 for bt in tiles}
    nxt = 0
    queue = [[] for _ in range(nwg)]      # items a workgroup holds, in index order
    step_of = [0] * nwg                   # barrier schedule: current step of the workgroup
    at_barrier = [False] * nwg
    arrived = {}
    finished = 0
    alive = list(range(resident))
    exited = set()

    def deps_done(k):
        s, (b, t) = k // T, tiles[k % T]
        nx, ny, walls, wx, rows = boxes[b]
        w, h, nb, nr = tile_geometry(nx, ny, wx, rows)
        return all(done[(b, d)] >= s for d in wait_set(nx, ny, walls, wx, rows, t % nb, t // nb))

    def run(k):
        nonlocal finished
        s, bt = k // T, tiles[k % T]
        assert done[bt] == s  # the steps of a tile run in order, each once
        if schedule == "dataflow":
            assert deps_done(k)
        done[bt] = s + 1
        finished += 1

    if schedule == "barrier":
        for g in range(nwg):
            queue[g] = [s * T + t for s in range(nsteps) for t in range(g, T, nwg)]
    while True:
        movable = []
        for g in alive:
            if g in exited:
                continue
            if schedule == "dataflow":
                if not queue[g] or deps_done(queue[g][0]):
                    movable.append(g)
            else:
                if at_barrier[g]:
                    if arrived.get(step_of[g], 0) == nwg:
                        movable.append(g)
                else:
                    movable.append(g)
        if not movable:
            return finished == total
        g = rng.choice(movable)
        if schedule == "dataflow":
            if not queue[g]:
                if nxt >= total:
                    exited.add(g)
                    continue
                queue[g] = list(range(nxt, min(nxt + chunk, total)))
                nxt += chunk
            else:
                run(queue[g].pop(0))
        else:
            if at_barrier[g]:
                at_barrier[g] = False
                step_of[g] += 1
            elif queue[g] and queue[g][0] // T == step_of[g]:
                run(queue[g].pop(0))
            elif step_of[g] < nsteps - 1:
                at_barrier[g] = True
                arrived[step_of[g]] = arrived.get(step_of[g], 0) + 1
            else:
                exited.add(g)


@pytest.mark.parametrize("resident", [1, 2, 5, 16])
def test_dataflow_schedule_completes_with_any_residency(resident):
    rng = random.Random(resident)
    boxes = BOXES[:6]
    for trial in range(3):
        for chunk in (1, 8):
            assert simulate(boxes, nsteps=4, nwg=16, resident=resident, schedule="dataflow", rng=rng, chunk=chunk)


def test_barrier_schedule_needs_every_workgroup_resident():
    rng = random.Random(7)
    boxes = BOXES[:4]
    assert simulate(boxes, nsteps=3, nwg=8, resident=8, schedule="barrier", rng=rng)
    assert not simulate(boxes, nsteps=3, nwg=8, resident=7, schedule="barrier", rng=rng)
