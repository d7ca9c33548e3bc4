"""Host emulation of the synchronisation of the cell sort's scatter.

The scatter ranks each particle among the particles of its cell with LDS
atomics on per-cell counts, reserves a destination range per cell with an
HBM atomic on the cell's cursor, copies particles to base + rank, and clears
the counts for the next round.  The emulation runs each wavefront's program
as a list of operations separated by barriers; between two barriers the
operations of different wavefronts may interleave in any order (the
hardware orders nothing else), and a schedule picks one interleaving.

Three programs are checked:

* the per-tile scatter with the counts cleared after the tile's last barrier
  (the ordering of the earlier kernel): a wavefront that reaches the next
  tile's rank atomics before another wavefront's clear of the same cell
  keeps a stale count, the clear then erases its contribution, and two
  particles get one destination while another slot is never written --
  particles lost;
* the same scatter with the clear moved before the last barrier: no
  interleaving loses a particle;
* the current scatter (one reservation per workgroup piece, cursors cleared
  between barriers): no interleaving loses a particle.
"""
import itertools
import random

import pytest

BARRIER = "barrier"


def run(programs, schedule):
    """Run wavefront programs (lists of callables and BARRIER markers) with
    the interleaving chosen by schedule(epoch, ready_waves) -> wave index."""
    pcs = [0] * len(programs)
    epoch = 0
    while True:
        ready = [w for w, p in enumerate(programs) if pcs[w] < len(p) and p[pcs[w]] != BARRIER]
        if ready:
            w = schedule(epoch, ready)
            programs[w][pcs[w]]()
            pcs[w] += 1
            continue
        if all(pcs[w] >= len(p) for w, p in enumerate(programs)):
            return
        # every wavefront is at a barrier (or done): release them together
        assert all(pcs[w] >= len(p) or p[pcs[w]] == BARRIER for w, p in enumerate(programs))
        for w, p in enumerate(programs):
            if pcs[w] < len(p):
                pcs[w] += 1
        epoch += 1


def per_tile_programs(tiles, n_waves, clear_before_last_barrier):
    """tiles[t][w] = list of (particle id, cell) of wavefront w in tile t."""
    sh = dict(cnt={}, gbase={}, cursor={}, dst={})
    cells = sorted({c for tile in tiles for wave in tile for _, c in wave})
    start, run_ = {}, 0
    total = {c: 0 for c in cells}
    for tile in tiles:
        for wave in tile:
            for _, c in wave:
                total[c] += 1
    for c in cells:
        start[c] = run_
        run_ += total[c]
    sh["cursor"] = dict(start)
    progs = [[] for _ in range(n_waves)]
    for t, tile in enumerate(tiles):
        for w in range(n_waves):
            p = progs[w]
            ranks = {}

            def rank(pid, c, ranks=ranks):
                old = sh["cnt"].get(c, 0)
                sh["cnt"][c] = old + 1
                ranks[pid] = old

            def reserve(pid, c, ranks=ranks):
                if ranks[pid] == 0:       # the cell's first particle of the tile
                    n = sh["cnt"][c]
                    sh["gbase"][c] = sh["cursor"][c]
                    sh["cursor"][c] += n

            def store(pid, c, ranks=ranks):
                sh["dst"].setdefault(sh["gbase"][c] + ranks[pid], []).append(pid)

            def clear(pid, c, ranks=ranks):
                if ranks[pid] == 0:
                    sh["cnt"][c] = 0

            mine = tile[w]
            p += [(lambda pid=pid, c=c: rank(pid, c)) for pid, c in mine] + [BARRIER]
            p += [(lambda pid=pid, c=c: reserve(pid, c)) for pid, c in mine] + [BARRIER]
            if clear_before_last_barrier:
                p += [(lambda pid=pid, c=c: clear(pid, c)) for pid, c in mine]
                p += [(lambda pid=pid, c=c: store(pid, c)) for pid, c in mine] + [BARRIER]
            else:
                p += [(lambda pid=pid, c=c: store(pid, c)) for pid, c in mine] + [BARRIER]
                p += [(lambda pid=pid, c=c: clear(pid, c)) for pid, c in mine]
    return progs, sh, run_


def piece_programs(tiles, n_waves):
    """The current scatter over one workgroup piece: histogram, barrier,
    reservation (counts become cursors), barrier, cursor atomics + stores,
    barrier, clear, barrier."""
    sh = dict(cnt={}, gbase={}, cursor={}, dst={})
    cells = sorted({c for tile in tiles for wave in tile for _, c in wave})
    sh["cursor"] = {c: 1000 * i for i, c in enumerate(cells)}
    n = sum(len(wave) for tile in tiles for wave in tile)
    progs = [[] for _ in range(n_waves)]
    for w in range(n_waves):
        p = progs[w]
        mine = [x for tile in tiles for x in tile[w]]

        def hist(c):
            sh["cnt"][c] = sh["cnt"].get(c, 0) + 1

        def reserve(c):   # one thread per cell: wave 0 takes them all here
            k = sh["cnt"].get(c, 0)
            if k:
                sh["gbase"][c] = sh["cursor"][c]
                sh["cursor"][c] += k
                sh["cnt"][c] = 0

        def place(pid, c):
            pos = sh["cnt"].get(c, 0)
            sh["cnt"][c] = pos + 1
            sh["dst"].setdefault(sh["gbase"][c] + pos, []).append(pid)

        def clear(c):
            sh["cnt"][c] = 0

        p += [(lambda c=c: hist(c)) for _, c in mine] + [BARRIER]
        if w == 0:
            p += [(lambda c=c: reserve(c)) for c in cells]
        p += [BARRIER]
        p += [(lambda pid=pid, c=c: place(pid, c)) for pid, c in mine] + [BARRIER]
        if w == 0:
            p += [(lambda c=c: clear(c)) for c in cells]
        p += [BARRIER]
    return progs, sh, n


def check(sh, n_particles):
    """(slots written more than once, particles lost).  A slot written twice
    keeps the last particle: the others are lost, and as many slots of the
    destination are never written (they hold stale data)."""
    shared = sum(1 for slot in sh["dst"].values() if len(slot) > 1)
    lost = sum(len(slot) - 1 for slot in sh["dst"].values())
    placed = {pid for slot in sh["dst"].values() for pid in slot}
    lost += n_particles - len(placed)
    return shared, lost


def two_tiles(n_waves=2):
    # tile 0: wavefront 0 holds the first particles of cells 3 and 4; tile 1:
    # every wavefront has particles of cell 4 (nearly sorted input)
    tiles = [[[(0, 3), (1, 4)], [(2, 4), (3, 4)]], [[(4, 4), (5, 5)], [(6, 4), (7, 4)]]]
    return tiles[:2] if n_waves == 2 else tiles


def adversary(late_wave, late_epoch):
    """Run late_wave's operations of late_epoch after everyone else's."""
    def pick(epoch, ready):
        if epoch == late_epoch and len(ready) > 1 and late_wave in ready:
            return next(w for w in ready if w != late_wave)
        return ready[0]
    return pick


def test_clear_after_the_last_barrier_loses_particles():
    tiles = two_tiles()
    n = sum(len(w) for t in tiles for w in t)
    # epoch 3 holds tile 0's clears and tile 1's rank atomics: wavefront 0
    # (which owns the rank-0 particle of cell 4) clears last
    progs, sh, _ = per_tile_programs(tiles, 2, clear_before_last_barrier=False)
    run(progs, adversary(0, 3))
    shared, lost = check(sh, n)
    assert shared > 0 and lost > 0, (shared, lost, sh["dst"])


@pytest.mark.parametrize("clear_before", [True, False])
def test_every_interleaving(clear_before):
    """In each of the seven epochs one of the two wavefronts runs all of its
    operations first, for every one of the 2^7 choices: the old ordering has
    losing schedules, the fixed one none."""
    tiles = two_tiles()
    n = sum(len(w) for t in tiles for w in t)
    bad = 0
    total = 0
    for bits in itertools.product([0, 1], repeat=7):
        def pick(epoch, ready, bits=bits):
            if len(ready) == 1:
                return ready[0]
            return ready[bits[epoch % len(bits)] % len(ready)]
        progs, sh, _ = per_tile_programs(tiles, 2, clear_before_last_barrier=clear_before)
        run(progs, pick)
        shared, lost = check(sh, n)
        bad += (shared > 0 or lost > 0)
        total += 1
    if clear_before:
        assert bad == 0
    else:
        assert bad > 0


@pytest.mark.parametrize("program", ["fixed per-tile", "per piece"])
def test_random_interleavings_keep_every_particle(program):
    rng = random.Random(7)
    for trial in range(300):
        n_waves = rng.randint(2, 4)
        n_tiles = rng.randint(1, 3)
        pid = 0
        tiles = []
        base = rng.randint(0, 5)
        for _ in range(n_tiles):
            tile = []
            for _ in range(n_waves):
                wave = []
                for _ in range(rng.randint(1, 4)):
                    wave.append((pid, base + rng.randint(0, 3)))
                    pid += 1
                tile.append(wave)
            tiles.append(tile)
        if program == "fixed per-tile":
            progs, sh, _ = per_tile_programs(tiles, n_waves, clear_before_last_barrier=True)
        else:
            progs, sh, _ = piece_programs(tiles, n_waves)
        run(progs, lambda epoch, ready: rng.choice(ready))
        assert check(sh, pid) == (0, 0), (program, trial)


def test_random_interleavings_of_the_old_ordering_lose_particles():
    rng = random.Random(11)
    losing = 0
    for trial in range(300):
        tiles = two_tiles()
        progs, sh, _ = per_tile_programs(tiles, 2, clear_before_last_barrier=False)
        run(progs, lambda epoch, ready: rng.choice(ready))
        losing += check(sh, 8) != (0, 0)
    assert losing > 0
