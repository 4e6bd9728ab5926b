"""The work order of the persistent forward, checked on the host: every (stage, slot, tile) once, every
item after the items it reads, and a simulated run of workgroups that claim items in that order and wait
for their dependencies finishes for any number of workgroups (no deadlock), with the slots of early
groups finishing first."""
import heapq

import numpy as np
import pytest

from paper_2409_02912_amd import synth

L = pytest.importorskip("paper_2409_02912_amd.libnrx")

CONV_KINDS = (0, 1, 2)


def _ragged(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        U = int(rng.integers(1, 5))
        out.append(dict(n_prb=int(rng.integers(4, 274)), n_ant=int(rng.choice([4, 8])), n_ue=U,
                        bits=[int(b) for b in rng.choice([2, 4, 6, 8], U)], slot_number=i % 20))
    return out


BATCHES = {
    "headline_like": [dict(n_prb=273, n_ant=8, n_ue=4, bits=[4] * 4, slot_number=i) for i in range(3)],
    "ragged": _ragged(24, 5),
    "three_ue_small": [dict(n_prb=p, n_ant=4, n_ue=3, bits=[2, 4, 6]) for p in (1, 2, 7, 30)],
    "one_slot": [dict(n_prb=1, n_ant=4, n_ue=1, bits=[2])],
}


def _deps(kinds, item, n_tiles):
    """(stage, slot, tile) triples an item (stage, slot, first tile, tiles) waits for."""
    stage, slot, ta, nt = item
    if stage == 0:
        return []
    tb = ta + nt
    if kinds[stage] in CONV_KINDS:
        return [(stage - 1, slot, t) for t in range(max(ta - 1, 0), min(tb, n_tiles[slot] - 1) + 1)]
    return [(stage - 1, slot, t) for t in range(ta, tb)]


def _simulate(items, kinds, n_tiles, n_wg, seed):
    """Event simulation: n_wg workgroups claim items in list order; an item starts once the tiles it depends
    on are finished and takes a random time.  Raises on deadlock (workgroups waiting, nothing running)."""
    rng = np.random.default_rng(seed)
    owner = {}
    for i, (st, sl, ta, nt) in enumerate(items):
        for t in range(ta, ta + nt):
            owner[(st, sl, t)] = i
    finished = set()
    waiting = {}            # item index -> workgroup, blocked on dependencies
    events = []             # (time, workgroup, item index)
    nxt = 0
    now = 0.0
    for wg in range(min(n_wg, len(items))):
        waiting[nxt] = wg
        nxt += 1

    def try_start():
        started = True
        while started:
            started = False
            for i in sorted(waiting):
                deps = {owner[d] for d in _deps(kinds, items[i], n_tiles)}
                assert all(d < i for d in deps)
                if deps <= finished:
                    wg = waiting.pop(i)
                    heapq.heappush(events, (now + float(rng.uniform(0.5, 2.0)), wg, i))
                    started = True
    try_start()
    while events:
        now, wg, i = heapq.heappop(events)
        finished.add(i)
        if nxt < len(items):
            waiting[nxt] = wg
            nxt += 1
        try_start()
        if not events and waiting:
            raise AssertionError(f"deadlock: {len(waiting)} workgroups wait, e.g. item {min(waiting)}")
    assert len(finished) == len(items)


@pytest.mark.parametrize("net", [(8, 128, 6, 2, 4), (4, 128, 8, 3, 8), (4, 128, 2, 0, 2)])
@pytest.mark.parametrize("batch", sorted(BATCHES))
def test_persistent_work_order(batch, net):
    B, d, C, R, m = net
    shapes = [dict(s, n_ant=min(s["n_ant"], B), bits=[min(b, m) for b in s["bits"]]) for s in BATCHES[batch]]
    model = L.nrx_model_create(B, d, C, R, m, L.NRX_BF16, flags=8)
    try:
        descs, _ = L.make_slots(shapes, m)
        st, sl, ti, nt, kinds = L.nrx_persist_schedule(model, descs)
    finally:
        L.nrx_model_destroy(model)
    # stages: StateInit, R message-passing rounds, two convs per block, readout
    assert len(kinds) == 2 + R + 2 * C
    assert kinds[0] == 0 and kinds[-1] == 4 and list(kinds).count(3) == R
    # tiles of whole REs, at most 512 rows; items of at most 4 consecutive tiles
    n_tiles = []
    for s in shapes:
        U = s["n_ue"]
        tr = (512 // U) * U
        n_tiles.append(-(-12 * s["n_prb"] * 14 * U // tr))
    assert np.all((nt >= 1) & (nt <= 4))
    items = list(zip(st.tolist(), sl.tolist(), ti.tolist(), nt.tolist()))
    covered = [(k, s, t) for (k, s, ta, n) in items for t in range(ta, ta + n)]
    expect = {(k, s, t) for k in range(len(kinds)) for s in range(len(shapes)) for t in range(n_tiles[s])}
    assert len(covered) == len(expect) and set(covered) == expect
    owner = {}
    for i, (k, s, ta, n) in enumerate(items):
        for t in range(ta, ta + n):
            owner[(k, s, t)] = i
    for i, it in enumerate(items):
        for dep in _deps(kinds, it, n_tiles):
            assert owner[dep] < i, (it, dep)
    # slots finish group by group: a slot's last readout comes before every item of later groups' slots
    last_ro = [max(owner[(len(kinds) - 1, s, t)] for t in range(n_tiles[s])) for s in range(len(shapes))]
    first_any = [min(owner[(0, s, t)] for t in range(n_tiles[s])) for s in range(len(shapes))]
    for a in range(len(shapes)):
        for b in range(len(shapes)):
            if first_any[b] > last_ro[a]:
                assert b > a
    for n_wg in (1, 3, 256):
        _simulate(items, kinds, n_tiles, n_wg, seed=n_wg)


def test_persistent_flag_needs_bf16_shared_layers():
    for prec, flags in ((L.NRX_FP32, 8), (L.NRX_FP8, 8), (L.NRX_BF16, 8 | 4)):
        with pytest.raises(L.NrxError) as e:
            L.nrx_model_create(4, 128, 2, 1, 4, prec, flags=flags)
        assert e.value.status == L.NRX_ERR_UNSUPPORTED
    with pytest.raises(L.NrxError) as e:
        L.nrx_model_create(4, 128, 2, 1, 4, L.NRX_BF16, flags=16)
    assert e.value.status == L.NRX_ERR_INVALID
    m = L.nrx_model_create(4, 128, 2, 1, 4, L.NRX_BF16, flags=0)
    try:
        descs, _ = L.make_slots([dict(n_prb=4, n_ant=4, n_ue=1, bits=[2])], 4)
        with pytest.raises(L.NrxError):
            L.nrx_persist_schedule(m, descs)
    finally:
        L.nrx_model_destroy(m)


def test_persistent_groups_of_the_uneven_workload():
    # the uneven 256-slot workload splits into many slot groups, so most slots finish well before the batch
    shapes = synth.ragged_shapes(256, seed=0)
    model = L.nrx_model_create(16, 128, 6, 2, 8, L.NRX_BF16, flags=8)
    try:
        descs, _ = L.make_slots(shapes, 8)
        st, sl, ti, nt, kinds = L.nrx_persist_schedule(model, descs)
    finally:
        L.nrx_model_destroy(model)
    ro = np.nonzero(st == len(kinds) - 1)[0]
    last = np.zeros(len(shapes))
    np.maximum.at(last, sl[ro], ro)
    frac = last / len(st)
    assert np.median(frac) < 0.6 and frac.max() == (len(st) - 1) / len(st)
