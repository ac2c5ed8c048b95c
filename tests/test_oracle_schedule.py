"""Pins for the window schedule (Algorithm 1 main/mature, Algorithm 2's
client replay, Sec. 4.2.1 slices, Fig. 5's prose example) and the per-frame
update size (Eq. 4 with Table 2's numbers).  CPU only."""
import numpy as np
import pytest

import oracle as O


def run_schedule(num_gs, swin, n_frames, deg=0):
    F = 11 + 3 * (deg + 1) ** 2
    rng = np.random.default_rng(0)
    params = rng.normal(size=(F, 2 * num_gs))
    birth, start, expire = O.genesis(num_gs, swin)
    O.schedule_expire(num_gs, swin, expire)
    records = []
    history = {}
    for st in range(1, n_frames + 1):
        rec = O.mature(st, num_gs, swin, params, birth, start, expire)
        records.append((st, rec))
        # "train" the window: perturb the optimisable slots so snapshots differ
        params[:, :num_gs] += rng.normal(size=(F, num_gs))
        history[st] = (params.copy(), birth.copy(), start.copy(), expire.copy())
    return records, history


@pytest.mark.parametrize("swin", [2, 3, 5, 10])
def test_one_slice_matures_per_frame(swin):
    num_gs = 20 * swin
    S = num_gs // swin
    records, history = run_schedule(num_gs, swin, 4 * swin)
    st, rec = records[0]
    assert len(rec["slots"]) == num_gs           # the client's first read
    for st, rec in records[1:]:
        slots = rec["slots"]
        assert len(slots) == S                   # exactly one slice per frame
        blocks = set((slots // S).tolist())
        assert len(blocks) == 1
        assert blocks.pop() == rec["birth"][0] % swin     # slice = birth mod swin
        assert np.all(rec["birth"] == rec["birth"][0])
        assert np.array_equal(slots, np.sort(slots))


@pytest.mark.parametrize("swin", [2, 3, 5, 10])
def test_every_window_frame_has_one_live_copy_per_slot(swin):
    num_gs = 10 * swin
    _, history = run_schedule(num_gs, swin, 3 * swin)
    for st, (_, birth, start, expire) in history.items():
        for f in range(st, st + swin):
            act = O.active(start, expire, f)
            per_slot = act[:num_gs].astype(int) + act[num_gs:].astype(int)
            assert np.all(per_slot == 1), (st, f)
            assert act.sum() == num_gs


def test_fig5_example_matured_and_optimisable_slices():
    """swin = 5: training frame N+1 in window [N, N+5) renders matured slices
    0, 1, 4 and optimisable slices 2, 3, and slice 2 matures after that
    window.  The reading reproduces this at N = 2 (mod 5)."""
    swin, num_gs = 5, 50
    S = num_gs // swin
    records, history = run_schedule(num_gs, swin, 20)
    for N in (7, 12, 17):
        _, birth, start, expire = history[N]     # state while training [N, N+5)
        act = O.active(start, expire, N + 1)
        opt = sorted(set((np.nonzero(act[:num_gs])[0] // S).tolist()))
        mat = sorted(set((np.nonzero(act[num_gs:])[0] // S).tolist()))
        assert opt == [2, 3] and mat == [0, 1, 4]
        _, rec = [r for r in records if r[0] == N + 1][0]
        assert set((rec["slots"] // S).tolist()) == {2}


def test_client_replay_equals_server_active_set():
    """Algorithm 2: the client keeps a buffer of num_gs slots in swin slices;
    update records are applied at their birth frame into slice birth mod swin.
    The client's live set at each frame equals the server's snapshots."""
    swin, num_gs = 4, 40
    S = num_gs // swin
    records, _ = run_schedule(num_gs, swin, 16)
    stream = [rec for _, rec in records]
    buf = {}
    first = stream[0]
    for j, slot in enumerate(first["slots"]):
        buf[int(slot)] = (first["params"][:, j], first["start"][j], first["expire"][j])
    events = stream[1:]
    for frame in range(0, 12):
        for rec in events:
            if rec["birth"][0] == frame:
                sl = rec["birth"][0] % swin
                assert np.all(rec["slots"] // S == sl)
                for j, slot in enumerate(rec["slots"]):
                    buf[int(slot)] = (rec["params"][:, j], rec["start"][j], rec["expire"][j])
        live = [s for s, (_, a, b) in buf.items() if a <= frame < b]
        assert len(live) == num_gs, frame
        # server side: the snapshot of every slot whose lifespan covers frame
        snaps = {}
        for rec in stream:
            for j, slot in enumerate(rec["slots"]):
                if rec["start"][j] <= frame < rec["expire"][j]:
                    snaps[int(slot)] = rec["params"][:, j]
        assert set(snaps) == set(live)
        for s in live:
            assert np.array_equal(buf[s][0], snaps[s])


def test_update_record_size_matches_table2():
    """Eq. 4: traffic per frame = (num_gs/swin) * bytes per Gaussian.  The
    DC-only record holds 14 FP32 values (mean 3, scale 3, rotation 4,
    opacity 1, DC colour 3) = 56 B; 200K/5 = 40K per frame -> 2.24 MB, i.e.
    the 2.1 MB (MiB) of Table 2.  With Table 6's precisions (fp16 mean and
    scale, uint8 rotation and opacity, full-precision DC) 29 B -> 1.16 MB,
    the 1.2 MB of the quantised row."""
    per_frame = 200_000 // 5
    assert per_frame == 40_000
    full = per_frame * 14 * 4
    assert round(full / 2 ** 20, 1) == 2.1
    quant = per_frame * (3 * 2 + 3 * 2 + 4 * 1 + 1 * 1 + 3 * 4)
    assert round(quant / 1e6, 1) == 1.2
