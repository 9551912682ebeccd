"""Run as a script by test_gpu_boundary.py in a fresh process: sdm_init on one
stream returns while a long spin still runs on another.

A fresh process is used because the HIP runtime maps streams onto a few
hardware queues (GPU_MAX_HW_QUEUES, 4 by default) in the order of their first
use; once a process has used more streams than that, two streams can share a
queue, and synchronising one then also waits for the other's work.  Here only
torch's default stream (the uploads), `side` and `busy` are ever used, so the
three sit on different queues.  Every device buffer is made, and used once by
an untimed sdm_init on `side`, before the first spin.  Exit status 0 when
sdm_init returned before the spin ended in every repetition."""
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    import torch

    from paper_2103_17238_amd import binding as B
    from paper_2103_17238_amd import inputs as I

    st = I.random_cells(8, 100, rng_seed=5)
    cfg = B.make_config(st.n_slots, st.n_cells, st.n_attr, st.dt, st.dv, st.kernel,
                        st.adaptive, st.b, st.seed)
    xi = torch.from_numpy(st.xi).cuda()
    v = torch.from_numpy(st.v).cuda()
    off = torch.from_numpy(st.cell_off).cuda()
    ws = B.workspace_tensor(B.sdm_workspace_bytes(cfg, st.cell_off))
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    B.sdm_free(B.sdm_init(cfg, xi, v, None, off, ws, side))
    side.synchronize()
    busy = torch.cuda.Stream()
    ok = True
    for rep in range(3):
        with torch.cuda.stream(busy):
            torch.cuda._sleep(400_000_000)
        ev = torch.cuda.Event()
        ev.record(busy)
        t0 = time.perf_counter()
        h = B.sdm_init(cfg, xi, v, None, off, ws, side)
        dt_init = time.perf_counter() - t0
        still_busy = not ev.query()
        busy.synchronize()
        dt_all = time.perf_counter() - t0
        print(f"rep {rep}: sdm_init {dt_init * 1e3:.2f} ms while the spin ran "
              f"{dt_all * 1e3:.2f} ms; spin still running at return: {still_busy}", flush=True)
        ok = ok and still_busy
        B.sdm_free(h)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main())
