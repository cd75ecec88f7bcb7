"""Pruning on the GPU (ss_prune_select, ss_gather_gaussians) against the
oracle's selection (oracle/prune.py) on the same FP32 score arrays: kept index
sets bit for bit, compacted parameters bit for bit, and the schedule of
Sec. 4.2.2-4.2.3 driven through the autograd path of a small fit."""
import numpy as np
import pytest
import torch

import scenegen
from oracle import prune as oprune

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pr():
    import paper_2412_00578_amd as ss
    from paper_2412_00578_amd import prune
    ss.lib()
    return prune


def _scores(n, seed):
    rng = np.random.default_rng(seed)
    s = (rng.standard_normal(n) ** 2 * rng.choice([1e-6, 1.0, 1e3], size=n)).astype(np.float32)
    s[rng.random(n) < 0.05] = 0.0
    s[rng.random(n) < 0.01] = -1.0
    s[rng.random(n) < 0.01] = np.nan
    s[rng.random(n) < 0.05] = np.float32(0.25)        # exact ties across the threshold
    return s


@pytest.mark.parametrize("n", [0, 1, 7, 4095, 4097, 70_001, 1_500_000])
def test_select_matches_oracle(pr, gpu_device, n):
    print(f"[case] prune select n={n}", flush=True)
    s = _scores(n, n + 3)
    t = torch.from_numpy(s).to(gpu_device)
    for ratio in (0.0, 0.3, 0.8, 1.0):
        got = pr.select(t, ratio)
        torch.cuda.synchronize()
        want = oprune.prune_select(s, ratio)
        assert np.array_equal(got.cpu().numpy().view(np.uint32), want), (n, ratio)


def test_select_on_a_pipeline_score(pr, gpu_device):
    """The score the adjoint accumulates (Sec. 4.2.1), pruned by 80 % and 30 %."""
    import paper_2412_00578_amd as ss
    print("[case] prune select on a pruning score", flush=True)
    sc, cam = scenegen.scene_c0(n=20_000, seed=4, sh_degree=1), scenegen.camera_c0()
    g = ss.Gaussians.from_scene(sc, gpu_device)
    score = ss.pruning_score(g, cam, "accutile")
    s = score.cpu().numpy()
    for ratio in (0.8, 0.3):
        got = pr.select(score, ratio).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, oprune.prune_select(s, ratio))


def test_gather_compacts_every_array(pr, gpu_device):
    import paper_2412_00578_amd as ss
    print("[case] gather", flush=True)
    sc = scenegen.scene_c0(n=50_001, seed=6, sh_degree=3)
    g = ss.Gaussians.from_scene(sc, gpu_device)
    keep_np = np.sort(np.random.default_rng(1).choice(sc.n, 12_345, replace=False)).astype(np.int32)
    keep = torch.from_numpy(keep_np).to(gpu_device)
    out = pr.gather(g, keep)
    torch.cuda.synchronize()
    for name in ("means", "scales", "quats", "opacity", "sh"):
        a = getattr(out, name).cpu().numpy()
        b = np.asarray(getattr(sc, name), np.float32)[keep_np]
        assert np.array_equal(a.reshape(b.shape), b), name
    empty = pr.gather(g, keep[:0])
    assert empty.n == 0


def test_schedule_through_a_fit(pr, gpu_device):
    """A short fit-to-target run through the autograd function with the
    paper's schedule scaled to 300 iterations: every prune keeps n -
    floor(p n) Gaussians, the kept ones are the top scores, and training
    continues on the compacted parameters."""
    import paper_2412_00578_amd as ss
    print("[case] schedule through a fit", flush=True)
    cams = scenegen.orbit_cameras(4, 12.0, 10.0, 320, 208)
    gt = ss.Gaussians.from_scene(scenegen.scene_blobs(20_000, 50), gpu_device)
    targets = [ss.Renderer(gpu_device).render(gt, c, "accutile").clone() for c in cams]
    sc = scenegen.scene_blobs(30_000, 51)
    raw = [torch.tensor(sc.means, device=gpu_device), torch.tensor(sc.scales).log().to(gpu_device),
           torch.tensor(sc.quats, device=gpu_device),
           torch.logit(torch.tensor(sc.opacity).clamp(1e-4, 1 - 1e-4)).to(gpu_device),
           torch.tensor(sc.sh, device=gpu_device)]
    events = dict((it, (r, kind)) for it, r, kind in pr.Schedule(total=300).events())
    n = want_n = sc.n
    for _, (r, _) in sorted(events.items()):
        want_n = oprune.n_keep(want_n, r)
    for it in range(300):
        if it in events:
            ratio = events[it][0]
            act = ss.Gaussians(raw[0], raw[1].exp(), raw[2], torch.sigmoid(raw[3]), raw[4], 3)
            score = sum(ss.pruning_score(act, c, "accutile") for c in cams)
            packed = ss.Gaussians(*[t.detach() for t in raw], 3)
            kept, keep = pr.prune(packed, score, ratio)
            want = oprune.prune_select(score.cpu().numpy(), ratio)
            assert np.array_equal(keep.cpu().numpy().view(np.uint32), want)
            assert kept.n == n - int(np.floor(ratio * n))
            n = kept.n
            raw = [kept.means, kept.scales, kept.quats, kept.opacity, kept.sh]
        params = [t.detach().requires_grad_(True) for t in raw]
        k = it % len(cams)
        img = ss.render(params[0], params[1].exp(), params[2], torch.sigmoid(params[3]),
                        params[4], cams[k], "accutile")
        loss = (img - targets[k]).abs().mean()
        loss.backward()
        with torch.no_grad():
            raw = [p - 1e-3 * torch.sign(p.grad) for p in params]   # signed-gradient step
    assert np.isfinite(float(loss))
    assert n == want_n
