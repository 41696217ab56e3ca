"""What the learned network gains (Hex 11x11), end to end on the GPU: the
training samples come from the library's random playouts, the network is
trained by its own forward/backward/Adam kernels, and the trained network is
judged against plain random playouts.

* value: on held-out positions the network's value is a far better
  estimate of the expected random-play outcome (the mean of 256 full random
  playouts from the position) than one full random playout, whose squared
  error is the outcome variance (about 0.9 here);
* policy: sampling moves from the network's policy beats the uniformly
  random mover from either seat (random against random: player 1 wins about
  52 % of Hex 11x11 games).

Thresholds leave room for the binomial noise of 4096 games (standard
deviation below 0.8 %) and for a short training run."""
import pytest
import torch

pytestmark = pytest.mark.gpu

ludax = pytest.importorskip("paper_2506_22609_amd.ludax")


@pytest.fixture(scope="module")
def trained():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_22609_amd import learn
    from paper_2506_22609_amd.workloads import init_net_params
    g = ludax.Game(3, 11, 11)
    data = learn.collect(g, 40000, seed=31, id_base=0)
    net = ludax.Net(11, 11, params=torch.from_numpy(init_net_params(3)).cuda())
    losses = learn.train(net, data, 1000, batch=4096, lr=1e-3, seed=1)
    return g, net, losses.cpu()


def test_training_lowers_the_value_loss(trained):
    _, _, losses = trained
    first, last = losses[:50, 0].mean().item(), losses[-50:, 0].mean().item()
    assert last < first - 0.04, (first, last)


def test_value_beats_a_single_random_playout(trained):
    from paper_2506_22609_amd import learn
    g, net, _ = trained
    ev = learn.collect(g, 600, seed=32, id_base=10**9)
    idx = torch.randperm(len(ev), generator=torch.Generator().manual_seed(0))[:2048].cuda()
    e = ev.take(idx)
    st = ludax.State(g, e.board.shape[0])
    ludax.init(g, st)
    st.board.copy_(e.board)
    st.to_move.copy_(e.to_move)
    st.ply.copy_((e.board != 0).sum(1).to(torch.int16))
    tr = learn.truth(g, st, 256, seed=33, id_base=2 * 10**9)
    one = st.clone()
    ludax.playout(g, one, 34, 3 * 10**9, stats=None)
    mse_playout = ((learn.outcome_p1(one) - tr) ** 2).mean().item()
    mse_net = ((net.estimate(st.clone()) - tr) ** 2).mean().item()
    mse_zero = (tr ** 2).mean().item()
    assert mse_net < 0.1 * mse_playout, (mse_net, mse_playout)
    assert mse_net < 0.6 * mse_zero, (mse_net, mse_zero)


@pytest.mark.parametrize("seat,need", [(1, 0.56), (2, 0.52)])
def test_policy_beats_the_random_mover(trained, seat, need):
    from paper_2506_22609_amd import learn
    g, net, _ = trained
    w, l, d = learn.play_vs_random(g, net, 4096, seat, 35, 4 * 10**9)
    assert w + l + d == 4096
    assert w / 4096 > need, (w, l, d)
