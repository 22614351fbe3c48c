"""The sliding-window stand-in for the SLAM's motion-probability maps and
the pseudo-frames at the sequence ends (Sec. 3.2, motion probability
estimation), host side (no GPU): the mirror index, the half-window failure
at the ends without pseudo-frames, and its repair."""
import numpy as np
import torch

from paper_2510_01119_amd.scene import motion_probability, pseudo_frame


def test_pseudo_frame_mirrors_the_ends():
    F = 6
    assert [pseudo_frame(j, F) for j in range(-3, 0)] == [3, 2, 1]
    assert [pseudo_frame(j, F) for j in range(F)] == list(range(F))
    assert [pseudo_frame(j, F) for j in range(F, F + 3)] == [4, 3, 2]
    # a window wider than the sequence folds back in
    assert pseudo_frame(-7, 4) == 1 and pseudo_frame(9, 4) == 3
    # one frame: every slot mirrors onto it (it shows no motion against itself)
    assert pseudo_frame(-1, 1) == 0 and pseudo_frame(2, 1) == 0
    s = torch.rand((1, 3, 3), generator=torch.Generator().manual_seed(2))
    assert torch.all(motion_probability(s, 2, 0.3, True) == 0)


def test_window_without_noise():
    """With no noise a frame's map is its own dynamic fraction times the
    share of its 2k slots that hold another frame: the first frame sees k of
    2k without pseudo-frames and 2k of 2k with them; the frame next to an end
    keeps 3 of 4 either way (its mirrored slot holds a copy of itself, which
    shows no motion)."""
    F, k = 7, 2
    s = torch.rand((F, 5, 6), generator=torch.Generator().manual_seed(1))
    plain = motion_probability(s, k, 0.0, pseudo_frames=False)
    pseudo = motion_probability(s, k, 0.0, pseudo_frames=True)
    share = np.array([(sum(0 <= i + d < F for d in (-2, -1, 1, 2))) / 4 for i in range(F)])
    assert np.allclose(share, [0.5, 0.75, 1, 1, 1, 0.75, 0.5])
    assert torch.allclose(plain, s * torch.tensor(share, dtype=s.dtype)[:, None, None])
    share_p = np.array([1, 0.75, 1, 1, 1, 0.75, 1])
    assert torch.allclose(pseudo, s * torch.tensor(share_p, dtype=s.dtype)[:, None, None])


def test_pseudo_frames_repeat_the_mirrored_pair():
    """A pseudo-frame is a copy of a real frame, so its slot repeats the
    evidence of the pair it mirrors: at frame 0 the slots -2, -1 equal +2,
    +1, so the map is the mean of the two real pairs; interior frames are
    the same with and without pseudo-frames."""
    F, k, sig = 8, 2, 0.3
    s = torch.full((F, 4, 4), 0.5)
    a = motion_probability(s, k, sig, True, torch.Generator().manual_seed(5))
    b = motion_probability(s, k, sig, False, torch.Generator().manual_seed(5))
    assert torch.allclose(a[2:F - 2], b[2:F - 2])
    # frame 0 without pseudo-frames holds half of the slots pseudo-frames fill twice
    assert torch.allclose(a[0], 2.0 * b[0])
    assert torch.allclose(a[F - 1], 2.0 * b[F - 1])
