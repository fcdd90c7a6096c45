"""Host-side checks of the video trackers' inputs (no GPU): a frame of the
wrong size, type or layout is refused before any upload, since the upload
copies H * W bytes from it into a device frame of that size."""
import numpy as np
import pytest
import torch

from paper_1910_06017_amd import video


def test_frames_of_the_tracker_size_pass():
    video._check_frames([torch.zeros((4, 6), dtype=torch.uint8) for _ in range(3)], 6, 4)


@pytest.mark.parametrize("bad", [
    torch.zeros((4, 7), dtype=torch.uint8),          # wrong width
    torch.zeros((5, 6), dtype=torch.uint8),          # wrong height
    torch.zeros((4, 6), dtype=torch.float32),        # wrong type
    torch.zeros((6, 4), dtype=torch.uint8).t(),      # right shape, not contiguous
    torch.zeros((2, 4, 6), dtype=torch.uint8),       # a stack, not a frame
    np.zeros((4, 6), dtype=np.uint8),                # not a tensor
])
def test_bad_frames_are_refused(bad):
    frames = [torch.zeros((4, 6), dtype=torch.uint8), bad]
    with pytest.raises(ValueError, match="frame 1"):
        video._check_frames(frames, 6, 4)


def test_boxes_must_be_m_by_4():
    video._check_boxes(np.zeros((3, 4), np.float32), 0)
    video._check_boxes(np.zeros((0, 4), np.float32), 0)
    for bad in (np.zeros(4, np.float32), np.zeros((3, 5), np.float32)):
        with pytest.raises(ValueError, match="seeds"):
            video._check_boxes(bad, 2)
