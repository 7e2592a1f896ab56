"""migrid: MI355X-native convolutional gridding and degridding."""
