"""MI355X-native ridge-directed circle Hough transform (ring detection)."""
