"""MI355X-native sliding-window Gaussian splatting (SwinGS hot path)."""
