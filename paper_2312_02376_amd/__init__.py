"""MI355X-native FFT-PIM apply (Ai & Lomakin, FFT periodic interpolation method)."""
