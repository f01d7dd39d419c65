"""MI355X-native Morse-Smale complex hot path (discrete gradient, critical
cells, 1-skeleton) behind a C ABI; see include/msc.h."""
