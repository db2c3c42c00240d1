"""MI355X-native spatio-directional mixture (SDMM) fitting, conditioning and sampling."""
